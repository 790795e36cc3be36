/*
 * Plain FP64 CPU oracle for the axisymmetric drift-diffusion fluid solver of
 * Ristivojevic & Petrovic, "Multigrid solver for axisymmetrical 2D fluid
 * equations" (arXiv:0811.4446).
 *
 * TEST INFRASTRUCTURE ONLY.  It exists to check the HIP library.  Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no source, header, table or helper with the HIP library.
 *
 * Layout: every field is a dense (nr+1) x (nz+1) row-major array of doubles.
 * Node (i, j) is at index i*(nz+1) + j.  i is the radial node (r_i = i*dr,
 * i = 0..nr), j the axial node (z_j given, j = 0..nz).  Rows j = 0 and j = nz
 * are electrode (Dirichlet) nodes; the unknowns are i = 0..nr, j = 1..nz-1.
 *
 * Every operator is stored in finite-volume (integrated) form with five
 * coefficients named after the blocks of the paper's linearised system
 * (Sec. 2, Eq. 14):
 *     a*x[i-1][j] + b*x[i][j] + c*x[i+1][j] + d*x[i][j-1] + e*x[i][j+1] = f
 * i.e. each row is the balance over the control volume of node (i, j).
 *
 * Control volumes (Sec. 2, grid definition): the radial extent of the cell of
 * node i is [r_{i-1/2}, r_{i+1/2}] clipped to [0, R]; the axial extent is
 * [z_{j-1/2}, z_{j+1/2}] with z_{j+1/2} the midpoint.  Per radian of azimuth:
 *     radial width  w_0 = dr^2/8,  w_i = r_i*dr,  w_nr = dr*(R - dr/4)/2
 *     axial width   dzc_j = (dz_{j-1} + dz_j)/2      (the paper's delta z)
 *     volume        vol_ij = w_i * dzc_j
 *     r-face i+1/2  area r_{i+1/2} * dzc_j
 *     z-face j+1/2  area w_i
 * With these widths the rows reproduce Eq. (12) and the axis row Eq. (13)
 * after division by vol and multiplication by -dr^2.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, nz) ((size_t)(i) * (size_t)((nz) + 1) + (size_t)(j))

/* ------------------------------------------------------------------ */
/* Geometry (Sec. 2: equidistant r nodes, non-equidistant z nodes).    */
/* ------------------------------------------------------------------ */

static double radial_width(int i, int nr, double R)
{
    double dr = R / nr;
    if (i == 0)
        return dr * dr / 8.0;
    if (i == nr)
        return 0.5 * dr * (R - 0.25 * dr);
    return (i * dr) * dr;
}

/* r_{i+1/2}: radius of the face between nodes i and i+1. */
static double face_radius(int i, int nr, double R)
{
    double dr = R / nr;
    return (i + 0.5) * dr;
}

/* Axial control-volume width of node j (1 <= j <= nz-1). */
static double axial_width(const double *z, int j)
{
    return 0.5 * (z[j + 1] - z[j - 1]);
}

double or_volume(int nr, int nz, double R, const double *z, int i, int j)
{
    (void)nz;
    return radial_width(i, nr, R) * axial_width(z, j);
}

/* ------------------------------------------------------------------ */
/* Bernoulli functions of the Scharfetter-Gummel flux (Sec. 2, F and G  */
/* after Eq. 11): F(x) = x/(exp(x)-1), G(x) = x exp(x)/(exp(x)-1).      */
/* G(x) = F(-x).  Near x = 0 the quotient cancels, so the Taylor series */
/* 1 - x/2 + x^2/12 - x^4/720 is used for |x| < 1e-3 (next term        */
/* x^6/30240 is below 1e-22).                                           */
/* ------------------------------------------------------------------ */

double or_bernoulli_F(double x)
{
    if (fabs(x) < 1e-3) {
        double x2 = x * x;
        return 1.0 - 0.5 * x + x2 / 12.0 - x2 * x2 / 720.0;
    }
    return x / expm1(x);
}

double or_bernoulli_G(double x)
{
    return or_bernoulli_F(-x);
}

/* ------------------------------------------------------------------ */
/* Poisson operator, Eq. (5) discretised as Eqs. (12)-(13).            */
/* Row (FV form): sum over faces area/dist*(V - V_nb)                   */
/*                = vol * k * (n_p - n_e),                              */
/* i.e. -div grad V = k (n_p - n_e) with k = e n0 / eps0.               */
/* r = 0: the axis face has zero area (the paper's axis row, Eq. 13).   */
/* r = R: no face (zero radial flux, half control volume).             */
/* The electrode rows are not assembled (their coefficients are zero). */
/* ------------------------------------------------------------------ */

/* wall != 0: Dirichlet wall at r = R (the paper's experiment, Sec. 3): the
 * nodes i = nr are fixed, their rows are the identity with right-hand side
 * Vwall[j] (NULL: 0, the correction equations of the coarse levels). */
void or_poisson_assemble_w(int nr, int nz, double R, const double *z, double k,
                           const double *ne, const double *np, int wall,
                           const double *Vwall, double *a, double *b, double *c,
                           double *d, double *e, double *f);

void or_poisson_assemble(int nr, int nz, double R, const double *z, double k,
                         const double *ne, const double *np,
                         double *a, double *b, double *c, double *d, double *e,
                         double *f)
{
    or_poisson_assemble_w(nr, nz, R, z, k, ne, np, 0, NULL, a, b, c, d, e, f);
}

void or_poisson_assemble_w(int nr, int nz, double R, const double *z, double k,
                           const double *ne, const double *np, int wall,
                           const double *Vwall, double *a, double *b, double *c,
                           double *d, double *e, double *f)
{
    double dr = R / nr;
    size_t n = (size_t)(nr + 1) * (nz + 1);
    memset(a, 0, n * sizeof(double));
    memset(b, 0, n * sizeof(double));
    memset(c, 0, n * sizeof(double));
    memset(d, 0, n * sizeof(double));
    memset(e, 0, n * sizeof(double));
    memset(f, 0, n * sizeof(double));
    for (int i = 0; i <= nr; ++i) {
        double w = radial_width(i, nr, R);
        for (int j = 1; j < nz; ++j) {
            size_t p = IDX(i, j, nz);
            if (wall && i == nr) {
                b[p] = 1.0;
                f[p] = Vwall ? Vwall[j] : 0.0;
                continue;
            }
            double dzc = axial_width(z, j);
            double ca = (i > 0) ? face_radius(i - 1, nr, R) * dzc / dr : 0.0;
            double cc = (i < nr) ? face_radius(i, nr, R) * dzc / dr : 0.0;
            double cd = w / (z[j] - z[j - 1]);
            double ce = w / (z[j + 1] - z[j]);
            a[p] = -ca;
            c[p] = -cc;
            d[p] = -cd;
            e[p] = -ce;
            b[p] = ca + cc + cd + ce;
            if (ne && np)
                f[p] = w * dzc * k * (np[p] - ne[p]);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Scharfetter-Gummel backward-Euler continuity operator, Eqs. (7)-(11). */
/* Row (FV form):                                                       */
/*   vol*(n - n^k)/dt + sum over faces area*phi_out = vol*S            */
/* Flux through face i+1/2 in +r (Eq. 8), per unit area:               */
/*   phi = D/dr * (n_i G(alpha) - n_{i+1} F(alpha)),                    */
/*   alpha = -s mu/D (V_{i+1} - V_i),  s = -1 electrons, +1 ions.       */
/* Axial flux through z_{j+1/2} in +z (Eq. 9) has the same form with    */
/* dz_j; its second term uses F (the printed G there cannot reduce to   */
/* the SG scheme, which needs zero flux for uniform n at alpha = 0).    */
/* dt_inv = 1/dt (0 gives the steady operator).                         */
/* ------------------------------------------------------------------ */

/* wall != 0: Dirichlet wall at r = R with density 0 there (Sec. 3): the
 * rows i = nr are the identity with right-hand side 0. */
void or_sg_assemble_w(int nr, int nz, double R, const double *z, int s,
                      double mu, double D, double dt_inv, int wall,
                      const double *V, const double *nk, const double *S,
                      double *a, double *b, double *c, double *d, double *e,
                      double *f);
/* mun, Dn non-NULL: node values of the mobility and the diffusion
 * coefficient (Sec. 2: field-dependent, supplied by lookup tables or a Monte
 * Carlo code); every face uses the arithmetic mean of its two nodes, and
 * alpha = -s mu_face/D_face (V_nb - V). */
void or_sg_assemble_t(int nr, int nz, double R, const double *z, int s,
                      double mu, double D, double dt_inv, int wall,
                      const double *mun, const double *Dn, const double *V,
                      const double *nk, const double *S, double *a, double *b,
                      double *c, double *d, double *e, double *f);

void or_sg_assemble(int nr, int nz, double R, const double *z, int s,
                    double mu, double D, double dt_inv,
                    const double *V, const double *nk, const double *S,
                    double *a, double *b, double *c, double *d, double *e,
                    double *f)
{
    or_sg_assemble_w(nr, nz, R, z, s, mu, D, dt_inv, 0, V, nk, S, a, b, c, d, e, f);
}

void or_sg_assemble_w(int nr, int nz, double R, const double *z, int s,
                      double mu, double D, double dt_inv, int wall,
                      const double *V, const double *nk, const double *S,
                      double *a, double *b, double *c, double *d, double *e,
                      double *f)
{
    or_sg_assemble_t(nr, nz, R, z, s, mu, D, dt_inv, wall, NULL, NULL, V, nk, S,
                     a, b, c, d, e, f);
}

/* Face coefficients: D of the face and q = -s mu/D, from the constants or
 * from the means of the two nodes' values. */
static void face_coef(int s, double mu, double D, const double *mun,
                      const double *Dn, size_t p, size_t pn, double *Df,
                      double *qf)
{
    if (mun && Dn) {
        double m = 0.5 * (mun[p] + mun[pn]);
        *Df = 0.5 * (Dn[p] + Dn[pn]);
        *qf = -(double)s * m / *Df;
    } else {
        *Df = D;
        *qf = -(double)s * mu / D;
    }
}

void or_sg_assemble_t(int nr, int nz, double R, const double *z, int s,
                      double mu, double D, double dt_inv, int wall,
                      const double *mun, const double *Dn, const double *V,
                      const double *nk, const double *S, double *a, double *b,
                      double *c, double *d, double *e, double *f)
{
    double dr = R / nr;
    size_t n = (size_t)(nr + 1) * (nz + 1);
    memset(a, 0, n * sizeof(double));
    memset(b, 0, n * sizeof(double));
    memset(c, 0, n * sizeof(double));
    memset(d, 0, n * sizeof(double));
    memset(e, 0, n * sizeof(double));
    memset(f, 0, n * sizeof(double));
    for (int i = 0; i <= nr; ++i) {
        double w = radial_width(i, nr, R);
        for (int j = 1; j < nz; ++j) {
            size_t p = IDX(i, j, nz);
            if (wall && i == nr) {
                b[p] = 1.0;
                continue;
            }
            double dzc = axial_width(z, j);
            double vol = w * dzc;
            double diag = vol * dt_inv;
            double Df, q;
            if (i < nr) { /* face i+1/2 */
                size_t pn = IDX(i + 1, j, nz);
                face_coef(s, mu, D, mun, Dn, p, pn, &Df, &q);
                double g = face_radius(i, nr, R) * dzc * Df / dr;
                double al = q * (V[pn] - V[p]);
                c[p] = -g * or_bernoulli_F(al);
                diag += g * or_bernoulli_G(al);
            }
            if (i > 0) { /* face i-1/2, outward is -r */
                size_t pn = IDX(i - 1, j, nz);
                face_coef(s, mu, D, mun, Dn, p, pn, &Df, &q);
                double g = face_radius(i - 1, nr, R) * dzc * Df / dr;
                double al = q * (V[p] - V[pn]);
                a[p] = -g * or_bernoulli_G(al);
                diag += g * or_bernoulli_F(al);
            }
            { /* face j+1/2 */
                size_t pn = IDX(i, j + 1, nz);
                face_coef(s, mu, D, mun, Dn, p, pn, &Df, &q);
                double g = w * Df / (z[j + 1] - z[j]);
                double al = q * (V[pn] - V[p]);
                e[p] = -g * or_bernoulli_F(al);
                diag += g * or_bernoulli_G(al);
            }
            { /* face j-1/2 */
                size_t pn = IDX(i, j - 1, nz);
                face_coef(s, mu, D, mun, Dn, p, pn, &Df, &q);
                double g = w * Df / (z[j] - z[j - 1]);
                double al = q * (V[p] - V[pn]);
                d[p] = -g * or_bernoulli_G(al);
                diag += g * or_bernoulli_F(al);
            }
            b[p] = diag;
            f[p] = vol * ((S ? S[p] : 0.0) + (nk ? nk[p] * dt_inv : 0.0));
        }
    }
}

/* ------------------------------------------------------------------ */
/* Operator application and residual on the unknown nodes.             */
/* ------------------------------------------------------------------ */

static double row_apply(int nr, int nz, const double *a, const double *b,
                        const double *c, const double *d, const double *e,
                        const double *x, int i, int j)
{
    size_t p = IDX(i, j, nz);
    double s = b[p] * x[p] + d[p] * x[p - 1] + e[p] * x[p + 1];
    if (i > 0)
        s += a[p] * x[IDX(i - 1, j, nz)];
    if (i < nr)
        s += c[p] * x[IDX(i + 1, j, nz)];
    return s;
}

/* y = A x on unknown nodes, 0 on electrode rows. */
void or_apply(int nr, int nz, const double *a, const double *b, const double *c,
              const double *d, const double *e, const double *x, double *y)
{
    for (int i = 0; i <= nr; ++i) {
        y[IDX(i, 0, nz)] = 0.0;
        y[IDX(i, nz, nz)] = 0.0;
        for (int j = 1; j < nz; ++j)
            y[IDX(i, j, nz)] = row_apply(nr, nz, a, b, c, d, e, x, i, j);
    }
}

/* r = f - A x on unknown nodes, 0 on electrode rows. */
void or_residual(int nr, int nz, const double *a, const double *b,
                 const double *c, const double *d, const double *e,
                 const double *f, const double *x, double *r)
{
    for (int i = 0; i <= nr; ++i) {
        r[IDX(i, 0, nz)] = 0.0;
        r[IDX(i, nz, nz)] = 0.0;
        for (int j = 1; j < nz; ++j)
            r[IDX(i, j, nz)] =
                f[IDX(i, j, nz)] - row_apply(nr, nz, a, b, c, d, e, x, i, j);
    }
}

/*
 * Relative residual in strong form (every row divided by its volume):
 *   || (f - A x)/vol ||_2 / || b_eff/vol ||_2
 * where b_eff = f minus the electrode-row terms of the rows next to the
 * electrodes (the right-hand side of the system in the unknowns alone).
 * If b_eff is zero the absolute strong-form residual norm is returned.
 */
double or_relres(int nr, int nz, double R, const double *z, const double *a,
                 const double *b, const double *c, const double *d,
                 const double *e, const double *f, const double *x)
{
    double rr = 0.0, bb = 0.0;
    for (int i = 0; i <= nr; ++i) {
        for (int j = 1; j < nz; ++j) {
            size_t p = IDX(i, j, nz);
            double vol = or_volume(nr, nz, R, z, i, j);
            double r = (f[p] - row_apply(nr, nz, a, b, c, d, e, x, i, j)) / vol;
            double be = f[p];
            if (j == 1)
                be -= d[p] * x[p - 1];
            if (j == nz - 1)
                be -= e[p] * x[p + 1];
            be /= vol;
            rr += r * r;
            bb += be * be;
        }
    }
    if (bb == 0.0)
        return sqrt(rr);
    return sqrt(rr / bb);
}

/* ------------------------------------------------------------------ */
/* Smoothers.  The paper names Gauss-Seidel among classical solvers     */
/* (Sec. 2, before Fig. 1); the multigrid details are not given there.  */
/* ------------------------------------------------------------------ */

/* One half-sweep of red-black point Gauss-Seidel: update every unknown
 * node with (i + j) % 2 == colour using the current neighbour values. */
void or_rbgs(int nr, int nz, const double *a, const double *b, const double *c,
             const double *d, const double *e, const double *f, double *x,
             int colour)
{
    for (int i = 0; i <= nr; ++i) {
        for (int j = 1; j < nz; ++j) {
            if (((i + j) & 1) != colour)
                continue;
            size_t p = IDX(i, j, nz);
            double s = f[p] - d[p] * x[p - 1] - e[p] * x[p + 1];
            if (i > 0)
                s -= a[p] * x[IDX(i - 1, j, nz)];
            if (i < nr)
                s -= c[p] * x[IDX(i + 1, j, nz)];
            x[p] = s / b[p];
        }
    }
}

/* One half-sweep of zebra z-line Gauss-Seidel: for every radial line i
 * with i % 2 == parity solve the tridiagonal system in j exactly
 * (Thomas algorithm), the neighbouring lines i-1 and i+1 held fixed.
 * work must hold 2*(nz+1) doubles. */
void or_zline(int nr, int nz, const double *a, const double *b, const double *c,
              const double *d, const double *e, const double *f, double *x,
              int parity, double *work)
{
    double *cp = work;          /* modified super-diagonal */
    double *rp = work + nz + 1; /* modified right-hand side */
    for (int i = parity; i <= nr; i += 2) {
        /* forward elimination over j = 1..nz-1 */
        for (int j = 1; j < nz; ++j) {
            size_t p = IDX(i, j, nz);
            double rhs = f[p];
            if (i > 0)
                rhs -= a[p] * x[IDX(i - 1, j, nz)];
            if (i < nr)
                rhs -= c[p] * x[IDX(i + 1, j, nz)];
            double sup = e[p];
            if (j == 1)
                rhs -= d[p] * x[p - 1]; /* electrode value */
            if (j == nz - 1) {
                rhs -= e[p] * x[p + 1];
                sup = 0.0;
            }
            if (j == 1) {
                cp[j] = sup / b[p];
                rp[j] = rhs / b[p];
            } else {
                double m = b[p] - d[p] * cp[j - 1];
                cp[j] = sup / m;
                rp[j] = (rhs - d[p] * rp[j - 1]) / m;
            }
        }
        /* back substitution */
        x[IDX(i, nz - 1, nz)] = rp[nz - 1];
        for (int j = nz - 2; j >= 1; --j)
            x[IDX(i, j, nz)] = rp[j] - cp[j] * x[IDX(i, j + 1, nz)];
    }
}

/* ------------------------------------------------------------------ */
/* Grid transfer between nested grids (coarse node (I,J) = fine node    */
/* (2I,2J); the coarse z nodes are every second fine z node).           */
/* Prolongation P: bilinear, with weights 1/2 in r (equidistant) and     */
/* weights by distance in z (non-equidistant).  Restriction = P^T,       */
/* applied to finite-volume (integrated) residuals.                     */
/* ------------------------------------------------------------------ */

/* Weight of the lower coarse node J for the fine node 2J+1. */
static double zweight_lower(const double *zf, int J)
{
    double h0 = zf[2 * J + 1] - zf[2 * J];
    double h1 = zf[2 * J + 2] - zf[2 * J + 1];
    return h1 / (h0 + h1);
}

/* xf += P ec on the fine unknown nodes (fine grid nrf x nzf). */
void or_prolong_add(int nrf, int nzf, const double *zf, const double *ec,
                    double *xf)
{
    int nzc = nzf / 2;
    for (int i = 0; i <= nrf; ++i) {
        for (int j = 1; j < nzf; ++j) {
            double v;
            /* value along the coarse z lines of the two radial parents */
            int I0 = i / 2, I1 = (i + 1) / 2;
            double cv[2];
            int Is[2] = {I0, I1};
            for (int t = 0; t < 2; ++t) {
                int I = Is[t];
                if (j % 2 == 0) {
                    cv[t] = ec[IDX(I, j / 2, nzc)];
                } else {
                    int J = j / 2;
                    double wl = zweight_lower(zf, J);
                    cv[t] = wl * ec[IDX(I, J, nzc)] + (1.0 - wl) * ec[IDX(I, J + 1, nzc)];
                }
            }
            if (i % 2 == 0)
                v = cv[0];
            else
                v = 0.5 * (cv[0] + cv[1]);
            xf[IDX(i, j, nzf)] += v;
        }
    }
}

/* fc = P^T rf (rf zero on fine electrode rows); coarse electrode rows 0. */
void or_restrict(int nrf, int nzf, const double *zf, const double *rf,
                 double *fc)
{
    int nrc = nrf / 2, nzc = nzf / 2;
    memset(fc, 0, (size_t)(nrc + 1) * (nzc + 1) * sizeof(double));
    for (int i = 0; i <= nrf; ++i) {
        for (int j = 1; j < nzf; ++j) {
            double r = rf[IDX(i, j, nzf)];
            /* scatter r to the coarse nodes with the prolongation weights */
            int nI = (i % 2 == 0) ? 1 : 2;
            int Is[2] = {i / 2, (i + 1) / 2};
            double wi[2] = {(i % 2 == 0) ? 1.0 : 0.5, 0.5};
            int nJ = (j % 2 == 0) ? 1 : 2;
            int Js[2];
            double wj[2];
            if (j % 2 == 0) {
                Js[0] = j / 2;
                wj[0] = 1.0;
            } else {
                int J = j / 2;
                double wl = zweight_lower(zf, J);
                Js[0] = J;
                wj[0] = wl;
                Js[1] = J + 1;
                wj[1] = 1.0 - wl;
            }
            for (int s = 0; s < nI; ++s)
                for (int t = 0; t < nJ; ++t)
                    fc[IDX(Is[s], Js[t], nzc)] += wi[s] * wj[t] * r;
        }
    }
    for (int I = 0; I <= nrc; ++I) {
        fc[IDX(I, 0, nzc)] = 0.0;
        fc[IDX(I, nzc, nzc)] = 0.0;
    }
}

/* ------------------------------------------------------------------ */
/* Direct solve of the whole system (coarsest grid): dense Gaussian     */
/* elimination with partial pivoting over the (nr+1)*(nz-1) unknowns.   */
/* The electrode values in x enter the right-hand side.                */
/* Returns 0, or -1 if a pivot is zero.                                 */
/* ------------------------------------------------------------------ */

int or_direct_solve(int nr, int nz, const double *a, const double *b,
                    const double *c, const double *d, const double *e,
                    const double *f, double *x)
{
    int m = nz - 1;
    int n = (nr + 1) * m;
    double *M = calloc((size_t)n * n, sizeof(double));
    double *rhs = calloc((size_t)n, sizeof(double));
    if (!M || !rhs) {
        free(M);
        free(rhs);
        return -1;
    }
#define U(i, j) ((i) * m + ((j) - 1))
    for (int i = 0; i <= nr; ++i) {
        for (int j = 1; j < nz; ++j) {
            size_t p = IDX(i, j, nz);
            int row = U(i, j);
            M[(size_t)row * n + row] = b[p];
            rhs[row] = f[p];
            if (i > 0)
                M[(size_t)row * n + U(i - 1, j)] = a[p];
            if (i < nr)
                M[(size_t)row * n + U(i + 1, j)] = c[p];
            if (j > 1)
                M[(size_t)row * n + U(i, j - 1)] = d[p];
            else
                rhs[row] -= d[p] * x[p - 1];
            if (j < nz - 1)
                M[(size_t)row * n + U(i, j + 1)] = e[p];
            else
                rhs[row] -= e[p] * x[p + 1];
        }
    }
    int status = 0;
    for (int k = 0; k < n && status == 0; ++k) {
        int piv = k;
        for (int r = k + 1; r < n; ++r)
            if (fabs(M[(size_t)r * n + k]) > fabs(M[(size_t)piv * n + k]))
                piv = r;
        if (M[(size_t)piv * n + k] == 0.0) {
            status = -1;
            break;
        }
        if (piv != k) {
            for (int t = 0; t < n; ++t) {
                double tmp = M[(size_t)k * n + t];
                M[(size_t)k * n + t] = M[(size_t)piv * n + t];
                M[(size_t)piv * n + t] = tmp;
            }
            double tmp = rhs[k];
            rhs[k] = rhs[piv];
            rhs[piv] = tmp;
        }
        for (int r = k + 1; r < n; ++r) {
            double l = M[(size_t)r * n + k] / M[(size_t)k * n + k];
            if (l == 0.0)
                continue;
            for (int t = k; t < n; ++t)
                M[(size_t)r * n + t] -= l * M[(size_t)k * n + t];
            rhs[r] -= l * rhs[k];
        }
    }
    if (status == 0) {
        for (int k = n - 1; k >= 0; --k) {
            double s = rhs[k];
            for (int t = k + 1; t < n; ++t)
                s -= M[(size_t)k * n + t] * rhs[t];
            rhs[k] = s / M[(size_t)k * n + k];
        }
        for (int i = 0; i <= nr; ++i)
            for (int j = 1; j < nz; ++j)
                x[IDX(i, j, nz)] = rhs[U(i, j)];
    }
#undef U
    free(M);
    free(rhs);
    return status;
}

/* ------------------------------------------------------------------ */
/* Multigrid hierarchy.  The paper applies "the multigrid method" to    */
/* its linear systems (Sec. 2, the paragraph after Eq. 14) without      */
/* giving the cycle; the components here are the plain textbook ones:   */
/* V(nu1, nu2) cycle, Gauss-Seidel smoothing (red-black points or zebra */
/* z-lines), restriction P^T, bilinear prolongation P, coarse operators */
/* rediscretised on the nested coarse grids (potential injected), and   */
/* a direct solve on the coarsest grid.                                 */
/* ------------------------------------------------------------------ */

typedef struct {
    int nr, nz;
    double R;
    double *z;
    double *a, *b, *c, *d, *e, *f, *x, *r, *V, *mu, *D;
} or_level;

typedef struct {
    int nlev, smoother, nu1, nu2, wall;
    or_level lev[20];
    double *work;
} or_mg;

/* Number of grid levels: min(nr, nz) / coarsest must be a power of two
 * 2^L and both nr and nz divisible by 2^L; returns L + 1, or -1. */
int or_levels(int nr, int nz, int coarsest)
{
    if (nr < 2 || nz < 2 || coarsest < 2)
        return -1;
    int m = nr < nz ? nr : nz;
    if (m % coarsest)
        return -1;
    int q = m / coarsest, L = 0;
    while (q > 1) {
        if (q & 1)
            return -1;
        q >>= 1;
        ++L;
    }
    if (nr % (1 << L) || nz % (1 << L))
        return -1;
    return L + 1;
}

static double *alloc_field(int nr, int nz)
{
    return calloc((size_t)(nr + 1) * (nz + 1), sizeof(double));
}

void or_mg_destroy(or_mg *h);
or_mg *or_mg_create_w(int nr, int nz, double R, const double *z, int coarsest,
                      int smoother, int nu1, int nu2, int wall);

or_mg *or_mg_create(int nr, int nz, double R, const double *z, int coarsest,
                    int smoother, int nu1, int nu2)
{
    return or_mg_create_w(nr, nz, R, z, coarsest, smoother, nu1, nu2, 0);
}

/* wall != 0: every level has the Dirichlet wall rows at r = R. */
or_mg *or_mg_create_w(int nr, int nz, double R, const double *z, int coarsest,
                      int smoother, int nu1, int nu2, int wall)
{
    int nlev = or_levels(nr, nz, coarsest);
    if (nlev < 1 || nlev > 20)
        return NULL;
    or_mg *h = calloc(1, sizeof(or_mg));
    h->nlev = nlev;
    h->smoother = smoother;
    h->nu1 = nu1;
    h->nu2 = nu2;
    h->wall = wall;
    for (int l = 0; l < nlev; ++l) {
        or_level *L = &h->lev[l];
        L->nr = nr >> l;
        L->nz = nz >> l;
        L->R = R;
        L->z = malloc((size_t)(L->nz + 1) * sizeof(double));
        for (int j = 0; j <= L->nz; ++j)
            L->z[j] = z[j << l]; /* nested: every 2^l-th fine node */
        L->a = alloc_field(L->nr, L->nz);
        L->b = alloc_field(L->nr, L->nz);
        L->c = alloc_field(L->nr, L->nz);
        L->d = alloc_field(L->nr, L->nz);
        L->e = alloc_field(L->nr, L->nz);
        L->f = alloc_field(L->nr, L->nz);
        L->x = (l == 0) ? NULL : alloc_field(L->nr, L->nz);
        L->r = alloc_field(L->nr, L->nz);
        L->V = alloc_field(L->nr, L->nz);
        L->mu = alloc_field(L->nr, L->nz);
        L->D = alloc_field(L->nr, L->nz);
    }
    h->work = malloc(2 * (size_t)(nz + 1) * sizeof(double));
    return h;
}

void or_mg_destroy(or_mg *h)
{
    if (!h)
        return;
    for (int l = 0; l < h->nlev; ++l) {
        or_level *L = &h->lev[l];
        free(L->z);
        free(L->a);
        free(L->b);
        free(L->c);
        free(L->d);
        free(L->e);
        free(L->f);
        free(L->x);
        free(L->r);
        free(L->V);
        free(L->mu);
        free(L->D);
    }
    free(h->work);
    free(h);
}

int or_mg_nlev(const or_mg *h) { return h->nlev; }

/* Copy coefficient `which` (0..5 = a, b, c, d, e, f) of level l out. */
void or_mg_get(const or_mg *h, int l, int which, double *out)
{
    const or_level *L = &h->lev[l];
    const double *src[6] = {L->a, L->b, L->c, L->d, L->e, L->f};
    memcpy(out, src[which], (size_t)(L->nr + 1) * (L->nz + 1) * sizeof(double));
}

/* Poisson on every level; the charge (and the wall potential Vwall, nz+1
 * values, with a Dirichlet wall) enters the finest right-hand side. */
void or_mg_assemble_poisson_w(or_mg *h, double k, const double *ne,
                              const double *np, const double *Vwall)
{
    for (int l = 0; l < h->nlev; ++l) {
        or_level *L = &h->lev[l];
        or_poisson_assemble_w(L->nr, L->nz, L->R, L->z, k, l == 0 ? ne : NULL,
                              l == 0 ? np : NULL, h->wall, l == 0 ? Vwall : NULL,
                              L->a, L->b, L->c, L->d, L->e, L->f);
    }
}

void or_mg_assemble_poisson(or_mg *h, double k, const double *ne,
                            const double *np)
{
    or_mg_assemble_poisson_w(h, k, ne, np, NULL);
}

/* SG continuity on every level; coarse levels see the potential injected
 * (coarse node value = coincident fine node value). */
/* SG operator on every level; coarse levels see the potential (and the
 * node transport mun, Dn when given) injected: coarse node value =
 * coincident fine node value. */
void or_mg_assemble_sg_t(or_mg *h, int s, double mu, double D, double dt_inv,
                         const double *V, const double *nk, const double *S,
                         const double *mun, const double *Dn)
{
    size_t n0 = (size_t)(h->lev[0].nr + 1) * (h->lev[0].nz + 1) * sizeof(double);
    int tr = mun && Dn;
    memcpy(h->lev[0].V, V, n0);
    if (tr) {
        memcpy(h->lev[0].mu, mun, n0);
        memcpy(h->lev[0].D, Dn, n0);
    }
    for (int l = 1; l < h->nlev; ++l) {
        or_level *F = &h->lev[l - 1], *C = &h->lev[l];
        for (int I = 0; I <= C->nr; ++I)
            for (int J = 0; J <= C->nz; ++J) {
                size_t pc = IDX(I, J, C->nz), pf = IDX(2 * I, 2 * J, F->nz);
                C->V[pc] = F->V[pf];
                C->mu[pc] = F->mu[pf];
                C->D[pc] = F->D[pf];
            }
    }
    for (int l = 0; l < h->nlev; ++l) {
        or_level *L = &h->lev[l];
        or_sg_assemble_t(L->nr, L->nz, L->R, L->z, s, mu, D, dt_inv, h->wall,
                         tr ? L->mu : NULL, tr ? L->D : NULL, L->V,
                         l == 0 ? nk : NULL, l == 0 ? S : NULL, L->a, L->b,
                         L->c, L->d, L->e, L->f);
    }
}

void or_mg_assemble_sg(or_mg *h, int s, double mu, double D, double dt_inv,
                       const double *V, const double *nk, const double *S)
{
    or_mg_assemble_sg_t(h, s, mu, D, dt_inv, V, nk, S, NULL, NULL);
}

static void smooth(or_mg *h, or_level *L, double *x, int sweeps)
{
    for (int s = 0; s < sweeps; ++s) {
        for (int colour = 0; colour < 2; ++colour) {
            if (h->smoother == 0)
                or_rbgs(L->nr, L->nz, L->a, L->b, L->c, L->d, L->e, L->f, x,
                        colour);
            else
                or_zline(L->nr, L->nz, L->a, L->b, L->c, L->d, L->e, L->f, x,
                         colour, h->work);
        }
    }
}

static int vcycle_level(or_mg *h, int l, double *x)
{
    or_level *L = &h->lev[l];
    if (l == h->nlev - 1)
        return or_direct_solve(L->nr, L->nz, L->a, L->b, L->c, L->d, L->e,
                               L->f, x);
    smooth(h, L, x, h->nu1);
    or_residual(L->nr, L->nz, L->a, L->b, L->c, L->d, L->e, L->f, x, L->r);
    or_level *C = &h->lev[l + 1];
    or_restrict(L->nr, L->nz, L->z, L->r, C->f);
    memset(C->x, 0, (size_t)(C->nr + 1) * (C->nz + 1) * sizeof(double));
    int st = vcycle_level(h, l + 1, C->x);
    or_prolong_add(L->nr, L->nz, L->z, C->x, x);
    smooth(h, L, x, h->nu2);
    return st;
}

/* One V-cycle on the finest level (x holds its electrode values). */
int or_mg_vcycle(or_mg *h, double *x) { return vcycle_level(h, 0, x); }

double or_mg_relres(const or_mg *h, const double *x)
{
    const or_level *L = &h->lev[0];
    return or_relres(L->nr, L->nz, L->R, L->z, L->a, L->b, L->c, L->d, L->e,
                     L->f, x);
}

/* V-cycles until the strong-form relative residual is <= rtol.
 * Returns 0 on convergence, -3 if max_cycles ran out, -4 if non-finite. */
int or_mg_solve(or_mg *h, double *x, double rtol, int max_cycles, int *cycles,
                double *relres)
{
    double rr = or_mg_relres(h, x);
    int k = 0;
    while (isfinite(rr) && rr > rtol && k < max_cycles) {
        or_mg_vcycle(h, x);
        rr = or_mg_relres(h, x);
        ++k;
    }
    if (cycles)
        *cycles = k;
    if (relres)
        *relres = rr;
    if (!isfinite(rr))
        return -4;
    return rr <= rtol ? 0 : -3;
}

/* ------------------------------------------------------------------ */
/* One backward-Euler step, Eq. (7), with the equations solved one      */
/* after the other: Poisson with the densities of step k, then the SG   */
/* continuity equation of the electrons and of the ions with the new    */
/* potential.  State arrays are updated in place; their electrode rows  */
/* are set to the boundary values first.                                */
/* ------------------------------------------------------------------ */

typedef struct {
    double mu_e, mu_p, D_e, D_p, k;
    double V_bottom, V_top, ne_bottom, ne_top, np_bottom, np_top;
} or_phys;

static void set_electrodes(int nr, int nz, double *u, double lo, double hi)
{
    for (int i = 0; i <= nr; ++i) {
        u[IDX(i, 0, nz)] = lo;
        u[IDX(i, nz, nz)] = hi;
    }
}

/* Wall r = R (Sec. 3): potential interpolated linearly in z between the
 * electrode values, densities 0. */
static void set_wall(int nr, int nz, const double *z, const or_phys *ph,
                     double *V, double *ne, double *np)
{
    for (int j = 0; j <= nz; ++j) {
        double t = (z[j] - z[0]) / (z[nz] - z[0]);
        V[IDX(nr, j, nz)] = ph->V_bottom + (ph->V_top - ph->V_bottom) * t;
        ne[IDX(nr, j, nz)] = 0.0;
        np[IDX(nr, j, nz)] = 0.0;
    }
}

int or_step_decoupled_w(int nr, int nz, double R, const double *z,
                        const or_phys *ph, double *V, double *ne, double *np,
                        const double *Se, const double *Sp, double dt,
                        int coarsest, int smoother, int nu1, int nu2,
                        double rtol, int max_cycles, int wall, int *cycles3,
                        double *relres3);

int or_step_decoupled(int nr, int nz, double R, const double *z,
                      const or_phys *ph, double *V, double *ne, double *np,
                      const double *Se, const double *Sp, double dt,
                      int coarsest, int smoother, int nu1, int nu2, double rtol,
                      int max_cycles, int *cycles3, double *relres3)
{
    return or_step_decoupled_w(nr, nz, R, z, ph, V, ne, np, Se, Sp, dt, coarsest,
                               smoother, nu1, nu2, rtol, max_cycles, 0, cycles3,
                               relres3);
}

/* wall != 0: Dirichlet wall at r = R (set_wall values) on every equation. */
int or_step_decoupled_w(int nr, int nz, double R, const double *z,
                        const or_phys *ph, double *V, double *ne, double *np,
                        const double *Se, const double *Sp, double dt,
                        int coarsest, int smoother, int nu1, int nu2,
                        double rtol, int max_cycles, int wall, int *cycles3,
                        double *relres3)
{
    or_mg *h = or_mg_create_w(nr, nz, R, z, coarsest, smoother, nu1, nu2, wall);
    if (!h)
        return -1;
    size_t n = (size_t)(nr + 1) * (nz + 1);
    double *nk = malloc(n * sizeof(double));
    double *Vw = malloc((size_t)(nz + 1) * sizeof(double));
    double dt_inv = 1.0 / dt;
    int st, worst = 0;
    set_electrodes(nr, nz, V, ph->V_bottom, ph->V_top);
    set_electrodes(nr, nz, ne, ph->ne_bottom, ph->ne_top);
    set_electrodes(nr, nz, np, ph->np_bottom, ph->np_top);
    if (wall)
        set_wall(nr, nz, z, ph, V, ne, np);
    for (int j = 0; j <= nz; ++j)
        Vw[j] = V[IDX(nr, j, nz)];

    or_mg_assemble_poisson_w(h, ph->k, ne, np, wall ? Vw : NULL);
    st = or_mg_solve(h, V, rtol, max_cycles, &cycles3[0], &relres3[0]);
    if (st < worst)
        worst = st;

    memcpy(nk, ne, n * sizeof(double));
    or_mg_assemble_sg(h, -1, ph->mu_e, ph->D_e, dt_inv, V, nk, Se);
    st = or_mg_solve(h, ne, rtol, max_cycles, &cycles3[1], &relres3[1]);
    if (st < worst)
        worst = st;

    memcpy(nk, np, n * sizeof(double));
    or_mg_assemble_sg(h, +1, ph->mu_p, ph->D_p, dt_inv, V, nk, Sp);
    st = or_mg_solve(h, np, rtol, max_cycles, &cycles3[2], &relres3[2]);
    if (st < worst)
        worst = st;

    free(nk);
    free(Vw);
    or_mg_destroy(h);
    return worst;
}

/* ------------------------------------------------------------------ */
/* Newton-Raphson blocks of the coupled system (Sec. 2, Eq. 14).        */
/* Unknowns per node u = (n_e, n_p, V).  The continuity rows depend on  */
/* V through alpha; this returns the derivative of one SG row          */
/*   F = sum over faces area*phi_out + vol*(n - n^k)*dt_inv - vol*S     */
/* with respect to V at the node and its four neighbours, as five       */
/* coefficient arrays (a, b, c, d, e: V_{i-1}, V_i, V_{i+1}, V_{j-1},    */
/* V_{j+1}).  Uses F'(x) = F(x)(1 - G(x))/x and G'(x) = F'(x) + 1; for  */
/* |x| < 0.1, where 1 - G(x) cancels, the Taylor series of F' from the   */
/* Bernoulli numbers: -1/2 + x/6 - x^3/180 + x^5/5040 - x^7/151200      */
/* + x^9/4790016 (next term below 1e-19 there).                         */
/* ------------------------------------------------------------------ */

double or_bernoulli_dF(double x)
{
    if (fabs(x) < 0.1) {
        double x2 = x * x;
        return -0.5 + x * (1.0 / 6.0 + x2 * (-1.0 / 180.0 + x2 * (1.0 / 5040.0
               + x2 * (-1.0 / 151200.0 + x2 * (1.0 / 4790016.0)))));
    }
    double F = or_bernoulli_F(x);
    return F * (1.0 - or_bernoulli_G(x)) / x;
}

void or_sg_dV_w(int nr, int nz, double R, const double *z, int s, double mu,
                double D, int wall, const double *V, const double *n, double *a,
                double *b, double *c, double *d, double *e);

void or_sg_dV(int nr, int nz, double R, const double *z, int s, double mu,
              double D, const double *V, const double *n, double *a, double *b,
              double *c, double *d, double *e)
{
    or_sg_dV_w(nr, nz, R, z, s, mu, D, 0, V, n, a, b, c, d, e);
}

void or_sg_dV_t(int nr, int nz, double R, const double *z, int s, double mu,
                double D, int wall, const double *mun, const double *Dn,
                const double *V, const double *n, double *a, double *b,
                double *c, double *d, double *e);

/* wall != 0: the wall rows (i = nr, identity) do not depend on V. */
void or_sg_dV_w(int nr, int nz, double R, const double *z, int s, double mu,
                double D, int wall, const double *V, const double *n, double *a,
                double *b, double *c, double *d, double *e)
{
    or_sg_dV_t(nr, nz, R, z, s, mu, D, wall, NULL, NULL, V, n, a, b, c, d, e);
}

/* mun, Dn: node transport as in or_sg_assemble_t (held fixed: the
 * derivative is with respect to V only). */
void or_sg_dV_t(int nr, int nz, double R, const double *z, int s, double mu,
                double D, int wall, const double *mun, const double *Dn,
                const double *V, const double *n, double *a, double *b,
                double *c, double *d, double *e)
{
    double dr = R / nr;
    size_t nn = (size_t)(nr + 1) * (nz + 1);
    memset(a, 0, nn * sizeof(double));
    memset(b, 0, nn * sizeof(double));
    memset(c, 0, nn * sizeof(double));
    memset(d, 0, nn * sizeof(double));
    memset(e, 0, nn * sizeof(double));
    for (int i = 0; i <= nr; ++i) {
        double w = radial_width(i, nr, R);
        for (int j = 1; j < nz; ++j) {
            size_t p = IDX(i, j, nz);
            if (wall && i == nr)
                continue;
            double dzc = axial_width(z, j);
            double center = 0.0;
            double Df, q;
            if (i < nr) { /* term g (G(al) n_p - F(al) n_{i+1}), al = q (V_{i+1} - V_p) */
                size_t pn = IDX(i + 1, j, nz);
                face_coef(s, mu, D, mun, Dn, p, pn, &Df, &q);
                double g = face_radius(i, nr, R) * dzc * Df / dr;
                double al = q * (V[pn] - V[p]);
                double dF = or_bernoulli_dF(al);
                double sl = g * ((dF + 1.0) * n[p] - dF * n[pn]);
                c[p] = q * sl;
                center -= q * sl;
            }
            if (i > 0) { /* term g (F(al) n_p - G(al) n_{i-1}), al = q (V_p - V_{i-1}) */
                size_t pn = IDX(i - 1, j, nz);
                face_coef(s, mu, D, mun, Dn, p, pn, &Df, &q);
                double g = face_radius(i - 1, nr, R) * dzc * Df / dr;
                double al = q * (V[p] - V[pn]);
                double dF = or_bernoulli_dF(al);
                double sl = g * (dF * n[p] - (dF + 1.0) * n[pn]);
                a[p] = -q * sl;
                center += q * sl;
            }
            {
                size_t pn = p + 1;
                face_coef(s, mu, D, mun, Dn, p, pn, &Df, &q);
                double g = w * Df / (z[j + 1] - z[j]);
                double al = q * (V[pn] - V[p]);
                double dF = or_bernoulli_dF(al);
                double sl = g * ((dF + 1.0) * n[p] - dF * n[pn]);
                e[p] = q * sl;
                center -= q * sl;
            }
            {
                size_t pn = p - 1;
                face_coef(s, mu, D, mun, Dn, p, pn, &Df, &q);
                double g = w * Df / (z[j] - z[j - 1]);
                double al = q * (V[p] - V[pn]);
                double dF = or_bernoulli_dF(al);
                double sl = g * (dF * n[p] - (dF + 1.0) * n[pn]);
                d[p] = -q * sl;
                center += q * sl;
            }
            b[p] = center;
        }
    }
}
