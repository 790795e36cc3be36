// Declarations of the learned warm-start network (wn_net.hip).
#pragma once
#include "mg_internal.h"

namespace mgf {

constexpr int kWnParams = 7 * 32 * 9 + 32 + 2 * (32 * 32 * 9 + 32) + 32 * 3 * 9 + 3;  // 21411
constexpr double kWnGain = 100.0;  // corrections are learned in units of 1/kWnGain

int64_t wn_scratch_size(int B, int H, int W);
int wn_forward_impl(const float *params, const float *in, float *out, int B, int H, int W, void *scratch,
                    hipStream_t st);
int wn_grad_impl(const float *params, const float *in, const float *target, int B, int H, int W, float *grad_out,
                 double *loss_host, void *scratch, hipStream_t st);
int wn_train_impl(float *params, float *m, float *v, int step, float lr, const float *in, const float *target,
                  int B, int H, int W, double *loss_host, void *scratch, hipStream_t st);
void launch_features(const Geom &g, const double *V, const double *ne, const double *np, double R, double d,
                     double vtop, double ratio, double *nscale, float *out, hipStream_t s);
void launch_targets(const Geom &g, const double *Vu, const double *neu, const double *npu, const double *Vf,
                    const double *nef, const double *npf, double vtop, const double *nscale, float *out,
                    hipStream_t s);
void launch_apply(const Geom &g, const double *Vu, const double *neu, const double *npu, const float *corr,
                  double vtop, const double *nscale, double *V, double *ne, double *np, const mg_physics &ph,
                  hipStream_t s);

}  // namespace mgf
