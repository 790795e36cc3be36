"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/mgfluid.h, and validates its arguments on the host
(mg_query is a pure host computation)."""
import os
import re

import numpy as np
import pytest

from paper_0811_4446_amd import inputs
from paper_0811_4446_amd import mgfluid as M

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mgfluid.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*(\w+)\s*\(", txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert "mg_setup" in names and "solve_steady" in names and "vcycle" in names
    lib = M.lib()
    for n in names:
        assert hasattr(lib, n), n
        assert n in M.SIGNATURES, n


def test_query_sizes():
    for N in (64, 256, 1024):
        pitch, ws = M.query(M.make_desc(N, N, inputs.z_cos(N)))
        assert pitch >= N + 1 and pitch % 16 == 0
        # three 5-point operators + rhs per level, plus work fields: at least
        # 18 level-0 fields, and the coarse levels add about a third
        assert ws >= 18 * (N + 1) * pitch * 8
    p32, ws32 = M.query(M.make_desc(256, 256, inputs.z_cos(256), prec=M.FP32_IR))
    assert ws32 > M.query(M.make_desc(256, 256, inputs.z_cos(256)))[1]


@pytest.mark.parametrize("kw,msg", [
    (dict(nr=60, nz=64), "cannot be coarsened"),
    (dict(nr=64, nz=64, coarsest=1), "cannot be coarsened"),
    (dict(nr=64, nz=64, abi=1), "abi_version"),
    (dict(nr=64, nz=64, wall=2), "r_outer_bc"),
    (dict(nr=64, nz=64, zbad="order"), "strictly increasing"),
    (dict(nr=64, nz=64, zbad="start"), "start at 0"),
    (dict(nr=64, nz=64, smoother=7), "smoother"),
    (dict(nr=64, nz=64, prec=9), "precision"),
    (dict(nr=64, nz=64, nu=(0, 0)), "smoothing"),
    (dict(nr=64, nz=2048), "z-line"),
])
def test_query_rejects_bad_grids(kw, msg):
    nr, nz = kw["nr"], kw["nz"]
    z = inputs.z_cos(nz)
    if kw.get("zbad") == "order":
        z = z.copy()
        z[5], z[6] = z[6], z[5]
    if kw.get("zbad") == "start":
        z = z + 0.1
    nu = kw.get("nu", (2, 2))
    d = M.make_desc(nr, nz, z, coarsest=kw.get("coarsest", 8), nu1=nu[0], nu2=nu[1],
                    smoother=kw.get("smoother", M.SMOOTH_ZEBRA), prec=kw.get("prec", M.FP64),
                    d=float(z[-1]) if kw.get("zbad") != "start" else 1.0)
    if "abi" in kw:
        d.abi_version = kw["abi"]
    if "wall" in kw:
        d.r_outer_bc = kw["wall"]
    with pytest.raises(M.MGError) as ei:
        M.query(d)
    assert ei.value.code == -1
    assert msg in str(ei.value)


def test_null_arguments_fail_before_device_work():
    lib = M.lib()
    assert lib.mg_query(None, None, None) == -1
    assert lib.mg_setup(None, None, 0, None, None) == -1
    assert lib.vcycle(None, 0, None, 1, None) == -1
    assert lib.sg_assemble(None, 0, None, None, 0.0) == -1
    assert lib.solve_steady(None, None, None, None, None) == -1
    assert lib.solve_steady_batches(None, 0, None, None, None) == -1
    assert b"null" in lib.mg_last_error()


def test_forward_noalloc_rejects_batches_beyond_one_launch():
    """2^24 tiles of 16 x 16 pixels is the launch limit of the fused forward
    pass; one more image's worth is refused before any device call (the fake
    addresses are never dereferenced)."""
    import ctypes
    lib = M.lib()
    fake = ctypes.c_void_p(1 << 20)
    tiles = 17 * 17  # one 257 x 257 image
    B = (1 << 24) // tiles + 1
    assert lib.wn_forward_noalloc(fake, fake, fake, B, 257, 257, None) == -1
    assert b"tiles" in lib.mg_last_error()
    assert lib.wn_forward_noalloc(fake, fake, fake, 0, 257, 257, None) == -1


def test_setup_rejects_small_workspace_without_touching_it():
    d = M.make_desc(64, 64, inputs.z_cos(64))
    pitch, ws = M.query(d)
    import ctypes
    h = ctypes.c_void_p()
    # a fake aligned address: the size check fails first, nothing is dereferenced
    code = M.lib().mg_setup(ctypes.byref(d), ctypes.c_void_p(1 << 20), ws - 8, None, ctypes.byref(h))
    assert code == -6


@pytest.mark.parametrize("nprob,krylov,msg", [(0, 20, "nprob"), (-3, 20, "nprob"), (70000, 20, "nprob"),
                                              (4, 0, "krylov_m")])
def test_batch_query_rejects_empty_and_oversized_batches(nprob, krylov, msg):
    import ctypes
    d = M.make_desc(64, 64, inputs.z_cos(64), krylov_m=krylov, coarsest=4)
    stride, total = ctypes.c_int64(0), ctypes.c_int64(0)
    code = M.lib().mg_batch_query(ctypes.byref(d), nprob, ctypes.byref(stride), ctypes.byref(total))
    assert code == -1  # MG_EINVAL
    assert msg in M.lib().mg_last_error().decode()


def test_batch_query_stride_covers_one_problem():
    import ctypes
    d = M.make_desc(64, 64, inputs.z_cos(64), krylov_m=20, coarsest=4)
    _, ws1 = M.query(d)
    stride, total = ctypes.c_int64(0), ctypes.c_int64(0)
    assert M.lib().mg_batch_query(ctypes.byref(d), 5, ctypes.byref(stride), ctypes.byref(total)) == 0
    assert stride.value >= ws1 and stride.value % 256 == 0
    assert total.value >= 5 * stride.value
