"""C-ABI contract checks that need no GPU: the library loads, exports every
function declared in include/pitmg.h, and rejects bad arguments on the host
before any device work."""
import ctypes as C

import numpy as np
import pytest

import paper_2405_04808_amd as pm
from paper_2405_04808_amd import pitmg as B


def test_library_exports_every_declared_function():
    lib = pm.load_library()
    names = pm.header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name


def test_default_options_and_status_strings():
    o = pm.default_options()
    assert (o.nu_pre, o.nu_post, o.coarse_maxit, o.restart, o.maxit) == (2, 2, 50, 30, 300)
    assert o.coarse_tol == 1e-3 and o.coarse_fixed_its == 0 and o.transfer_variant == 0
    assert o.apply_from_sweep == 1 and o.pair_sweeps == 2
    lib = pm.load_library()
    for code in range(-6, 2):
        assert lib.pitmg_status_string(code).decode() != "unknown status"


def _problem(p=2, q=1, n=16, levels=2, nstride=None):
    arr = C.c_void_p * levels
    fake = arr(*([0x1000] * levels))          # never dereferenced: validation fails first
    pb = B.pitmg_problem()
    pb.p, pb.q, pb.n, pb.n_levels = p, q, n, levels
    pb.N = C.cast(fake, C.POINTER(C.c_void_p))
    pb.V = C.cast(fake, C.POINTER(C.c_void_p))
    pb.Z = C.cast(fake, C.POINTER(C.c_void_p))
    pb.N_stride = p * p if nstride is None else nstride
    pb.V_stride = 0
    pb.Z_stride = p * q
    pb.blocks_on_device = 1
    return pb, fake


@pytest.mark.parametrize("kw,code", [
    (dict(n=0), pm.PITMG_ERR_INVALID),
    (dict(p=0), pm.PITMG_ERR_INVALID),
    (dict(n=12, levels=4), pm.PITMG_ERR_INVALID),        # 12 % 8 != 0
    (dict(nstride=3), pm.PITMG_ERR_INVALID),
    (dict(p=600, q=1), pm.PITMG_ERR_UNSUPPORTED),          # p, q <= 512
])
def test_setup_rejects_bad_problems_on_host(kw, code):
    lib = pm.load_library()
    pb, keep = _problem(**kw)
    h = C.c_void_p()
    rc = lib.pitmg_setup(C.byref(h), C.byref(pb), None, None)
    assert rc == code
    assert not h.value


def test_setup_rejects_bad_options_on_host():
    lib = pm.load_library()
    pb, keep = _problem()
    for field, val in [("restart", 0), ("nu_pre", -1), ("transfer_variant", 3),
                       ("coarse_maxit", 0), ("apply_from_sweep", 2), ("pair_sweeps", 3)]:
        o = pm.default_options(**{field: val})
        h = C.c_void_p()
        assert lib.pitmg_setup(C.byref(h), C.byref(pb), C.byref(o), None) == pm.PITMG_ERR_INVALID
        assert not h.value


def test_null_handle_calls_are_invalid():
    lib = pm.load_library()
    assert lib.pitmg_apply(None, 0, None, None) == pm.PITMG_ERR_INVALID
    assert lib.pitmg_vcycle(None, None, None) == pm.PITMG_ERR_INVALID
    assert lib.pitmg_fgmres_solve(None, None, None, 1e-10, 0, None) == pm.PITMG_ERR_INVALID
    assert lib.pitmg_setup(None, None, None, None) == pm.PITMG_ERR_INVALID
    lib.pitmg_destroy(None)
