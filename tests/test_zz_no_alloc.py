"""pitmg_coarse_solve_noalloc: the coarse GMRES + SGS solve with its scratch
in the library's static device array, against pitmg_coarse_solve (the same
kernels on the handle's buffers) and the oracle, through the C ABI.

Two calls in a row, the second on a smaller coarse system, then the first
system again: the array keeps the previous call's contents, so every call
must clear what has to start at zero.  A solve whose scratch exceeds the
array is refused.
"""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import make_problem
from oracle import OracleLevel, gmres_right
import paper_2405_04808_amd as pm

pytestmark = pytest.mark.gpu


def noalloc(s, b):
    out = s.empty(s.n_levels - 1)
    its = C.c_int(-1)
    s._order()
    rc = s.lib.pitmg_coarse_solve_noalloc(s.h, C.c_void_p(b.data_ptr()),
                                          C.c_void_p(out.data_ptr()), C.byref(its))
    torch.cuda.synchronize()
    return rc, out, its.value


def check(case, seed):
    prob, rng = make_problem(**case)
    s = pm.Solver(prob.levels, pm.default_options())
    lv = prob.levels[-1]
    ol = OracleLevel(lv.N, lv.V, lv.Z, factor_sgs=True)
    bh = rng.normal(size=ol.A.shape[0])
    b = torch.from_numpy(bh).to("cuda")
    before = s.device_bytes()
    ref, its_ref = s.coarse_solve(b)
    rc, got, its = noalloc(s, b)
    assert rc == pm.PITMG_OK, s.last_error()
    assert s.device_bytes() == before
    # same kernels in the same order on other buffers: bitwise equal
    assert its == its_ref
    assert torch.equal(got, ref)
    # and the oracle's GMRES + SGS on the same system
    xt, its_o = gmres_right(ol.At, bh[ol.perm], ol.sgs, 1e-3, 50)
    xo = np.empty_like(xt)
    xo[ol.perm] = xt
    assert its == its_o
    g = got.cpu().numpy()
    assert np.linalg.norm(g - xo) <= 1e-10 * np.linalg.norm(xo)
    s.close()
    return its


def test_noalloc_coarse_solve_two_calls_second_smaller():
    big = dict(kind="burgers", nx=64, nu=0.01, n=16, n_levels=2, seed=41)
    small = dict(kind="vanderpol", n=32, n_levels=3, seed=42)
    print("noalloc: Burgers p=64 coarse system", flush=True)
    check(big, 1)
    print("noalloc: van der Pol p=2 coarse system", flush=True)
    check(small, 2)
    print("noalloc: Burgers p=64 again", flush=True)
    check(big, 3)


def test_noalloc_refuses_oversized_scratch():
    prob, rng = make_problem(kind="burgers", nx=512, nu=0.01, n=8, n_levels=1, seed=43)
    s = pm.Solver(prob.levels, pm.default_options(coarse_maxit=200))
    b = torch.from_numpy(rng.normal(size=s.lens[0])).to("cuda")
    rc, _, _ = noalloc(s, b)
    assert rc == pm.PITMG_ERR_UNSUPPORTED
    assert "scratch" in s.last_error()
    s.close()
