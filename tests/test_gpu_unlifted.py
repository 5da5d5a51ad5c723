"""GPU parity of the system without virtual variables (Fig. 2, B = dF): the
operator product, the lifted hierarchy of the scaled blocks that the handle
builds on the device, and FGMRES preconditioned by the lifted cycle through
the lift / project maps, each against the FP64 oracle (oracle.unlifted).

Tolerances as for the lifted parity cases: 1e-13 for a product, the
conditioning bound of the block solves for a cycle in fixed-coarse-step mode,
and for a solve the same step count (+-1) with the solutions compared per
variable type at 1e-10 (or, when the counts differ, each within
||A^{-1}|| times its residual of the direct solution).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

torch = pytest.importorskip("torch")

from workloads import make_problem
from oracle import Hierarchy
from oracle.unlifted import assemble_unlifted, UnliftedSolver, ScaledLevel
import paper_2405_04808_amd as pm
from parity_util import dev, host, mg_opts, assert_types
from test_gpu_parity import inv_norm

pytestmark = pytest.mark.gpu

CASES = {
    "vdp64": dict(kind="vanderpol", n=64, n_levels=4, seed=51),
    "burgers_p12": dict(kind="burgers", nx=12, nu=0.01, n=32, n_levels=3, seed=52),
    "burgers_p64": dict(kind="burgers", nx=64, nu=0.01, n=32, n_levels=3, seed=53),
    "burgers_p128": dict(kind="burgers", nx=128, nu=0.01, n=16, n_levels=2, seed=54),
    "burgers_p64_theta05": dict(kind="burgers", nx=64, nu=0.01, n=16, n_levels=2, seed=55,
                                theta=0.5),
    "burgers_p256": dict(kind="burgers", nx=256, nu=0.01, n=8, n_levels=2, seed=56),
    # a dense shared V (non-diagonal mass matrix): the general product
    "burgers_p64_mass": dict(kind="burgers", nx=64, nu=0.01, n=16, n_levels=2, seed=57,
                             mass_offdiag=0.1),
}


def unl_types(got, ref, p, q, n, tol, what):
    bounds = [0, p * n, (p + q) * n, (2 * p + q) * n]
    for t, a, b in zip(("u", "z", "lam"), bounds[:-1], bounds[1:]):
        d = np.linalg.norm(np.asarray(got)[a:b] - ref[a:b])
        r = np.linalg.norm(ref[a:b])
        assert d <= tol * max(r, 1e-300), (what, t, d / max(r, 1e-300), tol)


@pytest.mark.parametrize("name", list(CASES))
def test_unlifted_apply_matches_oracle(name):
    prob, rng = make_problem(**CASES[name])
    s = pm.Solver(prob.levels, pm.default_options(unlifted=1))
    lv = prob.levels[0]
    A = assemble_unlifted(lv.N, lv.V, lv.Z)
    x = rng.normal(size=A.shape[0])
    print(f"unlifted apply {name}", flush=True)
    got = host(s.unlifted_apply(dev(x)))
    unl_types(got, A @ x, prob.p, prob.q, prob.n, 1e-13, name)
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_scaled_lifted_hierarchy_matches_oracle(name):
    # the lifted entry points of an unlifted handle act on the blocks
    # sqrt2 N_k, sqrt2 V_k, Z~_k that the handle scaled on the device
    prob, rng = make_problem(**CASES[name])
    s = pm.Solver(prob.levels, pm.default_options(unlifted=1, coarse_fixed_its=2))
    scaled = [ScaledLevel(lv) for lv in prob.levels]
    H = Hierarchy(scaled, mg_opts(s.options))
    r = rng.normal(size=prob.size)
    got = host(s.vcycle(dev(r)))
    # the bound of the other cycle parity cases, on the scaled coarsest blocks
    lc = prob.levels[-1]
    Nc, Zc = lc.N, lc.Z_full()
    S = 2 * Nc @ np.transpose(Nc, (0, 2, 1)) + Zc @ np.transpose(Zc, (0, 2, 1))
    tol = max(1e-10, 8 * 2.0 ** -53 * float(np.max(np.linalg.cond(S))))
    assert_types(got, H.vcycle(r), prob.p, prob.q, prob.n, tol, name)
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_unlifted_fgmres_matches_oracle(name):
    prob, rng = make_problem(**CASES[name])
    s = pm.Solver(prob.levels, pm.default_options(unlifted=1, restart=200, maxit=200))
    S = UnliftedSolver(prob.levels, mg_opts(s.options))
    b = rng.normal(size=S.A.shape[0])
    print(f"unlifted fgmres {name}", flush=True)
    xg, st, rc = s.unlifted_solve(dev(b), tol=1e-10)
    assert rc == pm.PITMG_OK and st["relres_true"] <= 1e-10
    x = host(xg)
    true = np.linalg.norm(b - S.A @ x) / np.linalg.norm(b)
    assert true <= 1.0001e-10
    xr, info = S.solve(b, tol=1e-10, restart=200, maxit=200)
    assert abs(st["iters"] - info["iters"]) <= 1, (st["iters"], info["iters"])
    p, q, n = prob.p, prob.q, prob.n
    if st["iters"] == info["iters"]:
        unl_types(x, xr, p, q, n, 1e-10, name)
    else:
        ninv, lu = inv_norm(S.A)
        xd = lu.solve(b)
        for y in (x, xr):
            r = np.linalg.norm(b - S.A @ y)
            assert np.linalg.norm(y - xd) <= 1.01 * ninv * r + 1e-12 * np.linalg.norm(xd)
    s.close()


def test_unlifted_entry_points_need_the_option():
    prob, rng = make_problem(**CASES["burgers_p12"])
    s = pm.Solver(prob.levels, pm.default_options())
    x = torch.zeros((2 * prob.p + prob.q) * prob.n, dtype=torch.float64, device="cuda")
    with pytest.raises(pm.PitmgError):
        s.unlifted_apply(x)
    with pytest.raises(pm.PitmgError):
        s.unlifted_solve(x)
    with pytest.raises(pm.PitmgError):
        s.set_options(unlifted=1)
    s.close()
