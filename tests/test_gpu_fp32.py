"""GPU checks of the FP32 smoother mode against the FP64 oracle.

With smoother_fp32 the blocks of every level above the coarsest are rounded
to FP32 and factored and applied in FP32.  One block solve then carries a
relative error of order cond(S_k) * u32 (u32 = 2^-24, S_k = N_k N_k^T +
Z~_k Z~_k^T), so a sweep is compared with the FP64 oracle at
64 * u32 * max_k cond(S_k), and a whole V-cycle at 64 * u32 * max cond times
the number of levels.  FGMRES still has to reach a true relative residual of
1e-10 (the finest residual, the coarse solve and the Krylov method stay
FP64); its solution is then checked against the oracle's FP64 solve at the
accuracy such a residual implies, and the step counts are compared.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import make_problem, make_rhs
from oracle import Hierarchy, OracleLevel
from oracle.multigrid import MGOptions
import paper_2405_04808_amd as pm

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
CASES = {
    "vdp64": dict(kind="vanderpol", n=64, n_levels=4, seed=11),
    "burgers_p12": dict(kind="burgers", nx=12, nu=0.01, n=32, n_levels=3, seed=12),
    "burgers_p64": dict(kind="burgers", nx=64, nu=0.01, n=32, n_levels=3, seed=16),
    "burgers_p64_theta05": dict(kind="burgers", nx=64, nu=0.01, n=16, n_levels=2, seed=15,
                                theta=0.5),
    "burgers_p150": dict(kind="burgers", nx=150, nu=0.02, n=8, n_levels=2, seed=14),
}


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def max_cond_S(lv):
    N = lv.N
    Z = lv.Z_full()
    S = N @ np.transpose(N, (0, 2, 1)) + Z @ np.transpose(Z, (0, 2, 1))
    return float(np.max(np.linalg.cond(S)))


def solver(name, **opt):
    prob, rng = make_problem(**CASES[name])
    b = make_rhs(prob, rng)
    opt.setdefault("smoother_fp32", 99)          # every level above the coarsest
    return prob, rng, b, pm.Solver(prob.levels, pm.default_options(**opt))


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_sweep_within_rounding_of_fp64_oracle(name):
    prob, rng, b, s = solver(name)
    for lev, lv in enumerate(prob.levels[:-1]):
        ol = OracleLevel(lv.N, lv.V, lv.Z)
        m = ol.A.shape[0]
        bb = rng.normal(size=m)
        y = rng.normal(size=m)
        yt = ol.jacobi(bb[ol.perm], y[ol.perm], s.options.omega)
        ref = np.empty_like(yt)
        ref[ol.perm] = yt
        got = host(s.jacobi_sweep(dev(bb), dev(y), level=lev))
        tol = 64 * U32 * max_cond_S(lv)
        assert rel(got, ref) <= tol, (name, lev, rel(got, ref), tol)
    s.close()


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_vcycle_within_rounding_of_fp64_oracle(name):
    prob, rng, b, s = solver(name, coarse_fixed_its=2)
    H = Hierarchy(prob.levels, MGOptions(coarse_fixed_its=2))
    r = rng.normal(size=prob.size)
    ref = H.vcycle(r)
    got = host(s.vcycle(dev(r)))
    cond = max(max_cond_S(lv) for lv in prob.levels[:-1])
    tol = 64 * U32 * cond * len(prob.levels)
    assert rel(got, ref) <= tol, (rel(got, ref), tol)
    s.close()


@pytest.mark.parametrize("name", ["vdp64", "burgers_p12", "burgers_p64", "burgers_p64_theta05"])
@pytest.mark.parametrize("levels32", [1, 99])
def test_fp32_smoother_fgmres_reaches_1e10(name, levels32):
    prob, rng, b, s = solver(name, restart=500, maxit=500, smoother_fp32=levels32)
    x, st, rc = s.solve(dev(b), tol=1e-10)
    x = host(x)
    assert rc == pm.PITMG_OK and st["converged"] == 1
    lv = prob.levels[0]
    A = OracleLevel(lv.N, lv.V, lv.Z).A
    true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
    assert true <= 1.01e-10
    H = Hierarchy(prob.levels)
    xr, info = H.solve(b, tol=1e-10, restart=500, maxit=500)
    # both iterates solve A x = b to 1e-10 in residual; their difference is
    # bounded by the residuals through A^{-1}
    Ad = A.toarray()
    bound = 2.02e-10 * np.linalg.norm(b) * np.linalg.norm(np.linalg.inv(Ad), 2)
    assert np.linalg.norm(x - xr) <= bound
    # rounding the smoother to FP32 weakens the preconditioner on the
    # near-null modes of A~; the step count may grow, but boundedly
    assert st["iters"] <= 2 * info["iters"] + 5
    s.close()


def test_fp32_option_fixed_at_setup():
    prob, rng, b, s = solver("burgers_p12")
    with pytest.raises(pm.PitmgError):
        s.set_options(smoother_fp32=0)
    s.close()
