"""End-to-end solves of the 512-node viscous Burgers workload (p = q = 512,
nu = 0.005, n = 4,096 steps, 10 levels: 10.5 M unknowns), with the FP64
smoother and with the FP32 smoother (factorisations and sweeps in FP32 on
every level above the coarsest; finest residual, coarse solve, Arnoldi and
FGMRES in FP64).

The assembled system is too large for the oracle's sparse assembly and its
FGMRES, so the check is P1: the true residual b - A~ x of the returned
iterate, formed on the host by the oracle's step-by-step product
(oracle.system.apply_blocks, pinned against the assembled operator on small
cases), meets the 1e-10 tolerance, and agrees with the residual the library
reports to 1 %.  The worst-case rounding bound of either evaluation,
2 k u || |A~| |x| || / ||b|| with k = 2p + q products per row, is printed:
here it is about 2e-8, far above the residual, because the solution is
large against b (|| |A~| |x| || is about 6e4 ||b||), so it cannot decide the
comparison; the two evaluations (the library's FP64 product on the GPU and
the oracle's on the host, in different summation orders) agreeing to a few
parts in 1e4 shows the rounding actually incurred is far smaller.  The
FP32 smoother's solution is compared with the FP64 one; both meet the same
residual tolerance, and their difference is printed (the forward error of
either is bounded only by cond(A~) times the residual).  The FGMRES restart length (200) keeps the
Krylov bases at 2 x 200 x 84 MB.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.system import apply_blocks
import paper_2405_04808_amd as pm
from parity_util import dev, host, full_config

pytestmark = pytest.mark.gpu

RESULTS = {}


@pytest.mark.parametrize("fp32", [0, 99])
def test_c3_solve_true_residual(fp32):
    prob, b = full_config("burgers512")
    print(f"c3 solve fp32={fp32}: size {prob.size}", flush=True)
    s = pm.Solver(prob.levels, pm.default_options(restart=200, maxit=800, smoother_fp32=fp32))
    xg, st, rc = s.solve(dev(b), tol=1e-10)
    assert rc == pm.PITMG_OK and st["converged"] == 1, (rc, st)
    x = host(xg)
    s.close()
    lv = prob.levels[0]
    nb = np.linalg.norm(b)
    true = np.linalg.norm(b - apply_blocks(lv.N, lv.V, lv.Z, x)) / nb
    k = 2 * prob.p + prob.q
    bound = 2 * k * 2.0 ** -53 * np.linalg.norm(apply_blocks(lv.N, lv.V, lv.Z, x,
                                                             magnitude=True)) / nb
    RESULTS[fp32] = x
    msg = (f"c3 fp32={fp32}: {st['iters']} FGMRES steps, residual {true:.3e} "
           f"(reported {st['relres_true']:.3e}, rounding bound {bound:.3e})")
    if fp32 and 0 in RESULTS:
        diff = np.linalg.norm(x - RESULTS[0]) / np.linalg.norm(RESULTS[0])
        msg += f", relative difference from the FP64-smoother solution {diff:.3e}"
    print(msg, flush=True)
    assert true <= 1.0e-10
    assert abs(true - st["relres_true"]) <= 0.01 * true
