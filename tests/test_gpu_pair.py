"""Two block Jacobi sweeps in one launch (pair_sweeps = 1), and the
pre- and post-smoothing of every level in one launch each (pair_sweeps = 2).

The two-sweep kernel hands each block's first-sweep coupling values to its
neighbours inside the launch, so its results must be bitwise those of two
one-sweep launches: the same arithmetic in the same order on the same
inputs.  The chained launch runs the same two-sweep blocks level after level
with dataflow flags between the levels (restriction on the way down,
interpolation on the way up), so it must be bitwise the level-by-level cycle
as well; where the cycle has another form it falls back to that cycle.  The cases force the one-step tiled sweep on every smoothed level,
including a finest level of 1,024 steps (1,025 work-groups, more than the
device holds at once, so the ticket order and the hand-off waits both
matter), with odd and even sweep counts, both transfer variants, the FP32
smoother and per-step V, Z~ (theta = 1/2).  One case is also checked against
the oracle's V-cycle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import make_problem, make_rhs
from oracle import Hierarchy
import paper_2405_04808_amd as pm
from parity_util import mg_opts, READINGS

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def tiled_everywhere(s, n_levels, shape=-1):
    s.set_sweep_shapes([shape] * (n_levels - 1) + [0])


def vcycle_pair(prob, r, shape=-1, **opt):
    outs = []
    for pair in (0, 1, 2):
        s = pm.Solver(prob.levels, pm.default_options(pair_sweeps=pair, **opt))
        tiled_everywhere(s, prob.n_levels, shape)
        outs.append(s.vcycle(dev(r)))
        torch.cuda.synchronize()
        s.close()
    return outs


@pytest.mark.parametrize("nx,n,n_levels", [(64, 40, 3), (128, 20, 3), (128, 1024, 8)])
@pytest.mark.parametrize("nu", [(2, 2), (3, 3), (1, 2), (4, 4)])
@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("reading", list(READINGS))
def test_pair_vcycle_bitwise(nx, n, n_levels, nu, variant, reading):
    if n == 1024 and (nu != (2, 2) or variant != 0):
        pytest.skip("the large grid runs once per reading, with the benchmark's sweep counts")
    prob, rng = make_problem(kind="burgers", nx=nx, nu=0.01, n=n, n_levels=n_levels, seed=31)
    r = rng.normal(size=prob.size)
    print(f"pair vcycle nx={nx} n={n} nu={nu} variant={variant} {reading}", flush=True)
    a, b, c = vcycle_pair(prob, r, nu_pre=nu[0], nu_post=nu[1], coarse_fixed_its=2,
                          transfer_variant=variant, **READINGS[reading])
    assert torch.equal(a, b)
    assert torch.equal(a, c)


@pytest.mark.parametrize("nx,n,n_levels", [(64, 40, 3), (128, 20, 3), (128, 1024, 8)])
@pytest.mark.parametrize("per", [1, 2, 3, 4])
@pytest.mark.parametrize("nu", [(2, 2), (3, 1)])
def test_pair_vcycle_bitwise_shared_block_groups(nx, n, n_levels, per, nu):
    # the FP64 shared-block sweep with 1-4 steps per work-group, two sweeps
    # per launch (ragged last groups at n = 20, 40)
    if n == 1024 and (per not in (3, 4) or nu != (2, 2)):
        pytest.skip("the large grid runs with the benchmark's sweep counts")
    prob, rng = make_problem(kind="burgers", nx=nx, nu=0.01, n=n, n_levels=n_levels, seed=36)
    r = rng.normal(size=prob.size)
    print(f"pair shared vcycle nx={nx} n={n} per={per} nu={nu}", flush=True)
    for variant in (0, 1):
        a, b, c = vcycle_pair(prob, r, shape=per, nu_pre=nu[0], nu_post=nu[1],
                              coarse_fixed_its=2, transfer_variant=variant)
        assert torch.equal(a, b)
        assert torch.equal(a, c)


@pytest.mark.parametrize("case", ["fp32", "theta05"])
def test_pair_vcycle_bitwise_fp32_and_per_step_blocks(case):
    if case == "fp32":
        prob, rng = make_problem(kind="burgers", nx=128, nu=0.01, n=40, n_levels=3, seed=32)
        opt = dict(smoother_fp32=2)
    else:
        prob, rng = make_problem(kind="burgers", nx=64, nu=0.01, n=32, n_levels=3, seed=33,
                                 theta=0.5)
        opt = {}
    r = rng.normal(size=prob.size)
    print(f"pair vcycle {case}", flush=True)
    a, b, c = vcycle_pair(prob, r, coarse_fixed_its=2, **opt)
    assert torch.equal(a, b)
    assert torch.equal(a, c)


def test_pair_vcycle_matches_oracle():
    prob, rng = make_problem(kind="burgers", nx=128, nu=0.01, n=24, n_levels=3, seed=34)
    s = pm.Solver(prob.levels, pm.default_options(coarse_fixed_its=2, pair_sweeps=1))
    tiled_everywhere(s, prob.n_levels)
    H = Hierarchy(prob.levels, mg_opts(s.options))
    r = rng.normal(size=prob.size)
    got = s.vcycle(dev(r)).cpu().numpy()
    ref = H.vcycle(r)
    # the bound of the other V-cycle parity cases whose coarse GMRES forms
    # A~ z from its SGS sweeps: 8 u max_k cond(S_k) on the coarsest level,
    # never tighter than 1e-10
    lv = prob.levels[-1]
    Zf = lv.Z_full()
    kappa = max(np.linalg.cond(lv.N[k] @ lv.N[k].T + Zf[k] @ Zf[k].T) for k in range(lv.n))
    tol = max(1e-10, 8 * 2.0 ** -53 * kappa)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= tol
    s.close()


@pytest.mark.parametrize("shape", [-1, 3])
def test_pair_fgmres_bitwise(shape):
    prob, rng = make_problem(kind="burgers", nx=64, nu=0.01, n=64, n_levels=4, seed=35)
    b = make_rhs(prob, rng)
    res = []
    for pair in (0, 1, 2):
        s = pm.Solver(prob.levels, pm.default_options(restart=200, maxit=400, pair_sweeps=pair))
        tiled_everywhere(s, prob.n_levels, shape)
        x, st, rc = s.solve(dev(b), tol=1e-10)
        torch.cuda.synchronize()
        assert rc == pm.PITMG_OK
        res.append((x.clone(), st["iters"]))
        s.close()
    for other in res[1:]:
        assert res[0][1] == other[1]
        assert torch.equal(res[0][0], other[0])


@pytest.mark.parametrize("nx,n,n_levels", [(64, 64, 4), (128, 48, 4), (128, 1024, 8)])
@pytest.mark.parametrize("variant", [0, 1])
def test_chain_runs_two_sweep_launches_per_cycle(nx, n, n_levels, variant):
    # the chained cycle issues one pre- and one post-smoothing launch per
    # V-cycle (the level-by-level cycle one of each per level) and matches it
    # bitwise over a whole FGMRES solve; n = 48 leaves an odd step count (3)
    # on the last level that smooths
    prob, rng = make_problem(kind="burgers", nx=nx, nu=0.01, n=n, n_levels=n_levels, seed=38)
    b = make_rhs(prob, rng)
    res = []
    for pair in (1, 2):
        s = pm.Solver(prob.levels, pm.default_options(transfer_variant=variant, pair_sweeps=pair))
        tiled_everywhere(s, prob.n_levels)
        s.profile(2)
        x, st, rc = s.solve(dev(b), tol=1e-10)
        torch.cuda.synchronize()
        assert rc == pm.PITMG_OK
        launches = s.profile_read()["jacobi"][0]
        cycles = st["iters"] + 1
        print(f"chain nx={nx} n={n} L={n_levels} variant={variant} pair={pair}: "
              f"{st['iters']} steps, {launches} sweep launches", flush=True)
        per = 2 if pair == 2 else 2 * (n_levels - 1)
        assert launches >= per * st["iters"] and launches <= per * cycles
        res.append((x.clone(), st["iters"]))
        s.close()
    assert res[0][1] == res[1][1]
    assert torch.equal(res[0][0], res[1][0])


def test_pair_handoff_wait_bound_reports_error():
    # force the hand-off's own bounded wait to run out from the host (a bound
    # of zero): every kernel still exits, and the solve reports the failure;
    # with the bound restored the same handle solves normally again
    prob, rng = make_problem(kind="burgers", nx=128, nu=0.01, n=1024, n_levels=8, seed=37)
    b = make_rhs(prob, rng)
    run_wait_bound_case(prob, b, 1)


def test_chain_wait_bound_reports_error():
    # the same with the chained cycle, whose blocks also wait for the
    # previous level's
    prob, rng = make_problem(kind="burgers", nx=128, nu=0.01, n=1024, n_levels=8, seed=39)
    b = make_rhs(prob, rng)
    run_wait_bound_case(prob, b, 2)


def run_wait_bound_case(prob, b, pair):
    s = pm.Solver(prob.levels, pm.default_options(restart=8, maxit=8, pair_sweeps=pair))
    tiled_everywhere(s, prob.n_levels)
    with pytest.raises(pm.PitmgError):
        s.set_handoff_wait(-1.0)
    s.set_handoff_wait(0.0)
    with pytest.raises(pm.PitmgError) as err:
        s.solve(dev(b), tol=1e-10)
    torch.cuda.synchronize()
    assert err.value.code == pm.PITMG_ERR_HIP
    assert "hand-off" in str(err.value)
    s.set_handoff_wait(2.0)
    x, st, rc = s.solve(dev(b), tol=1e-10)
    torch.cuda.synchronize()
    assert rc in (pm.PITMG_OK, pm.PITMG_NOT_CONVERGED) and st["iters"] == 8
    s.close()


@pytest.mark.parametrize("fp32,launches", [(99, 4), (2, 6)])
def test_chain_below_fp32_levels_bitwise(fp32, launches):
    # an FP32 finest level forms its residual explicitly, so it sweeps on its
    # own and the levels below it chain (all of them FP32 with smoother_fp32
    # = 99; only the FP64 levels 2-3 with smoother_fp32 = 2, the FP32 level 1
    # sweeping on its own too): per V-cycle the sweeps of the levels outside
    # the chain (one pre- and one post-smoothing launch each) plus the two
    # chained launches, and the same doubles as level by level
    prob, rng = make_problem(kind="burgers", nx=128, nu=0.01, n=64, n_levels=5, seed=40)
    r = rng.normal(size=prob.size)
    print(f"chain below FP32 levels: smoother_fp32={fp32}", flush=True)
    a, b, c = vcycle_pair(prob, r, coarse_fixed_its=2, smoother_fp32=fp32)
    assert torch.equal(a, b)
    assert torch.equal(a, c)
    s = pm.Solver(prob.levels, pm.default_options(coarse_fixed_its=2, smoother_fp32=fp32))
    tiled_everywhere(s, prob.n_levels)
    s.profile(2)
    s.vcycle(dev(r))
    torch.cuda.synchronize()
    assert s.profile_read()["jacobi"][0] == launches
    s.close()
