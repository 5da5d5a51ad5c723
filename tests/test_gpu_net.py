"""GPU parity of the learned coarse correction against the FP64 oracle.

The kernels multiply bfloat16 operands with FP32 accumulation.  They are
compared with oracle/coarse_net.py twice: with the oracle rounding at the
same points (bf16_points=True; the remaining differences are FP32 versus
FP64 accumulation and the rare bfloat16 rounding that this flips), and with
the plain FP64 network (the bfloat16 error itself).  Shapes span several
32-wide tiles with ragged tails (C = 60), the coarse shape of the benchmark
workload (C = 640) and of the 256-node Burgers workload (C = 1280).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import coarse_net as cn
from oracle import Hierarchy
from oracle.multigrid import MGOptions
from workloads import make_problem, make_rhs
import paper_2405_04808_amd as pm

pytestmark = pytest.mark.gpu

T = 8
H = 64
TOL_SAME_POINTS = 2e-3      # GPU vs oracle rounding at the same points
TOL_FP64 = 3e-2             # GPU vs plain FP64 network


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda")


def dev64(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.float64)


def params(C, seed, scale=1.0):
    return (cn.init_params(C, H, np.random.default_rng(seed)) * scale).astype(np.float32).astype(
        np.float64)


@pytest.mark.parametrize("C,batch", [(60, 1), (60, 37), (640, 1), (640, 64), (1280, 3)])
def test_forward_parity(C, batch):
    rng = np.random.default_rng(C + batch)
    theta = params(C, C, scale=2.0)
    x = rng.normal(size=(batch, T, C)).astype(np.float32).astype(np.float64)
    net = pm.Net(C, T, H, max_batch=max(batch, 4))
    net.set_params(theta)
    y = host(net.forward(dev32(x)))
    yq, _ = cn.forward(theta, x, C, H, bf16_points=True)
    y64, _ = cn.forward(theta, x, C, H)
    assert rel(y, yq) <= TOL_SAME_POINTS, rel(y, yq)
    assert rel(y, y64) <= TOL_FP64, rel(y, y64)
    net.close()


@pytest.mark.parametrize("C,batch", [(60, 5), (640, 32)])
def test_backward_parity(C, batch):
    rng = np.random.default_rng(100 + C)
    theta = params(C, C + 1, scale=2.0)
    x = rng.normal(size=(batch, T, C)).astype(np.float32).astype(np.float64)
    dy = (rng.normal(size=(batch, T, C)) * 1e-3).astype(np.float32).astype(np.float64)
    net = pm.Net(C, T, H, max_batch=batch)
    net.set_params(theta)
    g = host(net.backward(dev32(x), dev32(dy)))
    yq, cq = cn.forward(theta, x, C, H, bf16_points=True)
    gq = cn.backward(theta, cq, dy, C, H, bf16_points=True)
    y64, c64 = cn.forward(theta, x, C, H)
    g64 = cn.backward(theta, c64, dy, C, H)
    # per parameter block: W1, b1, W2, b2, W3, b3
    o = 0
    for name, k in zip(["W1", "b1", "W2", "b2", "W3", "b3"],
                       [H * C * 3, H, H * H * 3, H, C * H * 3, C]):
        assert rel(g[o:o + k], gq[o:o + k]) <= 5e-3, (name, rel(g[o:o + k], gq[o:o + k]))
        assert rel(g[o:o + k], g64[o:o + k]) <= 5e-2, (name, rel(g[o:o + k], g64[o:o + k]))
        o += k
    net.close()


def test_adam_parity():
    C = 60
    rng = np.random.default_rng(7)
    theta = params(C, 3)
    net = pm.Net(C, T, H, max_batch=4)
    net.set_params(theta)
    th, m, v = theta.copy(), np.zeros_like(theta), np.zeros_like(theta)
    for t in range(1, 4):
        g = rng.normal(size=theta.size).astype(np.float32).astype(np.float64)
        net.adam(dev32(g), 1e-3)
        th, m, v = cn.adam_step(th, g, m, v, t, 1e-3)
    got = net.get_params().astype(np.float64)
    assert np.max(np.abs(got - th)) <= 2e-7 * max(1.0, np.max(np.abs(th)))
    net.close()


def test_train_step_matches_oracle_step():
    C, count, batch = 60, 50, 16
    rng = np.random.default_rng(8)
    X = rng.normal(size=(count, T, C)).astype(np.float32).astype(np.float64)
    Y = (0.3 * rng.normal(size=(count, T, C))).astype(np.float32).astype(np.float64)
    idx = rng.integers(0, count, size=batch).astype(np.int32)
    idx[3] = -1                      # outside [0, count): a zero sample
    idx[9] = count
    theta = params(C, 9)
    net = pm.Net(C, T, H, max_batch=batch)
    net.set_params(theta)
    lr = 1e-3
    loss = net.train_step(torch.from_numpy(idx).to("cuda"), dev32(X), dev32(Y), lr)
    Xb = np.where((idx >= 0) & (idx < count), 1.0, 0.0)[:, None, None] * X[np.clip(idx, 0, count - 1)]
    Yb = np.where((idx >= 0) & (idx < count), 1.0, 0.0)[:, None, None] * Y[np.clip(idx, 0, count - 1)]
    yq, cq = cn.forward(theta, Xb, C, H, bf16_points=True)
    lq, dy = cn.mse(yq, Yb)
    gq = cn.backward(theta, cq, dy, C, H, bf16_points=True)
    assert abs(loss - lq) <= 1e-3 * lq
    th1, _, _ = cn.adam_step(theta, gq, np.zeros_like(theta), np.zeros_like(theta), 1, lr)
    got = net.get_params().astype(np.float64)
    # the first Adam step moves each parameter by about lr * sign(g); compare
    # where the sign is certain and count the rest
    sure = np.abs(gq) > 1e-2 * np.max(np.abs(gq))
    assert np.max(np.abs((got - theta)[sure] - (th1 - theta)[sure])) <= 1e-3 * lr
    assert np.mean(np.sign(got - theta) == np.sign(th1 - theta)) >= 0.98
    net.close()


def test_make_samples_parity():
    p, q, count = 12, 12, 9
    C = 4 * p + q
    rng = np.random.default_rng(10)
    r = rng.normal(size=(count, C * T)) * 10.0 ** rng.integers(-3, 3, size=(count, 1))
    e = rng.normal(size=(count, C * T))
    r[4] = 0.0                                    # zero residual: zero sample
    net = pm.Net(C, T, H, max_batch=4)
    X, Y = net.make_samples(p, q, dev64(r), dev64(e))
    X, Y = host(X), host(Y)
    for i in range(count):
        xs, ys = cn.make_sample(r[i], e[i], p, q, T)
        assert np.allclose(X[i], xs, rtol=2e-7, atol=1e-30)
        assert np.allclose(Y[i], ys, rtol=2e-7, atol=1e-30)
    net.close()


CASE = dict(kind="burgers", nx=12, nu=0.01, n=32, n_levels=3, seed=12)


def coarse_problem():
    prob, rng = make_problem(**CASE)
    return prob, rng, prob.p, prob.q, 4 * prob.p + prob.q


def test_vcycle_with_net_matches_oracle():
    prob, rng, p, q, C = coarse_problem()
    theta = params(C, 21, scale=0.5)
    H0 = Hierarchy(prob.levels, MGOptions())
    lvc = H0.levels[-1]

    def net_coarse(b_time):
        r = np.empty_like(b_time)
        r[lvc.perm] = b_time
        e = cn.coarse_correction(theta, r, p, q, T, H, bf16_points=True)
        return e[lvc.perm]

    H0.coarse_solve = net_coarse
    r = rng.normal(size=prob.size)
    ref = H0.vcycle(r)
    s = pm.Solver(prob.levels, pm.default_options(coarse_mode=1))
    net = pm.Net(C, T, H, max_batch=1)
    net.set_params(theta)
    s.attach_net(net)
    got = host(s.vcycle(dev64(r)))
    assert rel(got, ref) <= 5e-3, rel(got, ref)
    s.close()
    net.close()


def test_net_shape_must_match():
    prob, rng, p, q, C = coarse_problem()
    s = pm.Solver(prob.levels, pm.default_options())
    net = pm.Net(C + 1, T, H, max_batch=1)
    with pytest.raises(pm.PitmgError):
        s.attach_net(net)
    with pytest.raises(pm.PitmgError):
        s.set_options(coarse_mode=1)
        s.solve(dev64(make_rhs(prob, rng)))
    s.close()
    net.close()


def test_pairs_recorded_from_plain_coarse_solves():
    prob, rng, p, q, C = coarse_problem()
    b = make_rhs(prob, rng)
    s = pm.Solver(prob.levels, pm.default_options(restart=200, maxit=200))
    lc = C * T
    R = torch.zeros((5, lc), dtype=torch.float64, device="cuda")
    E = torch.zeros_like(R)
    s.arm_pairs(R, E, 5)
    x, st, rc = s.solve(dev64(b), tol=1e-10)
    assert s.pair_count() == 5 and st["coarse_calls"] >= 5
    Rh, Eh = host(R), host(E)
    from oracle import OracleLevel
    lv = prob.levels[-1]
    Ac = OracleLevel(lv.N, lv.V, lv.Z).A
    for i in range(5):
        # each pair is a coarse solve to the coarse tolerance (1e-3)
        assert np.linalg.norm(Rh[i]) > 0
        assert np.linalg.norm(Rh[i] - Ac @ Eh[i]) <= 1.01e-3 * np.linalg.norm(Rh[i])
    s.close()


def test_fgmres_with_net_and_stall_rule():
    prob, rng, p, q, C = coarse_problem()
    b = make_rhs(prob, rng)
    net = pm.Net(C, T, H, max_batch=1)
    net.set_params(params(C, 22, scale=0.5))
    # never stalls: every V-cycle uses the network, FGMRES still converges
    s = pm.Solver(prob.levels, pm.default_options(restart=300, maxit=300, coarse_mode=1,
                                                  stall_ratio=1e9))
    s.attach_net(net)
    x, st, rc = s.solve(dev64(b), tol=1e-10)
    A = prob.levels[0]
    assert rc == pm.PITMG_OK and st["converged"] == 1
    assert st["fallback_at"] == -1 and st["net_calls"] == st["iters"] and st["coarse_calls"] == 0
    from oracle import OracleLevel
    Ao = OracleLevel(A.N, A.V, A.Z).A
    assert np.linalg.norm(b - Ao @ host(x)) <= 1.01e-10 * np.linalg.norm(b)
    # stalls at once: the rule switches to GMRES + SGS after stall_steps steps
    s.set_options(restart=300, maxit=300, coarse_mode=1, stall_ratio=1e-12, stall_steps=2)
    x, st, rc = s.solve(dev64(b), tol=1e-10)
    assert rc == pm.PITMG_OK and st["fallback_at"] == 3
    assert st["net_calls"] == 3 and st["coarse_calls"] == st["iters"] - 3
    s.close()
    net.close()
