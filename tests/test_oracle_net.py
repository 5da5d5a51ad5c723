"""Pins of the learned coarse correction's FP64 reference (oracle/coarse_net.py).

Each function is checked against something other than itself: PyTorch's
conv1d and autograd (an independent implementation of the same definitions),
central finite differences, the closed form of Adam under a constant
gradient, PyTorch's Adam, PyTorch's bfloat16 conversion and hand-worked
rounding ties, and the inverse relation of the two vector layouts.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import coarse_net as cn
from oracle.system import type_offsets


def torch_net(theta, x, C, H):
    W1, b1, W2, b2, W3, b3 = [torch.tensor(a) for a in cn.unpack(theta, C, H)]
    xt = torch.tensor(x).permute(0, 2, 1)                       # B, C, T
    F = torch.nn.functional
    h1 = torch.tanh(F.conv1d(xt, W1, b1, padding=1))
    h2 = torch.tanh(F.conv1d(h1, W2, b2, padding=1))
    return F.conv1d(h2, W3, b3, padding=1).permute(0, 2, 1)


def small(C=6, H=4, T=5, B=3, seed=0):
    rng = np.random.default_rng(seed)
    theta = cn.init_params(C, H, rng) * 3.0
    x = rng.normal(size=(B, T, C))
    return theta, x, C, H


def test_param_count_and_layout():
    C, H = 10, 4
    assert cn.param_count(C, H) == 4 * 10 * 3 + 4 + 4 * 4 * 3 + 4 + 10 * 4 * 3 + 10
    theta = np.arange(cn.param_count(C, H), dtype=float)
    W1, b1, W2, b2, W3, b3 = cn.unpack(theta, C, H)
    assert W1.shape == (H, C, 3) and W3.shape == (C, H, 3)
    assert W1[0, 0, 1] == 1 and b1[0] == H * C * 3 and b3[-1] == theta[-1]


def test_forward_matches_torch_conv1d():
    theta, x, C, H = small()
    y, _ = cn.forward(theta, x, C, H)
    ref = torch_net(theta, x, C, H).numpy()
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_forward_t1_and_t2_padding():
    # the zero padding is what a width-3 filter sees at both ends
    for T in (1, 2):
        theta, x, C, H = small(T=T, seed=T)
        y, _ = cn.forward(theta, x, C, H)
        assert np.allclose(y, torch_net(theta, x, C, H).numpy(), rtol=0, atol=1e-12)


def test_backward_matches_torch_autograd():
    theta, x, C, H = small(seed=3)
    tgt = np.random.default_rng(4).normal(size=x.shape)
    y, cache = cn.forward(theta, x, C, H)
    loss, dy = cn.mse(y, tgt)
    g = cn.backward(theta, cache, dy, C, H)
    th = torch.tensor(theta, requires_grad=True)
    parts, o = [], 0
    for sh in [(H, C, 3), (H,), (H, H, 3), (H,), (C, H, 3), (C,)]:
        k = int(np.prod(sh))
        parts.append(th[o:o + k].reshape(sh))
        o += k
    F = torch.nn.functional
    xt = torch.tensor(x).permute(0, 2, 1)
    h1 = torch.tanh(F.conv1d(xt, parts[0], parts[1], padding=1))
    h2 = torch.tanh(F.conv1d(h1, parts[2], parts[3], padding=1))
    yt = F.conv1d(h2, parts[4], parts[5], padding=1).permute(0, 2, 1)
    lt = ((yt - torch.tensor(tgt)) ** 2).mean()
    lt.backward()
    assert abs(float(lt.detach()) - loss) <= 1e-12 * loss
    assert np.max(np.abs(g - th.grad.numpy())) <= 1e-11 * np.max(np.abs(g))


def test_backward_matches_central_differences():
    theta, x, C, H = small(C=5, H=3, T=4, B=2, seed=5)
    tgt = np.random.default_rng(6).normal(size=x.shape)

    def L(th):
        return cn.mse(cn.forward(th, x, C, H)[0], tgt)[0]

    y, cache = cn.forward(theta, x, C, H)
    g = cn.backward(theta, cache, cn.mse(y, tgt)[1], C, H)
    rng = np.random.default_rng(7)
    for i in rng.choice(theta.size, size=40, replace=False):
        h = 1e-6
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (L(tp) - L(tm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_adam_constant_gradient_closed_form():
    # with a constant gradient the bias-corrected moments are exactly g and
    # g^2, so every step moves by lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3])
    th = np.array([1.0, 1.0, 1.0])
    m = np.zeros(3)
    v = np.zeros(3)
    lr, eps = 0.01, 1e-8
    for t in range(1, 6):
        th, m, v = cn.adam_step(th, g, m, v, t, lr)
    expect = 1.0 - 5 * lr * g / (np.abs(g) + eps)
    assert np.allclose(th, expect, rtol=0, atol=1e-14)


def test_adam_matches_torch():
    rng = np.random.default_rng(8)
    th0 = rng.normal(size=20)
    p = torch.nn.Parameter(torch.tensor(th0))
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    th, m, v = th0.copy(), np.zeros(20), np.zeros(20)
    for t in range(1, 8):
        g = rng.normal(size=20)
        p.grad = torch.tensor(g)
        opt.step()
        th, m, v = cn.adam_step(th, g, m, v, t, 1e-3)
    assert np.max(np.abs(th - p.detach().numpy())) <= 1e-12


def test_bf16_rounding_ties_and_torch():
    one = 1.0
    ulp = 2.0 ** -7
    assert cn.bf16(np.array([one]))[0] == 1.0
    assert cn.bf16(np.array([one + ulp / 2]))[0] == 1.0             # tie -> even (down)
    assert cn.bf16(np.array([one + 1.5 * ulp]))[0] == one + 2 * ulp  # tie -> even (up)
    assert cn.bf16(np.array([one + 0.75 * ulp]))[0] == one + ulp
    assert cn.bf16(np.array([-3.0]))[0] == -3.0
    x = np.random.default_rng(9).normal(size=10000) * 10.0 ** np.random.default_rng(10).integers(
        -8, 8, size=10000)
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(cn.bf16(x), ref)


def test_node_major_layout_round_trip_and_offsets():
    p, q, T = 3, 2, 4
    C = 4 * p + q
    x = np.arange(C * T, dtype=float)
    y = cn.node_major(x, p, q, T)
    assert y.shape == (T, C)
    assert np.array_equal(cn.type_major(y, p, q), x)
    off = type_offsets(p, q, T)
    # row t = (u_t, v_t, z_t, lambda_t, mu_t), each read at its type's offset
    t = 2
    assert np.array_equal(y[t, :p], x[off["u"] + t * p: off["u"] + (t + 1) * p])
    assert np.array_equal(y[t, p:2 * p], x[off["v"] + t * p: off["v"] + (t + 1) * p])
    assert np.array_equal(y[t, 2 * p:2 * p + q], x[off["z"] + t * q: off["z"] + (t + 1) * q])
    assert np.array_equal(y[t, 2 * p + q:3 * p + q], x[off["lam"] + t * p: off["lam"] + (t + 1) * p])
    assert np.array_equal(y[t, 3 * p + q:], x[off["mu"] + t * p: off["mu"] + (t + 1) * p])


def test_coarse_correction_special_cases():
    p, q, T, H = 2, 1, 8, 4
    C = 4 * p + q
    theta = np.zeros(cn.param_count(C, H))
    *_, b3 = cn.unpack(theta, C, H)
    b3[:] = np.arange(C) + 1.0
    r = np.random.default_rng(11).normal(size=C * T)
    e = cn.coarse_correction(theta, r, p, q, T, H)
    # zero weights: y = b3 in every row, scaled by rms(r)
    assert np.allclose(e, cn.rms(r) * cn.type_major(np.tile(b3, (T, 1)), p, q))
    assert np.all(cn.coarse_correction(theta, np.zeros(C * T), p, q, T, H) == 0.0)
    # scale equivariance: e(a r) = a e(r) for a > 0
    theta = cn.init_params(C, H, np.random.default_rng(12))
    e1 = cn.coarse_correction(theta, r, p, q, T, H)
    e2 = cn.coarse_correction(theta, 7.5 * r, p, q, T, H)
    assert np.allclose(e2, 7.5 * e1, rtol=1e-12, atol=0)


def test_bf16_points_stay_close_to_fp64():
    theta, x, C, H = small(C=32, H=16, T=8, B=4, seed=13)
    y, _ = cn.forward(theta, x, C, H)
    yq, _ = cn.forward(theta, x, C, H, bf16_points=True)
    assert np.linalg.norm(yq - y) <= 3e-2 * np.linalg.norm(y)


def test_training_steps_reduce_the_loss():
    C, H, T = 8, 8, 4
    rng = np.random.default_rng(14)
    X = rng.normal(size=(64, T, C))
    A = rng.normal(size=(C, C)) / np.sqrt(C)
    Y = X @ A.T                                          # a learnable linear map
    theta = cn.init_params(C, H, rng)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    first = None
    for t in range(1, 301):
        y, cache = cn.forward(theta, X, C, H)
        loss, dy = cn.mse(y, Y)
        first = loss if first is None else first
        theta, m, v = cn.adam_step(theta, cn.backward(theta, cache, dy, C, H), m, v, t, 1e-2)
    assert loss < 0.2 * first
