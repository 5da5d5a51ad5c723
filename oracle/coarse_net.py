"""Learned coarse-grid correction: plain FP64 reference (TEST INFRASTRUCTURE).

The coarsest-level solve of the V-cycle (GMRES + symmetric block
Gauss-Seidel to a relative tolerance, Sec. 5.3.4) may be replaced by a small
network; FGMRES admits a preconditioner that changes from step to step, which
is why the paper uses it (Sec. 5.3.4, last paragraph).  The paper itself has
no learned component: this module defines the network as this project reads
it, so that the GPU kernels can be checked against something written from the
definitions.

Network (over the T coarse steps, one sample = one coarse residual):

    x  = r_c / s,   s = rms(r_c) = ||r_c||_2 / sqrt(len)      (s = 0 -> e_c = 0)
    h1 = tanh(conv(W1, b1, x))     W1: [H][C][3]
    h2 = tanh(conv(W2, b2, h1))    W2: [H][H][3]
    y  = conv(W3, b3, h2)          W3: [C][H][3]
    e_c = s * y

with conv(W, b, x)[t, o] = b[o] + sum_{c, d} W[o, c, d] x[t + d - 1, c] and x
taken as zero outside 0 <= t < T (a width-3 cross-correlation in time with
zero padding).  Samples are node-major, x[t, :] = (u_t, v_t, z_t, lambda_t,
mu_t), so C = 4p + q.  The flat parameter vector is
[W1, b1, W2, b2, W3, b3], each row-major.

Training minimises the mean squared error over all entries of y against the
normalised target e_c / s, with Adam (Kingma and Ba, 2015: bias-corrected
first and second moments).

bf16=True reproduces the rounding points of the GPU kernels, which multiply
bfloat16 operands and accumulate in FP32: the network input, the weights, the
hidden activations and, in the backward pass, the output gradients of each
layer are rounded to bfloat16 (round to nearest even, from FP32) before they
enter a product.  Everything else here stays FP64.
"""
from __future__ import annotations

import numpy as np

from workloads import coarse_net_params

WIDTH = 3


# ---------------------------------------------------------------------------
# parameters
# ---------------------------------------------------------------------------

def param_count(C: int, H: int) -> int:
    return H * C * WIDTH + H + H * H * WIDTH + H + C * H * WIDTH + C


def unpack(theta: np.ndarray, C: int, H: int):
    """Views (W1, b1, W2, b2, W3, b3) of the flat parameter vector."""
    shapes = [(H, C, WIDTH), (H,), (H, H, WIDTH), (H,), (C, H, WIDTH), (C,)]
    out, o = [], 0
    for sh in shapes:
        k = int(np.prod(sh))
        out.append(theta[o:o + k].reshape(sh))
        o += k
    if o != theta.size:
        raise ValueError("parameter vector has the wrong length")
    return out


def init_params(C: int, H: int, rng: np.random.Generator) -> np.ndarray:
    """Seeded initial parameters (drawn by the shared input generators)."""
    return coarse_net_params(C, H, int(rng.integers(0, 2 ** 31)), WIDTH)


# ---------------------------------------------------------------------------
# bfloat16 rounding (round to nearest, ties to even, from FP32)
# ---------------------------------------------------------------------------

def bf16(a: np.ndarray) -> np.ndarray:
    u = np.ascontiguousarray(np.asarray(a, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _q(a, on):
    return bf16(a) if on else a


# ---------------------------------------------------------------------------
# layers
# ---------------------------------------------------------------------------

def conv(W: np.ndarray, b: np.ndarray, x: np.ndarray) -> np.ndarray:
    """x: [B, T, Cin] -> [B, T, Cout]; width-3 cross-correlation, zero padding."""
    B, T, _ = x.shape
    xp = np.zeros((B, T + 2, x.shape[2]))
    xp[:, 1:T + 1] = x
    y = np.broadcast_to(b, (B, T, W.shape[0])).copy()
    for d in range(WIDTH):
        y += xp[:, d:d + T, :] @ W[:, :, d].T
    return y


def conv_backward(W: np.ndarray, x: np.ndarray, dy: np.ndarray):
    """Gradients of conv(W, b, x) for the output gradient dy: (dW, db, dx)."""
    B, T, Cin = x.shape
    xp = np.zeros((B, T + 2, Cin))
    xp[:, 1:T + 1] = x
    dW = np.empty_like(W)
    for d in range(WIDTH):
        dW[:, :, d] = dy.reshape(-1, dy.shape[2]).T @ xp[:, d:d + T, :].reshape(-1, Cin)
    db = dy.sum(axis=(0, 1))
    # x[t'] feeds y[t' - d + 1] through tap d
    dyp = np.zeros((B, T + 2, dy.shape[2]))
    dyp[:, 1:T + 1] = dy
    dx = np.zeros((B, T, Cin))
    for d in range(WIDTH):
        dx += dyp[:, 2 - d:2 - d + T, :] @ W[:, :, d]
    return dW, db, dx


def forward(theta: np.ndarray, x: np.ndarray, C: int, H: int, bf16_points: bool = False):
    """y = net(x) for x: [B, T, C]; returns (y, cache for backward)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, C, H)
    q = bf16_points
    x0 = _q(np.asarray(x, dtype=np.float32).astype(np.float64) if q else x, q)
    Wq = [_q(W, q) for W in (W1, W2, W3)]
    h1 = np.tanh(conv(Wq[0], b1, x0))
    if q:
        h1 = np.asarray(h1, dtype=np.float32).astype(np.float64)
    h1q = _q(h1, q)
    h2 = np.tanh(conv(Wq[1], b2, h1q))
    if q:
        h2 = np.asarray(h2, dtype=np.float32).astype(np.float64)
    h2q = _q(h2, q)
    y = conv(Wq[2], b3, h2q)
    return y, (x0, h1, h1q, h2, h2q, Wq)


def backward(theta: np.ndarray, cache, dy: np.ndarray, C: int, H: int,
             bf16_points: bool = False) -> np.ndarray:
    """Gradient of a scalar loss with output gradient dy w.r.t. the flat
    parameter vector (same layout)."""
    q = bf16_points
    x0, h1, h1q, h2, h2q, Wq = cache
    g3 = _q(dy, q)
    dW3, db3, dh2 = conv_backward(Wq[2], h2q, g3)
    g2 = _q(dh2 * (1.0 - h2 * h2), q)
    dW2, db2, dh1 = conv_backward(Wq[1], h1q, g2)
    g1 = _q(dh1 * (1.0 - h1 * h1), q)
    dW1, db1, _ = conv_backward(Wq[0], x0, g1)
    return np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])


def mse(y: np.ndarray, target: np.ndarray):
    """Mean squared error over all entries and its gradient w.r.t. y."""
    d = y - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(theta, grad, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# coarse vectors <-> samples
# ---------------------------------------------------------------------------

def node_major(x_type: np.ndarray, p: int, q: int, T: int) -> np.ndarray:
    """Type-major coarse vector [u | v | z | lambda | mu] -> [T, 4p+q]."""
    u = x_type[:T * p].reshape(T, p)
    v = x_type[T * p:2 * T * p].reshape(T, p)
    z = x_type[2 * T * p:2 * T * p + T * q].reshape(T, q)
    lam = x_type[2 * T * p + T * q:3 * T * p + T * q].reshape(T, p)
    mu = x_type[3 * T * p + T * q:].reshape(T, p)
    return np.concatenate([u, v, z, lam, mu], axis=1)


def type_major(y: np.ndarray, p: int, q: int) -> np.ndarray:
    """Inverse of node_major."""
    u, v = y[:, :p], y[:, p:2 * p]
    z, lam, mu = y[:, 2 * p:2 * p + q], y[:, 2 * p + q:3 * p + q], y[:, 3 * p + q:]
    return np.concatenate([u.ravel(), v.ravel(), z.ravel(), lam.ravel(), mu.ravel()])


def rms(r: np.ndarray) -> float:
    return float(np.linalg.norm(r) / np.sqrt(r.size))


def make_sample(r_type: np.ndarray, e_type: np.ndarray, p: int, q: int, T: int):
    """Normalised training pair (x, target), each [T, 4p+q]."""
    s = rms(r_type)
    if s == 0.0:
        return np.zeros((T, 4 * p + q)), np.zeros((T, 4 * p + q))
    return node_major(r_type / s, p, q, T), node_major(e_type / s, p, q, T)


def coarse_correction(theta: np.ndarray, r_type: np.ndarray, p: int, q: int, T: int, H: int,
                      bf16_points: bool = False) -> np.ndarray:
    """e_c = s * net(r_c / s) for one type-major coarse residual."""
    s = rms(r_type)
    if s == 0.0:
        return np.zeros_like(r_type)
    x = node_major(r_type / s, p, q, T)[None]
    y, _ = forward(theta, x, 4 * p + q, H, bf16_points)
    return s * type_major(y[0], p, q)
