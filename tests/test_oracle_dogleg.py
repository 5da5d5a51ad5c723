"""Pins of the oracle's Burgers residual, its Jacobian, the minimum-norm
step and Powell's dogleg (oracle/dogleg.py; Sec. 6, Sec. 6.2, Sec. 3).

Each pin checks against something other than the oracle's own formula:
finite differences of F for B = dF, a manufactured PDE solution for the
consistency (order one in h and dt) of F, the pseudo-inverse for the
minimum-norm step, a hand-worked two-dimensional dogleg, and a plain
step-by-step Newton time integration for the gamma -> infinity limit of the
continuation.
"""
import numpy as np
import pytest

from oracle.dogleg import (BurgersSpec, continuation, dogleg_solve, dogleg_step,
                           forward_euler_newton, jacobian, min_norm_step, residual,
                           step_initial_state)


def spec(nx=8, n=6, gamma=1e2, T=1.0, w0=None):
    w0 = step_initial_state(nx) if w0 is None else w0
    return BurgersSpec(nx=nx, n=n, T=T, gamma=gamma, w0=w0)


@pytest.mark.parametrize("nu", [0.05, 0.0])
def test_jacobian_matches_central_differences(nu):
    s = spec()
    rng = np.random.default_rng(5)
    x = rng.normal(size=s.size)
    B = jacobian(s, x, nu).toarray()
    eps = 1e-6
    fd = np.empty_like(B)
    for j in range(s.size):
        e = np.zeros(s.size)
        e[j] = eps
        fd[:, j] = (residual(s, x + e, nu) - residual(s, x - e, nu)) / (2 * eps)
    assert np.abs(B - fd).max() <= 1e-6 * max(1.0, np.abs(B).max())


def test_residual_is_first_order_consistent():
    """u = sin(pi x) e^{-t} with the control that makes it an exact PDE
    solution: the discrete residual falls like h + dt (upwind differences
    and backward Euler are first order)."""
    nu, gamma = 0.1, 1e3
    errs = []
    for m in (32, 64, 128):
        s = BurgersSpec(nx=m - 1, n=m, T=0.5, gamma=gamma,
                        w0=np.sin(np.pi * np.arange(1, m) / m))
        xg = np.arange(1, m) / m
        t = s.dt * np.arange(1, s.n + 1)[:, None]
        u = np.sin(np.pi * xg)[None, :] * np.exp(-t)
        z = -u + nu * np.pi ** 2 * u + u * np.pi * np.cos(np.pi * xg)[None, :] * np.exp(-t)
        F = residual(s, np.concatenate([u.ravel(), gamma * z.ravel()]), nu)
        errs.append(np.abs(F).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 1.6 < r1 < 2.4 and 1.6 < r2 < 2.4, errs


def test_min_norm_step_is_the_pseudoinverse_solution():
    s = spec(nx=6, n=5)
    rng = np.random.default_rng(7)
    x = np.abs(rng.normal(size=s.size))
    B = jacobian(s, x, 0.03)
    F = residual(s, x, 0.03)
    sn = min_norm_step(B, F)
    ref = -np.linalg.pinv(B.toarray()) @ F
    assert np.linalg.norm(sn - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.linalg.norm(B @ sn + F) <= 1e-10 * np.linalg.norm(F)


def test_dogleg_step_cases():
    """B = diag(1, 10), F = (1, 1): s_N = (-1, -0.1), g = (1, 10),
    B g = (1, 100), tau = 101 / 10001."""
    B = np.diag([1.0, 10.0])
    F = np.array([1.0, 1.0])
    sN = np.array([-1.0, -0.1])
    g = B.T @ F
    Bg = B @ g
    s, kind = dogleg_step(sN, g, Bg, 2.0)
    assert kind == "newton" and np.allclose(s, sN)
    tau = 101.0 / 10001.0
    sC = -tau * g
    s, kind = dogleg_step(sN, g, Bg, 0.05)                 # |s_C| ~ 0.1015 > 0.05
    assert kind == "cauchy" and np.allclose(s, -0.05 * g / np.linalg.norm(g))
    delta = 0.5                                           # between |s_C| and |s_N|
    s, kind = dogleg_step(sN, g, Bg, delta)
    assert kind == "dogleg"
    assert abs(np.linalg.norm(s) - delta) < 1e-12
    beta = (s - sC) @ (sN - sC) / ((sN - sC) @ (sN - sC))
    assert 0.0 < beta < 1.0
    assert np.allclose(s, sC + beta * (sN - sC))
    # the model decreases along the dogleg path
    m = lambda d: 0.5 * np.sum((F + B @ d) ** 2)
    assert m(sN) < m(s) < m(sC) < m(np.zeros(2))


def test_continuation_reaches_the_forward_solution():
    """With gamma = 1e5 the minimum-norm steps leave the control near zero,
    so the states approach those of plain step-by-step Newton time
    integration (z = 0); every viscosity of the continuation converges in a
    few iterations (Table 6 reports 2 to 9), and near the solution the
    Gauss-Newton steps converge superlinearly.  At nu = 0 the states at
    t = 1 approach the entropy solution u(x, 1) = x of the step (the
    rarefaction from the left boundary has just reached the shock)."""
    s = spec(nx=48, n=48, gamma=1e5)
    nus = [1e-1, 1e-2, 1e-3, 1e-4, 0.0]
    out = continuation(s, nus, ftol=1e-10)
    for nu, x, info in out:
        assert info.converged, (nu, info.fnorms)
        assert info.iters <= 10
        u, zt = x[:s.nx * s.n].reshape(s.n, s.nx), x[s.nx * s.n:]
        U = forward_euler_newton(s, nu)
        assert np.linalg.norm(u - U) <= 1e-6 * np.linalg.norm(U), nu
        assert np.linalg.norm(zt / s.gamma) <= 1e-6 * np.linalg.norm(U)
        assert u.min() >= -1e-9 and u.max() <= 1.0 + 1e-9     # upwind: no over- or undershoot
    # superlinear: the last accepted reductions of the first stage
    f = out[0][2].fnorms
    assert f[-1] / f[-2] < 0.1 * (f[-2] / f[-3]) or f[-1] <= 1e-10 * f[0]
    # inviscid states at t = 1 against u = x away from the two boundary layers
    xg = np.arange(1, s.nx + 1) / (s.nx + 1)
    u1 = out[-1][1][(s.n - 1) * s.nx:s.n * s.nx]
    mid = (xg > 0.15) & (xg < 0.75)
    assert np.abs(u1[mid] - xg[mid]).max() < 0.1


def test_dogleg_from_a_far_start_takes_restricted_steps():
    """A start away from the solution (states 2 u_0) with a small initial
    radius: the iteration takes Cauchy steps (the steepest-descent boundary
    point) and dogleg steps first, then Gauss-Newton steps, and converges."""
    s = spec(nx=12, n=8, gamma=1e5)
    x0 = np.concatenate([np.tile(2.0 * s.w0, s.n), np.zeros(s.n * s.nx)])
    x, info = dogleg_solve(s, x0, 1e-2, ftol=1e-10, delta0=0.5, maxit=100)
    assert info.converged
    assert info.kinds[0] == "cauchy" and "dogleg" in info.kinds and info.kinds[-1] == "newton"
    U = forward_euler_newton(s, 1e-2)
    assert np.linalg.norm(x[:s.nx * s.n].reshape(s.n, s.nx) - U) <= 1e-6 * np.linalg.norm(U)
