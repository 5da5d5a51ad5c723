"""Powell's dogleg for the discrete Burgers equation F(u, z~) = 0, with its
Gauss-Newton steps from minimum-norm augmented systems (Sec. 6, the
nonlinear solver applied to Burgers' equation in Sec. 6.2 and Table 6; the
minimum-norm problem of Sec. 3).  Test infrastructure: only tests/, the
package's smoke check and the benchmark's CPU baseline use it.

Unknowns x = (u, z~) in the unlifted type-major order [u_1..u_n | z~_1..z~_n]
(p = q = nx per step): the states u_k at steps k = 1..n and the scaled
controls z~_k = gamma z_k, so that dF/dz~ = -(df/dz) / gamma is the block
Z~ of the augmented systems (the control scaling of Sec. 4).

The state equation, backward Euler in time (theta = 1) on n steps of
dt = T / n and upwind differences in space on nx interior nodes of [0, 1]
(h = 1 / (nx + 1), homogeneous Dirichlet values, Sec. 6.2), the convective
term in flux form, (u^2 / 2)_x by the backward (upwind, u >= 0) difference:

    F_k(u, z~) = (u_k - u_{k-1}) / dt - f(u_k, z~_k / gamma),   u_0 = w0,
    f_i(w, z)  = nu (w_{i+1} - 2 w_i + w_{i-1}) / h^2 - (w_i^2 - w_{i-1}^2) / (2 h) + z_i.

(The flux form is the reading for this nonlinear solve: with the
convective term as w_i (w_i - w_{i-1}) / h the inviscid discrete equation
keeps the shock of the step at rest and has further roots, and the
continuation stalls at small viscosities.)

B = dF, one row block per step: dF_k/du_k = I/dt - df/du(u_k) (the block
N_k of the systems: diagonal 1/dt + 2 nu/h^2 + u_i/h, sub-diagonal
-(nu/h^2 + u_{i-1}/h), super-diagonal -nu/h^2), dF_k/du_{k-1} = -I/dt (V),
dF_k/dz~_k = -I/gamma (Z~).

Dogleg (Powell's hybrid method in its trust-region form), one iteration at
x with residual F, Jacobian B and radius delta:
  * Gauss-Newton step s_N: the minimum-norm solution of B s = -F, from the
    augmented system [[I, B^T], [B, 0]] (s, y) = (0, -F);
  * Cauchy step s_C = -tau g, g = B^T F, tau = |g|^2 / |B g|^2 (the
    minimiser of the model m(s) = |F + B s|^2 / 2 along -g);
  * s = s_N if |s_N| <= delta; else -(delta / |g|) g if |s_C| >= delta;
    else s_C + beta (s_N - s_C) with beta in (0, 1] and |s| = delta;
  * rho = (|F(x)|^2 - |F(x + s)|^2) / (|F|^2 - |F + B s|^2); the step is
    taken when rho > eta; delta becomes |s| / 4 when rho < 1/4 and doubles
    when rho > 3/4 and the step reached the boundary.
Readings (the paper names the method, not these constants): eta = 1e-4;
delta starts at |s_N| of the first iteration (the first step is a full
Gauss-Newton step); the iteration stops when |F(x)| <= ftol |F(x_start)| at
the start of that viscosity, and the linear tolerance 1e-6 of Sec. 6 bounds
the inexactness of s_N (here s_N is exact: a sparse direct solve).
Continuation (Sec. 6.2): the solution for each viscosity is the starting
point for the next.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class BurgersSpec:
    nx: int
    n: int
    T: float
    gamma: float
    w0: np.ndarray               # (nx,) state at t = 0

    @property
    def h(self) -> float:
        return 1.0 / (self.nx + 1)

    @property
    def dt(self) -> float:
        return self.T / self.n

    @property
    def size(self) -> int:
        return 2 * self.nx * self.n


def step_initial_state(nx: int) -> np.ndarray:
    """u_0 of Sec. 6.2: 1 on (0, 1/2], 0 on (1/2, 1), at the interior nodes."""
    x = np.arange(1, nx + 1) / (nx + 1)
    return np.where(x <= 0.5, 1.0, 0.0)


def split(spec: BurgersSpec, x: np.ndarray):
    p, n = spec.nx, spec.n
    return x[:p * n].reshape(n, p), x[p * n:].reshape(n, p)


def residual(spec: BurgersSpec, x: np.ndarray, nu: float) -> np.ndarray:
    """F(u, z~) stacked over the steps, (n p,)."""
    u, zt = split(spec, x)
    h, dt = spec.h, spec.dt
    prev = np.vstack([spec.w0[None, :], u[:-1]])
    left = np.zeros_like(u)
    left[:, 1:] = u[:, :-1]
    right = np.zeros_like(u)
    right[:, :-1] = u[:, 1:]
    f = nu * (right - 2.0 * u + left) / (h * h) - (u * u - left * left) / (2.0 * h) \
        + zt / spec.gamma
    return ((u - prev) / dt - f).reshape(-1)


def jacobian(spec: BurgersSpec, x: np.ndarray, nu: float) -> sp.csr_matrix:
    """B = dF, (n p) x (2 n p), columns in the order [u | z~]."""
    u, _ = split(spec, x)
    p, n, h, dt = spec.nx, spec.n, spec.h, spec.dt
    a = nu / (h * h)
    rows, cols, vals = [], [], []
    idx = np.arange(p)
    for k in range(n):
        r0 = k * p
        uk = u[k]
        # d/du_k of (u_k / dt - f): diagonal, sub- and super-diagonal
        rows += [r0 + idx, r0 + idx[1:], r0 + idx[:-1]]
        cols += [r0 + idx, r0 + idx[:-1], r0 + idx[1:]]
        vals += [1.0 / dt + 2.0 * a + uk / h, -(a + uk[:-1] / h), -a * np.ones(p - 1)]
        if k > 0:                               # d/du_{k-1}
            rows.append(r0 + idx)
            cols.append(r0 - p + idx)
            vals.append(-np.ones(p) / dt)
        rows.append(r0 + idx)                   # d/dz~_k
        cols.append(n * p + r0 + idx)
        vals.append(-np.ones(p) / spec.gamma)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n * p, 2 * n * p))


def min_norm_step(B: sp.csr_matrix, F: np.ndarray) -> np.ndarray:
    """The minimum-norm s with B s = -F, from the augmented system
    [[I, B^T], [B, 0]] (s, y) = (0, -F) (Sec. 3), solved directly."""
    m, nv = B.shape
    A = sp.bmat([[sp.identity(nv), B.T], [B, None]], format="csc")
    rhs = np.concatenate([np.zeros(nv), -F])
    return spla.spsolve(A, rhs)[:nv]


def dogleg_step(sN: np.ndarray, g: np.ndarray, Bg: np.ndarray, delta: float):
    """The dogleg point for radius delta: (s, kind) with kind "newton",
    "cauchy" (the steepest-descent boundary point) or "dogleg"."""
    nN = np.linalg.norm(sN)
    if nN <= delta:
        return sN.copy(), "newton"
    gg = float(g @ g)
    if gg == 0.0:
        return sN * (delta / nN), "newton"
    tau = gg / float(Bg @ Bg)
    sC = -tau * g
    nC = np.linalg.norm(sC)
    if nC >= delta:
        return -(delta / np.sqrt(gg)) * g, "cauchy"
    # |sC + beta d| = delta, d = sN - sC, beta in (0, 1]
    d = sN - sC
    a = float(d @ d)
    b = 2.0 * float(sC @ d)
    c = nC * nC - delta * delta
    beta = (-b + np.sqrt(b * b - 4.0 * a * c)) / (2.0 * a)
    return sC + beta * d, "dogleg"


@dataclass
class DoglegInfo:
    iters: int = 0
    accepted: int = 0
    converged: bool = False
    fnorms: List[float] = field(default_factory=list)
    kinds: List[str] = field(default_factory=list)


def dogleg_solve(spec: BurgersSpec, x0: np.ndarray, nu: float, ftol: float = 1e-8,
                 maxit: int = 50, eta: float = 1e-4, delta0: Optional[float] = None):
    """Powell's dogleg for F(x) = 0 from x0 (module docstring)."""
    x = np.array(x0, dtype=np.float64)
    F = residual(spec, x, nu)
    f0 = np.linalg.norm(F)
    info = DoglegInfo(fnorms=[f0])
    delta = delta0
    if f0 == 0.0:
        info.converged = True
        return x, info
    for _ in range(maxit):
        if np.linalg.norm(F) <= ftol * f0:
            info.converged = True
            break
        B = jacobian(spec, x, nu)
        sN = min_norm_step(B, F)
        g = B.T @ F
        Bg = B @ g
        if delta is None:
            delta = np.linalg.norm(sN)
        s, kind = dogleg_step(sN, g, Bg, delta)
        ns = np.linalg.norm(s)
        ff = float(F @ F)
        pred = ff - float(np.sum((F + B @ s) ** 2))
        Fn = residual(spec, x + s, nu)
        ared = ff - float(Fn @ Fn)
        rho = ared / pred if pred > 0.0 else -1.0
        if rho < 0.25:
            delta = 0.25 * ns
        elif rho > 0.75 and ns >= 0.99 * delta:
            delta = 2.0 * delta
        info.iters += 1
        info.kinds.append(kind)
        if rho > eta:
            x = x + s
            F = Fn
            info.accepted += 1
        info.fnorms.append(float(np.linalg.norm(F)))
    else:
        info.converged = bool(np.linalg.norm(F) <= ftol * f0)
    return x, info


def continuation(spec: BurgersSpec, nus: Sequence[float], x0: Optional[np.ndarray] = None,
                 **kw):
    """Dogleg solves for the viscosities in order, each from the previous
    solution (Sec. 6.2); x0 defaults to u_k = w0 for every step, z~ = 0."""
    if x0 is None:
        x0 = np.concatenate([np.tile(spec.w0, spec.n), np.zeros(spec.n * spec.nx)])
    x = x0
    out = []
    for nu in nus:
        x, info = dogleg_solve(spec, x, nu, **kw)
        out.append((nu, x.copy(), info))
    return out


def forward_euler_newton(spec: BurgersSpec, nu: float, tol: float = 1e-13, maxit: int = 50):
    """The states with z = 0, step by step: Newton's method on
    (u_k - u_{k-1}) / dt - f(u_k, 0) = 0 for k = 1..n (a reference for the
    limit gamma -> infinity, where the minimum-norm steps leave the control
    at zero)."""
    p, n, h, dt = spec.nx, spec.n, spec.h, spec.dt
    a = nu / (h * h)
    U = np.empty((n, p))
    prev = spec.w0.copy()
    for k in range(n):
        w = prev.copy()
        for _ in range(maxit):
            left = np.concatenate([[0.0], w[:-1]])
            right = np.concatenate([w[1:], [0.0]])
            G = (w - prev) / dt - (a * (right - 2.0 * w + left) - (w * w - left * left) / (2.0 * h))
            J = sp.diags([-(a + w[:-1] / h), 1.0 / dt + 2.0 * a + w / h,
                          -a * np.ones(p - 1)], [-1, 0, 1], format="csc")
            dw = spla.spsolve(J, -G)
            w = w + dw
            if np.linalg.norm(dw) <= tol * max(1.0, np.linalg.norm(w)):
                break
        U[k] = w
        prev = w
    return U
