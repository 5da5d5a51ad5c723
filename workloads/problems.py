"""Model problems and the per-level Jacobian blocks of the lifted constraint.

Blocks follow Sec. 4.1 eq. (blocks) with the virtual-variable substitution of
Sec. 5.1: for step k on a grid of step dt, with physical state w_k, physical
virtual state w_{k-1} (the lifted iterate has v = u) and physical control
zeta_k,

    N_k  = ( M - theta*dt*du f(w_k, zeta_k) ) / dt
    V_k  = ( -M - (1-theta)*dt*du f(w_{k-1}, zeta_k) ) / dt      (k >= 2)
    Z~_k = ( -theta*dt*dz f(w_k, zeta_k)
             - (1-theta)*dt*dz f(w_{k-1}, zeta_k) ) / (gamma*dt)

V_1 multiplies v_0 := 0 and is never used.  The Euclidean variables of
Sec. 4.1 relate to the physical ones by u = sqrt(dt) w and
z = gamma sqrt(dt) zeta; the blocks only need the physical point.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Tuple

import numpy as np


# ---------------------------------------------------------------------------
# Right-hand sides du f and dz f of the two model ODEs
# ---------------------------------------------------------------------------

def vanderpol_jacobians(mu: float = 0.1, q: int = 1) -> Callable:
    """du f and dz f of the van der Pol system of Sec. 6.1.

    f(u, z) = (u2 [+ z1], mu (1 - u1^2) u2 - u1 + z_last).  With q = 2 both
    equations carry a control (as in the paper); with q = 1 only the second
    one does.  Returns jac(w, zeta) -> (du f (m,2,2), dz f (2,q)); dz f does
    not depend on the point, so it is returned once.
    """
    if q not in (1, 2):
        raise ValueError("van der Pol supports q = 1 or 2")

    def jac(w: np.ndarray, zeta: np.ndarray):
        u1, u2 = w[:, 0], w[:, 1]
        m = w.shape[0]
        du = np.zeros((m, 2, 2))
        du[:, 0, 1] = 1.0
        du[:, 1, 0] = -2.0 * mu * u1 * u2 - 1.0
        du[:, 1, 1] = mu * (1.0 - u1 * u1)
        dz = np.zeros((2, q))
        if q == 1:
            dz[1, 0] = 1.0
        else:
            dz[0, 0] = 1.0
            dz[1, 1] = 1.0
        return du, dz

    return jac


def vanderpol_rhs(mu: float = 0.1, q: int = 1) -> Callable:
    """f itself for van der Pol (used by finite-difference checks)."""
    def f(w: np.ndarray, zeta: np.ndarray) -> np.ndarray:
        u1, u2 = w[..., 0], w[..., 1]
        out = np.empty(w.shape)
        out[..., 0] = u2 + (zeta[..., 0] if q == 2 else 0.0)
        out[..., 1] = mu * (1.0 - u1 * u1) * u2 - u1 + zeta[..., q - 1]
        return out
    return f


def burgers_jacobians(nx: int, nu: float) -> Callable:
    """du f and dz f of the semi-discrete viscous Burgers equation.

    Upwind finite differences on nx interior nodes of [0, 1] with spacing
    h = 1/(nx+1) and homogeneous Dirichlet values:
        f_i = nu (w_{i+1} - 2 w_i + w_{i-1}) / h^2 - w_i (w_i - w_{i-1}) / h + z_i
    (backward difference for the convective term; Sec. 6.2).  dz f = I.
    """
    h = 1.0 / (nx + 1)
    a = nu / (h * h)

    def jac(w: np.ndarray, zeta: np.ndarray):
        m = w.shape[0]
        wl = np.zeros_like(w)
        wl[:, 1:] = w[:, :-1]
        du = np.zeros((m, nx, nx))
        idx = np.arange(nx)
        du[:, idx, idx] = -2.0 * a - (2.0 * w - wl) / h
        du[:, idx[1:], idx[:-1]] = a + w[:, 1:] / h
        du[:, idx[:-1], idx[1:]] = a
        dz = np.eye(nx)
        return du, dz

    return jac


def burgers_step_state(nx: int) -> np.ndarray:
    """The initial state of Sec. 6.2 at the nx interior nodes of [0, 1]
    (h = 1/(nx+1)): 1 on (0, 1/2], 0 on (1/2, 1)."""
    x = np.arange(1, nx + 1) / (nx + 1)
    return np.where(x <= 0.5, 1.0, 0.0)


def burgers_rhs(nx: int, nu: float) -> Callable:
    h = 1.0 / (nx + 1)

    def f(w: np.ndarray, zeta: np.ndarray) -> np.ndarray:
        wl = np.zeros_like(w)
        wl[..., 1:] = w[..., :-1]
        wr = np.zeros_like(w)
        wr[..., :-1] = w[..., 1:]
        return nu * (wr - 2.0 * w + wl) / (h * h) - w * (w - wl) / h + zeta
    return f


# ---------------------------------------------------------------------------
# Lifted blocks on one grid
# ---------------------------------------------------------------------------

@dataclass
class Level:
    """Blocks of one time level.  V and Z are (n,p,p)/(n,p,q) arrays, or
    (1,p,p)/(1,p,q) when identical for every step (``shared``)."""
    n: int
    dt: float
    N: np.ndarray
    V: np.ndarray
    Z: np.ndarray
    shared: bool = False

    def V_full(self) -> np.ndarray:
        return np.broadcast_to(self.V, (self.n,) + self.V.shape[1:]) if self.shared else self.V

    def Z_full(self) -> np.ndarray:
        return np.broadcast_to(self.Z, (self.n,) + self.Z.shape[1:]) if self.shared else self.Z


def lifted_blocks(w: np.ndarray, zeta: np.ndarray, w0: np.ndarray, dt: float,
                  theta: float, gamma: float, jac: Callable,
                  M: Optional[np.ndarray] = None, compress: bool = True) -> Level:
    """Blocks N_k, V_k, Z~_k (k = 1..n) at physical point (w, zeta).

    w: (n,p) states, zeta: (n,q) controls, w0: (p,) the state at t = 0 (the
    physical value of v_0).  If theta == 1 and dz f does not depend on the
    point, V_k and Z~_k are the same for every k and are returned once.
    """
    n, p = w.shape
    q = zeta.shape[1]
    if M is None:
        M = np.eye(p)
    wprev = np.vstack([w0[None, :], w[:-1]])
    du_k, dz_k = jac(w, zeta)
    N = (M[None] - theta * dt * du_k) / dt
    const_dz = dz_k.ndim == 2
    if theta == 1.0 and const_dz and compress:
        V = (-M / dt)[None].copy()
        Z = (-(dt * dz_k) / (gamma * dt))[None].copy()
        return Level(n=n, dt=dt, N=N, V=V, Z=Z, shared=True)
    du_p, dz_p = jac(wprev, zeta)
    V = (-M[None] - (1.0 - theta) * dt * du_p) / dt
    if const_dz:
        dz_k = np.broadcast_to(dz_k, (n, p, q))
        dz_p = np.broadcast_to(dz_p, (n, p, q))
    Z = (-theta * dt * dz_k - (1.0 - theta) * dt * dz_p) / (gamma * dt)
    return Level(n=n, dt=dt, N=N, V=np.ascontiguousarray(V),
                 Z=np.ascontiguousarray(Z), shared=False)


# ---------------------------------------------------------------------------
# Whole hierarchies
# ---------------------------------------------------------------------------

@dataclass
class Problem:
    kind: str
    p: int
    q: int
    n: int
    n_levels: int
    gamma: float
    theta: float
    T: float
    levels: List[Level]
    w: np.ndarray          # finest physical states (n,p)
    zeta: np.ndarray       # finest physical controls (n,q)
    w0: np.ndarray
    params: dict = field(default_factory=dict)

    @property
    def size(self) -> int:
        return (4 * self.p + self.q) * self.n


def coarsen_point(w: np.ndarray, zeta: np.ndarray, variant: int = 0, c: int = 2):
    """Restrict a linearisation point to the grid of c times the step.

    States by injection, controls by averaging (Sec. 5.3.1).  variant 0 takes
    the first fine step c(k-1)+1 of coarse step k, as printed for c = 2;
    variant 1 (c = 2 only) takes step 2k, which sits at the same time as
    coarse step k.
    """
    ws = w[0::c] if variant == 0 else w[c - 1::c]
    zc = zeta.reshape(zeta.shape[0] // c, c, *zeta.shape[1:]).mean(axis=1)
    return ws, zc


def make_problem(kind: str, n: int, n_levels: int, seed: int, *, p: int = None,
                 nx: int = None, nu: float = 0.01, mu: float = 0.1, q: int = None,
                 gamma: float = 100.0, theta: float = 1.0, T: float = 1.0,
                 state_scale: float = 0.5, control_scale: float = 0.5,
                 noise: float = 0.1, transfer_variant: int = 0,
                 compress: bool = True, rng: Optional[np.random.Generator] = None,
                 coarsen: int = 2, mass_offdiag: float = 0.0
                 ) -> Tuple[Problem, np.random.Generator]:
    """Build a seeded problem hierarchy.

    Draw order with ``np.random.default_rng(seed)`` (the right-hand side is
    drawn afterwards from the same generator by :func:`make_rhs`):
      van der Pol: w (n,2) ~ N(0, state_scale^2), zeta (n,q) ~ N(0, control_scale^2)
      Burgers:     xi (n,nx) ~ N(0,1), w = sin(pi x) + noise*xi,
                   zeta (n,nx) ~ N(0, control_scale^2)
    mass_offdiag (Burgers): M = I + mass_offdiag * (the nearest-neighbour
    couplings), a non-diagonal mass matrix (so V_k = -M/dt is a dense shared
    block) for exercising the general block paths; 0 gives M = I.
    """
    if n % (coarsen ** (n_levels - 1)) != 0:
        raise ValueError("n must be divisible by coarsen^(n_levels-1)")
    if rng is None:
        rng = np.random.default_rng(seed)
    if kind == "vanderpol":
        q = 1 if q is None else q
        p = 2
        w = rng.normal(0.0, state_scale, size=(n, 2))
        zeta = rng.normal(0.0, control_scale, size=(n, q))
        jac = vanderpol_jacobians(mu=mu, q=q)
        w0 = np.array([1.0, 1.0])
        params = dict(mu=mu)
    elif kind == "burgers":
        if nx is None:
            raise ValueError("burgers needs nx")
        p = q = nx
        x = np.arange(1, nx + 1) / (nx + 1)
        xi = rng.normal(0.0, 1.0, size=(n, nx))
        w = np.sin(np.pi * x)[None, :] + noise * xi
        zeta = rng.normal(0.0, control_scale, size=(n, nx))
        jac = burgers_jacobians(nx, nu)
        w0 = np.sin(np.pi * x)
        params = dict(nu=nu, nx=nx)
        if mass_offdiag:
            M = np.eye(nx) + mass_offdiag * (np.eye(nx, k=1) + np.eye(nx, k=-1))
            params["M"] = M
    else:
        raise ValueError(f"unknown problem kind {kind!r}")

    levels = []
    wl, zl = w, zeta
    for lev in range(n_levels):
        nl = n // coarsen ** lev
        dt = T / nl
        levels.append(lifted_blocks(wl, zl, w0, dt, theta, gamma, jac, M=params.get("M"),
                                    compress=compress))
        if lev + 1 < n_levels:
            wl, zl = coarsen_point(wl, zl, transfer_variant, coarsen)
    prob = Problem(kind=kind, p=p, q=q, n=n, n_levels=n_levels, gamma=gamma,
                   theta=theta, T=T, levels=levels, w=w, zeta=zeta, w0=w0,
                   params=params)
    return prob, rng


def make_rhs(prob: Problem, rng: np.random.Generator, count: int = 1) -> np.ndarray:
    """Right-hand side(s) ~ N(0,1) in type-major order [u|v|z|lambda|mu]."""
    if count == 1:
        return rng.normal(0.0, 1.0, size=prob.size)
    return rng.normal(0.0, 1.0, size=(count, prob.size))


# The workloads measured in this project (sizes from the project's benchmark
# list; the paper's own runs use an SQP driver that is out of scope).
CONFIGS = {
    "vdp256": dict(kind="vanderpol", n=256, n_levels=6, seed=1, q=1),
    "burgers128": dict(kind="burgers", nx=128, nu=0.01, n=1024, n_levels=8, seed=2),
    "burgers512": dict(kind="burgers", nx=512, nu=0.005, n=4096, n_levels=10, seed=3),
    "burgers256": dict(kind="burgers", nx=256, nu=0.01, n=2048, n_levels=9, seed=5),
}


def config_problem(name: str, **over):
    """Problem and right-hand side of a named workload (same seed for both)."""
    cfg = dict(CONFIGS[name])
    cfg.update(over)
    prob, rng = make_problem(**cfg)
    b = make_rhs(prob, rng)
    return prob, b


def coarse_net_params(C: int, H: int, seed: int, width: int = 3) -> np.ndarray:
    """Seeded initial parameters of the coarse-correction network: the flat
    vector [W1 (H,C,width), b1 (H), W2 (H,H,width), b2 (H), W3 (C,H,width),
    b3 (C)], each entry uniform in +-1/sqrt(fan_in) of its layer, rounded to
    FP32.  Draw order: W1, b1, W2, b2, W3, b3 from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    parts = []
    for (o, i) in ((H, C), (H, H), (C, H)):
        a = 1.0 / np.sqrt(i * width)
        parts.append(rng.uniform(-a, a, size=o * i * width))
        parts.append(rng.uniform(-a, a, size=o))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def batch_mix(seed: int = 4, count: int = 64, vdp_n=(256, 1024, 4096), burgers_nx=(64, 128, 256),
              burgers_n=(512, 1024, 2048, 4096)):
    """An uneven batch of independent systems (make_problem keyword sets).

    The first half are van der Pol with n drawn from vdp_n; the second half
    viscous Burgers (nu = 0.01) with nx drawn from burgers_nx and n from
    burgers_n.  Every system coarsens to 8 steps (n_levels = log2(n) - 2) and
    takes seed 4000 + i.  Draw order from default_rng(seed): for each system
    in turn, its n (van der Pol) or its nx then n (Burgers).
    """
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        if i < count // 2:
            n = int(rng.choice(list(vdp_n)))
            cfg = dict(kind="vanderpol", n=n, seed=4000 + i)
        else:
            nx = int(rng.choice(list(burgers_nx)))
            n = int(rng.choice(list(burgers_n)))
            cfg = dict(kind="burgers", nx=nx, nu=0.01, n=n, seed=4000 + i)
        cfg["n_levels"] = int(np.log2(n)) - 2
        out.append(cfg)
    return out
