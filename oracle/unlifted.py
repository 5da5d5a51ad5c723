"""The augmented system without virtual variables (Fig. 2, B = dF) and its
preconditioning by the lifted multigrid cycle through lift and project maps.

Unlifted type-major order: x = [u_1..u_n | z_1..z_n | lambda_1..lambda_n].
B = dF has one row block per time step (the theta-method constraint):

    lambda_k row:  K_k at u_k,  C_k at u_{k-1} (k >= 2),  B_k at z_k,

and A = [[I, B^T], [B, 0]] (eq. (augsys)).  At a linearisation point with
v = u the lifted blocks are these blocks: N_k = K_k, V_k = C_k (O_k with
u_{k-1} in place of v_{k-1}), Z~_k = B_k (Sec. 5.1).

Lift and project (the paper gives none; this is the choice that makes the
lifted solve exact).  Let A~' be the lifted operator built from the scaled
blocks (sqrt(2) N_k, sqrt(2) V_k, Z~_k) and E the map

    E(u, z, lambda) = (u / sqrt2, u / sqrt2, z, lambda, 0)   (lifted order u, v, z, lambda, mu),

whose transpose is E^T(u, v, z, lambda, mu) = ((u + v) / sqrt2, z, lambda).
Then
  * A = E^T A~' E (the identity on the states splits evenly between u and
    v, and the scaled blocks take the 1/sqrt2 back), and
  * A^{-1} = E^T A~'^{-1} E: if (u, z, lambda) solves A x = r, the lifted
    vector (u/sqrt2, u/sqrt2, z, lambda, mu) solves A~' y = E r for the mu
    that the u rows leave (the u and v rows of A~' sum to sqrt2 times the u
    row of A, and the mu rows hold with v = u), and A~' is nonsingular.
So M = E^T MG'(E r), with MG' one cycle on the hierarchy of scaled blocks,
is the lifted preconditioner carried to the unlifted system, exact when the
cycle is an exact solve.  Flexible GMRES runs on A with M (Sec. 5.3.4).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .multigrid import Hierarchy, MGOptions
from .krylov import fgmres

SQRT2 = np.sqrt(2.0)


def unlifted_offsets(p: int, q: int, n: int):
    return dict(u=0, z=p * n, lam=(p + q) * n, end=(2 * p + q) * n)


def assemble_unlifted(N, V, Z) -> sp.csr_matrix:
    """A = [[I, B^T], [B, 0]] with B = dF in the unlifted type-major order.
    N: (n,p,p) (K_k), V: (n,p,p) (C_k; step 1 unused), Z: (n,p,q) (B_k)."""
    N = np.asarray(N, dtype=np.float64)
    n, p, _ = N.shape
    q = Z.shape[2]
    V = np.broadcast_to(V, (n, p, p))
    Z = np.broadcast_to(Z, (n, p, q))
    rows, cols, vals = [], [], []

    def put(block, r0, c0):
        r, c = np.nonzero(block)
        rows.append(r0 + r)
        cols.append(c0 + c)
        vals.append(block[r, c])

    for k in range(n):
        put(N[k], k * p, k * p)                     # K_k at u_k
        if k >= 1:
            put(V[k], k * p, (k - 1) * p)           # C_k at u_{k-1}
        put(Z[k], k * p, p * n + k * q)             # B_k at z_k
    B = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(p * n, (p + q) * n))
    A = sp.bmat([[sp.identity((p + q) * n, format="csr"), B.T],
                 [B, sp.csr_matrix((p * n, p * n))]], format="csr")
    A.eliminate_zeros()
    return A


def lift(r: np.ndarray, p: int, q: int, n: int) -> np.ndarray:
    """E r: unlifted (u, z, lambda) -> lifted (u/sqrt2, u/sqrt2, z, lambda, 0)."""
    pn, qn = p * n, q * n
    u, z, lam = r[:pn], r[pn:pn + qn], r[pn + qn:]
    return np.concatenate([u / SQRT2, u / SQRT2, z, lam, np.zeros(pn)])


def project(y: np.ndarray, p: int, q: int, n: int) -> np.ndarray:
    """E^T y: lifted (u, v, z, lambda, mu) -> unlifted ((u + v)/sqrt2, z, lambda)."""
    pn, qn = p * n, q * n
    u, v = y[:pn], y[pn:2 * pn]
    z, lam = y[2 * pn:2 * pn + qn], y[2 * pn + qn:3 * pn + qn]
    return np.concatenate([(u + v) / SQRT2, z, lam])


class ScaledLevel:
    """A level's blocks with N_k and V_k multiplied by sqrt2 (the lifted
    problem whose solve E^T A~'^{-1} E is the unlifted inverse)."""

    def __init__(self, lv):
        self.n = lv.N.shape[0]
        self.N = SQRT2 * np.asarray(lv.N)
        self.V = SQRT2 * np.asarray(lv.V)
        self.Z = np.asarray(lv.Z)


class UnliftedSolver:
    """FGMRES on the unlifted system with the lifted cycle through E."""

    def __init__(self, levels, opts: MGOptions = None):
        lv0 = levels[0]
        self.n, self.p, _ = np.asarray(lv0.N).shape
        self.q = lv0.Z.shape[2]
        self.A = assemble_unlifted(lv0.N, lv0.V, lv0.Z)
        self.H = Hierarchy([ScaledLevel(lv) for lv in levels], opts)

    def precondition(self, r: np.ndarray) -> np.ndarray:
        p, q, n = self.p, self.q, self.n
        return project(self.H.vcycle(lift(r, p, q, n)), p, q, n)

    def solve(self, b: np.ndarray, tol: float = 1e-10, restart: int = 30, maxit: int = 300):
        self.H.coarse_its = []
        x, info = fgmres(self.A, b, self.precondition, tol, restart=restart, maxit=maxit)
        info["coarse_its"] = list(self.H.coarse_its)
        return x, info
