"""Restriction and interpolation in time (Sec. 5.3.1), type-major vectors.

For every variable type except the control (u, v, lambda, mu), with fine
steps 1..n and coarse steps 1..n/2:
    interpolation: s^f_{2k-1} = s^c_k,  s^f_{2k} = (s^c_k + s^c_{k+1}) / 2
    restriction:   s^c_k = s^f_{2k-1}
and for the control (piecewise constant in time):
    interpolation: z^f_{2k-1} = z^f_{2k} = z^c_k
    restriction:   z^c_k = (z^f_{2k-1} + z^f_{2k}) / 2.

The printed interpolation reaches s^c_{n/2+1} at k = n/2, a coarse step that
does not exist.  variant 0 (default) keeps the printed formulas and takes
s^c_{n/2+1} := s^c_{n/2}.  variant 1 aligns coarse step k with fine step 2k
(both end at time 2k*dt): s^c_k = s^f_{2k}, s^f_{2k} = s^c_k,
s^f_{2k-1} = (s^c_{k-1} + s^c_k)/2 with s^c_0 := 0.

Scale of the interface multiplier (mu_scale).  Sec. 5.3.1 leaves the
transfers open ("supports alternatives"); the printed formulas fix only the
pattern.  In the Euclidean variables of Sec. 4.1 every type except mu is
sqrt(dt) times a function of time, so a common factor between the grids
cancels in P MG R (the coarse GMRES is homogeneous).  The u_k row of the
lifted system balances N_k^T lambda_k + mu_k, and N_k = (M - theta dt du f)/dt,
so mu is 1/dt times a lambda-sized function: the same function on the grid
of step 2 dt has half the mu coefficient relative to the other types.
mu_scale multiplies the mu block of the interpolation (coarse -> fine) and,
keeping R proportional to the transpose pattern of P, the mu rows of the
restriction.  mu_scale = 1 is the printed, unscaled transfer; 2 is the
step ratio.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def _node_R(nf: int, variant: int) -> sp.csr_matrix:
    nc = nf // 2
    R = sp.lil_matrix((nc, nf))
    for k in range(1, nc + 1):
        R[k - 1, (2 * k - 1 if variant == 0 else 2 * k) - 1] = 1.0
    return R.tocsr()


def _node_P(nf: int, variant: int) -> sp.csr_matrix:
    nc = nf // 2
    P = sp.lil_matrix((nf, nc))
    for k in range(1, nc + 1):
        if variant == 0:
            P[2 * k - 2, k - 1] = 1.0                    # s^f_{2k-1} = s^c_k
            kk = k + 1 if k < nc else nc                 # s^c_{n/2+1} := s^c_{n/2}
            P[2 * k - 1, k - 1] += 0.5                   # s^f_{2k}
            P[2 * k - 1, kk - 1] += 0.5
        else:
            P[2 * k - 1, k - 1] = 1.0                    # s^f_{2k} = s^c_k
            P[2 * k - 2, k - 1] += 0.5                   # s^f_{2k-1}
            if k >= 2:
                P[2 * k - 2, k - 2] += 0.5               # s^c_0 := 0
    return P.tocsr()


def _ctrl_R(nf: int) -> sp.csr_matrix:
    nc = nf // 2
    R = sp.lil_matrix((nc, nf))
    for k in range(1, nc + 1):
        R[k - 1, 2 * k - 2] = 0.5
        R[k - 1, 2 * k - 1] = 0.5
    return R.tocsr()


def _ctrl_P(nf: int) -> sp.csr_matrix:
    nc = nf // 2
    P = sp.lil_matrix((nf, nc))
    for k in range(1, nc + 1):
        P[2 * k - 2, k - 1] = 1.0
        P[2 * k - 1, k - 1] = 1.0
    return P.tocsr()


def restriction(p: int, q: int, nf: int, variant: int = 0,
                mu_scale: float = 1.0) -> sp.csr_matrix:
    """Type-major restriction from nf steps to nf/2 steps; the mu rows are
    multiplied by mu_scale."""
    if nf % 2:
        raise ValueError("n must be even to coarsen")
    Rs = sp.kron(_node_R(nf, variant), sp.identity(p))
    Rz = sp.kron(_ctrl_R(nf), sp.identity(q))
    return sp.block_diag([Rs, Rs, Rz, Rs, mu_scale * Rs], format="csr")


def interpolation(p: int, q: int, nf: int, variant: int = 0,
                  mu_scale: float = 1.0) -> sp.csr_matrix:
    """Type-major interpolation from nf/2 steps to nf steps; the mu block is
    multiplied by mu_scale."""
    if nf % 2:
        raise ValueError("n must be even to coarsen")
    Ps = sp.kron(_node_P(nf, variant), sp.identity(p))
    Pz = sp.kron(_ctrl_P(nf), sp.identity(q))
    return sp.block_diag([Ps, Ps, Pz, Ps, mu_scale * Ps], format="csr")
