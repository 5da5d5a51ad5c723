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

Coarsening by a factor c > 2 (Sec. 6 reports trying larger factors), with
coarse steps 1..n/c and variant 0's alignment: injection
s^c_k = s^f_{c(k-1)+1}, linear interpolation
s^f_{c(k-1)+1+i} = ((c-i) s^c_k + i s^c_{k+1}) / c for i = 0..c-1 (with
s^c_{n/c+1} := s^c_{n/c}), the control averaged over and copied to the c
fine steps of a coarse step.  For c = 2 these are the formulas above.  The
mu block takes mu_scale^(log2 c): one factor mu_scale per halving of the
step.
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


def _node_R_c(nf: int, c: int) -> sp.csr_matrix:
    nc = nf // c
    R = sp.lil_matrix((nc, nf))
    for k in range(1, nc + 1):
        R[k - 1, c * (k - 1)] = 1.0                      # s^c_k = s^f_{c(k-1)+1}
    return R.tocsr()


def _node_P_c(nf: int, c: int) -> sp.csr_matrix:
    nc = nf // c
    P = sp.lil_matrix((nf, nc))
    for k in range(1, nc + 1):
        kk = k + 1 if k < nc else nc                     # s^c_{nc+1} := s^c_{nc}
        for i in range(c):
            P[c * (k - 1) + i, k - 1] += (c - i) / c
            if i:
                P[c * (k - 1) + i, kk - 1] += i / c
    return P.tocsr()


def _ctrl_R_c(nf: int, c: int) -> sp.csr_matrix:
    nc = nf // c
    R = sp.lil_matrix((nc, nf))
    for k in range(1, nc + 1):
        for i in range(c):
            R[k - 1, c * (k - 1) + i] = 1.0 / c
    return R.tocsr()


def _ctrl_P_c(nf: int, c: int) -> sp.csr_matrix:
    nc = nf // c
    P = sp.lil_matrix((nf, nc))
    for k in range(1, nc + 1):
        for i in range(c):
            P[c * (k - 1) + i, k - 1] = 1.0
    return P.tocsr()


def _mu_factor(mu_scale: float, c: int) -> float:
    return float(mu_scale) ** np.log2(c)


def _factor_parts(nf: int, variant: int, c: int):
    if c < 2 or c & (c - 1):
        raise ValueError("the coarsening factor must be a power of 2")
    if nf % c:
        raise ValueError("n must be divisible by the coarsening factor")
    if c == 2:
        return _node_R(nf, variant), _node_P(nf, variant), _ctrl_R(nf), _ctrl_P(nf)
    if variant != 0:
        raise ValueError("transfer variant 1 is defined for a factor of 2 only")
    return _node_R_c(nf, c), _node_P_c(nf, c), _ctrl_R_c(nf, c), _ctrl_P_c(nf, c)


def restriction(p: int, q: int, nf: int, variant: int = 0,
                mu_scale: float = 1.0, c: int = 2) -> sp.csr_matrix:
    """Type-major restriction from nf steps to nf/c steps; the mu rows are
    multiplied by mu_scale^(log2 c)."""
    nR, _, zR, _ = _factor_parts(nf, variant, c)
    Rs = sp.kron(nR, sp.identity(p))
    Rz = sp.kron(zR, sp.identity(q))
    return sp.block_diag([Rs, Rs, Rz, Rs, _mu_factor(mu_scale, c) * Rs], format="csr")


def interpolation(p: int, q: int, nf: int, variant: int = 0,
                  mu_scale: float = 1.0, c: int = 2) -> sp.csr_matrix:
    """Type-major interpolation from nf/c steps to nf steps; the mu block is
    multiplied by mu_scale^(log2 c)."""
    _, nP, _, zP = _factor_parts(nf, variant, c)
    Ps = sp.kron(nP, sp.identity(p))
    Pz = sp.kron(zP, sp.identity(q))
    return sp.block_diag([Ps, Ps, Pz, Ps, _mu_factor(mu_scale, c) * Ps], format="csr")
