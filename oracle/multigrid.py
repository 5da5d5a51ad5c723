"""Block smoothers, the V-cycle and the preconditioned outer solve.

Everything here acts on time-major vectors y = Q x, b~ = P b (eq. (augsysp2))
of one level, with A~ = P A Q^T split as L + D + L^T (Sec. 5.3.2):

  block Jacobi (eq. (jacobi)), with weight omega:
        y <- y + omega D^{-1} (b~ - A~ y)
  (omega = 1 is the printed, undamped sweep; see MGOptions.omega)
  symmetric block Gauss-Seidel (Sec. 5.3.4), used as the right
  preconditioner of the coarse GMRES:
        M = (D + L) D^{-1} (D + L^T),   M^{-1} r = (D+L^T)^{-1} D (D+L)^{-1} r
  V-cycle (Alg. 1, recursed level by level, zero initial guess on each
  level): pre-smooth, restrict b - A y, recurse, interpolate and add,
  post-smooth; on the last level GMRES + SGS to a relative tolerance.
  Outer solve: flexible GMRES preconditioned by one V-cycle (Sec. 5.3.4, 6).

Factorisations are SuperLU (scipy.sparse.linalg.splu) of the assembled
sparse block parts; nothing uses the derived Schur-complement formulas.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .system import assemble_A, time_major_perm, block_bounds, split_blocks
from .transfer import restriction, interpolation
from .krylov import gmres_right, fgmres


class OracleLevel:
    """One level: the time-major operator and factorisations of its parts."""

    def __init__(self, N, V, Z, factor_sgs: bool = False):
        N = np.asarray(N, dtype=np.float64)
        self.n, self.p, _ = N.shape
        self.q = Z.shape[2]
        V = np.broadcast_to(V, (self.n, self.p, self.p))
        Z = np.broadcast_to(Z, (self.n, self.p, self.q))
        self.A = assemble_A(N, V, Z)                       # type-major
        self.perm = time_major_perm(self.p, self.q, self.n)
        self.At = self.A[self.perm][:, self.perm].tocsc()  # P A Q^T
        self.bounds = block_bounds(self.p, self.q, self.n)
        self.D, self.L, self.U = split_blocks(self.At.tocsr(), self.bounds)
        self.D_lu = spla.splu(self.D.tocsc())
        self.sgs_lo = self.sgs_up = None
        if factor_sgs:
            self.factor_sgs()

    def factor_sgs(self):
        self.sgs_lo = spla.splu((self.D + self.L).tocsc())
        self.sgs_up = spla.splu((self.D + self.U).tocsc())

    # -- smoothers ----------------------------------------------------------
    def jacobi(self, b: np.ndarray, y: np.ndarray, omega: float = 1.0) -> np.ndarray:
        """One block Jacobi sweep, first form of eq. (jacobi), with the
        correction D^{-1}(b - A~ y) weighted by omega (1 = as printed)."""
        return y + omega * self.D_lu.solve(b - self.At @ y)

    def sgs(self, r: np.ndarray) -> np.ndarray:
        """M^{-1} r for the symmetric block Gauss-Seidel splitting."""
        a = self.sgs_lo.solve(r)                 # (D + L) a = r
        return self.sgs_up.solve(self.D @ a)     # (D + L^T) y = D a

    def fgs(self, r: np.ndarray) -> np.ndarray:
        return self.sgs_lo.solve(r)

    def bgs(self, r: np.ndarray) -> np.ndarray:
        return self.sgs_up.solve(r)

    def smooth(self, kind: str, b: np.ndarray, y: np.ndarray, omega: float) -> np.ndarray:
        """One smoothing sweep y + omega M^{-1}(b - A~ y) of the given kind."""
        if kind == "jacobi":
            return self.jacobi(b, y, omega)
        if self.sgs_lo is None:
            self.factor_sgs()
        r = b - self.At @ y
        d = {"fgs": self.fgs, "bgs": self.bgs, "sgs": self.sgs}[kind](r)
        return y + omega * d


@dataclass
class MGOptions:
    """Cycle parameters.

    omega: weight of the block Jacobi correction.  The permuted matrix is
    block tridiagonal (Fig. 5), so conjugating I - D^{-1} A~ by the block
    sign pattern diag((-1)^k) negates it: its spectrum is symmetric about 0,
    and each slow smooth error mode (eigenvalue near +1) has an oscillating
    twin near -1 that no coarse grid represents.  The printed sweep
    (omega = 1) leaves that twin as slow as the smooth mode, and the cycle
    converges no faster than its smoother.  omega = 1/2 maps the spectrum
    [-rho, rho] into [(1-rho)/2, (1+rho)/2]: every oscillating twin is damped
    by at least 1/2 per sweep, and the smooth modes are left to the coarse
    grid (the weighted Jacobi smoother of the multigrid texts cited in
    Sec. 5.3).
    mu_scale: scale of the interface multiplier in the transfers (see
    oracle.transfer); 1 = the printed transfers.
    cycle: "V" (the cycle of Alg. 1, one coarse correction per level), "W" or
    "F" (Sec. 6 reports trying both): every level above the coarsest makes
    two coarse corrections, the second from the coarse residual the first
    leaves, e2 = MG_{l+1}(r_c - A~_{l+1} e1); W recurses with W in both, F
    with F in the first and V in the second.  Counting a move down to the
    next level and back up as two sequential steps, a 4-level V, F and W cycle
    take 6, 18 and 28 (the counts Sec. 6 gives); Hierarchy.calls records the
    levels entered.
    smoother: the fixed-point iteration of the smoothing sweeps,
    y <- y + omega M^{-1} (b - A~ y), with the splittings of Sec. 5.3.4:
    "jacobi" M = D, "fgs" M = D + L (forward block Gauss-Seidel), "bgs"
    M = D + L^T (backward), "sgs" M = (D + L) D^{-1} (D + L^T).
    coarsen: the step ratio between consecutive levels (2 as in Alg. 1;
    larger powers of 2 as Sec. 6 reports trying), see oracle.transfer.
    """
    nu_pre: int = 2
    nu_post: int = 2
    coarse_tol: float = 1e-3
    coarse_maxit: int = 50
    coarse_fixed_its: int = 0
    transfer_variant: int = 0
    omega: float = 0.5
    mu_scale: float = 2.0
    cycle: str = "V"
    smoother: str = "jacobi"
    coarsen: int = 2


class Hierarchy:
    """The multigrid hierarchy of one problem (blocks given per level)."""

    def __init__(self, levels, opts: Optional[MGOptions] = None):
        """levels: list of objects with N (n,p,p), V, Z arrays (V/Z may be
        (1,p,p)/(1,p,q) when shared by every step)."""
        self.opts = opts or MGOptions()
        self.levels: List[OracleLevel] = []
        for i, lv in enumerate(levels):
            last = i == len(levels) - 1
            self.levels.append(OracleLevel(lv.N, lv.V, lv.Z, factor_sgs=last))
        self.R, self.P = [], []
        for i in range(len(self.levels) - 1):
            f, c = self.levels[i], self.levels[i + 1]
            cf = self.opts.coarsen
            if c.n * cf != f.n:
                raise ValueError("levels must divide the step count by the coarsening factor")
            Rt = restriction(f.p, f.q, f.n, self.opts.transfer_variant,
                             self.opts.mu_scale, cf)
            Pt = interpolation(f.p, f.q, f.n, self.opts.transfer_variant,
                               self.opts.mu_scale, cf)
            # time-major transfers: R~ = P_c R Q_f^T, P~ = P_f P Q_c^T
            self.R.append(Rt[c.perm][:, f.perm].tocsr())
            self.P.append(Pt[f.perm][:, c.perm].tocsr())
        self.coarse_its: List[int] = []
        self.calls: List[int] = []                # levels entered by mg()

    # -- multigrid ------------------------------------------------------------
    def coarse_solve(self, b: np.ndarray) -> np.ndarray:
        lv = self.levels[-1]
        o = self.opts
        x, its = gmres_right(lv.At, b, lv.sgs, o.coarse_tol, o.coarse_maxit,
                             o.coarse_fixed_its)
        self.coarse_its.append(its)
        return x

    def mg(self, lev: int, b: np.ndarray, cycle: Optional[str] = None) -> np.ndarray:
        """MG_lev(b): one cycle from a zero initial guess (Alg. 1; the W and F
        variants of MGOptions.cycle)."""
        if lev == len(self.levels) - 1:
            return self.coarse_solve(b)
        cycle = cycle or self.opts.cycle
        if cycle not in ("V", "W", "F"):
            raise ValueError("cycle must be V, W or F")
        lv = self.levels[lev]
        o = self.opts
        y = np.zeros_like(b)
        for _ in range(o.nu_pre):                 # pre-smooth
            y = lv.smooth(o.smoother, b, y, o.omega)
        r = b - lv.At @ y                         # residual
        rc = self.R[lev] @ r                      # restrict
        e = self._enter(lev + 1, rc, cycle)       # coarse correction
        if cycle != "V":                          # the second one (W, F)
            rc2 = rc - self.levels[lev + 1].At @ e
            e = e + self._enter(lev + 1, rc2, "W" if cycle == "W" else "V")
        y = y + self.P[lev] @ e                   # interpolate and add
        for _ in range(o.nu_post):                # post-smooth
            y = lv.smooth(o.smoother, b, y, o.omega)
        return y

    def _enter(self, lev: int, b: np.ndarray, cycle: str) -> np.ndarray:
        self.calls.append(lev)
        return self.mg(lev, b, cycle)

    # -- type-major front end -------------------------------------------------
    def to_time(self, x: np.ndarray, lev: int = 0) -> np.ndarray:
        return x[self.levels[lev].perm]

    def to_type(self, y: np.ndarray, lev: int = 0) -> np.ndarray:
        x = np.empty_like(y)
        x[self.levels[lev].perm] = y
        return x

    def vcycle(self, r_type: np.ndarray) -> np.ndarray:
        """One V-cycle applied to a type-major vector (zero initial guess)."""
        return self.to_type(self.mg(0, self.to_time(r_type)))

    def apply(self, x_type: np.ndarray) -> np.ndarray:
        return self.levels[0].A @ x_type

    def solve(self, b_type: np.ndarray, tol: float = 1e-10, restart: int = 30,
              maxit: int = 300, x0: np.ndarray = None):
        """FGMRES on A~ y = b~ preconditioned by one V-cycle per step."""
        self.coarse_its = []
        bt = self.to_time(b_type)
        y0 = None if x0 is None else self.to_time(x0)
        y, info = fgmres(self.levels[0].At, bt, lambda v: self.mg(0, v), tol,
                         restart=restart, maxit=maxit, x0=y0)
        info["coarse_its"] = list(self.coarse_its)
        return self.to_type(y), info


def direct_solve(level, b_type: np.ndarray) -> np.ndarray:
    """The plain definition y* = A^{-1} b (sparse LU of the whole matrix)."""
    N = np.asarray(level.N)
    n, p, _ = N.shape
    q = level.Z.shape[2]
    V = np.broadcast_to(level.V, (n, p, p))
    Z = np.broadcast_to(level.Z, (n, p, q))
    A = assemble_A(N, V, Z).tocsc()
    return spla.splu(A).solve(b_type)
