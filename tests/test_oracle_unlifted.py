"""Pins of the unlifted augmented system (Fig. 2, B = dF) and of the lift /
project maps that carry the lifted multigrid cycle to it (oracle.unlifted):
the printed block pattern, the operator identity A = E^T A~' E against the
independently assembled lifted operator, the exactness of E^T A~'^{-1} E,
and FGMRES on the unlifted system with the lifted cycle."""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.system import assemble_A
from oracle.unlifted import (assemble_unlifted, lift, project, unlifted_offsets, ScaledLevel,
                             UnliftedSolver, SQRT2)
from oracle.multigrid import MGOptions
from workloads import make_problem, make_rhs
from test_oracle_pins import random_level, _read_pattern

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _slices(p, q, n):
    o = unlifted_offsets(p, q, n)
    sl = {}
    for k in range(1, n + 1):
        for t, w in (("u", p), ("z", q), ("lam", p)):
            s = o[t] + (k - 1) * w
            sl[f"{t}{k}"] = slice(s, s + w)
    return sl


def test_fig2_unlifted_pattern_and_blocks():
    p, q, n = 2, 1, 4
    lv = random_level(n, p, q, 31)
    A = assemble_unlifted(lv.N, lv.V_full(), lv.Z_full()).toarray()
    sl = _slices(p, q, n)
    names = {"K": lv.N, "C": lv.V_full(), "B": lv.Z_full()}
    covered = np.zeros(A.shape, dtype=bool)
    _, entries = _read_pattern("fig2_pattern_n4.txt")
    for r, c, tok in entries:
        blk = A[sl[r], sl[c]]
        if tok == "I":
            np.testing.assert_array_equal(blk, np.eye(blk.shape[0]))
        else:
            M = names[tok[0]][int(tok[1]) - 1]
            np.testing.assert_array_equal(blk, M.T if tok.endswith("^T") else M)
        covered[sl[r], sl[c]] = True
    assert np.all(A[~covered] == 0.0)
    np.testing.assert_array_equal(A, A.T)


@pytest.mark.parametrize("p,q,n", [(2, 1, 6), (3, 2, 5)])
def test_unlifted_operator_is_the_lifted_one_through_e(p, q, n):
    """A = E^T A~' E with A~' the lifted operator of the blocks sqrt2 N_k,
    sqrt2 V_k, Z~_k (assembled by oracle.system, independently)."""
    lv = random_level(n, p, q, 32)
    A = assemble_unlifted(lv.N, lv.V_full(), lv.Z_full()).toarray()
    Al = assemble_A(SQRT2 * lv.N, SQRT2 * lv.V_full(), lv.Z_full())
    m = A.shape[0]
    E = np.column_stack([lift(e, p, q, n) for e in np.eye(m)])
    np.testing.assert_allclose(E.T @ (Al @ E), A, rtol=0, atol=1e-13)
    # E^T is the adjoint of E, and project is E^T
    y = np.random.default_rng(1).normal(size=E.shape[0])
    np.testing.assert_allclose(project(y, p, q, n), E.T @ y, rtol=0, atol=1e-14)


@pytest.mark.parametrize("p,q,n", [(2, 1, 6), (3, 2, 5)])
def test_lifted_inverse_through_e_is_the_unlifted_inverse(p, q, n):
    """E^T A~'^{-1} E = A^{-1}: the lift / project maps lose nothing when the
    lifted system is solved exactly.  With the unscaled blocks they would
    solve the system whose state identity is doubled instead."""
    lv = random_level(n, p, q, 33)
    A = assemble_unlifted(lv.N, lv.V_full(), lv.Z_full())
    Al = assemble_A(SQRT2 * lv.N, SQRT2 * lv.V_full(), lv.Z_full())
    r = np.random.default_rng(2).normal(size=A.shape[0])
    x = spla.spsolve(A.tocsc(), r)
    y = spla.spsolve(Al.tocsc(), lift(r, p, q, n))
    np.testing.assert_allclose(project(y, p, q, n), x, rtol=0, atol=1e-10 * np.linalg.norm(x))
    # the lifted solution has v = u and mu as the u rows leave it
    pn = p * n
    np.testing.assert_allclose(y[:pn], y[pn:2 * pn], rtol=0, atol=1e-10 * np.linalg.norm(x))
    Al1 = assemble_A(lv.N, lv.V_full(), lv.Z_full())
    y1 = spla.spsolve(Al1.tocsc(), lift(r, p, q, n))
    assert np.linalg.norm(project(y1, p, q, n) - x) > 1e-3 * np.linalg.norm(x)


@pytest.mark.parametrize("cfg", [dict(kind="vanderpol", n=64, n_levels=4, seed=34),
                                 dict(kind="burgers", nx=12, nu=0.01, n=32, n_levels=3,
                                      seed=35)])
def test_unlifted_fgmres_with_the_lifted_cycle(cfg):
    """FGMRES on the unlifted system, preconditioned by E^T MG'(E r), reaches
    1e-10 in about as many steps as the lifted solve, and its solution is the
    direct one."""
    from oracle import Hierarchy
    prob, rng = make_problem(**cfg)
    p, q, n = prob.p, prob.q, prob.n
    lv = prob.levels[0]
    S = UnliftedSolver(prob.levels, MGOptions())
    b = np.random.default_rng(3).normal(size=S.A.shape[0])
    x, info = S.solve(b, tol=1e-10, restart=100, maxit=100)
    assert info["converged"]
    xd = spla.spsolve(S.A.tocsc(), b)
    assert np.linalg.norm(S.A @ x - b) <= 1e-10 * np.linalg.norm(b) * 1.0001
    lifted = Hierarchy(prob.levels, MGOptions()).solve(make_rhs(prob, rng), tol=1e-10,
                                                       restart=100, maxit=100)[1]["iters"]
    assert info["iters"] <= lifted + 4, (info["iters"], lifted)
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)
