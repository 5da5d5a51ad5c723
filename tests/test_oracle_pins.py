"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: the block
patterns printed in Figs. 4 and 5, the spectral radii of Table 2, finite
differences of the scaled discrete constraint, closed forms of the augmented
spectrum, brute-force Krylov minimisers and dense direct solves.
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from workloads import make_problem, make_rhs
from workloads.problems import (lifted_blocks, vanderpol_jacobians, vanderpol_rhs,
                                burgers_jacobians, burgers_rhs, coarsen_point, Level)
import oracle
from oracle import (assemble_A, assemble_B, time_major_perm, block_bounds,
                    split_blocks, restriction, interpolation, gmres_right, fgmres,
                    OracleLevel, Hierarchy, direct_solve, type_offsets)
from oracle.multigrid import MGOptions

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def random_level(n, p, q, seed, shared=False):
    rng = np.random.default_rng(seed)
    N = rng.normal(size=(n, p, p)) + 3 * np.eye(p)
    if shared:
        V = rng.normal(size=(1, p, p))
        Z = rng.normal(size=(1, p, q))
    else:
        V = rng.normal(size=(n, p, p))
        Z = rng.normal(size=(n, p, q))
    return Level(n=n, dt=1.0 / n, N=N, V=V, Z=Z, shared=shared)


# ---------------------------------------------------------------------------
# Figures 4 and 5: block patterns at n = 4
# ---------------------------------------------------------------------------

def _read_pattern(name):
    order, entries = None, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            parts = line.split()
            if parts[0] == "order":
                order = [t for t in parts[1:] if t != "|"]
            else:
                entries.append(tuple(parts))
    return order, entries


def _var_slices(p, q, n):
    o = type_offsets(p, q, n)
    sl = {}
    for k in range(1, n + 1):
        for t, w in (("u", p), ("v", p), ("z", q), ("lam", p), ("mu", p)):
            s = o[t] + (k - 1) * w
            sl[f"{t}{k}"] = slice(s, s + w)
    return sl


def _expected_block(tok, lv, p, q):
    if tok == "I":
        return None, 1.0
    if tok == "-I":
        return None, -1.0
    name, k = tok[0], int(tok[1])
    tr = tok.endswith("^T")
    M = {"N": lv.N, "V": lv.V_full(), "Z": lv.Z_full()}[name][k - 1]
    return (M.T if tr else M), None


def _check_pattern(A, order_index, entries, lv, p, q, n):
    """A: dense matrix; order_index: var -> slice in A's ordering."""
    covered = np.zeros(A.shape, dtype=bool)
    for r, c, tok in entries:
        rs, cs = order_index[r], order_index[c]
        blk = A[rs, cs]
        M, s = _expected_block(tok, lv, p, q)
        if M is None:
            np.testing.assert_array_equal(blk, s * np.eye(blk.shape[0]))
        else:
            np.testing.assert_array_equal(blk, M)
        covered[rs, cs] = True
    assert np.all(A[~covered] == 0.0), "nonzero outside the printed blocks"


def test_fig4_type_major_pattern():
    p, q, n = 2, 1, 4
    lv = random_level(n, p, q, 11)
    A = assemble_A(lv.N, lv.V, lv.Z).toarray()
    _, entries = _read_pattern("fig4_pattern_n4.txt")
    _check_pattern(A, _var_slices(p, q, n), entries, lv, p, q, n)


def test_fig5_time_major_pattern_and_blocks():
    p, q, n = 2, 1, 4
    lv = random_level(n, p, q, 12)
    A = assemble_A(lv.N, lv.V, lv.Z)
    perm = time_major_perm(p, q, n)
    At = A[perm][:, perm].toarray()
    order, entries = _read_pattern("fig5_pattern_n4.txt")
    widths = {"u": p, "v": p, "z": q, "lam": p, "mu": p}
    idx, pos = {}, 0
    for var in order:
        w = widths[var.rstrip("0123456789")]
        idx[var] = slice(pos, pos + w)
        pos += w
    assert pos == At.shape[0]
    # the permutation itself must produce the printed variable order
    sl = _var_slices(p, q, n)
    np.testing.assert_array_equal(
        perm, np.concatenate([np.arange(sl[v].start, sl[v].stop) for v in order]))
    _check_pattern(At, idx, entries, lv, p, q, n)
    # block-tridiagonal: the block split leaves only +I couplings between
    # u_k and mu_k, one block apart (Sec. 5.3.2)
    bounds = block_bounds(p, q, n)
    D, L, U = split_blocks(A[perm][:, perm].tocsr(), bounds)
    Ld = L.toarray()
    assert np.all(np.isin(Ld, [0.0, 1.0]))
    for k in range(1, n):
        rows = idx[f"mu{k}"]
        cols = idx[f"u{k}"]
        np.testing.assert_array_equal(Ld[rows, cols], np.eye(p))
    assert Ld.sum() == p * (n - 1) + p          # mu_1..mu_n rows, one identity each
    np.testing.assert_array_equal(U.toarray(), Ld.T)


# ---------------------------------------------------------------------------
# Algebraic invariants of the augmented matrix
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p,q,n", [(2, 1, 8), (3, 2, 6)])
def test_symmetry_inertia_and_spectrum(p, q, n):
    lv = random_level(n, p, q, 5)
    A = assemble_A(lv.N, lv.V, lv.Z)
    assert (A != A.T).nnz == 0
    Ad = A.toarray()
    ev = np.linalg.eigvalsh(Ad)
    # inertia of [[I, B^T], [B, 0]] with B of full row rank 2pn
    assert np.sum(ev > 1e-10) == (2 * p + q) * n
    assert np.sum(ev < -1e-10) == 2 * p * n
    # closed form: eigenvalues 1 (multiplicity cols - rows) and
    # (1 +- sqrt(1 + 4 sigma^2)) / 2 for every singular value sigma of B
    s = np.linalg.svd(assemble_B(lv.N, lv.V, lv.Z).toarray(), compute_uv=False)
    closed = np.concatenate([np.ones(q * n), (1 + np.sqrt(1 + 4 * s * s)) / 2,
                             (1 - np.sqrt(1 + 4 * s * s)) / 2])
    np.testing.assert_allclose(np.sort(ev), np.sort(closed), rtol=1e-10, atol=1e-10)


def _scaled_lifted_constraint(f, u, v, z, dt, theta, gamma, w0, M):
    """F~(u, v, z) in Euclidean variables, written from Sec. 4.1 and 5.1:
    lambda rows  dt^{-1/2} c~_k(dt^{-1/2} u, dt^{-1/2} v, (gamma^2 dt)^{-1/2} z)
    mu rows      u - v."""
    n = u.shape[0]
    U = u / np.sqrt(dt)
    Vv = v / np.sqrt(dt)
    Zp = z / (gamma * np.sqrt(dt))
    out = np.empty((2, n, u.shape[1]))
    for k in range(n):
        vprev = Vv[k - 1] if k > 0 else None
        vphys = vprev if vprev is not None else w0          # physical v_0
        mvprev = M @ vprev if vprev is not None else 0.0    # v_0 := 0 in M v_{k-1}
        c = (M @ U[k] - mvprev
             - dt * (theta * f(U[k], Zp[k]) + (1 - theta) * f(vphys, Zp[k])))
        out[0, k] = c / np.sqrt(dt)
        out[1, k] = u[k] - v[k]
    return out.reshape(-1)


@pytest.mark.parametrize("kind", ["vanderpol", "burgers"])
@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_blocks_match_finite_differences_of_scaled_constraint(kind, theta):
    """Central differences of F~ reproduce the assembled B~ = dF~ (Sec. 5.1)."""
    n, gamma = 6, 7.0
    rng = np.random.default_rng(3)
    if kind == "vanderpol":
        p, q = 2, 2
        jac, f = vanderpol_jacobians(0.3, q), vanderpol_rhs(0.3, q)
        w = rng.normal(0, 0.5, size=(n, p))
        w0 = np.array([1.0, 1.0])
    else:
        p = q = 5
        jac, f = burgers_jacobians(p, 0.05), burgers_rhs(p, 0.05)
        w = 0.5 + 0.2 * rng.normal(size=(n, p))
        w0 = np.sin(np.pi * np.arange(1, p + 1) / (p + 1))
    zeta = rng.normal(0, 0.5, size=(n, q))
    dt = 0.3 / n
    lv = lifted_blocks(w, zeta, w0, dt, theta, gamma, jac, compress=False)
    B = assemble_B(lv.N, lv.V, lv.Z).toarray()
    M = np.eye(p)
    u = np.sqrt(dt) * w
    v = np.sqrt(dt) * w                     # the lifted iterate has v = u
    z = gamma * np.sqrt(dt) * zeta
    x0 = np.concatenate([u.ravel(), v.ravel(), z.ravel()])

    def F(x):
        uu = x[:n * p].reshape(n, p)
        vv = x[n * p:2 * n * p].reshape(n, p)
        zz = x[2 * n * p:].reshape(n, q)
        return _scaled_lifted_constraint(f, uu, vv, zz, dt, theta, gamma, w0, M)

    J = np.empty_like(B)
    h = 1e-6
    for j in range(x0.size):
        e = np.zeros_like(x0)
        e[j] = h
        J[:, j] = (F(x0 + e) - F(x0 - e)) / (2 * h)
    assert np.max(np.abs(J - B)) <= 1e-6 * max(1.0, np.max(np.abs(B)))


def test_theorem1_invertibility():
    """D is nonsingular when every N_k is invertible (Thm. 1).  The condition
    is sufficient, not necessary: the block of step k is singular exactly when
    [N_k, Z~_k] loses row rank, e.g. N_k singular and Z~_k = 0."""
    p, q, n = 3, 2, 5
    lv = random_level(n, p, q, 21)
    ol = OracleLevel(lv.N, lv.V, lv.Z)
    D = ol.D.toarray()
    assert np.linalg.matrix_rank(D) == D.shape[0]
    N = lv.N.copy()
    N[2] = 0.0
    N[2][0, 0] = 1.0                       # rank-deficient N_3
    D2 = OracleLevel(N, lv.V, lv.Z).D.toarray()
    assert np.linalg.matrix_rank(D2) == D2.shape[0]      # Z~ restores the rank
    Z = lv.Z.copy()
    Z[2] = 0.0
    A3 = assemble_A(N, lv.V, Z)
    perm = time_major_perm(p, q, n)
    D3 = split_blocks(A3[perm][:, perm].tocsr(), block_bounds(p, q, n))[0].toarray()
    assert np.linalg.matrix_rank(D3) < D3.shape[0]


# ---------------------------------------------------------------------------
# Transfers (Sec. 5.3.1)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("variant", [0, 1])
def test_transfers(variant):
    p, q, nf = 2, 3, 16
    R = restriction(p, q, nf, variant)
    P = interpolation(p, q, nf, variant)
    nc = nf // 2
    np.testing.assert_array_equal((R @ P).toarray(), np.eye((4 * p + q) * nc))
    o_f, o_c = type_offsets(p, q, nf), type_offsets(p, q, nc)
    # interpolation reproduces data linear in the step index (node types),
    # away from the one-sided end of each variant
    kc = np.arange(1, nc + 1)
    xc = np.zeros((4 * p + q) * nc)
    a = np.array([0.3, -1.2])
    sc = (kc[:, None] * a[None, :]).ravel()          # s^c_k = k * a
    xc[o_c["u"]:o_c["v"]] = sc
    xc[o_c["mu"]:] = sc
    zc = np.arange(nc * q, dtype=float)
    xc[o_c["z"]:o_c["lam"]] = zc
    xf = P @ xc
    uf = xf[o_f["u"]:o_f["v"]].reshape(nf, p)
    kf = np.arange(1, nf + 1)
    # coarse step k sits at fine step 2k-1 (variant 0) or 2k (variant 1)
    pos = (kf + 1) / 2.0 if variant == 0 else kf / 2.0
    good = slice(0, nf - 1) if variant == 0 else slice(1, nf)
    np.testing.assert_allclose(uf[good], (pos[:, None] * a[None, :])[good], rtol=0, atol=1e-14)
    # control: piecewise constant interpolation, restriction averages pairs
    zf = xf[o_f["z"]:o_f["lam"]].reshape(nf, q)
    np.testing.assert_array_equal(zf[0::2], zf[1::2])
    np.testing.assert_array_equal(zf[0::2].ravel(), zc)
    y = np.random.default_rng(0).normal(size=(4 * p + q) * nf)
    zr = (R @ y)[o_c["z"]:o_c["lam"]].reshape(nc, q)
    yz = y[o_f["z"]:o_f["lam"]].reshape(nf, q)
    np.testing.assert_allclose(zr, 0.5 * (yz[0::2] + yz[1::2]), rtol=0, atol=1e-15)
    # injection of node variables
    ur = (R @ y)[o_c["u"]:o_c["v"]].reshape(nc, p)
    yu = y[o_f["u"]:o_f["v"]].reshape(nf, p)
    np.testing.assert_array_equal(ur, yu[0::2] if variant == 0 else yu[1::2])
    # mu_scale multiplies exactly the mu rows of R and the mu block of P
    R2 = restriction(p, q, nf, variant, mu_scale=2.0)
    P2 = interpolation(p, q, nf, variant, mu_scale=2.0)
    dR = (R2 - R).toarray()
    dP = (P2 - P).toarray()
    np.testing.assert_array_equal(dR[:o_c["mu"]], 0.0)
    np.testing.assert_array_equal(dR[o_c["mu"]:], R.toarray()[o_c["mu"]:])
    np.testing.assert_array_equal(dP[:, :o_c["mu"]], 0.0)
    np.testing.assert_array_equal(dP[:, o_c["mu"]:], P.toarray()[:, o_c["mu"]:])


# ---------------------------------------------------------------------------
# Smoothers (Sec. 5.3.2, 5.3.4) and Table 2
# ---------------------------------------------------------------------------

def test_jacobi_two_forms_and_exact_limit():
    p, q, n = 3, 2, 6
    lv = random_level(n, p, q, 8)
    ol = OracleLevel(lv.N, lv.V, lv.Z)
    rng = np.random.default_rng(1)
    b = rng.normal(size=ol.At.shape[0])
    y = rng.normal(size=ol.At.shape[0])
    y1 = ol.jacobi(b, y)
    # second form of eq. (jacobi): D^{-1} (b - (L + L^T) y)
    y2 = np.linalg.solve(ol.D.toarray(), b - (ol.L + ol.U) @ y)
    np.testing.assert_allclose(y1, y2, rtol=1e-11, atol=1e-11)
    # with the coupling blocks removed one sweep solves the system exactly
    ol.At = ol.D.tocsc()
    y3 = ol.jacobi(b, y)
    np.testing.assert_allclose(ol.D @ y3, b, rtol=1e-11, atol=1e-11)


def test_sgs_preconditioner_properties():
    p, q, n = 2, 1, 5
    lv = random_level(n, p, q, 9)
    ol = OracleLevel(lv.N, lv.V, lv.Z, factor_sgs=True)
    m = ol.At.shape[0]
    Minv = np.column_stack([ol.sgs(e) for e in np.eye(m)])
    # M = (D+L) D^{-1} (D+L^T) is symmetric for symmetric A~, and M - A~ =
    # L D^{-1} L^T is zero except in the rows/columns touched by L
    np.testing.assert_allclose(Minv, Minv.T, rtol=1e-9, atol=1e-9)
    M = np.linalg.inv(Minv)
    Dd, Ld = ol.D.toarray(), ol.L.toarray()
    np.testing.assert_allclose(M - ol.At.toarray(), Ld @ np.linalg.solve(Dd, Ld.T),
                               rtol=1e-8, atol=1e-8)


@pytest.mark.parametrize("n", [64, 128])
def test_table2_spectral_radii(n):
    """Block Jacobi spectral radii per level track Table 2.  The paper's first
    SQP iterate is not given; a constant iterate (w = 0) is used, so the band
    is 0.06.  Both the gamma = 1 (radius ~1) and gamma = 100 (radius well
    below 1, falling with the level) regimes must be reproduced."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table2_spectral_radii.txt"))
            if l.strip() and not l.startswith("#")]
    jac = vanderpol_jacobians(mu=0.1, q=2)
    prev = 2.0
    for r in rows:
        if int(r[0]) != n:
            continue
        nl = n >> (int(r[1]) - 1)
        for g, ref in ((1.0, float(r[2])), (100.0, float(r[3]))):
            w = np.zeros((nl, 2))
            lv = lifted_blocks(w, np.zeros((nl, 2)), np.ones(2), 8.0 / nl, 0.5, g, jac)
            ol = OracleLevel(lv.N, lv.V, lv.Z)
            A, D = ol.At.toarray(), ol.D.toarray()
            rho = np.max(np.abs(np.linalg.eigvals(np.eye(len(A)) - np.linalg.solve(D, A))))
            assert abs(rho - ref) <= 0.06, (n, r[1], g, rho, ref)
            if g == 100.0:
                assert rho < prev
                prev = rho


# ---------------------------------------------------------------------------
# Krylov solvers
# ---------------------------------------------------------------------------

def _krylov_minimiser(A, b, Minv, k):
    """argmin over x in M^{-1} K_k(A M^{-1}, b) of ||b - A x||, by brute force."""
    K = [b]
    for _ in range(k - 1):
        K.append(A @ (Minv @ K[-1]))
    Q, _ = np.linalg.qr(np.column_stack(K))
    Y = Minv @ Q
    c = np.linalg.lstsq(A @ Y, b, rcond=None)[0]
    return Y @ c


def test_gmres_right_matches_bruteforce_minimiser():
    rng = np.random.default_rng(4)
    m = 30
    A = rng.normal(size=(m, m)) + 4 * np.eye(m)
    Minv = np.linalg.inv(np.diag(np.diag(A)) + 0.5 * np.tril(A, -1))
    b = rng.normal(size=m)
    for k in (1, 3, 7):
        x, its = gmres_right(A, b, lambda r: Minv @ r, tol=0.0, maxit=50, fixed_its=k)
        assert its == k
        np.testing.assert_allclose(x, _krylov_minimiser(A, b, Minv, k), rtol=1e-8, atol=1e-10)
    # exact preconditioner: one step
    x, its = gmres_right(A, b, lambda r: np.linalg.solve(A, r), tol=1e-12, maxit=50)
    assert its == 1
    np.testing.assert_allclose(A @ x, b, rtol=1e-10, atol=1e-10)
    # k distinct eigenvalues: convergence in at most k steps
    Dg = np.diag(np.repeat([1.0, 2.0, 5.0], 10))
    x, its = gmres_right(Dg, b, lambda r: r, tol=1e-12, maxit=50)
    assert its <= 3
    np.testing.assert_allclose(Dg @ x, b, rtol=1e-9, atol=1e-9)


def test_fgmres_equals_gmres_for_fixed_preconditioner():
    rng = np.random.default_rng(6)
    m = 40
    A = rng.normal(size=(m, m)) + 5 * np.eye(m)
    Minv = np.linalg.inv(np.triu(A))
    b = rng.normal(size=m)
    x, info = fgmres(A, b, lambda r: Minv @ r, tol=1e-30, restart=6, maxit=6)
    assert info["iters"] == 6
    np.testing.assert_allclose(x, _krylov_minimiser(A, b, Minv, 6), rtol=1e-8, atol=1e-10)
    x, info = fgmres(A, b, lambda r: np.linalg.solve(A, r), tol=1e-12)
    assert info["iters"] == 1 and info["relres_true"] < 1e-12
    # restarted run still reaches the tolerance
    A2 = np.eye(m) + 0.05 * rng.normal(size=(m, m))
    x, info = fgmres(A2, b, lambda r: r, tol=1e-10, restart=5, maxit=200)
    assert info["converged"] and info["iters"] > 5 and info["relres_true"] < 1e-9


# ---------------------------------------------------------------------------
# Multigrid and the whole solve
# ---------------------------------------------------------------------------

def test_single_level_cycle_is_an_exact_solve():
    """With no coarsening the cycle is the coarse GMRES+SGS solve; at a tight
    tolerance it inverts A~ and FGMRES needs one step."""
    prob, rng = make_problem("vanderpol", n=8, n_levels=1, seed=7)
    b = make_rhs(prob, rng)
    H = Hierarchy(prob.levels, MGOptions(coarse_tol=1e-14, coarse_maxit=200))
    xd = direct_solve(prob.levels[0], b)
    np.testing.assert_allclose(H.vcycle(b), xd, rtol=1e-9, atol=1e-9 * np.abs(xd).max())
    x, info = H.solve(b, tol=1e-10)
    assert info["iters"] <= 2


def test_vcycle_is_consistent_two_grid():
    """Two levels, exact coarse solve: the error propagation of the cycle is
    S^nu (I - P A_c^{-1} R A) S^nu (Alg. 1)."""
    prob, rng = make_problem("vanderpol", n=16, n_levels=2, seed=3)
    H = Hierarchy(prob.levels, MGOptions(nu_pre=2, nu_post=1))
    lu = spla.splu(H.levels[1].At.tocsc())
    H.coarse_solve = lambda r: lu.solve(r)
    A = H.levels[0].At.toarray()
    m = A.shape[0]
    E = np.column_stack([H.mg(0, e) for e in np.eye(m)])
    S = np.eye(m) - H.opts.omega * np.linalg.solve(H.levels[0].D.toarray(), A)
    Ac = H.levels[1].At.toarray()
    CG = np.eye(m) - H.P[0].toarray() @ np.linalg.solve(Ac, H.R[0].toarray() @ A)
    T = S @ CG @ S @ S
    np.testing.assert_allclose(np.eye(m) - E @ A, T, rtol=1e-8, atol=1e-8)


@pytest.mark.parametrize("kind,kw", [("vanderpol", dict(n=16, n_levels=2)),
                                     ("burgers", dict(n=16, n_levels=2, nx=4))])
def test_whole_solve_matches_dense_direct_solve(kind, kw):
    prob, rng = make_problem(kind, seed=17, **kw)
    b = make_rhs(prob, rng)
    H = Hierarchy(prob.levels)
    x, info = H.solve(b, tol=1e-13, restart=200, maxit=400)
    assert info["converged"]
    lv = prob.levels[0]
    A = assemble_A(lv.N, lv.V_full(), lv.Z_full()).toarray()
    xd = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xd) / np.linalg.norm(xd) <= 1e-9
    assert info["relres_true"] <= 2e-13


def test_coarse_solve_tolerance_and_counts():
    """The coarse GMRES stops at the first step whose residual estimate is
    below 1e-3 relative (Sec. 5.3.4); its true residual agrees."""
    prob, rng = make_problem("burgers", nx=6, n=8, n_levels=1, seed=2)
    H = Hierarchy(prob.levels)
    b = make_rhs(prob, rng)
    lv = H.levels[0]
    x, its = gmres_right(lv.At, lv.to_time(b) if hasattr(lv, "to_time") else b[lv.perm],
                         lv.sgs, 1e-3, 50)
    bt = b[lv.perm]
    assert np.linalg.norm(bt - lv.At @ x) <= 1e-3 * np.linalg.norm(bt) * (1 + 1e-8)
    if its > 1:
        x1, _ = gmres_right(lv.At, bt, lv.sgs, 0.0, 50, fixed_its=its - 1)
        assert np.linalg.norm(bt - lv.At @ x1) > 1e-3 * np.linalg.norm(bt)


def test_single_block_helpers_match_the_assembled_operator():
    # block indices, dense diagonal blocks and couplings written one block at
    # a time agree with the assembled A~ and its time-major splitting
    from oracle.system import (block_index, diagonal_block, block_coupling, assemble_A,
                               time_major_perm, block_bounds, split_blocks)
    prob, rng = make_problem(kind="burgers", nx=4, nu=0.01, n=6, n_levels=1, seed=77)
    lv = prob.levels[0]
    p, q, n = prob.p, prob.q, lv.N.shape[0]
    A = assemble_A(lv.N, lv.V_full(), lv.Z_full()).toarray()
    perm = time_major_perm(p, q, n)
    bounds = block_bounds(p, q, n)
    assert np.array_equal(np.concatenate([block_index(p, q, n, k) for k in range(1, n + 2)]),
                          perm)
    y = rng.normal(size=A.shape[0])
    Vf, Zf = lv.V_full(), lv.Z_full()
    for k in range(1, n + 2):
        idx = block_index(p, q, n, k)
        kk = min(k, n) - 1
        D = diagonal_block(lv.N[kk], Vf[kk], Zf[kk], k, n)
        assert np.array_equal(D, A[np.ix_(idx, idx)])
        # the coupling is the rest of block k's rows of A~ y
        full = A[idx] @ y
        assert np.allclose(D @ y[idx] + block_coupling(y, p, q, n, k), full, rtol=0, atol=1e-12)


@pytest.mark.parametrize("shared", [False, True])
def test_blockwise_apply_matches_the_assembled_operator(shared):
    # the step-by-step product used where the assembled matrix is too large
    from oracle.system import apply_blocks
    lv = random_level(7, 3, 2, 21, shared=shared)
    A = assemble_A(lv.N, lv.V_full(), lv.Z_full())
    x = np.random.default_rng(5).normal(size=A.shape[0])
    np.testing.assert_allclose(apply_blocks(lv.N, lv.V, lv.Z, x), A @ x, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(apply_blocks(lv.N, lv.V, lv.Z, x, magnitude=True),
                               abs(A) @ abs(x), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("c", [2, 4, 8])
def test_transfers_coarsening_factor(c):
    """Coarsening by c: R P = I, interpolation reproduces data linear in time
    (coarse step k at fine step c(k-1)+1) away from the one-sided end,
    control averaged over / copied to the c fine steps, and the mu block
    scaled by mu_scale^(log2 c).  For c = 2 the factor-c forms are the
    printed ones (variant 0)."""
    p, q, nf = 2, 3, 32
    nc = nf // c
    R = restriction(p, q, nf, 0, c=c)
    P = interpolation(p, q, nf, 0, c=c)
    np.testing.assert_allclose((R @ P).toarray(), np.eye((4 * p + q) * nc), rtol=0, atol=1e-15)
    if c == 2:
        np.testing.assert_array_equal(R.toarray(), restriction(p, q, nf, 0).toarray())
        np.testing.assert_array_equal(P.toarray(), interpolation(p, q, nf, 0).toarray())
    o_f, o_c = type_offsets(p, q, nf), type_offsets(p, q, nc)
    a = np.array([0.7, -0.4])
    xc = np.zeros((4 * p + q) * nc)
    kc = np.arange(1, nc + 1)
    xc[o_c["lam"]:o_c["mu"]] = (kc[:, None] * a[None, :]).ravel()
    zc = np.random.default_rng(1).normal(size=nc * q)
    xc[o_c["z"]:o_c["lam"]] = zc
    xf = P @ xc
    lf = xf[o_f["lam"]:o_f["mu"]].reshape(nf, p)
    kf = np.arange(1, nf + 1)
    pos = (kf - 1) / c + 1.0                           # fine step in coarse units
    good = slice(0, nf - c + 1)
    np.testing.assert_allclose(lf[good], (pos[:, None] * a[None, :])[good], rtol=0, atol=1e-13)
    zf = xf[o_f["z"]:o_f["lam"]].reshape(nc, c, q)
    for i in range(c):
        np.testing.assert_array_equal(zf[:, i, :].ravel(), zc)
    y = np.random.default_rng(2).normal(size=(4 * p + q) * nf)
    yz = y[o_f["z"]:o_f["lam"]].reshape(nc, c, q)
    np.testing.assert_allclose((R @ y)[o_c["z"]:o_c["lam"]].reshape(nc, q), yz.mean(axis=1),
                               rtol=0, atol=1e-15)
    yu = y[o_f["v"]:o_f["z"]].reshape(nf, p)
    np.testing.assert_array_equal((R @ y)[o_c["v"]:o_c["z"]].reshape(nc, p), yu[0::c])
    Rm = restriction(p, q, nf, 0, mu_scale=2.0, c=c).toarray()
    np.testing.assert_allclose(Rm[o_c["mu"]:], c * R.toarray()[o_c["mu"]:], rtol=0, atol=0)
    with pytest.raises(ValueError):
        restriction(p, q, nf, 1, c=4) if c != 2 else restriction(p, q, 30, 0, c=4)
