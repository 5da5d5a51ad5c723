"""The lifted augmented system and its time-major block structure.

Type-major vector order (Fig. 4): x = [u_1..u_n | v_1..v_n | z_1..z_n |
lambda_1..lambda_n | mu_1..mu_n], each u_k, v_k, lambda_k, mu_k of length p
and z_k of length q.

B~ = dF~ (Sec. 5.1) has one row block per constraint:
  lambda_k row (theta-method constraint with virtual variables):
      N_k at u_k,  V_k at v_{k-1} (k >= 2; v_0 := 0),  Z~_k at z_k
  mu_k row (scaled u = v condition, transplanted to u - v):
      +I at u_k,  -I at v_k
and the augmented matrix is A = [[I, B~^T], [B~, 0]] (eq. (augsys)).

Time-major order (Fig. 5): block 1 = (u_1, z_1, lambda_1); block k = 2..n
= (v_{k-1}, u_k, z_k, lambda_k, mu_{k-1}); block n+1 = (v_n, mu_n).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def type_offsets(p: int, q: int, n: int):
    """Start index of each variable type in the type-major vector."""
    return dict(u=0, v=p * n, z=2 * p * n, lam=2 * p * n + q * n,
                mu=3 * p * n + q * n, end=(4 * p + q) * n)


def assemble_B(N, V, Z) -> sp.csr_matrix:
    """B~ with rows [lambda rows (pn) ; mu rows (pn)] and columns
    [u (pn) ; v (pn) ; z (qn)].  N: (n,p,p), V: (n,p,p), Z: (n,p,q)."""
    n, p, _ = N.shape
    q = Z.shape[2]
    rows, cols, vals = [], [], []

    def put(block, r0, c0):
        r, c = np.nonzero(block)          # zero entries are not stored
        rows.append(r0 + r)
        cols.append(c0 + c)
        vals.append(block[r, c])

    lam0, mu0 = 0, p * n                      # row offsets
    u0, v0, z0 = 0, p * n, 2 * p * n          # column offsets
    eye = np.eye(p)
    for k in range(n):                        # 0-based k is step k+1
        put(N[k], lam0 + k * p, u0 + k * p)           # N_k at u_k
        if k >= 1:
            put(V[k], lam0 + k * p, v0 + (k - 1) * p)  # V_k at v_{k-1}
        put(Z[k], lam0 + k * p, z0 + k * q)           # Z~_k at z_k
        put(eye, mu0 + k * p, u0 + k * p)             # +u_k
        put(-eye, mu0 + k * p, v0 + k * p)            # -v_k
    B = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(2 * p * n, (2 * p + q) * n))
    return B


def assemble_A(N, V, Z) -> sp.csr_matrix:
    """Lifted augmented matrix in type-major order, A = [[I, B^T], [B, 0]]."""
    B = assemble_B(N, V, Z)
    m, ncol = B.shape
    A = sp.bmat([[sp.identity(ncol, format="csr"), B.T],
                 [B, sp.csr_matrix((m, m))]], format="csr")
    A.eliminate_zeros()
    return A


def time_major_perm(p: int, q: int, n: int) -> np.ndarray:
    """Index array perm with y = x[perm] (type-major -> time-major, Fig. 5)."""
    o = type_offsets(p, q, n)

    def rng(t, k, w):   # indices of variable t at step k (1-based)
        s = o[t] + (k - 1) * w
        return np.arange(s, s + w)

    parts = [rng("u", 1, p), rng("z", 1, q), rng("lam", 1, p)]
    for k in range(2, n + 1):
        parts += [rng("v", k - 1, p), rng("u", k, p), rng("z", k, q),
                  rng("lam", k, p), rng("mu", k - 1, p)]
    parts += [rng("v", n, p), rng("mu", n, p)]
    perm = np.concatenate(parts)
    assert perm.size == o["end"] and np.unique(perm).size == perm.size
    return perm


def block_bounds(p: int, q: int, n: int) -> np.ndarray:
    """Offsets of the n+1 diagonal blocks in the time-major vector."""
    sizes = [2 * p + q] + [4 * p + q] * (n - 1) + [2 * p]
    return np.concatenate([[0], np.cumsum(sizes)])


def split_blocks(At: sp.csr_matrix, bounds: np.ndarray):
    """Block diagonal D, strictly lower block part L and strictly upper block
    part U of a time-major matrix (Sec. 5.3.2)."""
    C = At.tocoo()
    blk = np.searchsorted(bounds, np.arange(At.shape[0]), side="right") - 1
    br, bc = blk[C.row], blk[C.col]
    def pick(mask):
        return sp.csr_matrix((C.data[mask], (C.row[mask], C.col[mask])), shape=At.shape)
    return pick(br == bc), pick(br > bc), pick(br < bc)


# ---------------------------------------------------------------------------
# One time-major block at a time (for sizes whose assembled matrix is too
# large to form): indices, the dense diagonal block D_k and its right-hand
# side, written from the operator rows of the lifted system (Fig. 4, Fig. 5).
# ---------------------------------------------------------------------------

def block_index(p: int, q: int, n: int, k: int) -> np.ndarray:
    """Type-major indices of time-major block k (1-based), in the block's
    order: block 1 (u_1, z_1, lambda_1); 2 <= k <= n (v_{k-1}, u_k, z_k,
    lambda_k, mu_{k-1}); block n+1 (v_n, mu_n)."""
    o = type_offsets(p, q, n)

    def rng(t, kk, w):
        s = o[t] + (kk - 1) * w
        return np.arange(s, s + w)

    if k == 1:
        return np.concatenate([rng("u", 1, p), rng("z", 1, q), rng("lam", 1, p)])
    if k == n + 1:
        return np.concatenate([rng("v", n, p), rng("mu", n, p)])
    return np.concatenate([rng("v", k - 1, p), rng("u", k, p), rng("z", k, q),
                           rng("lam", k, p), rng("mu", k - 1, p)])


def diagonal_block(Nk: np.ndarray, Vk: np.ndarray, Zk: np.ndarray, k: int, n: int) -> np.ndarray:
    """Dense D_k from the rows of A~ restricted to block k's own unknowns:
    u_k: u_k + N_k^T lambda_k;  v_{k-1}: v_{k-1} + V_k^T lambda_k - mu_{k-1};
    z_k: z_k + Z_k^T lambda_k;  lambda_k: N_k u_k + V_k v_{k-1} + Z_k z_k;
    mu_{k-1}: -v_{k-1} (its u_{k-1} term couples to block k-1).  Block n+1
    holds v_n (v_n - mu_n, V_{n+1} := 0) and mu_n (-v_n)."""
    p, q = Nk.shape[0], Zk.shape[1]
    I = np.eye(p)
    if k == n + 1:
        return np.block([[I, -I], [-I, np.zeros((p, p))]])
    if k == 1:
        return np.block([[I, np.zeros((p, q)), Nk.T],
                         [np.zeros((q, p)), np.eye(q), Zk.T],
                         [Nk, Zk, np.zeros((p, p))]])
    Zp, Zq, Zqp = np.zeros((p, p)), np.zeros((p, q)), np.zeros((q, p))
    return np.block([
        [I, Zp, Zq, Vk.T, -I],
        [Zp, I, Zq, Nk.T, Zp],
        [Zqp, Zqp, np.eye(q), Zk.T, Zqp],
        [Vk, Nk, Zk, Zp, Zp],
        [-I, Zp, Zq, Zp, Zp],
    ])


def block_coupling(y: np.ndarray, p: int, q: int, n: int, k: int) -> np.ndarray:
    """((L + L^T) y) on block k: the u_k row sees +mu_k (block k+1) and the
    mu_{k-1} row sees +u_{k-1} (block k-1); block n+1's mu_n row sees +u_n."""
    o = type_offsets(p, q, n)
    if k == n + 1:
        return np.concatenate([np.zeros(p), y[o["u"] + (n - 1) * p: o["u"] + n * p]])
    mu_k = y[o["mu"] + (k - 1) * p: o["mu"] + k * p]
    if k == 1:
        return np.concatenate([mu_k, np.zeros(q + p)])
    u_km1 = y[o["u"] + (k - 2) * p: o["u"] + (k - 1) * p]
    return np.concatenate([np.zeros(p), mu_k, np.zeros(q + p), u_km1])


def apply_blocks(N, V, Z, x: np.ndarray, magnitude: bool = False) -> np.ndarray:
    """A~ x in type-major order from the operator rows of the lifted system
    (Fig. 4), step by step with dense products, for sizes whose assembled
    matrix is too large to form.  N: (n,p,p), V: (n,p,p), Z: (n,p,q), each
    possibly of leading size 1 (shared by every step):
      u_k:      u_k + N_k^T lambda_k + mu_k
      v_k:      v_k + V_{k+1}^T lambda_{k+1} - mu_k      (V_{n+1} := 0)
      z_k:      z_k + Z_k^T lambda_k
      lambda_k: N_k u_k + V_k v_{k-1} + Z_k z_k          (v_0 := 0)
      mu_k:     u_k - v_k
    magnitude=True gives |A~| |x| instead (every entry and every sign taken
    positive), the scale of the rounding error of a computed product.
    """
    N = np.asarray(N)
    sg = -1.0
    if magnitude:
        N, V, Z, x, sg = np.abs(N), np.abs(V), np.abs(Z), np.abs(x), 1.0
    n, p, _ = N.shape
    q = Z.shape[2]
    o = type_offsets(p, q, n)
    u = x[o["u"]:o["v"]].reshape(n, p)
    v = x[o["v"]:o["z"]].reshape(n, p)
    z = x[o["z"]:o["lam"]].reshape(n, q)
    lam = x[o["lam"]:o["mu"]].reshape(n, p)
    mu = x[o["mu"]:o["end"]].reshape(n, p)
    vprev = np.vstack([np.zeros((1, p)), v[:-1]])
    Vb = np.broadcast_to(V, (n, p, p))
    Zb = np.broadcast_to(Z, (n, p, q))
    out = np.empty_like(x)
    out[o["u"]:o["v"]] = (u + np.einsum("kij,ki->kj", N, lam) + mu).ravel()
    vt = np.einsum("kij,ki->kj", Vb[1:], lam[1:])
    out[o["v"]:o["z"]] = (v + sg * mu + np.vstack([vt, np.zeros((1, p))])).ravel()
    out[o["z"]:o["lam"]] = (z + np.einsum("kij,ki->kj", Zb, lam)).ravel()
    lrow = np.einsum("kij,kj->ki", N, u) + np.einsum("kij,kj->ki", Zb, z)
    lrow[1:] += np.einsum("kij,kj->ki", Vb[1:], vprev[1:])
    out[o["lam"]:o["mu"]] = lrow.ravel()
    out[o["mu"]:o["end"]] = (u + sg * v).ravel()
    return out
