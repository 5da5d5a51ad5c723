"""GMRES with a right preconditioner, and flexible GMRES (Saad 1993).

Both are written from the definition: the k-th iterate minimises the
residual 2-norm over the (preconditioned) Krylov space, with the basis built
by modified Gram-Schmidt and the small (k+1) x k Hessenberg least-squares
problem solved densely with numpy.linalg.lstsq at every step.  All in FP64.

GMRES preconditioned on the right by M^{-1} (coarse solver, Sec. 5.3.4):
    x_k = M^{-1} V_k y_k,   y_k = argmin || beta e_1 - H_k y ||.
Flexible GMRES (outer solver, Sec. 6): the preconditioner may change from
one step to the next, so the preconditioned vectors z_j = M_j(v_j) are kept
and x_k = x_0 + Z_k y_k.
"""
from __future__ import annotations

import numpy as np


def _lsq(H: np.ndarray, beta: float):
    rhs = np.zeros(H.shape[0])
    rhs[0] = beta
    y = np.linalg.lstsq(H, rhs, rcond=None)[0]
    res = np.linalg.norm(rhs - H @ y)
    return y, res


def gmres_right(A, b: np.ndarray, prec, tol: float, maxit: int,
                fixed_its: int = 0):
    """Right-preconditioned GMRES from x0 = 0, no restart.

    Stops when the residual estimate ||beta e1 - H y|| <= tol * ||b||, at
    maxit steps, or -- if fixed_its > 0 -- after exactly fixed_its steps
    (no tolerance test), which makes the result independent of where the
    residual lands relative to tol.  Returns (x, steps).
    """
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros_like(b), 0
    nsteps = fixed_its if fixed_its > 0 else maxit
    V = [b / beta]
    H = np.zeros((nsteps + 1, nsteps))
    k = 0
    y = None
    for j in range(nsteps):
        w = A @ prec(V[j])
        wnorm0 = np.linalg.norm(w)
        for i in range(j + 1):
            H[i, j] = np.dot(w, V[i])
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        k = j + 1
        y, res = _lsq(H[:k + 1, :k], beta)
        if fixed_its <= 0 and res <= tol * beta:
            break
        if H[j + 1, j] <= 1e-14 * wnorm0:
            break
        V.append(w / H[j + 1, j])
    x = prec(np.column_stack(V[:k]) @ y)
    return x, k


def fgmres(A, b: np.ndarray, prec, tol: float, restart: int = 30,
           maxit: int = 300, x0: np.ndarray = None):
    """Flexible GMRES with restart.

    prec(v) -> z may be nonlinear.  A cycle ends when its residual estimate
    reaches tol * ||b|| (or at breakdown / restart length / maxit); the solve
    is converged only when the true residual ||b - A x|| <= tol * ||b||, so
    a cycle whose estimate met the tolerance but whose true residual did not
    is followed by another cycle from the new residual.  Returns (x, info)
    with the step count, the history of relative residual estimates and the
    true relative residual at the end.
    """
    x = np.zeros_like(b) if x0 is None else x0.astype(np.float64).copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return np.zeros_like(b), dict(iters=0, history=[], relres_true=0.0,
                                      converged=True)
    total = 0
    hist = []
    converged = False
    while True:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta <= tol * bnorm:
            converged = True
            break
        if total >= maxit:
            break
        V = [r / beta]
        Zs = []
        H = np.zeros((restart + 1, restart))
        k = 0
        y = None
        stop = False
        for j in range(restart):
            Zs.append(prec(V[j]))
            w = A @ Zs[j]
            wnorm0 = np.linalg.norm(w)
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            k = j + 1
            total += 1
            y, res = _lsq(H[:k + 1, :k], beta)
            hist.append(res / bnorm)
            if res <= tol * bnorm or H[j + 1, j] <= 1e-14 * wnorm0:
                break                      # end of cycle; true residual decides
            if total >= maxit:
                stop = True
                break
            V.append(w / H[j + 1, j])
        x = x + np.column_stack(Zs[:k]) @ y
        if stop:
            break
    relres = np.linalg.norm(b - A @ x) / bnorm
    converged = relres <= tol
    return x, dict(iters=total, history=hist, relres_true=relres,
                   converged=converged)
