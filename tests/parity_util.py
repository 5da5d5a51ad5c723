"""Helpers shared by the GPU parity tests: host/device copies, the oracle's
cycle options that mirror the library's, and comparisons of type-major
vectors one variable type at a time (u, v, z, lambda, mu), so that an error
confined to a small slot (z carries 1/gamma; v and mu can be small) cannot
hide in one global norm."""
import functools

import numpy as np

from oracle import type_offsets
from oracle.multigrid import MGOptions

# the two readings of the smoother weight and the interface multiplier's
# transfer scale: the library's defaults, and the cycle exactly as printed
READINGS = {"weighted": dict(omega=0.5, mu_scale=2.0),
            "printed": dict(omega=1.0, mu_scale=1.0)}
TYPES = ("u", "v", "z", "lam", "mu")


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def mg_opts(o):
    """Oracle cycle options equal to the library options o."""
    return MGOptions(nu_pre=o.nu_pre, nu_post=o.nu_post, coarse_tol=o.coarse_tol,
                     coarse_maxit=o.coarse_maxit, coarse_fixed_its=o.coarse_fixed_its,
                     transfer_variant=o.transfer_variant, omega=o.omega,
                     mu_scale=o.mu_scale, cycle="VWF"[o.cycle],
                     smoother=("jacobi", "fgs", "bgs", "sgs")[o.smoother],
                     coarsen=o.coarsen)


def omega_at(o, lev, n_levels):
    """Smoother weight the library applies on level lev: the option above the
    coarsest level, 1 on the coarsest (its sweeps are exact block solves)."""
    return o.omega if lev < n_levels - 1 else 1.0


def sweep_ref(ol, b, y, omega):
    """Oracle block Jacobi sweep of type-major b, y (y None = 0)."""
    yt = ol.jacobi(b[ol.perm], np.zeros_like(b) if y is None else y[ol.perm], omega)
    ref = np.empty_like(yt)
    ref[ol.perm] = yt
    return ref


def type_errors(got, ref, p, q, n):
    """Relative 2-norm error of each variable type (type-major vectors)."""
    o = type_offsets(p, q, n)
    bounds = [o["u"], o["v"], o["z"], o["lam"], o["mu"], o["end"]]
    out = {}
    for t, a, b in zip(TYPES, bounds[:-1], bounds[1:]):
        d = np.linalg.norm(np.asarray(got)[a:b] - np.asarray(ref)[a:b])
        r = np.linalg.norm(np.asarray(ref)[a:b])
        out[t] = d / r if r > 0 else (0.0 if d == 0 else np.inf)
    return out


def assert_types(got, ref, p, q, n, tol, what=""):
    """Every variable type within tol (relative to that type's own norm)."""
    err = type_errors(got, ref, p, q, n)
    bad = {t: e for t, e in err.items() if not e <= tol}
    assert not bad, (what, tol, err)
    return err


def cond_S_max(lv):
    """max_k cond(S_k), S_k = N_k N_k^T + Z~_k Z~_k^T, on one level."""
    N, Z = lv.N, lv.Z_full()
    S = N @ np.transpose(N, (0, 2, 1)) + Z @ np.transpose(Z, (0, 2, 1))
    return float(np.max(np.linalg.cond(S)))


def sweep_tol(lv):
    """Tolerance of one block Jacobi sweep on level lv against the oracle's
    SuperLU of D_k: the library solves each block through the Schur
    complement S_k and the inverse of its Cholesky factor, whose rounding
    grows with cond(S_k) = cond([N_k Z~_k])^2: 64 u max_k cond(S_k), never
    tighter than 1e-11."""
    return max(1e-11, 64 * 2.0 ** -53 * cond_S_max(lv))


def coarse_identity_tol(prob):
    """Tolerance of a V-cycle whose coarse GMRES forms A~ z from its SGS sweeps.

    The library takes A~ z = v + L d (forward sweep a, backward correction
    d = z - a), exact in exact arithmetic.  In floating point it carries the
    residual of the coarse block solves, which go through the Schur
    complement S_k: about u cond(S_k) relative (u = 2^-53), so the bound is
    8 u max_k cond(S_k) on the coarsest level, and never tighter than the
    1e-10 of the explicit product.
    """
    return max(1e-10, 8 * 2.0 ** -53 * cond_S_max(prob.levels[-1]))


@functools.lru_cache(maxsize=2)
def full_config(name):
    """config_problem(name), built once per test session: the 512-node Burgers
    workload takes about half a minute and 20 GB of host memory to build."""
    from workloads import config_problem
    return config_problem(name)
