"""ctypes binding of libpitmg.so (declarations: include/pitmg.h).

The functions keep the C names (pitmg_setup, pitmg_apply, pitmg_jacobi_sweep,
pitmg_coarse_solve, pitmg_vcycle, pitmg_fgmres_solve, ...) and only marshal
arguments.  Device memory and the stream come from PyTorch; every step of the
solve runs in the HIP library.  There is no fallback: if the library is not
built, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import List, Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpitmg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "pitmg.h")

PITMG_OK = 0
PITMG_NOT_CONVERGED = 1
PITMG_ERR_INVALID = -1
PITMG_ERR_SINGULAR = -2
PITMG_ERR_NONFINITE = -3
PITMG_ERR_HIP = -4
PITMG_ERR_OOM = -5
PITMG_ERR_UNSUPPORTED = -6

PROFILE_CLASSES = ("factor", "jacobi", "apply", "transfer", "coarse", "krylov")


class pitmg_problem(C.Structure):
    _fields_ = [("p", C.c_int), ("q", C.c_int), ("n", C.c_int), ("n_levels", C.c_int),
                ("N", C.POINTER(C.c_void_p)), ("V", C.POINTER(C.c_void_p)),
                ("Z", C.POINTER(C.c_void_p)), ("N_stride", C.c_longlong),
                ("V_stride", C.c_longlong), ("Z_stride", C.c_longlong),
                ("blocks_on_device", C.c_int)]


class pitmg_options(C.Structure):
    _fields_ = [("nu_pre", C.c_int), ("nu_post", C.c_int), ("coarse_tol", C.c_double),
                ("coarse_maxit", C.c_int), ("coarse_fixed_its", C.c_int),
                ("restart", C.c_int), ("maxit", C.c_int), ("transfer_variant", C.c_int),
                ("smoother_fp32", C.c_int), ("coarse_mode", C.c_int), ("stall_ratio", C.c_double),
                ("stall_steps", C.c_int), ("vcycle_graph", C.c_int),
                ("apply_from_sweep", C.c_int),
                ("pair_sweeps", C.c_int),
                ("omega", C.c_double),
                ("mu_scale", C.c_double),
                ("cycle", C.c_int),
                ("smoother", C.c_int),
                ("unlifted", C.c_int),
                ("coarsen", C.c_int)]


class pitmg_stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("converged", C.c_int), ("relres_est", C.c_double),
                ("relres_true", C.c_double), ("coarse_calls", C.c_int),
                ("coarse_its_total", C.c_int), ("ms_solve", C.c_double),
                ("net_calls", C.c_int), ("fallback_at", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class pitmg_burgers(C.Structure):
    _fields_ = [("nx", C.c_int), ("n", C.c_int), ("n_levels", C.c_int), ("T", C.c_double),
                ("gamma", C.c_double), ("w0", C.POINTER(C.c_double))]


class pitmg_dogleg_params(C.Structure):
    _fields_ = [("ftol", C.c_double), ("lin_tol", C.c_double), ("maxit", C.c_int),
                ("eta", C.c_double)]


class pitmg_dogleg_stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("accepted", C.c_int), ("converged", C.c_int),
                ("solves", C.c_int), ("fgmres_iters", C.c_int), ("coarse_calls", C.c_int),
                ("coarse_its", C.c_int), ("fnorm0", C.c_double), ("fnorm", C.c_double),
                ("ms", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PitmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pitmg error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libpitmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with "
                          "`python -m paper_2405_04808_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(path)
    vp, i, d = C.c_void_p, C.c_int, C.c_double
    sig = {
        "pitmg_default_options": (None, [C.POINTER(pitmg_options)]),
        "pitmg_setup": (i, [C.POINTER(vp), C.POINTER(pitmg_problem), C.POINTER(pitmg_options), vp]),
        "pitmg_refactor": (i, [vp, C.POINTER(pitmg_problem)]),
        "pitmg_set_options": (i, [vp, C.POINTER(pitmg_options)]),
        "pitmg_apply": (i, [vp, i, vp, vp]),
        "pitmg_jacobi_sweep": (i, [vp, i, vp, vp, vp]),
        "pitmg_coarse_solve": (i, [vp, vp, vp, C.POINTER(i)]),
        "pitmg_coarse_solve_noalloc": (i, [vp, vp, vp, C.POINTER(i)]),
        "pitmg_vcycle": (i, [vp, vp, vp]),
        "pitmg_fgmres_solve": (i, [vp, vp, vp, d, i, C.POINTER(pitmg_stats)]),
        "pitmg_unlifted_apply": (i, [vp, vp, vp]),
        "pitmg_unlifted_fgmres_solve": (i, [vp, vp, vp, d, i, C.POINTER(pitmg_stats)]),
        "pitmg_fgmres_solve_batch": (i, [C.POINTER(vp), i, C.POINTER(vp), C.POINTER(vp), d, i,
                                         C.POINTER(pitmg_stats), C.POINTER(i)]),
        "pitmg_profile_enable": (i, [vp, i]),
        "pitmg_profile_read": (i, [vp, i, C.POINTER(i), C.POINTER(d), C.POINTER(d)]),
        "pitmg_profile_reset": (i, [vp]),
        "pitmg_profile_sample": (i, [vp, i]),
        "pitmg_failed_block": (i, [vp, C.POINTER(i), C.POINTER(i)]),
        "pitmg_device_bytes": (C.c_longlong, [vp]),
        "pitmg_level_info": (i, [vp, i, C.POINTER(i), C.POINTER(i)]),
        "pitmg_default_dogleg_params": (None, [C.POINTER(pitmg_dogleg_params)]),
        "pitmg_burgers_residual": (i, [C.POINTER(pitmg_burgers), d, vp, vp, vp]),
        "pitmg_burgers_dogleg": (i, [C.POINTER(pitmg_burgers), C.POINTER(pitmg_options),
                                     C.POINTER(d), i, vp, C.POINTER(pitmg_dogleg_params),
                                     C.POINTER(pitmg_dogleg_stats), vp]),
        "pitmg_burgers_last_error": (C.c_char_p, []),
        "pitmg_net_param_count": (C.c_longlong, [i, i]),
        "pitmg_net_create": (i, [C.POINTER(vp), i, i, i, i, vp]),
        "pitmg_net_set_params": (i, [vp, vp, i]),
        "pitmg_net_get_params": (i, [vp, vp]),
        "pitmg_net_forward": (i, [vp, i, vp, vp]),
        "pitmg_net_backward": (i, [vp, i, vp, vp, vp]),
        "pitmg_net_adam": (i, [vp, vp, C.c_float]),
        "pitmg_net_train_step": (i, [vp, i, vp, i, vp, vp, C.c_float, C.POINTER(d)]),
        "pitmg_net_make_samples": (i, [vp, i, i, i, vp, vp, vp, vp]),
        "pitmg_net_last_error": (C.c_char_p, [vp]),
        "pitmg_net_destroy": (None, [vp]),
        "pitmg_coarse_net_attach": (i, [vp, vp]),
        "pitmg_coarse_pairs_arm": (i, [vp, vp, vp, i]),
        "pitmg_coarse_pairs_count": (i, [vp]),
        "pitmg_autotune": (i, [vp, C.POINTER(i)]),
        "pitmg_set_sweep_shapes": (i, [vp, C.POINTER(i)]),
        "pitmg_set_handoff_wait": (i, [vp, C.c_double]),
        "pitmg_status_string": (C.c_char_p, [i]),
        "pitmg_last_error": (C.c_char_p, [vp]),
        "pitmg_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def header_functions(path: str = HEADER) -> List[str]:
    """Names of the functions declared in include/pitmg.h."""
    txt = open(path).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pitmg_[a-z_]+)\s*\(", txt)))


def default_options(**over) -> pitmg_options:
    o = pitmg_options()
    load_library().pitmg_default_options(C.byref(o))
    for k, v in over.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Solver:
    """One handle of the HIP solver over device copies of the blocks.

    levels: sequence with .N (n_l,p,p), .V, .Z numpy arrays per level (V/Z of
    leading size 1 when shared by every step); they are uploaded once into
    torch device tensors which the library borrows.
    """

    def __init__(self, levels: Sequence, options: Optional[pitmg_options] = None,
                 device: str = "cuda", stream=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the solver runs on a GPU device")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.options = options if options is not None else default_options()
        self.h = C.c_void_p()
        self._upload(levels)
        # the library works on self.stream: the uploads (on the current
        # stream) must be complete before setup reads the blocks
        self._order()
        pb = self._problem()
        with torch.cuda.device(self.device):
            rc = self.lib.pitmg_setup(C.byref(self.h), C.byref(pb), C.byref(self.options),
                                      C.c_void_p(self.stream.cuda_stream))
        if rc < 0:
            msg = self.last_error()
            self.close()
            raise PitmgError(rc, msg)

    # -- blocks -----------------------------------------------------------------
    def _upload(self, levels):
        torch = self.torch
        lv0 = levels[0]
        self.p = lv0.N.shape[1]
        self.q = lv0.Z.shape[2]
        self.n = lv0.N.shape[0]
        self.n_levels = len(levels)
        self.shared_V = lv0.V.shape[0] == 1 and self.n > 1
        self.shared_Z = lv0.Z.shape[0] == 1 and self.n > 1
        # the library borrows these arrays with the sizes the options imply:
        # level l holds n / coarsen^l steps
        c = int(getattr(self.options, "coarsen", 2) or 2)
        for l, lv in enumerate(levels):
            nl = self.n // c ** l
            ok = (self.n % c ** l == 0 and lv.N.shape[0] == nl
                  and lv.V.shape[0] in ((1,) if self.shared_V else (nl,))
                  and lv.Z.shape[0] in ((1,) if self.shared_Z else (nl,)))
            if not ok:
                raise ValueError(f"level {l} does not hold n / {c}^{l} = {nl} steps")
        self.dN, self.dV, self.dZ = [], [], []
        for lv in levels:
            self.dN.append(torch.as_tensor(lv.N, dtype=torch.float64).contiguous().to(self.device))
            self.dV.append(torch.as_tensor(lv.V, dtype=torch.float64).contiguous().to(self.device))
            self.dZ.append(torch.as_tensor(lv.Z, dtype=torch.float64).contiguous().to(self.device))
        self.lens = [(4 * self.p + self.q) * lv.N.shape[0] for lv in levels]

    def _problem(self) -> pitmg_problem:
        arr = C.c_void_p * self.n_levels
        self._pN = arr(*[t.data_ptr() for t in self.dN])
        self._pV = arr(*[t.data_ptr() for t in self.dV])
        self._pZ = arr(*[t.data_ptr() for t in self.dZ])
        pb = pitmg_problem()
        pb.p, pb.q, pb.n, pb.n_levels = self.p, self.q, self.n, self.n_levels
        pb.N = C.cast(self._pN, C.POINTER(C.c_void_p))
        pb.V = C.cast(self._pV, C.POINTER(C.c_void_p))
        pb.Z = C.cast(self._pZ, C.POINTER(C.c_void_p))
        pb.N_stride = self.p * self.p
        pb.V_stride = 0 if self.shared_V else self.p * self.p
        pb.Z_stride = 0 if self.shared_Z else self.p * self.q
        pb.blocks_on_device = 1
        return pb

    def refactor(self, levels):
        """New blocks (same sizes): copy into the borrowed tensors, re-factor."""
        for l, lv in enumerate(levels):
            self.dN[l].copy_(self.torch.as_tensor(lv.N, dtype=self.torch.float64))
            self.dV[l].copy_(self.torch.as_tensor(lv.V, dtype=self.torch.float64))
            self.dZ[l].copy_(self.torch.as_tensor(lv.Z, dtype=self.torch.float64))
        self._check(self.lib.pitmg_refactor(self.h, C.byref(self._problem())))

    def refactor_device(self):
        """Re-factor from the (already updated) device block tensors."""
        self._check(self.lib.pitmg_refactor(self.h, C.byref(self._problem())))

    # -- calls ------------------------------------------------------------------
    def _order(self):
        """Make the solver's stream wait for work queued on the current stream
        (inputs written there); a no-op when they are the same stream."""
        cur = self.torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            self.stream.wait_stream(cur)

    def _check(self, rc):
        if rc < 0:
            raise PitmgError(rc, self.last_error())
        return rc

    def last_error(self) -> str:
        s = self.lib.pitmg_last_error(self.h)
        return s.decode() if s else ""

    def empty(self, level: int = 0):
        return self.torch.empty(self.lens[level], dtype=self.torch.float64, device=self.device)

    def set_options(self, **over):
        o = pitmg_options()
        C.memmove(C.byref(o), C.byref(self.options), C.sizeof(o))
        for k, v in over.items():
            setattr(o, k, v)
        self._check(self.lib.pitmg_set_options(self.h, C.byref(o)))
        self.options = o

    def apply(self, x, level: int = 0, out=None):
        out = self.empty(level) if out is None else out
        self._order()
        self._check(self.lib.pitmg_apply(self.h, level, _ptr(x), _ptr(out)))
        return out

    def jacobi_sweep(self, b, y_in=None, level: int = 0, out=None):
        out = self.empty(level) if out is None else out
        self._order()
        self._check(self.lib.pitmg_jacobi_sweep(self.h, level, _ptr(b), _ptr(y_in), _ptr(out)))
        return out

    def coarse_solve(self, b, out=None):
        out = self.empty(self.n_levels - 1) if out is None else out
        its = C.c_int(0)
        self._order()
        self._check(self.lib.pitmg_coarse_solve(self.h, _ptr(b), _ptr(out), C.byref(its)))
        return out, its.value

    def vcycle(self, r, out=None):
        out = self.empty(0) if out is None else out
        self._order()
        self._check(self.lib.pitmg_vcycle(self.h, _ptr(r), _ptr(out)))
        return out

    def solve(self, b, tol: float = 1e-10, x0=None, out=None):
        """Returns (x, stats dict, status code >= 0)."""
        x = out if out is not None else self.empty(0)
        use_x0 = 0
        if x0 is not None:
            x.copy_(x0)
            use_x0 = 1
        st = pitmg_stats()
        self._order()
        rc = self._check(self.lib.pitmg_fgmres_solve(self.h, _ptr(b), _ptr(x), float(tol),
                                                     use_x0, C.byref(st)))
        return x, st.as_dict(), rc

    # -- the system without virtual variables (options.unlifted = 1) -----------
    def unlifted_len(self) -> int:
        return (2 * self.p + self.q) * self.n

    def unlifted_apply(self, x, out=None):
        """y = A x for the unlifted system (Fig. 2), vectors [u | z | lambda]."""
        y = out if out is not None else self.torch.empty(self.unlifted_len(), dtype=self.torch.float64,
                                                         device=self.device)
        self._order()
        self._check(self.lib.pitmg_unlifted_apply(self.h, _ptr(x), _ptr(y)))
        return y

    def unlifted_solve(self, b, tol: float = 1e-10, x0=None, out=None):
        """FGMRES on the unlifted system with the lifted cycle through the
        lift / project maps; returns (x, stats dict, status code >= 0)."""
        x = out if out is not None else self.torch.empty(self.unlifted_len(),
                                                         dtype=self.torch.float64,
                                                         device=self.device)
        use_x0 = 0
        if x0 is not None:
            x.copy_(x0)
            use_x0 = 1
        st = pitmg_stats()
        self._order()
        rc = self._check(self.lib.pitmg_unlifted_fgmres_solve(self.h, _ptr(b), _ptr(x),
                                                              float(tol), use_x0, C.byref(st)))
        return x, st.as_dict(), rc

    # -- profiling --------------------------------------------------------------
    def profile(self, on=True):
        """True / 1: time every launch; 2: the block Jacobi sweep only; False / 0: off."""
        level = int(on) if not isinstance(on, bool) else (1 if on else 0)
        self._check(self.lib.pitmg_profile_enable(self.h, level))

    def profile_sample(self, every: int):
        """Time the sweeps of every `every`-th V-cycle only."""
        self._check(self.lib.pitmg_profile_sample(self.h, int(every)))

    def profile_reset(self):
        self._check(self.lib.pitmg_profile_reset(self.h))

    def profile_read(self):
        out = {}
        for c, name in enumerate(PROFILE_CLASSES):
            n = C.c_int(0)
            ms = C.c_double(0)
            by = C.c_double(0)
            self._check(self.lib.pitmg_profile_read(self.h, c, C.byref(n), C.byref(ms), C.byref(by)))
            out[name] = (n.value, ms.value)
        return out

    def failed_block(self):
        lv, k = C.c_int(0), C.c_int(0)
        self.lib.pitmg_failed_block(self.h, C.byref(lv), C.byref(k))
        return lv.value, k.value

    def device_bytes(self) -> int:
        return self.lib.pitmg_device_bytes(self.h)

    def level_info(self, level: int) -> dict:
        """Step count and sweep form of one level: fp32 (FP32 sweeps),
        diag_vz (shared diagonal V and Z~ used through their diagonals) and
        gin (one-step sweeps on W = G^{-1} N)."""
        n, f = C.c_int(), C.c_int()
        self._check(self.lib.pitmg_level_info(self.h, level, C.byref(n), C.byref(f)))
        return dict(n=n.value, fp32=bool(f.value & 1), diag_vz=bool(f.value & 2),
                    gin=bool(f.value & 4))

    def autotune(self):
        """Pick each level's sweep launch shape by timing; returns the choices."""
        cfg = (C.c_int * self.n_levels)()
        self._check(self.lib.pitmg_autotune(self.h, cfg))
        return list(cfg)

    def set_handoff_wait(self, seconds: float):
        """Bound of each neighbour wait of the two-sweep launches (seconds)."""
        self._check(self.lib.pitmg_set_handoff_wait(self.h, C.c_double(seconds)))

    def set_sweep_shapes(self, cfg):
        """Set each level's sweep launch shape (as returned by autotune)."""
        arr = (C.c_int * self.n_levels)(*cfg)
        self._check(self.lib.pitmg_set_sweep_shapes(self.h, arr))

    # -- learned coarse correction ------------------------------------------------
    def attach_net(self, net: Optional["Net"]):
        """Use net for the coarse solve when coarse_mode = 1 (None detaches)."""
        self._net = net
        self._check(self.lib.pitmg_coarse_net_attach(self.h, net.h if net is not None else None))

    def arm_pairs(self, r, e, cap: int):
        """Record (r_c, e_c) of the next GMRES+SGS coarse solves into r, e
        (device FP64 [cap][len_c])."""
        self._pairs = (r, e)
        self._check(self.lib.pitmg_coarse_pairs_arm(self.h, _ptr(r), _ptr(e), int(cap)))

    def pair_count(self) -> int:
        return self.lib.pitmg_coarse_pairs_count(self.h)

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.pitmg_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(solvers: Sequence["Solver"], bs, tol: float = 1e-10, outs=None):
    """pitmg_fgmres_solve_batch over distinct solvers: returns (xs, stats
    dicts, status codes, overall code).  bs: device FP64 right-hand sides."""
    lib = load_library()
    n = len(solvers)
    xs = list(outs) if outs is not None else [s.empty(0) for s in solvers]
    H = (C.c_void_p * n)(*[s.h.value for s in solvers])
    R = (C.c_void_p * n)(*[b.data_ptr() for b in bs])
    X = (C.c_void_p * n)(*[x_.data_ptr() for x_ in xs])
    st = (pitmg_stats * n)()
    status = (C.c_int * n)()
    for s_ in solvers:
        s_._order()
    rc = lib.pitmg_fgmres_solve_batch(H, n, R, X, float(tol), 0, st, status)
    if rc < 0:
        bad = [i for i in range(n) if status[i] < 0]
        msg = solvers[bad[0]].last_error() if bad else ""
        raise PitmgError(rc, f"system {bad[0] if bad else '?'}: {msg}")
    return xs, [st[i].as_dict() for i in range(n)], [status[i] for i in range(n)], rc


class Burgers:
    """Burgers' equation F(u, z~) = 0 on the device (pitmg_burgers_*): nx
    interior nodes, n steps on [0, T], control scaling gamma, initial state
    w0 (numpy, nx).  Vectors x = [u | z~] are torch FP64 device tensors of
    2 nx n values; every computation runs in the HIP library."""

    def __init__(self, nx: int, n: int, n_levels: int, T: float, gamma: float, w0):
        import numpy as np
        self.lib = load_library()
        self._w0 = np.ascontiguousarray(w0, dtype=np.float64)
        if self._w0.shape != (nx,):
            raise ValueError("w0 must hold nx values")
        self.spec = pitmg_burgers(nx, n, n_levels, float(T), float(gamma),
                                  self._w0.ctypes.data_as(C.POINTER(C.c_double)))

    def _stream(self, x):
        import torch
        return C.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)

    def _err(self, rc):
        raise PitmgError(rc, self.lib.pitmg_burgers_last_error().decode())

    def residual(self, x, nu: float, out=None):
        import torch
        out = out if out is not None else torch.empty(self.spec.nx * self.spec.n,
                                                      dtype=torch.float64, device=x.device)
        rc = self.lib.pitmg_burgers_residual(C.byref(self.spec), float(nu), _ptr(x), _ptr(out),
                                             self._stream(x))
        if rc < 0:
            self._err(rc)
        return out

    def dogleg(self, x, nus: Sequence[float], options: Optional[pitmg_options] = None,
               ftol: float = 1e-8, lin_tol: float = 1e-6, maxit: int = 50, eta: float = 1e-4):
        """Continuation over nus from x (updated in place); returns (stats
        dicts, status code >= 0)."""
        dp = pitmg_dogleg_params(float(ftol), float(lin_tol), int(maxit), float(eta))
        k = len(nus)
        arr = (C.c_double * k)(*[float(v) for v in nus])
        st = (pitmg_dogleg_stats * k)()
        o = options if options is not None else default_options()
        rc = self.lib.pitmg_burgers_dogleg(C.byref(self.spec), C.byref(o), arr, k, _ptr(x),
                                           C.byref(dp), st, self._stream(x))
        if rc < 0:
            self._err(rc)
        return [st[i].as_dict() for i in range(k)], rc


class Net:
    """The learned coarse correction's network (pitmg_net_*): C channels over
    T coarse steps, H hidden channels, batches up to max_batch.  Tensors are
    torch device tensors; every computation runs in the HIP library."""

    def __init__(self, C: int, T: int, H: int = 64, max_batch: int = 256, device: str = "cuda",
                 stream=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.device = torch.device(device)
        self.C, self.T, self.H, self.max_batch = C, T, H, max_batch
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.h = _c_void_p()
        with torch.cuda.device(self.device):
            rc = self.lib.pitmg_net_create(_byref(self.h), C, T, H, max_batch,
                                           _c_void_p(self.stream.cuda_stream))
        if rc < 0:
            raise PitmgError(rc, "pitmg_net_create failed")
        self.P = int(self.lib.pitmg_net_param_count(C, H))

    def _check(self, rc):
        if rc < 0:
            msg = self.lib.pitmg_net_last_error(self.h)
            raise PitmgError(rc, msg.decode() if msg else "")
        return rc

    def set_params(self, theta):
        t = self.torch.as_tensor(theta, dtype=self.torch.float32).contiguous().to(self.device)
        self._check(self.lib.pitmg_net_set_params(self.h, _ptr(t), 1))

    def get_params(self):
        import numpy as np
        out = np.empty(self.P, dtype=np.float32)
        self._check(self.lib.pitmg_net_get_params(self.h, out.ctypes.data))
        return out

    def forward(self, x, out=None):
        b = x.shape[0]
        y = out if out is not None else self.torch.empty_like(x)
        self._check(self.lib.pitmg_net_forward(self.h, b, _ptr(x), _ptr(y)))
        return y

    def backward(self, x, dy, grad=None):
        g = grad if grad is not None else self.torch.empty(self.P, dtype=self.torch.float32,
                                                           device=self.device)
        self._check(self.lib.pitmg_net_backward(self.h, x.shape[0], _ptr(x), _ptr(dy), _ptr(g)))
        return g

    def adam(self, grad, lr: float):
        self._check(self.lib.pitmg_net_adam(self.h, _ptr(grad), float(lr)))

    def train_step(self, idx, X, Y, lr: float) -> float:
        loss = _c_double(0.0)
        self._check(self.lib.pitmg_net_train_step(self.h, idx.shape[0], _ptr(idx), X.shape[0],
                                                  _ptr(X), _ptr(Y), float(lr), _byref(loss)))
        return loss.value

    def make_samples(self, p: int, q: int, r, e):
        """Normalised node-major samples (X, Y) from type-major pairs r, e."""
        n = r.shape[0]
        X = self.torch.empty((n, self.T, self.C), dtype=self.torch.float32, device=self.device)
        Y = self.torch.empty_like(X)
        self._check(self.lib.pitmg_net_make_samples(self.h, n, p, q, _ptr(r), _ptr(e), _ptr(X),
                                                    _ptr(Y)))
        return X, Y

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.lib.pitmg_net_destroy(self.h)
            self.h = _c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_c_void_p = C.c_void_p
_c_double = C.c_double
_byref = C.byref
