"""Training and evaluation of the learned coarse-grid correction.

The network (include/pitmg.h, pitmg_net_*) learns the map from a coarsest-
level right-hand side r_c to the GMRES + SGS coarse solution e_c.  The pairs
come from the method itself: solves with the plain coarse solve record every
coarsest-level (r_c, e_c) of their V-cycles (pitmg_coarse_pairs_arm).  The
samples are normalised and laid out node-major by pitmg_net_make_samples;
training runs pitmg_net_train_step (bfloat16 MFMA products, FP32 Adam) over
shuffled mini-batches.  Everything numerical runs in the HIP library; this
module only sequences the calls and reports.

Problems are given as (levels, b) pairs: the per-level Jacobian blocks (as
accepted by Solver) and a type-major right-hand side.
"""
from __future__ import annotations

import time
from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np

from . import pitmg as pm


def collect_pairs(problems: Iterable[Tuple[Sequence, np.ndarray]], options, max_pairs: int,
                  tol: float = 1e-10, device: str = "cuda", progress=None):
    """Solve each problem with GMRES + SGS on the coarsest grid and record
    its coarsest-level (r_c, e_c) pairs, up to max_pairs in total.

    Returns (R, E, info): FP64 device tensors [count][len_c] and per-solve
    statistics."""
    import torch
    R = E = None
    count = 0
    info = []
    s, cur = None, None
    for levels, b in problems:
        if levels is not cur:            # consecutive right-hand sides of one point share a handle
            if s is not None:
                s.close()
            s, cur = pm.Solver(levels, options, device=device), levels
        lc = s.lens[-1]
        if R is None:
            R = torch.empty((max_pairs, lc), dtype=torch.float64, device=device)
            E = torch.empty_like(R)
        left = max_pairs - count
        s.arm_pairs(R[count:], E[count:], left)
        t0 = time.perf_counter()
        _, st, _ = s.solve(torch.from_numpy(b).to(device), tol=tol)
        got = s.pair_count()
        info.append({"iters": st["iters"], "pairs": got, "s": time.perf_counter() - t0})
        count += got
        if progress is not None:
            progress(len(info), count)
        if count >= max_pairs:
            break
    if s is not None:
        s.close()
    return R[:count], E[:count], info


def train(net: "pm.Net", X, Y, epochs: int, batch: int, lr: float, seed: int,
          val_frac: float = 0.1) -> Dict:
    """Adam on shuffled mini-batches of (X, Y); the last val_frac of the
    samples (after one seeded permutation) are held out for validation."""
    import torch
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    nval = max(1, int(round(val_frac * n)))
    tr, va = perm[:n - nval], perm[n - nval:]
    va_t = torch.from_numpy(va.astype(np.int64)).to(X.device)
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        order = rng.permutation(tr).astype(np.int32)
        idx = torch.from_numpy(order).to(X.device)
        losses = []
        for s in range(0, len(order), batch):
            b = idx[s:s + batch]
            losses.append(net.train_step(b, X, Y, lr))
        hist.append({"epoch": ep, "train_loss": float(np.mean(losses)),
                     "val_rel_err": validate(net, X[va_t], Y[va_t])})
    return {"history": hist, "train_s": time.perf_counter() - t0, "train": int(len(tr)),
            "val": int(nval)}


def validate(net: "pm.Net", X, Y) -> float:
    """Mean over samples of ||net(x) - y|| / ||y||."""
    import torch
    errs = []
    for s in range(0, X.shape[0], net.max_batch):
        y = net.forward(X[s:s + net.max_batch].contiguous())
        t = Y[s:s + net.max_batch]
        num = torch.linalg.vector_norm((y - t).reshape(y.shape[0], -1), dim=1)
        den = torch.linalg.vector_norm(t.reshape(t.shape[0], -1), dim=1).clamp_min(1e-30)
        errs.append((num / den).cpu())
    return float(torch.cat(errs).mean())


def ablation(problems: Iterable[Tuple[Sequence, np.ndarray]], options, net: "pm.Net",
             stall_ratio: float, tol: float = 1e-10, device: str = "cuda",
             time_coarse: bool = False) -> List[Dict]:
    """Each problem solved four ways: GMRES + SGS on the coarsest grid; the
    network throughout; the network under the stall rule (stall_ratio); and
    a zero coarse correction (a network with all parameters zero).  With
    time_coarse, also the event-timed cost of the coarsest-level correction
    per V-cycle in each mode."""
    import torch
    zero = pm.Net(net.C, net.T, net.H, max_batch=1, device=device)
    zero.set_params(np.zeros(zero.P, dtype=np.float32))
    out = []
    base = {k: getattr(options, k) for k, _ in options._fields_}
    for levels, b in problems:
        s = pm.Solver(levels, options, device=device)
        db = torch.from_numpy(b).to(device)
        row = {}
        for name, mode, ratio, n_ in (("plain", 0, base["stall_ratio"], net),
                                      ("net", 1, 1e300, net),
                                      ("net_stall_rule", 1, stall_ratio, net),
                                      ("zero_correction", 1, 1e300, zero)):
            s.attach_net(n_)
            s.set_options(**dict(base, coarse_mode=mode, stall_ratio=ratio))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st, rc = s.solve(db, tol=tol)
            torch.cuda.synchronize()
            row[name] = {"iters": st["iters"], "ms": round((time.perf_counter() - t0) * 1e3, 1),
                         "converged": st["converged"], "relres_true": st["relres_true"],
                         "net_calls": st["net_calls"], "fallback_at": st["fallback_at"]}
            if time_coarse:
                # the coarsest-level correction alone, timed with events
                s.profile(True)
                s.profile_reset()
                r = torch.randn(s.lens[0], dtype=torch.float64, device=device)
                e = s.empty(0)
                for _ in range(20):
                    s.vcycle(r, out=e)
                n_calls, ms = s.profile_read()["coarse"]
                s.profile(False)
                row[name]["coarse_ms_per_vcycle"] = round(ms / 20, 4)
        s.attach_net(None)
        s.close()
        out.append(row)
    zero.close()
    return out
