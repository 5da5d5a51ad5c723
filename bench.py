#!/usr/bin/env python3
"""Benchmark: augmented-system solves per second to 1e-10 relative residual.

One step = the whole hot path on one synthetic linearisation point: factor
every time-step block of every level from the Jacobian blocks already in HBM
(S_k = N N^T + Z Z^T, Cholesky, inverse factor), then FGMRES preconditioned
by one parallel-in-time V-cycle per step, from x0 = 0 to ||b - A~x|| <=
1e-10 ||b||.  value = steps per second on one MI355X.

The roofline object covers the dominant kernel, the block Jacobi sweep: its
algorithmic bytes (every Jacobian / factor block read once per sweep plus the
vectors, shared blocks once per launch) over its launch durations, measured
during the timed steps with start/stop events that the sweep's own kernel
dispatches record on the solver's stream.  "traffic" is the HBM traffic per
sweep launch from the committed FETCH_SIZE / WRITE_SIZE counter summary
(calibrated against a copy kernel), and null once the sweep's sources differ
from those the counters were taken with; the counter runs use --counters.

Beside the FP64 solve, the line reports the V-cycle's algorithmic HBM rate
with the FP64 smoother and with the FP32 smoother (every level above the
coarsest), one FP32-smoother solve of the same system, the learned coarse
correction (pairs, training, held-out ablation) and an uneven batch of
independent systems solved one by one and as a batch.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
COUNTERS = os.path.join(ROOT, "profiles", "k_jacobi_burgers128_hbm_counters.md")

WORKLOADS = {
    # the measured workload: viscous Burgers, 128 nodes, 1024 steps
    "burgers128": dict(cfg="burgers128", restart=300, maxit=300,
                       desc="viscous Burgers nx=128 (p=q=128), nu=0.01, n=1024 steps, "
                            "8 levels (coarsest 8 steps), gamma=100, V(2,2) weighted block "
                            "Jacobi (omega 1/2), mu transfer scale 2, coarse GMRES+SGS tol "
                            "1e-3, FGMRES tol 1e-10"),
    # the large-block workload (FP64 and FP32 smoothers); its assembled system
    # (10.5 M unknowns, about 3e9 nonzeros) is beyond the oracle, so it has no
    # CPU baseline
    "burgers512": dict(cfg="burgers512", restart=200, maxit=800,
                       desc="viscous Burgers nx=512 (p=q=512), nu=0.005, n=4096 steps, "
                            "10 levels (coarsest 8 steps), gamma=100, V(2,2) weighted block "
                            "Jacobi (omega 1/2), mu transfer scale 2, coarse GMRES+SGS tol "
                            "1e-3, FGMRES(200) tol 1e-10"),
    # the learned-coarse-correction workload: the bench line is the plain
    # solve; the learned leg trains on 20,000 pairs of this size.  Its
    # assembled system (2.6 M unknowns, about 3e8 nonzeros) is beyond the
    # oracle's direct factorisation, so it has no CPU baseline
    "burgers256": dict(cfg="burgers256", restart=200, maxit=400,
                       desc="viscous Burgers nx=256 (p=q=256), nu=0.01, n=2048 steps, "
                            "9 levels (coarsest 8 steps), gamma=100, V(2,2) weighted block "
                            "Jacobi (omega 1/2), mu transfer scale 2, coarse GMRES+SGS tol "
                            "1e-3, FGMRES(200) tol 1e-10"),
    "vdp256": dict(cfg="vdp256", restart=300, maxit=300,
                   desc="van der Pol p=2 q=1, n=256 steps, 6 levels, gamma=100, V(2,2) "
                        "weighted block Jacobi (omega 1/2), mu transfer scale 2, "
                        "FGMRES tol 1e-10"),
}


def sweep_bytes(p, q, n, shared_V, shared_Z, mat_bytes=8):
    """Algorithmic HBM bytes of one block Jacobi sweep on a level of n steps,
    the unit of the method's cost model: per time-step block N_k, the lower
    triangle of G_k^{-1} and, unless shared by every step, V_k and Z~_k, each
    of mat_bytes per entry; the right-hand side and the previous iterate read
    and the new iterate written, 3 (4p+q) FP64 values.  Shared blocks count
    once per sweep; block n+1 holds 2p values."""
    mats = p * p + (0 if shared_V else p * p) + (0 if shared_Z else p * q) + p * (p + 1) // 2
    total = n * (mats * mat_bytes + 3 * (4 * p + q) * 8) + 3 * (2 * p) * 8
    total += ((p * p if shared_V else 0) + (p * q if shared_Z else 0)) * mat_bytes
    return float(total)


def vector_bytes(p, q, n):
    """The vector part of sweep_bytes (no blocks)."""
    return float(n * 3 * (4 * p + q) * 8 + 3 * (2 * p) * 8)


def level_pairs(p, q, L, shapes, pair_sweeps, shared=True, fp32_levels=0):
    """Per level above the coarsest: how two sweeps share a launch, or None.
    "tiled": the one-step kernel (p = q in {64, 128}), which keeps each
    step's blocks in registers for both sweeps; "shared": the FP64
    shared-block kernel (shape 1-4, or the built-in rule 0, with shared V
    and Z~), which reads its blocks again for the second sweep."""
    ok = pair_sweeps and p == q and p in (64, 128)
    out = []
    for lev in range(L - 1):
        c = shapes[lev]
        if not ok:
            out.append(None)
        elif c == -1 or not shared:
            out.append("tiled")
        elif lev >= fp32_levels:
            out.append("shared")
        else:
            out.append(None)
    return out


def vcycle_launches(L, nu_pre, nu_post, pairs):
    """(level, sweeps in the launch) of every sweep launch of one V-cycle, in
    the library's pattern: on a paired level sweeps go two per launch, an odd
    one last on its own."""
    out = []
    for lev in range(L - 1):
        for nu in (nu_pre, nu_post):
            s_ = 0
            while s_ < nu:
                two = pairs[lev] is not None and s_ + 1 < nu
                out.append((lev, 2 if two else 1))
                s_ += 2 if two else 1
    return out


def chained(L, nu_pre, nu_post, pairs, pair_sweeps):
    """Whether the library runs the pre-smoothing of every level above the
    coarsest in one launch and the post-smoothing in another (pair_sweeps 2,
    the one-step kernel on every such level, V(2,2), at most 8 such levels)."""
    return (pair_sweeps == 2 and nu_pre == 2 and nu_post == 2 and 2 <= L - 1 <= 8
            and all(pr == "tiled" for pr in pairs))


def vcycle_sweeps(p, q, n, L, nu_pre, nu_post, shared_V, shared_Z, pairs, mat_bytes=8,
                  chain=False):
    """Sweep bytes of one V-cycle and its number of sweep launches: (bytes
    with the blocks counted once per sweep, bytes with the blocks counted
    once per launch, launches).  A chained cycle has the same sweeps in two
    launches."""
    per_sweep = per_launch = 0.0
    launches = vcycle_launches(L, nu_pre, nu_post, pairs)
    for lev, k in launches:
        nl = n >> lev
        one = sweep_bytes(p, q, nl, shared_V, shared_Z, mat_bytes)
        per_sweep += k * one
        per_launch += one + (k - 1) * vector_bytes(p, q, nl)
    return per_sweep, per_launch, 2 if chain else len(launches)


def vcycle_bytes(p, q, n, L, nu_pre, nu_post, shared_V, shared_Z, mat_bytes=8, fp64_residual=False,
                 pairs=None):
    """Algorithmic bytes of one V-cycle: the sweeps of every level above the
    coarsest (blocks once per sweep), the coarse right-hand sides written,
    the coarsest right-hand side and correction, and, with an FP32 smoother,
    the explicit FP64 finest residual (blocks and two vectors read, one
    written)."""
    pairs = pairs or [None] * (L - 1)
    tot, _, _ = vcycle_sweeps(p, q, n, L, nu_pre, nu_post, shared_V, shared_Z, pairs, mat_bytes)
    for lev in range(L - 1):
        tot += 8.0 * (4 * p + q) * (n >> (lev + 1))
    nc = n >> (L - 1)
    tot += 8.0 * 2 * (4 * p + q) * nc
    if fp64_residual:
        mats = p * p + (0 if shared_V else p * p) + (0 if shared_Z else p * q)
        tot += 8.0 * (n * mats + 3 * (4 * p + q) * n)
    return tot


def cpu_baseline(name):
    """Time one whole solve of the FP64 oracle on the same system: its setup
    (assembly and SuperLU factorisations of every level) and its FGMRES to a
    true relative residual of 1e-10."""
    from workloads import config_problem
    from oracle import Hierarchy
    from oracle.multigrid import MGOptions
    cores = len(os.sched_getaffinity(0))
    wl = WORKLOADS[name]
    prob, b = config_problem(wl["cfg"])
    t1 = time.perf_counter()
    H = Hierarchy(prob.levels, MGOptions())
    t2 = time.perf_counter()
    _, info = H.solve(b, tol=1e-10, restart=wl["restart"], maxit=wl["maxit"])
    t3 = time.perf_counter()
    return {"value": 1.0 / (t3 - t1), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"one whole oracle solve of the same system: setup (assembly + SuperLU "
                      f"of every level, {t2 - t1:.1f} s) and FGMRES to 1e-10 ({info['iters']} "
                      f"steps, {t3 - t2:.1f} s); SciPy/SuperLU single-threaded, numpy BLAS on "
                      f"{cores} threads",
            "oracle_iters": info["iters"], "converged": bool(info["converged"])}


def learned_leg(pm, torch, wl, train_seeds=range(50000, 50008), held_out=(60000, 60001),
                rhs_per_point=8, max_pairs=8000):
    """Learned coarse correction on the benchmark workload: record the
    coarsest-level pairs of plain solves on other linearisation points
    (rhs_per_point seeded right-hand sides each, as an SQP step solves
    several systems per point), train the network, then solve held-out
    points four ways (plain, network, network under a stall rule, zero
    correction)."""
    import numpy as np
    from paper_2405_04808_amd import coarse_training as ct
    from workloads import config_problem, coarse_net_params

    def probs(seeds, per=1):
        for sd in seeds:
            prob, b = config_problem(wl["cfg"], seed=sd)
            rng = np.random.default_rng(sd + 1)
            for j in range(per):
                yield prob.levels, (b if j == 0 else rng.normal(size=b.shape))

    opts = pm.default_options(restart=wl["restart"], maxit=wl["maxit"])
    t0 = time.perf_counter()
    def progress(solves, pairs):
        if solves % 25 == 0:
            print(f"# learned: {solves} solves, {pairs} pairs, "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    R, E, info = ct.collect_pairs(probs(train_seeds, rhs_per_point), opts, max_pairs=max_pairs,
                                  progress=progress)
    t_pairs = time.perf_counter() - t0
    print(f"# learned: {R.shape[0]} pairs from {len(info)} solves in {t_pairs:.1f} s",
          file=sys.stderr, flush=True)
    prob0, _ = config_problem(wl["cfg"])
    p, q = prob0.p, prob0.q
    C, T, H = 4 * p + q, prob0.levels[-1].N.shape[0], 64
    net = pm.Net(C, T, H, max_batch=256)
    net.set_params(coarse_net_params(C, H, 0).astype("float32"))
    X, Y = net.make_samples(p, q, R, E)
    del R, E
    tr = ct.train(net, X, Y, epochs=30, batch=256, lr=1e-3, seed=1)
    print(f"# learned: trained in {tr['train_s']:.1f} s, validation error "
          f"{tr['history'][-1]['val_rel_err']:.3f}", file=sys.stderr, flush=True)
    abl = ct.ablation(probs(held_out), opts, net, stall_ratio=0.999, time_coarse=True)
    net.close()
    return {"network": f"conv1d width 3: {C}->{H}->{H}->{C} channels over {T} coarse steps, "
                       "tanh, bf16 MFMA products, FP32 accumulation and Adam",
            "pairs": int(X.shape[0]), "pair_solves": len(info), "pairs_s": round(t_pairs, 1),
            "train_samples": tr["train"], "val_samples": tr["val"], "epochs": 30,
            "batch": 256, "lr": 1e-3, "train_s": round(tr["train_s"], 2),
            "val_rel_err": round(tr["history"][-1]["val_rel_err"], 4),
            "stall_rule": "ratio 0.999 on 2 consecutive steps",
            "held_out": {str(sd): row for sd, row in zip(held_out, abl)}}


def batch_leg(pm, torch, count=64):
    """Uneven batch: 64 independent systems, half van der Pol (n in {256,
    1024, 4096}), half viscous Burgers (nx in {64, 128, 256}, n in {512 ..
    4096}), FP32 smoother and FP64 outer solve, solved one after another, as
    one batch (phases interleaved over one stream per system), and as a batch
    with captured V-cycles and tuned sweeps.  Fresh handles for each mode;
    setup and tuning are timed apart from the solves."""
    from workloads import batch_mix, make_problem, make_rhs
    cfgs = batch_mix(count=count)
    probs = []
    for c in cfgs:
        prob, rng = make_problem(**c)
        probs.append((prob, make_rhs(prob, rng)))
    bs = [torch.from_numpy(b).to("cuda") for _, b in probs]
    torch.cuda.synchronize()
    out = {"systems": count,
           "mix": f"{count // 2} van der Pol (n in [256, 1024, 4096]), {count - count // 2} "
                  "viscous Burgers (nx in [64, 128, 256], n in [512, 1024, 2048, 4096]); seeds "
                  "4000+i; coarsest 8 steps; FP32 smoother on every level above the coarsest, "
                  "FGMRES(60) in FP64 to 1e-10",
           "sizes": [[c["kind"], c.get("nx", 2), c["n"]] for c in cfgs]}
    seq_its = None
    for mode in ("sequential", "batch", "batch_graph_tuned"):
        ts = time.perf_counter()
        ss = []
        for prob, _ in probs:
            o = pm.default_options(restart=60, maxit=600, smoother_fp32=99,
                                   vcycle_graph=1 if "graph" in mode else 0)
            ss.append(pm.Solver(prob.levels, o, stream=torch.cuda.Stream()))
        torch.cuda.synchronize()
        setup = time.perf_counter() - ts
        tune = 0.0
        if mode.endswith("tuned"):
            ta = time.perf_counter()
            for s_ in ss:
                s_.autotune()
            tune = time.perf_counter() - ta
        torch.cuda.synchronize()
        ta = time.perf_counter()
        if mode == "sequential":
            st = [s_.solve(b, tol=1e-10)[1] for s_, b in zip(ss, bs)]
        else:
            _, st, _, _ = pm.solve_batch(ss, bs, tol=1e-10)
        torch.cuda.synchronize()
        el = time.perf_counter() - ta
        its = [x["iters"] for x in st]
        row = {"s": round(el, 3), "systems_per_s": round(count / el, 3),
               "setup_s": round(setup, 2), "tune_s": round(tune, 2), "fgmres_iters_total": sum(its),
               "all_converged_1e-10": all(x["converged"] == 1 and x["relres_true"] <= 1.01e-10
                                          for x in st)}
        if seq_its is None:
            seq_its = its
        else:
            row["iters_same_as_sequential"] = its == seq_its
        out[mode] = row
        print(f"# batch {mode}: {el:.2f} s", file=sys.stderr, flush=True)
        for s_ in ss:
            s_.close()
        del ss
        torch.cuda.empty_cache()
    out["speedup_batch"] = round(out["sequential"]["s"] / out["batch"]["s"], 2)
    out["speedup_batch_graph_tuned"] = round(out["sequential"]["s"] / out["batch_graph_tuned"]["s"], 2)
    return out


def variants_leg(pm, torch, prob, db, wl, reps=2):
    """The cycle and smoother variants of Sec. 5.3.4 and Sec. 6 on the
    benchmark system: FGMRES steps and time per solve (blocks already
    factored; the Gauss-Seidel handles also form N_k^T S_k^{-1} V_k at
    setup, outside the timing)."""
    out = {}
    names = {0: "jacobi", 1: "fgs", 2: "bgs", 3: "sgs"}
    for cycle, smoother in ((0, 0), (1, 0), (2, 0), (0, 1), (0, 2), (0, 3), (1, 3)):
        key = f"{'VWF'[cycle]}-{names[smoother]}"
        s_ = pm.Solver(prob.levels, pm.default_options(restart=wl["restart"], maxit=wl["maxit"],
                                                        cycle=cycle, smoother=smoother),
                       device="cuda:0")
        x_ = s_.empty(0)
        _, st, _ = s_.solve(db, tol=1e-10, out=x_)            # warm-up
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(reps):
            _, st, rc = s_.solve(db, tol=1e-10, out=x_)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - ta) * 1e3 / reps
        out[key] = {"fgmres_iters": st["iters"], "ms_per_solve": round(ms, 2),
                    "ms_per_fgmres_step": round(ms / max(st["iters"], 1), 3),
                    "relres_true": st["relres_true"], "converged": st["converged"] == 1}
        print(f"# variant {key}: {st['iters']} steps, {ms:.1f} ms", file=sys.stderr, flush=True)
        s_.close()
    out["note"] = ("V/W/F cycle with block Jacobi (jacobi), forward / backward / symmetric "
                   "block Gauss-Seidel (fgs / bgs / sgs) smoothing, omega 1/2, V(2,2); "
                   "solve only (no refactor); the Gauss-Seidel sweeps are chains in time")
    return out


# Table 6 of the paper (viscosity: dogleg iterations, SGS steps per coarse
# solve, FGMRES steps per solve), for context only: its iterates come from
# the paper's own runs.
TABLE6 = {"0.1": (2, 1.00, 2.00), "0.01": (7, 1.00, 5.62), "0.001": (9, 1.00, 11.00),
          "0.0001": (6, 1.00, 7.33), "0.0": (5, 1.00, 12.80)}


def dogleg_leg(pm, torch, nx=512, n=512, levels=7, gamma=1e5):
    """The nonlinear solve of Sec. 6.2 / Table 6 on the GPU: Burgers'
    equation with the step initial state, 512 steps on [0, 1], seven levels,
    gamma = 1e5, V(4,4), viscosity continuation 1e-1 .. 1e-4, 0; Powell's
    dogleg with minimum-norm Gauss-Newton steps (unlifted FGMRES to 1e-6).
    The whole continuation is timed once (from the step initial state)."""
    import numpy as np
    from workloads import burgers_step_state
    nus = [1e-1, 1e-2, 1e-3, 1e-4, 0.0]
    w0 = burgers_step_state(nx)
    b = pm.Burgers(nx, n, levels, 1.0, gamma, w0)
    x = torch.from_numpy(np.concatenate([np.tile(w0, n), np.zeros(n * nx)])).to("cuda:0")
    opts = pm.default_options(nu_pre=4, nu_post=4, restart=100, maxit=400)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats, rc = b.dogleg(x, nus, opts, ftol=1e-8, lin_tol=1e-6)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    stages = []
    for nu, st in zip(nus, stats):
        stages.append({"nu": nu, "dogleg_iters": st["iters"], "accepted": st["accepted"],
                       "converged": st["converged"] == 1,
                       "sgs_per_coarse_solve": round(st["coarse_its"] / max(st["coarse_calls"], 1), 2),
                       "fgmres_per_solve": round(st["fgmres_iters"] / max(st["solves"], 1), 2),
                       "solves": st["solves"], "ms": round(st["ms"], 1),
                       "fnorm_start": st["fnorm0"], "fnorm_end": st["fnorm"],
                       "table6": TABLE6.get(repr(nu))})
        print(f"# dogleg nu={nu}: {st['iters']} iterations, "
              f"{st['fgmres_iters'] / max(st['solves'], 1):.2f} FGMRES steps per solve",
              file=sys.stderr, flush=True)
    u1 = x[(n - 1) * nx:n * nx].cpu().numpy()
    xg = np.arange(1, nx + 1) / (nx + 1)
    mid = (xg > 0.1) & (xg < 0.8)
    return {"problem": f"Burgers nx={nx} (p=q={nx}), n={n} steps on [0,1], {levels} levels, "
                       f"gamma={gamma:g}, step initial state, flux-form upwind convection, "
                       "V(4,4) weighted block Jacobi, unlifted FGMRES(100) to 1e-6, "
                       "dogleg stop |F| <= 1e-8 |F(start)| per viscosity",
            "status": rc, "total_s": round(total, 3), "stages": stages,
            "inviscid_u_t1_vs_x_maxdev_mid": float(np.abs(u1[mid] - xg[mid]).max()),
            "table6_columns": "dogleg iterations, SGS per coarse solve, FGMRES per solve"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="burgers128", choices=list(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="do not time the sweep launches (value only)")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-smoother leg")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-coarse-correction leg (pairs, training, ablation)")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven-batch leg")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the cycle / smoother variants leg")
    ap.add_argument("--no-dogleg", action="store_true",
                    help="skip the Burgers dogleg / continuation leg (Table 6)")
    ap.add_argument("--no-setup6", action="store_true",
                    help="skip the refactor + 6 solves measurement")
    ap.add_argument("--sweep-shapes", default=None,
                    help="comma-separated sweep launch shape per level instead of tuning "
                         "(as reported in config.sweep_shapes)")
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--counters", action="store_true",
                    help="counter-collection run: one solve cut at 40 FGMRES steps (the same "
                         "launches per V-cycle), then a 256 MiB copy kernel for calibration")
    args = ap.parse_args()
    if args.counters:
        args.steps, args.warmup = 1, 0
        args.no_cpu_baseline = args.no_profile = args.no_fp32 = args.no_learned = True
        args.no_variants = True
        args.no_batch = True
        args.no_dogleg = True
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only; --gpus {args.gpus} is not "
              "supported (the time-parallel path shards by time blocks, see the design "
              "notes, but no multi-GPU run exists)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2405_04808_amd as pm
    from workloads import config_problem

    wl = WORKLOADS[args.workload]
    prob, b = config_problem(wl["cfg"])
    its_cap = 40 if args.counters else wl["maxit"]
    opts = pm.default_options(restart=min(wl["restart"], its_cap), maxit=its_cap)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    solver = pm.Solver(prob.levels, opts, device="cuda:0")
    # setup-time tuning of each level's sweep launch shape (not timed)
    if args.sweep_shapes:
        sweep_shapes = [int(c) for c in args.sweep_shapes.split(",")]
        solver.set_sweep_shapes(sweep_shapes)
    else:
        sweep_shapes = solver.autotune()
    db = torch.from_numpy(b).to(dev)
    x = solver.empty(0)
    torch.cuda.synchronize()
    print(f"# workload {args.workload}: size {prob.size}, levels {prob.n_levels}, "
          f"device bytes {solver.device_bytes() / 1e9:.2f} GB", file=sys.stderr, flush=True)

    def step():
        solver.refactor_device()
        _, st, rc = solver.solve(db, tol=1e-10, out=x)
        return st, rc

    for w in range(args.warmup):
        st, rc = step()
        print(f"# warmup {w}: iters {st['iters']} relres {st['relres_true']:.3e} "
              f"{st['ms_solve']:.1f} ms", file=sys.stderr, flush=True)

    profile = not args.no_profile
    if profile:
        solver.profile(2)              # the sweep's own dispatch events only,
        solver.profile_sample(16)      # on every 16th V-cycle (same launch mix)
        solver.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for s in range(args.steps):
        st, rc = step()
        stats.append(st)
        print(f"# step {s}: iters {st['iters']} relres {st['relres_true']:.3e}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    prof = solver.profile_read() if profile else None
    if profile:
        solver.profile(False)
        # per-class breakdown from one more step with every launch timed
        # (outside the timed region: the brackets slow the step down)
        solver.profile(True)
        solver.profile_sample(1)
        solver.profile_reset()
        step()
        classes = solver.profile_read()
        solver.profile(False)

    # one linearisation point as the method uses it: refactor, then about six
    # solves (the projected-CG usage of Sec. 6); outside the timed steps
    setup6 = None
    if not args.counters and not args.no_setup6:
        torch.cuda.synchronize()
        ta = time.perf_counter()
        solver.refactor_device()
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for _ in range(6):
            solver.solve(db, tol=1e-10, out=x)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        setup6 = {"refactor_ms": round((tb - ta) * 1e3, 3),
                  "six_solves_s": round(tc - tb, 3), "total_s": round(tc - ta, 3)}
        print(f"# refactor + 6 solves: {tc - ta:.2f} s", file=sys.stderr, flush=True)

    iters = [s["iters"] for s in stats]
    ok = all(s["converged"] == 1 and s["relres_true"] <= 1.01e-10 for s in stats)
    p, q, n, L = prob.p, prob.q, prob.n, prob.n_levels
    shared_V, shared_Z = solver.shared_V, solver.shared_Z
    pairs = level_pairs(p, q, L, sweep_shapes, opts.pair_sweeps, shared=shared_V and shared_Z)

    if args.counters:
        # plain copy kernel of known size for calibrating FETCH_SIZE / WRITE_SIZE
        src = torch.ones(32 << 20, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"counters_run": True, "fgmres_iters": iters,
                          "copy_bytes": src.numel() * 8}))
        solver.close()
        return

    roofline = None
    kern = None
    if prof:
        # algorithmic bytes of the Jacobi launches of the timed steps: whole
        # V-cycles' sweeps, so bytes per launch is the V-cycle's sweep bytes
        # over its sweep launches
        chain = chained(L, opts.nu_pre, opts.nu_post, pairs, opts.pair_sweeps)
        per_sweep, per_launch_once, nlaunch = vcycle_sweeps(p, q, n, L, opts.nu_pre,
                                                            opts.nu_post, shared_V, shared_Z,
                                                            pairs, chain=chain)
        launches, ms = prof["jacobi"]
        alg_bytes = per_sweep / nlaunch * launches
        achieved = alg_bytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        once = per_launch_once / nlaunch * launches / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        from paper_2405_04808_amd.rocprof_summary import read_traffic
        # the counter profile covers the Burgers nx=128 workload only
        rec = read_traffic(COUNTERS) if args.workload == "burgers128" else None
        names = {0: "built-in", -1: "k_jacobi_tiled<%d, %d, double>" % (p // 32, p // 16)}
        kname = ("block Jacobi sweep, levels 0..%d chained: k_jacobi_chain<%d, %d, double>, "
                 "one launch for the pre-smoothing and one for the post-smoothing of every "
                 "level, two sweeps per level" % (L - 2, p // 32, p // 16)) if chain else \
            "block Jacobi sweep, levels 0..%d: " % (L - 2) + ", ".join(
            ("k_jacobi_tiled2<%d, %d, double> (two sweeps per launch)" % (p // 32, p // 16)
             if pairs[lev] == "tiled" else
             "k_jacobi_shared_nl2<%d, %d> x%d steps (two sweeps per launch)" % (p // 32, p // 16, c)
             if pairs[lev] == "shared" else
             names.get(c) or "k_jacobi_shared_nl<%d, %d> x%d steps" % (p // 32, p // 16, c))
            for lev, c in enumerate(sweep_shapes[:L - 1]))
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": rec["traffic_bytes_per_launch"] if rec else None,
                    "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated)",
                    "kernel": kname,
                    "bytes_unit": "per sweep: N_k, lower G_k^{-1} per step (V, Z~ shared, once), "
                                  "right-hand side, previous and new iterate; a two-sweep "
                                  "launch counts two sweeps",
                    "achieved_blocks_once_per_launch": round(once, 1),
                    "frac_blocks_once_per_launch": round(once / HBM_PEAK_GBS, 4),
                    "launches": launches, "sample": "sweeps of every 16th V-cycle",
                    "avg_launch_us": round(ms * 1e3 / max(launches, 1), 2),
                    "alg_bytes_per_launch": round(alg_bytes / max(launches, 1))}
        kern = {k: {"launches": v[0], "ms_total": round(v[1], 3)} for k, v in classes.items()}
        kern["note"] = "one extra untimed step with every launch bracketed by events"

    def vcycle_rate(s_, mat_bytes, fp64_res, lev_pairs=None, reps=20):
        """ms per V-cycle (back-to-back calls on the solver's stream) and its
        algorithmic GB/s."""
        g = torch.Generator(device="cpu").manual_seed(7)
        r = torch.randn(prob.size, generator=g, dtype=torch.float64).to(dev)
        e = s_.empty(0)
        s_.vcycle(r, out=e)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            s_.vcycle(r, out=e)
        ev1.record()
        torch.cuda.synchronize()
        ms_ = ev0.elapsed_time(ev1) / reps
        by = vcycle_bytes(p, q, n, L, opts.nu_pre, opts.nu_post, shared_V, shared_Z, mat_bytes,
                          fp64_res, lev_pairs)
        return {"ms": round(ms_, 4), "alg_GB": round(by / 1e9, 4),
                "GBps": round(by / (ms_ * 1e-3) / 1e9, 1)}

    vc = {"fp64": vcycle_rate(solver, 8, False, pairs)}
    fp32 = None
    if not args.no_fp32:
        s32 = pm.Solver(prob.levels, pm.default_options(restart=wl["restart"], maxit=wl["maxit"],
                                                        smoother_fp32=99), device="cuda:0")
        # the same setup-time tuning as the FP64 solver (not timed)
        shapes32 = s32.autotune()
        pairs32 = level_pairs(p, q, L, shapes32, opts.pair_sweeps, shared=shared_V and shared_Z,
                              fp32_levels=L - 1)
        vc["fp32"] = vcycle_rate(s32, 4, True, pairs32)
        x32 = s32.empty(0)
        _, st32, _ = s32.solve(db, tol=1e-10, out=x32)           # warm-up
        torch.cuda.synchronize()
        ta = time.perf_counter()
        st32s = []
        for _ in range(2):
            s32.refactor_device()
            _, st32, _ = s32.solve(db, tol=1e-10, out=x32)
            st32s.append(st32)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        diff = float(torch.linalg.vector_norm(x32 - x) / torch.linalg.vector_norm(x))
        fp32 = {"smoother": "FP32 on every level above the coarsest; FP64 finest residual, "
                            "coarse solve, Arnoldi and FGMRES",
                "sweep_shapes": list(shapes32),
                "ms_per_step": round((tb - ta) * 1e3 / 2, 3), "fgmres_iters": [t["iters"] for t in st32s],
                "relres_true": max(t["relres_true"] for t in st32s),
                "rel_diff_vs_fp64_solution": diff}
        s32.close()

    learned = None
    if not args.no_learned and args.workload == "burgers128":
        learned = learned_leg(pm, torch, wl)
    elif not args.no_learned and args.workload == "burgers256":
        # 20,000 pairs: 8 points, up to 100 right-hand sides each
        learned = learned_leg(pm, torch, wl, rhs_per_point=100, max_pairs=20000)

    variants = None
    if not args.no_variants and args.workload == "burgers128":
        variants = variants_leg(pm, torch, prob, db, wl)

    batch = None
    if not args.no_batch and args.workload == "burgers128":
        batch = batch_leg(pm, torch, count=args.batch_count)

    dogleg = None
    if not args.no_dogleg and args.workload == "burgers128":
        dogleg = dogleg_leg(pm, torch)

    cpu = None
    if not args.no_cpu_baseline and args.workload not in ("burgers512", "burgers256"):
        cpu = cpu_baseline(args.workload)

    out = {
        "metric": "augmented-system solves/sec to 1e-10 rel. residual",
        "value": round(1e3 / ms_per_step, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded linearisation point and N(0,1) right-hand side)",
        "config": {"workload": wl["desc"], "p": p, "q": q, "n": n, "levels": L,
                   "step": "refactor all levels + FGMRES solve from x0=0",
                   "sweep_shapes": sweep_shapes,
                   "fgmres_restart": opts.restart, "vector_len": prob.size},
        "fgmres_iters": iters,
        "converged_1e-10": ok,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "vcycle_hbm": vc,
        "fp32_smoother": fp32,
        "cycle_variants": variants,
        "learned_coarse": learned,
        "uneven_batch": batch,
        "burgers_dogleg": dogleg,
        "kernel_ms": kern,
        "refactor_plus_6_solves": setup6,
    }
    print(json.dumps(out))
    solver.close()


if __name__ == "__main__":
    main()
