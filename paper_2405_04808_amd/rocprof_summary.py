"""Summaries of rocprofv3 CSV output for the profiles kept with the sources.

Two kinds of run are summarised:

* a kernel trace (``rocprofv3 --kernel-trace --stats -f csv``): the per-kernel
  table of ``*_kernel_stats.csv`` (calls, total, average, min, max);
* two counter runs (``rocprofv3 --pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``,
  ``-f csv``) of a program that launches the block Jacobi sweep and then a
  plain copy kernel of known size.  The counters are in KiB per dispatch; the
  copy kernel reads and writes a known number of bytes, so
  bytes = counter * 1024 * (known KiB / copy counter) calibrates each counter
  against the device.  The result is the HBM traffic per sweep launch,
  averaged over every sweep dispatch of the run, beside the algorithmic
  bytes.

* a matrix-core run (``rocprofv3 --pmc SQ_INSTS_VALU_MFMA_MOPS_F64
  SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE``):
  per kernel, the matrix-core FLOP per dispatch (MOPS x 512), the rate over
  the dispatch's duration against the device's dense peak for the type, and
  the busy fraction SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / XCDs x
  SIMDs) (GRBM_GUI_ACTIVE is summed over the XCDs).

The counter summary ends with one machine-readable line,
``traffic: {json}``, which bench.py reads together with a hash of the sweep
kernel's sources; the figure is only used while that hash matches.

    python -m paper_2405_04808_amd.rocprof_summary stats DIR --title T --command C
    python -m paper_2405_04808_amd.rocprof_summary counters --fetch DIR --write DIR \\
        --kernel k_jacobi_shared --copy-kernel elementwise --copy-bytes B ...
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
SWEEP_SOURCES = ("csrc/pitmg_jacobi_tiled.hip", "csrc/pitmg_tiled.h", "csrc/pitmg_device.h")


def _code_only(text: str) -> str:
    """The source without comments and whitespace: what the compiler sees
    (string literals in these kernels contain no comment markers)."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return re.sub(r"\s+", "", text)


def sweep_source_hash() -> str:
    """sha256 over the code of the register-tiled sweep kernels (comments and
    whitespace left out, so documentation edits keep the counters valid)."""
    h = hashlib.sha256()
    for rel in SWEEP_SOURCES:
        with open(os.path.join(HERE, rel), encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def _find(directory: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    return hits[-1]


def _short(name: str, width: int = 60) -> str:
    name = re.sub(r"\s+", " ", name).replace("(anonymous namespace)::", "")
    name = re.sub(r"^void ", "", name)
    name = re.sub(r"\(.*$", "", name).replace("pitmg::", "")
    return name if len(name) <= width else name[: width - 3] + "..."


def stats_table(directory: str, top: int = 25) -> str:
    path = _find(directory, "kernel_stats.csv")
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | total ms | avg us | % | min us | max us |",
           "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append("| `{}` | {} | {:.1f} | {:.2f} | {:.1f} | {:.2f} | {:.2f} |".format(
            _short(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e6,
            float(r["AverageNs"]) / 1e3, float(r["Percentage"]), float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3))
    return "\n".join(out)


def _first_dispatch(rows, pattern):
    """Smallest Dispatch_Id of the kernels matching pattern (0 if none or no
    pattern).  With k_dots, whose first dispatch opens the first solve, the
    dispatches before it (setup, factorisation, sweep tuning) are left out."""
    if not pattern:
        return 0
    rx = re.compile(pattern)
    ids = [int(r["Dispatch_Id"]) for r in rows if rx.search(r["Kernel_Name"])]
    return min(ids) if ids else 0


def counter_means(directory: str, counter: str, after_first: str = None):
    """{kernel name: {grid size: [values]}} for one counter, over the
    dispatches after the first one of the kernels matching after_first."""
    path = _find(directory, "counter_collection.csv")
    rows = list(csv.DictReader(open(path)))
    first = _first_dispatch(rows, after_first)
    out = defaultdict(lambda: defaultdict(list))
    for r in rows:
        if r["Counter_Name"] != counter or int(r["Dispatch_Id"]) <= first:
            continue
        out[r["Kernel_Name"]][int(r["Grid_Size"])].append(float(r["Counter_Value"]))
    return out


def _select(table, pattern: str, exclude_grids=()):
    rx = re.compile(pattern)
    names = [k for k in table if rx.search(k)]
    if not names:
        raise KeyError(f"no kernel matches {pattern!r}")
    merged = defaultdict(list)
    for k in names:
        for g, vals in table[k].items():
            if g not in exclude_grids:
                merged[g].extend(vals)
    return names, merged


def per_grid_durations(directory: str, pattern: str, after_first: str = None):
    """{grid size: [durations in us]} of the dispatches of kernels matching
    pattern, from *_kernel_trace.csv, after the first dispatch matching
    after_first (if given)."""
    path = _find(directory, "kernel_trace.csv")
    rows = list(csv.DictReader(open(path)))
    first = _first_dispatch(rows, after_first)
    rx = re.compile(pattern)
    out = defaultdict(list)
    for r in rows:
        if int(r["Dispatch_Id"]) > first and rx.search(r["Kernel_Name"]):
            g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            out[g].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    return out


def summarise_counters(fetch_dir, write_dir, kernel, copy_kernel, copy_bytes, exclude_grids=(),
                       after_first=None):
    f_tab = counter_means(fetch_dir, "FETCH_SIZE", after_first)
    w_tab = counter_means(write_dir, "WRITE_SIZE", after_first)
    names, f_sweep = _select(f_tab, kernel, exclude_grids)
    _, w_sweep = _select(w_tab, kernel, exclude_grids)
    _, f_copy = _select(f_tab, copy_kernel)
    _, w_copy = _select(w_tab, copy_kernel)
    known_kib = copy_bytes / 1024.0
    f_copy_all = [v for vals in f_copy.values() for v in vals]
    w_copy_all = [v for vals in w_copy.values() for v in vals]
    cf = known_kib / (sum(f_copy_all) / len(f_copy_all))
    cw = known_kib / (sum(w_copy_all) / len(w_copy_all))
    rows = []
    tot_f = tot_w = cnt = 0.0
    for g in sorted(f_sweep, reverse=True):
        fv, wv = f_sweep[g], w_sweep.get(g, [])
        mf = sum(fv) / len(fv)
        mw = sum(wv) / len(wv) if wv else float("nan")
        rows.append((g, len(fv), mf, mw, mf * 1024 * cf, mw * 1024 * cw))
        tot_f += sum(fv)
        tot_w += sum(wv)
        cnt += len(fv)
    per_launch = (tot_f / cnt) * 1024 * cf + (tot_w / cnt) * 1024 * cw
    return {"kernels": names, "rows": rows, "fetch_factor": cf, "write_factor": cw,
            "copy_fetch_kib": sum(f_copy_all) / len(f_copy_all),
            "copy_write_kib": sum(w_copy_all) / len(w_copy_all), "copy_known_kib": known_kib,
            "dispatches": int(cnt), "traffic_bytes_per_launch": per_launch}


MFMA_PEAK_TFLOPS = {"F64": 78.6, "F32": 157.3}


def mfma_table(directory: str, kernel: str) -> str:
    """Per kernel matching `kernel`: dispatches, average duration, matrix-core
    FLOP per dispatch, TFLOP/s and its fraction of the dense peak, busy %."""
    path = _find(directory, "counter_collection.csv")
    agent = list(csv.DictReader(open(_find(directory, "agent_info.csv"))))
    gpu = [a for a in agent if int(a["Simd_Count"]) > 0][0]
    simds, xcc = int(gpu["Simd_Count"]), int(gpu["Num_Xcc"])
    rx = re.compile(kernel)
    disp = defaultdict(dict)
    for r in csv.DictReader(open(path)):
        if not rx.search(r["Kernel_Name"]):
            continue
        d = disp[(r["Kernel_Name"], int(r["Grid_Size"]) // int(r["Workgroup_Size"]),
                  r["Dispatch_Id"])]
        d[r["Counter_Name"]] = float(r["Counter_Value"])
        d["ns"] = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
    per = defaultdict(list)
    for (name, wgs, _), d in disp.items():
        per[(name, wgs)].append(d)
    out = ["| kernel | work-groups | dispatches | avg ms | MFMA GFLOP / dispatch | TFLOP/s | "
           "peak | frac | MFMA busy |", "|---|---|---|---|---|---|---|---|---|"]
    for (name, wgs), ds in sorted(per.items(), key=lambda kv: -sum(d["ns"] for d in kv[1])):
        ns = sum(d["ns"] for d in ds) / len(ds)
        f64 = sum(d.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0) for d in ds) / len(ds) * 512
        f32 = sum(d.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0) for d in ds) / len(ds) * 512
        typ, flop = ("F64", f64) if f64 >= f32 else ("F32", f32)
        busy = sum(d.get("SQ_VALU_MFMA_BUSY_CYCLES", 0) for d in ds)
        active = sum(d.get("GRBM_GUI_ACTIVE", 0) for d in ds) / xcc * simds
        rate = flop / (ns * 1e-9) / 1e12
        out.append("| `{}` | {} | {} | {:.3f} | {:.1f} | {:.2f} | {} {} | {:.3f} | {:.1f} % |".format(
            _short(name), wgs, len(ds), ns / 1e6, flop / 1e9, rate, MFMA_PEAK_TFLOPS[typ], typ,
            rate / MFMA_PEAK_TFLOPS[typ], 100.0 * busy / active if active else 0.0))
    return "\n".join(out)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    a.add_argument("--title", required=True)
    a.add_argument("--command", required=True)
    a.add_argument("--note", default="")
    a.add_argument("--per-grid", default=None,
                   help="kernel regex: add its dispatch durations grouped by grid size")
    a.add_argument("--exclude-grid", type=int, action="append", default=[])
    a.add_argument("--after-first", default=None,
                   help="kernel regex: count only dispatches after its first dispatch")
    a.add_argument("--out", required=True)
    b = sub.add_parser("counters")
    b.add_argument("--fetch", required=True)
    b.add_argument("--write", required=True)
    b.add_argument("--kernel", required=True)
    b.add_argument("--copy-kernel", required=True)
    b.add_argument("--copy-bytes", type=float, required=True)
    b.add_argument("--title", required=True)
    b.add_argument("--command", action="append", required=True)
    b.add_argument("--note", default="")
    b.add_argument("--exclude-grid", type=int, action="append", default=[],
                   help="grid size (work-items) whose dispatches are left out")
    b.add_argument("--after-first", default=None,
                   help="kernel regex: count only dispatches after its first dispatch")
    b.add_argument("--out", required=True)
    m = sub.add_parser("mfma")
    m.add_argument("--dir", action="append", required=True, help="LABEL=DIR")
    m.add_argument("--kernel", required=True)
    m.add_argument("--title", required=True)
    m.add_argument("--command", action="append", required=True)
    m.add_argument("--note", default="")
    m.add_argument("--out", required=True)
    args = ap.parse_args(argv)

    if args.cmd == "mfma":
        txt = [f"# {args.title}", "", "Commands (from the repository root, MI355X, ROCm 7.2):", "",
               "```"] + args.command + ["```", ""]
        if args.note:
            txt += [args.note, ""]
        for spec in args.dir:
            label, d = spec.rsplit("=", 1)
            txt += [f"## {label}", "", mfma_table(d, args.kernel), ""]
        open(args.out, "w").write("\n".join(txt))
        return 0

    if args.cmd == "stats":
        txt = [f"# {args.title}", "", "Command (from the repository root, MI355X, ROCm 7.2):", "",
               "```", args.command, "```", ""]
        if args.note:
            txt += [args.note, ""]
        txt += [stats_table(args.dir), ""]
        if args.per_grid:
            d = per_grid_durations(args.dir, args.per_grid, args.after_first)
            txt += [f"Dispatches of `{args.per_grid}` by grid size (work-items):", "",
                    "| grid | dispatches | avg us | total ms |", "|---|---|---|---|"]
            keep = []
            for g in sorted(d, reverse=True):
                v = d[g]
                mark = " (left out below)" if g in args.exclude_grid else ""
                txt.append(f"| {g}{mark} | {len(v)} | {sum(v) / len(v):.2f} | {sum(v) / 1e3:.1f} |")
                if g not in args.exclude_grid:
                    keep += v
            txt += ["", "Average over the {} dispatches not left out: {:.2f} us.".format(
                len(keep), sum(keep) / max(len(keep), 1)), ""]
        open(args.out, "w").write("\n".join(txt))
        return 0

    s = summarise_counters(args.fetch, args.write, args.kernel, args.copy_kernel,
                           args.copy_bytes, tuple(args.exclude_grid), args.after_first)
    txt = [f"# {args.title}", "", "Commands (from the repository root, MI355X, ROCm 7.2):", "",
           "```"] + args.command + ["```", ""]
    if args.note:
        txt += [args.note, ""]
    txt += ["Calibration: the copy kernel moves {:.0f} KiB each way; FETCH_SIZE read {:.0f} KiB "
            "and WRITE_SIZE {:.0f} KiB per dispatch, so the factors are {:.4f} (fetch) and "
            "{:.4f} (write).".format(s["copy_known_kib"], s["copy_fetch_kib"],
                                     s["copy_write_kib"], s["fetch_factor"], s["write_factor"]),
            "", "Sweep kernel(s): " + ", ".join(f"`{_short(k, 80)}`" for k in s["kernels"]), "",
            "| grid (work-groups x threads) | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB "
            "| fetched MB (calibrated) | written MB (calibrated) |",
            "|---|---|---|---|---|---|"]
    for g, c, mf, mw, bf, bw in s["rows"]:
        txt.append(f"| {g} | {c} | {mf:.0f} | {mw:.0f} | {bf / 1e6:.2f} | {bw / 1e6:.2f} |")
    rec = {"kernel": args.kernel, "traffic_bytes_per_launch": round(s["traffic_bytes_per_launch"]),
           "dispatches": s["dispatches"], "fetch_factor": round(s["fetch_factor"], 5),
           "write_factor": round(s["write_factor"], 5), "sources_sha256": sweep_source_hash()}
    txt += ["", "Average over all {} sweep dispatches: {:.2f} MB per launch.".format(
        s["dispatches"], s["traffic_bytes_per_launch"] / 1e6), "", "traffic: " + json.dumps(rec),
        ""]
    open(args.out, "w").write("\n".join(txt))
    return 0


def read_traffic(path: str):
    """The traffic record of a counter summary, or None if absent or stale."""
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic: "):
            rec = json.loads(line[len("traffic: "):])
            return rec if rec.get("sources_sha256") == sweep_source_hash() else None
    return None


if __name__ == "__main__":
    sys.exit(main())
