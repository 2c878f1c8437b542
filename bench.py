"""Throughput of the multigrid F-cycle solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload annulus4097]

Default workload annulus4097: the polar annulus r in [0.5, 1], theta
periodic, mapped to the unit square (Q1 finite elements with kx = 4 pi r,
ky = 1/(4 pi r)), 4097 x 4096 nodes (16,773,120 unknowns; FP64 x, b and the
defect take 403 MB, beyond the 256 MB last-level cache), f = N(0, 1) (seed
3), x0 = 0, four-colour Gauss-Seidel 2/2, F-cycle over 11 levels, solved to
a 1e-10 relative residual (||b - A x_k|| <= 1e-10 ||b - A x_0||) with inputs
resident in device memory.  `value` = unknowns solved per second in the
headline precision (FP32 cycles inside FP64 defect correction); the FP64
form is timed beside it and the two solutions are compared.  `roofline`
reports the dominant finest-level fused pass timed with HIP events on the
solver's stream; `cpu_baseline` times the CPU oracle on a bounded sample of
the same workload with one process and with one process per core.  Other
workloads: aniso1025, batch256, grf2049, sphere2049 (see their functions).
Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TOL = 1e-10
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="annulus4097",
                    choices=["aniso1025", "annulus4097", "batch256", "grf2049", "sphere2049"])
    ap.add_argument("--nu", type=int, default=2)
    ap.add_argument("--smoother", default=None,
                    choices=["tri_x", "tri_y", "adi", "gstri_x", "gstri_y", "gsadi"],
                    help="aniso1025 / annulus4097 with a line smoother instead of the workload's point smoother")
    ap.add_argument("--omega", type=float, default=0.8, help="damping of the TRI and ADI line smoothers")
    ap.add_argument("--sor", type=float, default=1.0,
                    help="aniso1025 / annulus4097: SOR factor of the point Gauss-Seidel smoother (1 = Gauss-Seidel)")
    ap.add_argument("--x0", default="zero", choices=["zero", "uniform", "nested"],
                    help="start vector; nested = mg_start_nested inside the timed region")
    ap.add_argument("--levels", type=int, default=0, help="number of levels (0 = coarsen as far as possible)")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--inner-cycles", type=int, default=None,
                    help="mixed form: FP32 F-cycles per FP64 residual (default: 3 on annulus4097 with the point "
                         "smoother, whose cycles contract by about 0.9 each, else 1)")
    ap.add_argument("--tune", default="auto", choices=["auto", "off", "refresh"],
                    help="tile shapes and coarse threshold: autotuned (cached), the fixed rule, or measured again")
    ap.add_argument("--max-cycles", type=int, default=20000)
    ap.add_argument("--eps", type=float, default=None, help="one eps of the workload only (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="timed budget of each oracle sample (one process, then one per core)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain device copy of 512 MiB (HBM counter calibration)")
    ap.add_argument("--stats-summary", metavar="KERNEL_STATS_CSV",
                    help="print a markdown summary of a rocprofv3 --stats kernel_stats.csv and exit")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print the HBM traffic summary of two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of "
                         "this bench with --calibrate-copy, and exit")
    ap.add_argument("--trace", metavar="KERNEL_TRACE_CSV",
                    help="with --stats-summary: also break the time down by kernel and grid size (level)")
    ap.add_argument("--counters-summary", nargs="+", metavar="COUNTER_CSV",
                    help="print a markdown summary of rocprofv3 --pmc counter_collection.csv files (SQ counters "
                         "per dispatch of each kernel) and exit")
    ap.add_argument("--durations", metavar="KERNEL_STATS_CSV",
                    help="with --counters-summary: kernel durations for per-CU issue rates")
    ap.add_argument("--command", default="", help="command line recorded in a summary")
    return ap.parse_args()


COPY_BYTES = 512 << 20
PROFILES = os.path.join(ROOT, "profiles")


def calibrate_copy():
    """One device-to-device copy of COPY_BYTES: the reference a counter-based
    byte count is scaled by."""
    import torch

    a = torch.zeros(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()


def source_digest() -> str:
    """sha256 over the compile flags and the kernel sources: a stored counter
    measurement is only reported while the kernels it was taken on are
    unchanged."""
    import hashlib

    from paper_0805_3041_amd.build import flags_key

    d = hashlib.sha256(flags_key().encode() + b"\0")
    csrc = os.path.join(ROOT, "paper_0805_3041_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                d.update(name.encode() + b"\0" + f.read())
    return d.hexdigest()


def stored_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from profiles/<workload>_traffic.md, or
    None when absent or taken on other kernel sources."""
    path = os.path.join(PROFILES, f"{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    digest, found = None, None
    for line in open(path):
        line = line.strip().strip("`")
        if line.startswith("source_sha256:"):
            digest = line.split(":", 1)[1].strip()
        if line.startswith("traffic_bytes_per_launch[") and kernel in line:
            found = float(line.rsplit(":", 1)[1])
    if digest != source_digest():
        return None
    return found


def _csv_rows(path):
    import csv

    with open(path) as f:
        return list(csv.DictReader(f))


def trace_breakdown(path: str, top: int = 30) -> list:
    """Markdown rows: time per (kernel, grid size) from a kernel_trace.csv;
    the grid size tells the levels of one kernel apart."""
    acc = {}
    for r in _csv_rows(path):
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        key = (name, int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]), int(r["Workgroup_Size_X"]))
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        a = acc.setdefault(key, [0, 0.0])
        a[0] += 1
        a[1] += d
    out = ["", "Time by kernel and grid (workgroups = grid / workgroup size; one grid size per level):", "",
           "| calls | total ms | avg us | workgroups | kernel |", "|---|---|---|---|---|"]
    for (name, grid, wg), (n, t) in sorted(acc.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append(f"| {n} | {t / 1e3:.3f} | {t / n:.2f} | {grid // wg} | `{name}` |")
    return out


# counters of a --counters-summary table, in this order, and derived ratios
SQ_ORDER = ["SQ_WAVES", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS",
            "SQ_INSTS_SMEM", "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_INSTS_BRANCH", "SQ_ACTIVE_INST_ANY",
            "SQ_ACTIVE_INST_VALU", "SQ_ACTIVE_INST_LDS", "SQ_ACTIVE_INST_SCA", "SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
            "SQ_WAIT_INST_LDS", "SQ_LDS_BANK_CONFLICT"]
CHIP_CUS, CLOCK_GHZ = 256, 2.4


def counters_summary(paths, durations, command: str) -> str:
    """Per kernel: each SQ counter's mean per dispatch over the given
    counter_collection.csv files, and the ratios that tell what bounds it.
    With kernel durations, instructions per CU per cycle at 2.4 GHz (a CU
    issues at most one VALU and one SALU wave-instruction per cycle)."""
    per = {}
    for path in paths:
        seen = {}
        for r in _csv_rows(path):
            name = r["Kernel_Name"].split("(")[0].replace("void ", "")
            c = per.setdefault(name, {})
            c[r["Counter_Name"]] = c.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            seen.setdefault((name, r["Counter_Name"]), set()).add(r["Dispatch_Id"])
        for (name, cn), ds in seen.items():
            per[name][cn] /= len(ds)
    dur = {}
    if durations:
        for r in _csv_rows(durations):
            dur[r["Name"].split("(")[0].replace("void ", "")] = float(r["AverageNs"])
    names = sorted(per)
    out = ["# SQ counters per dispatch (rocprofv3 --pmc)", "", f"Command: `{command}`", "",
           "| counter | " + " | ".join(f"`{n}`" for n in names) + " |", "|---|" + "---|" * len(names)]
    for cn in SQ_ORDER:
        if any(cn in per[n] for n in names):
            out.append(f"| {cn} | " + " | ".join(f"{per[n].get(cn, float('nan')):.4g}" for n in names) + " |")

    def ratio(n, a, b):
        x, y = per[n].get(a), per[n].get(b)
        return f"{x / y:.3f}" if x is not None and y else "-"

    out.append("| SALU / VALU instructions | " + " | ".join(ratio(n, "SQ_INSTS_SALU", "SQ_INSTS_VALU") for n in names) + " |")
    out.append("| waiting (any) / wave cycles | " + " | ".join(ratio(n, "SQ_WAIT_ANY", "SQ_WAVE_CYCLES") for n in names) + " |")
    out.append("| waiting on dependencies / wave cycles | " + " | ".join(ratio(n, "SQ_WAIT_INST_ANY", "SQ_WAVE_CYCLES") for n in names) + " |")
    out.append("| issuing / wave cycles | " + " | ".join(ratio(n, "SQ_ACTIVE_INST_ANY", "SQ_WAVE_CYCLES") for n in names) + " |")
    out.append("| LDS bank conflicts / LDS active | " + " | ".join(ratio(n, "SQ_LDS_BANK_CONFLICT", "SQ_ACTIVE_INST_LDS") for n in names) + " |")
    if dur:
        def per_cu(n, cn):
            if cn not in per[n] or n not in dur:
                return "-"
            cycles = dur[n] * CLOCK_GHZ
            return f"{per[n][cn] / CHIP_CUS / cycles:.2f}"
        out.append("| average duration us | " + " | ".join(f"{dur.get(n, float('nan')) / 1e3:.2f}" for n in names) + " |")
        out.append("| VALU issue per CU per cycle | " + " | ".join(per_cu(n, "SQ_INSTS_VALU") for n in names) + " |")
        out.append("| SALU issue per CU per cycle | " + " | ".join(per_cu(n, "SQ_INSTS_SALU") for n in names) + " |")
        out.append("| LDS instructions per CU per cycle | " + " | ".join(per_cu(n, "SQ_INSTS_LDS") for n in names) + " |")
    return "\n".join(out) + "\n"


def stats_summary(path: str, command: str, trace: str = None) -> str:
    rows = _csv_rows(path)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = ["# rocprofv3 kernel statistics", "", f"Command: `{command}`", "",
           f"Total kernel time: {tot / 1e6:.3f} ms", "",
           "| calls | total ms | avg us | min us | max us | % | kernel |", "|---|---|---|---|---|---|---|"]
    for r in rows[:25]:
        name = r["Name"].split("(")[0].replace("void ", "")
        out.append(f"| {int(r['Calls'])} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} | `{name}` |")
    if trace:
        out += trace_breakdown(trace)
    return "\n".join(out) + "\n"


def _per_dispatch(path, counter):
    """{dispatch id: (kernel name, counter value summed over its rows)}."""
    acc = {}
    for r in _csv_rows(path):
        if r["Counter_Name"] != counter:
            continue
        key = r["Dispatch_Id"]
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        v = acc.get(key, (name, 0.0))[1] + float(r["Counter_Value"])
        acc[key] = (name, v)
    return acc


def traffic_summary(fetch_csv: str, write_csv: str, command: str) -> str:
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the finest-level fused
    passes, each scaled by what the same counter reads for the COPY_BYTES
    device copy."""
    fetch = _per_dispatch(fetch_csv, "FETCH_SIZE")
    write = _per_dispatch(write_csv, "WRITE_SIZE")

    def copy_kib(acc):
        vals = [v for n, v in acc.values() if "copy" in n.lower() or "Copy" in n]
        return max(vals) if vals else None

    cf, cw = copy_kib(fetch), copy_kib(write)
    exp_kib = COPY_BYTES / 1024
    out = ["# HBM traffic of the finest-level fused passes (rocprofv3 FETCH_SIZE / WRITE_SIZE)", "",
           f"Command: `{command}`", "",
           f"Calibration: a {COPY_BYTES >> 20} MiB device copy reads FETCH_SIZE {cf:.0f} KiB and writes "
           f"WRITE_SIZE {cw:.0f} KiB (expected {exp_kib:.0f} KiB each); scale factors "
           f"{exp_kib / cf:.4f} (read), {exp_kib / cw:.4f} (write).", "",
           "| kernel | dispatches | FETCH_SIZE KiB / dispatch | WRITE_SIZE KiB / dispatch | scaled bytes / launch |",
           "|---|---|---|---|---|"]
    per_kernel = {}
    for acc, which in ((fetch, 0), (write, 1)):
        for n, v in acc.values():
            if "k_pre" in n or "k_post" in n:
                if ", true," not in n:
                    continue
                per_kernel.setdefault(n, ([], []))[which].append(v)
    lines = []
    for n, (fv, wv) in sorted(per_kernel.items()):
        if not fv or not wv:
            continue
        f_avg, w_avg = sum(fv) / len(fv), sum(wv) / len(wv)
        bytes_ = (f_avg * exp_kib / cf + w_avg * exp_kib / cw) * 1024
        out.append(f"| `{n}` | {len(fv)} | {f_avg:.0f} | {w_avg:.0f} | {bytes_:.4g} |")
        lines.append(f"traffic_bytes_per_launch[{n}]: {bytes_:.6g}")
    out += ["", *lines, f"source_sha256: {source_digest()}", ""]
    return "\n".join(out)


# Mixed form on annulus4097: FP32 F-cycles per FP64 residual.  Its cycles
# contract the error by about 0.905 each (230 to 1e-10), so three FP32
# cycles per outer step lose nothing to FP32 rounding (the inner residual
# falls by 0.74, far above FP32's 1e-7), need 77 outer steps (231 cycles)
# instead of 230, and form the FP64 residual a third as often.
ANNULUS_INNER = 3

# Algorithmic bytes per stored fine node of the finest-level fused passes
# (5-point operator): reads and writes the pass cannot avoid.
#   FP64 pre-pass : read x, b; write smoothed x; write coarse b and x (1/4 node each)
#   FP64 post-pass: read smoothed x, b, coarse x (1/4); write x
#   FP32 pre-pass (mixed, finest level): the correction e starts at 0 and is
#                   not read: read r; write smoothed e; coarse b and x
#   FP32 post-pass (mixed, finest level): read smoothed e, r, coarse e (1/4);
#                   read and write the FP64 iterate (e itself is left as it
#                   is: the next pre-pass does not read it)
#   FP32 pre-pass forming the residual itself (mixed, finest level, when
#                   the solver reports forms_residual): read the FP64 x and
#                   b; write r (for the passes after it), smoothed e, coarse
#                   b and x; no separate residual kernel runs
BYTES_PER_NODE = {
    ("fp64", 0): 8 + 8 + 8 + 2 + 2,
    ("fp64", 1): 8 + 8 + 2 + 8,
    ("mixed", 0): 4 + 4 + 1 + 1,
    ("mixed", 1): 4 + 4 + 1 + 8 + 8,
}
BYTES_PER_NODE_PRE_RESID = 8 + 8 + 4 + 4 + 1 + 1
# Mixed form with K > 1 inner cycles per outer step: the finest passes of
# the other K - 1 inner cycles are plain FP32 passes (pre: read e, r; write
# smoothed e, coarse b and x; post: read smoothed e, r, coarse e; write e).
BYTES_PER_NODE_MIXED_INNER = {0: 4 + 4 + 4 + 1 + 1, 1: 4 + 4 + 1 + 4}


def pass_bytes_per_node(s, head, which, inner=1):
    """Algorithmic bytes per finest node of solver s's finest fused pass,
    averaged over the launches of one outer step of `inner` cycles (the
    launch mix that mg_profile_pass times with reps a multiple of inner)."""
    if head != "mixed":
        return BYTES_PER_NODE[(head, which)]
    first = BYTES_PER_NODE[(head, which)]
    if which == 0 and s.pass_info(0, 0).get("forms_residual"):
        first = BYTES_PER_NODE_PRE_RESID
    return (first + (inner - 1) * BYTES_PER_NODE_MIXED_INNER[which]) / inner
# Level 1 (a coarse level: plain post-pass, 4- or 8-byte values):
#   pre-pass : read x, b; write t; write coarse b and x (1/4 node each) = 3.5 w
#   post-pass: read t, b, coarse x (1/4); write x                      = 3.25 w
BYTES_PER_NODE_L1 = {
    ("fp64", 0): 28, ("fp64", 1): 26,
    ("mixed", 0): 14, ("mixed", 1): 13,
}


def fine_levels_roofline(s, rhs, scratch, head, times0, reps, inner=1):
    """Algorithmic bytes of the fused passes of levels 0 and 1 (the levels
    that carry most of a cycle's bytes) over their summed device time."""
    shape1 = s.level_shape(1) if s.nlevels > 1 else None
    total_b = sum(pass_bytes_per_node(s, head, w, inner) for w in (0, 1)) * rhs.numel()
    total_t = times0[0] + times0[1]
    per = {}
    if shape1 is not None:
        try:
            t1 = {w: s.profile_pass(rhs, scratch, 1, w, reps=reps) for w in (0, 1)}
        except Exception:
            t1 = None
        if t1 is not None:
            n1 = shape1[0] * shape1[1]
            total_b += sum(BYTES_PER_NODE_L1[(head, w)] for w in (0, 1)) * n1
            total_t += t1[0] + t1[1]
            per = {"level1_pre_us": t1[0], "level1_post_us": t1[1]}
    ach = total_b / (total_t * 1e-6) / 1e9
    return {"achieved": ach, "frac": ach / HBM_PEAK_GBS, "unit": "GB/s", "bytes": total_b, "us": total_t, **per}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


# ----------------------------------------------------------------------------- CPU baseline (the oracle)
#
# The oracle (FP64, scipy.sparse) runs F-cycles of a bounded sample of the
# workload: one process, then one process per host core (up to the 16 cores a
# one-GPU share has), each on its own copy of the sample problem, started
# together.  Both rates are unknown-cycles per second; they become unknowns/s
# to tolerance once the GPU run has given the cycle counts.  The pools run
# before anything touches the GPU (the workers are forked).

MAX_POOL = 16


def pool_size() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(MAX_POOL, n))


def _oracle_sample(spec):
    """(step, unknowns per step) of one oracle sample problem."""
    import numpy as np

    from oracle import mg_oracle as O
    import workloads as W

    kind = spec["kind"]
    opts = O.Options(smoother=spec.get("smoother", "rbgs"), nu_pre=spec.get("nu", 2), nu_post=spec.get("nu", 2),
                     omega=spec.get("omega", 0.8), sor=spec.get("sor", 1.0))
    n = spec["n"]
    if kind == "grf":
        a, f, ustar = W.grf_problem(n, 5)
        g = O.Grid(n, n)
        return (lambda: O.adjoint_gradient(g, a, f, ustar)), g.n_unknowns
    if kind == "annulus":
        g = O.Grid(n, n - 1, periodic_y=True)
        kx, ky = W.annulus_cell_coefficients(n)
        h = O.hierarchy_q1(g, kx, ky, opts, separable=True)
        b = g.pack(W.annulus_rhs(n, n - 1, 3))
    elif kind == "sphere":
        g = O.Grid(n, n)
        kx, ky = W.sphere_cell_coefficients(n, n)
        h = O.hierarchy_q1(g, kx, ky, opts)
        b = g.pack(W.normal_field(n, n, 3))
    else:  # 5-point anisotropic problem
        g = O.Grid(n, n)
        h = O.hierarchy_5pt(g, spec["eps"], 1.0, opts)
        b = g.pack(W.aniso_rhs(n, 2))
    state = {"x": np.zeros(g.n_unknowns)}

    def step():
        state["x"] = O.mg_cycle(h, 0, state["x"], b, "F")

    return step, g.n_unknowns


def _oracle_worker(spec, seconds, barrier, queue):
    from threadpoolctl import threadpool_limits

    with threadpool_limits(1):
        step, unknowns = _oracle_sample(spec)
        barrier.wait(timeout=600)
        done = 0
        t0 = time.perf_counter()
        while done < 2 or time.perf_counter() - t0 < seconds:
            step()
            done += 1
        queue.put((unknowns, done, time.perf_counter() - t0))


def oracle_rates(spec, seconds):
    """Oracle throughput in unknown-steps per second with one process and with
    pool_size() processes (one sample problem each, timed together)."""
    import multiprocessing as mp

    ctx = mp.get_context("fork")
    out = {}
    for procs in sorted({1, pool_size()}):
        barrier, queue = ctx.Barrier(procs), ctx.Queue()
        ps = [ctx.Process(target=_oracle_worker, args=(spec, seconds, barrier, queue)) for _ in range(procs)]
        for p in ps:
            p.start()
        res = [queue.get(timeout=seconds + 900) for _ in ps]
        for p in ps:
            p.join(timeout=60)
        if any(p.exitcode != 0 for p in ps):
            raise RuntimeError("an oracle worker failed")
        out[procs] = {"rate": sum(u * d / t for u, d, t in res), "steps": sum(d for _, d, _ in res),
                      "seconds": max(t for _, _, t in res), "unknowns": res[0][0]}
    out["what"] = _describe(spec)
    return out


def _describe(spec):
    return {"annulus": "FP64 F-cycles on the {n}x{m} annulus", "sphere": "FP64 F-cycles of the {n}x{n} spherical "
            "problem", "grf": "oracle gradients (direct forward + adjoint solves, dL/da) at {n}x{n}",
            "aniso": "FP64 F-cycles of the eps={eps:g} 5-point problem at {n}x{n}"}[spec["kind"]].format(
        n=spec["n"], m=spec["n"] - 1, eps=spec.get("eps", 1.0))


def cpu_baseline_from_rates(rates, steps_per_unknown_solved, scale_note):
    """unknowns/s to tolerance of the oracle: its unknown-step rate divided by
    the steps one solved unknown needs (cycles to tolerance, or 1 for a
    gradient), for all cores ("value") and for one core ("single_core")."""
    procs = max(k for k in rates if isinstance(k, int))
    one = rates[1]
    many = rates[procs]
    return {
        "value": many["rate"] / steps_per_unknown_solved,
        "unit": "unknowns/s",
        "cores": procs,
        "kind": "oracle",
        "sample": f"{rates['what']}: {procs} processes (one core each) ran {many['steps']} steps in "
                  f"{many['seconds']:.1f} s, one process {one['steps']} steps in {one['seconds']:.1f} s; "
                  f"{scale_note} (extrapolated)",
        "single_core": {"value": one["rate"] / steps_per_unknown_solved, "cores": 1},
        "host_cpu": cpu_model(),
        "host_threads_available": os.cpu_count(),
    }


def baseline_spec(args):
    """The oracle sample of each workload."""
    w = args.workload
    sm = args.smoother
    if w == "annulus4097":
        return {"kind": "annulus", "n": 1025, "smoother": sm or "gs4c", "nu": args.nu, "omega": args.omega,
                "sor": args.sor}
    if w == "aniso1025":
        eps = min(__import__("workloads").ANISO_EPS) if args.eps is None else args.eps
        return {"kind": "aniso", "n": 1025, "eps": eps, "smoother": sm or "rbgs", "nu": args.nu,
                "omega": args.omega, "sor": args.sor}
    if w == "batch256":
        return {"kind": "aniso", "n": 257, "eps": 1e-2, "smoother": "rbgs", "nu": args.nu}
    if w == "sphere2049":
        return {"kind": "sphere", "n": 257, "smoother": sm or "gs4c", "nu": args.nu, "omega": args.omega,
                "sor": args.sor}
    if w == "grf2049":
        return {"kind": "grf", "n": 129}
    raise ValueError(w)


def oracle_sampled_residual(x_stored, rows=4000, seed=51):
    """The oracle's FP64 residual b - A x of an annulus4097 solution at `rows`
    sampled nodes, each row assembled from its cells' element matrices; returns
    the relative 2-norm estimated from the samples (sqrt of the mean square
    times the number of unknowns, over ||b||) and the largest sampled entry."""
    import numpy as np

    from oracle import mg_oracle as O
    import workloads as W

    nx, ny = 4097, 4096
    g = O.Grid(nx, ny, periodic_y=True)
    kx, ky = W.annulus_cell_coefficients(nx)
    KX = np.broadcast_to(kx, (g.ncy, g.ncx))
    KY = np.broadcast_to(ky, (g.ncy, g.ncx))
    b = W.annulus_rhs(nx, ny, 3)
    rng = np.random.default_rng(seed)
    r = []
    for _ in range(rows):
        i = int(rng.integers(1, nx - 1))
        j = int(rng.integers(0, ny))
        row = O.q1_row(g, KX, KY, i, j)
        r.append(b[j, i] - sum(v * x_stored[jq, iq] for (jq, iq), v in row.items()))
    r = np.array(r)
    est = math.sqrt(float(np.mean(r * r)) * g.n_unknowns) / float(np.linalg.norm(b))
    return {"rows": rows, "est_rel_res": est, "max_abs": float(np.abs(r).max())}


def annulus(args, rates=None):
    """Workload annulus4097: r in [0.5, 1], theta periodic, mapped to the unit
    square (Q1, kx = 4 pi r, ky = 1/(4 pi r) per radial cell), 4097 radial x
    4096 angular nodes (16,773,120 unknowns), f = N(0, 1) (seed 3), x0 = 0,
    four-colour Gauss-Seidel 2/2, F-cycle over 11 levels down to 5 x 4.  The
    mixed form (FP32 cycles inside FP64 defect correction) is the headline,
    the FP64 form is timed beside it, and the two solutions are compared."""
    import torch

    import workloads as W
    from paper_0805_3041_amd import mg

    nx, ny = 4097, 4096
    kx, ky = W.annulus_cell_coefficients(nx)
    kxt, kyt = torch.tensor(kx, device="cuda"), torch.tensor(ky, device="cuda")
    rhs = torch.tensor(W.annulus_rhs(nx, ny, 3), device="cuda")
    unknowns = (nx - 2) * ny

    smoother = args.smoother or "gs4c"

    # (line smoothers reach 1e-10 in a few cycles: one per outer step)
    inner = (1 if args.smoother else ANNULUS_INNER) if args.inner_cycles is None else args.inner_cycles

    def make(precision):
        return mg.Solver(nx, ny, periodic_y=True, kx=kxt, ky=kyt, kx_1d_along_x=True, smoother=smoother,
                         nu_pre=args.nu, nu_post=args.nu, omega=args.omega, sor=args.sor, precision=precision,
                         levels=args.levels, tune=args.tune, inner_cycles=inner if precision == "mixed" else 1)

    def f_cycles(info, precision):  # a mixed outer step runs `inner` F-cycles
        return info.cycles * (inner if precision == "mixed" else 1)

    def start(s, x):
        if args.x0 == "nested":
            s.nested_start(rhs, x)
        else:
            x.zero_()

    def run(s, steps, warmup, label):
        x = torch.zeros_like(rhs)
        for _ in range(warmup):
            start(s, x)
            s.solve(rhs, x, TOL, args.max_cycles, history=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = None
        for _ in range(steps):
            start(s, x)
            info = s.solve(rhs, x, TOL, args.max_cycles, history=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if info.status != mg.MG_OK:
            raise SystemExit(f"{label} solve did not converge: {mg.status_string(info.status)} "
                             f"rel_res {info.rel_res:.3e}")
        return wall, info, x

    head = args.precision
    other = "fp64" if head == "mixed" else "mixed"
    s = make(head)
    wall_h, info_h, x_h = run(s, args.steps, args.warmup, head)
    scratch = torch.zeros_like(rhs)
    if args.smoother:
        roofline = line_roofline(s, rhs, scratch, head, nx, ny, True, smoother, 1)
    else:
        k = inner if head == "mixed" else 1
        reps = k * max(1, 20 // k)  # whole outer steps
        times = {which: s.profile_pass(rhs, scratch, 0, which, reps=reps) for which in (0, 1)}
        dom = 1 if times[1] >= times[0] else 0
        kernel_name = s.pass_kernel_name(0, dom)
        levels01 = fine_levels_roofline(s, rhs, scratch, head, times, reps, k)
        bpn = pass_bytes_per_node(s, head, dom, k)
        alg_bytes = bpn * nx * ny
        achieved = alg_bytes / (times[dom] * 1e-6) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic("annulus4097", kernel_name),
                    "kernel": kernel_name, "avg_us": times[dom], "bytes_per_launch": alg_bytes,
                    "bytes_per_node": bpn, "nodes": nx * ny,
                    "other_pass_us": times[1 - dom], "levels_0_1": levels01}
        if k > 1:
            roofline["launch_mix"] = (f"averaged over the {k} launches of an outer step: the first pre-pass from "
                                      f"e = 0, the last post-pass adding e into the FP64 iterate, the other "
                                      f"{k - 1} plain FP32 passes")
    s.close()
    del scratch
    s = make(other)
    steps_o = max(1, args.steps // 2)
    wall_o, info_o, x_o = run(s, steps_o, 1, other)
    s.close()
    x_m, x_64 = (x_h, x_o) if head == "mixed" else (x_o, x_h)
    err_vs_fp64 = float((x_m - x_64).abs().max() / x_64.abs().max())
    if args.calibrate_copy:
        calibrate_copy()
    smoothing = SMOOTHER_NAMES[smoother] if args.smoother else "four-colour GS"
    if not args.smoother and args.sor != 1.0:
        smoothing = f"four-colour SOR (omega {args.sor:g})"
    info_m, info_64 = (info_h, info_o) if head == "mixed" else (info_o, info_h)
    out = {
        "metric": "unknowns/s to 1e-10 rel. residual",
        "value": unknowns * args.steps / wall_h,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall_h / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-inner/f64-outer" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "annulus4097: polar annulus r in [0.5,1], theta periodic, mapped to the unit square, "
                               f"Q1 with kx=4 pi r, ky=1/(4 pi r), 4097x4096 nodes, f = N(0,1), {smoothing} "
                               f"{args.nu}/{args.nu}, F-cycle to "
                               + (f"{args.levels} levels" if args.levels else "5x4")
                               + f", x0={'nested' if args.x0 == 'nested' else '0'}, tol 1e-10", "precision": head,
                   "inner_cycles": inner, "tune": args.tune},
        "roofline": roofline,
        "cycles": f_cycles(info_h, head),
        "outer_steps": info_m.cycles,
        "rel_res": info_h.rel_res,
        "us_per_cycle": 1e6 * info_h.seconds / max(1, f_cycles(info_h, head)),
        f"value_{other}": unknowns * steps_o / wall_o,
        f"cycles_{other}": f_cycles(info_o, other),
        f"rel_res_{other}": info_o.rel_res,
        f"us_per_cycle_{other}": 1e6 * info_o.seconds / max(1, f_cycles(info_o, other)),
        "speedup_mixed_over_fp64": ((wall_o / steps_o) / (wall_h / args.steps)) if head == "mixed"
        else ((wall_h / args.steps) / (wall_o / steps_o)),
        "mixed_vs_fp64_max_rel_diff": err_vs_fp64,
    }
    if rates is not None:
        cb = cpu_baseline_from_rates(rates, info_64.cycles,
                                     f"rate per unknown-cycle applied to 4097x4096 and the {info_64.cycles} "
                                     f"cycles of the FP64 solve")
        cb["oracle_residual_of_mixed_solution"] = oracle_sampled_residual(x_m.cpu().numpy())
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


# Line sweep, per node of the lines it solves.  The kernels that hold a
# line in LDS (k_line_cr, k_line_y) read b and the off-line neighbours (each
# once; Jacobi: x itself once) and write x: 3 values.  The thread-per-line
# Thomas kernel (k_line, lines too long for LDS) also reads the two Thomas
# factors and writes and re-reads the forward-sweep value: 7 values.  Both
# add six bands when the coefficients vary in 2-D.
LINE_VALUES_PER_NODE = {"lds": 3, "thomas": 7}
# y lines of at least this many unknowns whose four LDS arrays for 4 lines
# fit in 140 KB run k_line_y (segments), other LDS-fitting lines k_line_cr
LINE_Y_MIN = 128

SMOOTHER_NAMES = {"tri_x": "TRI (x lines)", "tri_y": "TRI (y lines)", "adi": "ADI", "gstri_x": "GSTRI (x lines)",
                  "gstri_y": "GSTRI (y lines)", "gsadi": "GSADI"}


def line_roofline(s, rhs, scratch, head, nx, ny, periodic_y, smoother, stencil, bands_2d=False, reps=20, cells=0):
    """Roofline of the first line sweep of the finest level (one launch)."""
    us = s.profile_pass(rhs, scratch, 0, 2, reps=reps)
    w = 4 if head == "mixed" else 8
    first_y = smoother in ("tri_y", "gstri_y")
    jac = smoother in ("tri_x", "tri_y", "adi")
    if first_y:
        lines = [i for i in range(1, nx - 1) if jac or i % 2 == 0]
        m = ny - 2
    else:
        rows = range(0, ny) if periodic_y else range(1, ny - 1)
        lines = [j for j in rows if jac or j % 2 == 0]
        m = nx - 2
    nodes = len(lines) * m
    t = "float" if head == "mixed" else "double"
    if first_y and m >= LINE_Y_MIN and 4 * 4 * (m + m // 32 + 1) * w <= 140 * 1024:
        kernel = "k_line_y"
    elif 4 * m * w <= 140 * 1024:
        kernel = "k_line_cr"
    else:
        kernel = "k_line"
    bpn = (LINE_VALUES_PER_NODE["thomas" if kernel == "k_line" else "lds"] + (6 if bands_2d else 0) + cells) * w
    alg = bpn * nodes
    ach = alg / (us * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": None, "kernel": f"mg::{kernel}<{t}, {stencil}>", "avg_us": us, "bytes_per_launch": alg,
            "bytes_per_node": bpn, "nodes": nodes}


def _roofline_single(n, eps, head, nu):
    """Roofline of the finest-level fused pass of one n x n 5-point problem
    (the kernels every batched group runs, one problem slot per launch)."""
    import torch

    import workloads as W
    from paper_0805_3041_amd import mg

    s = mg.Solver(n, n, eps_x=eps, smoother="rbgs", nu_pre=nu, nu_post=nu, precision=head)
    rhs = torch.tensor(W.aniso_rhs(n, 2), device="cuda")
    scratch = torch.zeros_like(rhs)
    times = {which: s.profile_pass(rhs, scratch, 0, which, reps=50) for which in (0, 1)}
    dom = 1 if times[1] >= times[0] else 0
    kernel = s.pass_kernel_name(0, dom)
    bpn = pass_bytes_per_node(s, head, dom)
    s.close()
    alg = bpn * n * n
    ach = alg / (times[dom] * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": None, "kernel": kernel, "avg_us": times[dom], "bytes_per_launch": alg,
            "bytes_per_node": bpn, "nodes": n * n, "other_pass_us": times[1 - dom],
            "note": f"one {n}x{n} problem of the batch"}


def batch256(args, rates=None):
    """Workload batch256: 256 independent 5-point problems, n drawn uniformly
    from {129, 257, 513, 1025} and eps = 10^U(-3, 0) (seed 4), rhs_i = N(0, 1)
    (seed 1000 + i), x0 = 0, red-black GS 2/2, F-cycles until every problem
    reaches 1e-10 (converged problems are masked out of later cycles)."""
    import torch

    import workloads as W
    from paper_0805_3041_amd import mg

    ns, eps = W.batch_problems(256, 4)
    rhs = [torch.tensor(W.batch_rhs(n, i), device="cuda") for i, n in enumerate(ns)]
    unknowns = sum((n - 2) ** 2 for n in ns)

    def run(B, steps, warmup):
        xs = [torch.zeros_like(r) for r in rhs]
        for _ in range(warmup):
            for x in xs:
                x.zero_()
            B.solve(rhs, xs, TOL, args.max_cycles)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = None
        for _ in range(steps):
            for x in xs:
                x.zero_()
            _, infos = B.solve(rhs, xs, TOL, args.max_cycles)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, infos

    head = args.precision
    other = "fp64" if head == "mixed" else "mixed"
    B = mg.BatchedSolver([(n, n) for n in ns], eps, smoother="rbgs", nu_pre=args.nu, nu_post=args.nu, precision=head,
                         tune=args.tune)
    wall_h, infos_h = run(B, args.steps, args.warmup)
    schedule = B.schedule()
    B.close()
    bad = [i for i, info in enumerate(infos_h) if info.status != mg.MG_OK]
    if bad:
        raise SystemExit(f"{len(bad)} batched problems did not converge (first: {bad[0]})")
    B = mg.BatchedSolver([(n, n) for n in ns], eps, smoother="rbgs", nu_pre=args.nu, nu_post=args.nu,
                         precision=other, tune=args.tune)
    steps_o = max(1, args.steps // 2)
    wall_o, infos_o = run(B, steps_o, 1)
    B.close()
    bad = [i for i, info in enumerate(infos_o) if info.status != mg.MG_OK]
    if bad:
        raise SystemExit(f"{len(bad)} batched {other} problems did not converge (first: {bad[0]})")
    cycles = [info.cycles for info in infos_h]
    out = {
        "metric": "unknowns/s to 1e-10 rel. residual",
        "value": unknowns * args.steps / wall_h,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall_h / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-inner/f64-outer" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "batch256: 256 problems -(eps u_xx + u_yy) = N(0,1), n in {129,257,513,1025} "
                               f"drawn uniformly, eps = 10^U(-3,0) (seed 4), {unknowns} unknowns, red-black GS "
                               f"{args.nu}/{args.nu}, F-cycle, x0=0, tol 1e-10", "precision": head},
        "roofline": _roofline_single(1025, 1e-3, head, args.nu),
        "cycles": {"min": min(cycles), "max": max(cycles), "sum": sum(cycles)},
        "schedule": schedule,
        f"value_{other}": unknowns * steps_o / wall_o,
        "speedup_mixed_over_fp64": ((wall_o / steps_o) / (wall_h / args.steps)) if head == "mixed"
        else ((wall_h / args.steps) / (wall_o / steps_o)),
    }
    if rates is not None:
        work = sum((m - 2) ** 2 * c for m, c in zip(ns, cycles))
        out["cpu_baseline"] = cpu_baseline_from_rates(
            rates, work / unknowns, "rate per unknown-cycle applied to each problem's unknowns times its cycles")
    print(json.dumps(out), flush=True)


# Cell coefficients (grf2049): the finest fused passes form the 9-point
# couplings from the per-cell coefficient a (kx = ky = a, one FP64 value per
# cell, one cell per node) instead of reading six bands per node.
CELL_BYTES_ISO = 8


def _roofline_grf(n, at, ft, calibrate=False):
    """Roofline of the finest-level fused passes of the grf2049 operator (the
    solver the forward and adjoint solves build)."""
    import torch

    from paper_0805_3041_amd import mg

    s = mg.Solver(n, n, kx=at, ky=at, smoother="gs4c")
    scratch = torch.zeros_like(ft)
    times = {which: s.profile_pass(ft, scratch, 0, which, reps=20) for which in (0, 1)}
    dom = 1 if times[1] >= times[0] else 0
    kernel = s.pass_kernel_name(0, dom)
    s.close()
    if calibrate:
        calibrate_copy()
    bpn = BYTES_PER_NODE[("fp64", dom)] + CELL_BYTES_ISO
    alg = bpn * n * n
    ach = alg / (times[dom] * 1e-6) / 1e9
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": stored_traffic("grf2049", kernel), "kernel": kernel, "avg_us": times[dom],
            "bytes_per_launch": alg, "bytes_per_node": bpn, "nodes": n * n, "other_pass_us": times[1 - dom]}


def grf2049(args, rates=None):
    """Workload grf2049: -div(a grad u) = f on 2049^2 nodes (2048^2 cells),
    a = exp(g), g a Gaussian random field (squared-exponential covariance,
    length 0.1, sigma 1, seed 5), f = 2 pi^2 sin(pi x) sin(pi y), loss
    0.5 ||u - u*||^2; one step = rebuild of every level's operator for a (in
    one handle kept across steps) + forward solve + adjoint solve + dL/da,
    dL/df (FP64, four-colour GS 2/2, both solves to 1e-10)."""
    import torch

    import workloads as W
    from paper_0805_3041_amd import autograd as AG

    n = 2049
    a, f, ustar = W.grf_problem(n, 5)
    at = torch.tensor(a, device="cuda")
    ft = torch.tensor(f, device="cuda")
    us = torch.tensor(ustar, device="cuda")
    unknowns = (n - 2) ** 2

    # one handle for every step, as in a gradient loop: each step rebuilds
    # the operators for its coefficient in place (the first sets up)
    gsolve = AG.GradientSolver(n, n, tol=TOL, max_cycles=args.max_cycles)

    def step():
        aa = at.clone().requires_grad_(True)
        ff = ft.clone().requires_grad_(True)
        u = gsolve(aa, ff)
        loss = 0.5 * torch.sum((u - us) ** 2)
        loss.backward()
        return aa.grad, ff.grad

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        da, df = step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gsolve.close()
    out = {
        "metric": "unknowns/s to 1e-10 rel. residual (forward + adjoint gradient)",
        "value": unknowns * args.steps / wall,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "grf2049: -div(a grad u) = 2 pi^2 sin(pi x) sin(pi y) on 2049^2 nodes, a = exp(GRF, "
                               "length 0.1, sigma 1, seed 5) per cell, Q1, four-colour GS 2/2, F-cycle; forward + "
                               "adjoint solve to 1e-10 and dL/da, dL/df of 0.5 ||u - u*||^2; one handle across steps, "
                               "every level's operator rebuilt from a each step", "precision": "fp64"},
        "roofline": _roofline_grf(n, at, ft, args.calibrate_copy),
        "grad_norms": {"dL_da": float(torch.linalg.vector_norm(da)), "dL_df": float(torch.linalg.vector_norm(df))},
    }
    if rates is not None:
        out["cpu_baseline"] = cpu_baseline_from_rates(
            rates, 1.0, f"rate per unknown applied unchanged to {unknowns} unknowns (direct solves grow faster "
                        "than linearly, so this overstates the CPU rate at full size)")
    print(json.dumps(out), flush=True)


def sphere2049(args, rates=None):
    """Workload sphere2049: -Laplace(u) in spherical coordinates (axisymmetric
    shell section r in [0.5, 1], theta in [0.1 pi, 0.9 pi], the weak form
    weighted by r^2 sin(theta)) mapped to the unit square, 2049^2 nodes, Q1
    with per-cell kx = r^2 sin(theta) Lt/Lr and ky = sin(theta) Lr/Lt (two
    arrays varying in both directions), f = N(0,1) (seed 3); four-colour GS
    2/2 or the --smoother line smoother, F-cycle to 1e-10."""
    import torch

    import workloads as W
    from paper_0805_3041_amd import mg

    n = 2049
    kx, ky = W.sphere_cell_coefficients(n, n)
    kxt, kyt = torch.tensor(kx, device="cuda"), torch.tensor(ky, device="cuda")
    rhs = torch.tensor(W.normal_field(n, n, 3), device="cuda")
    unknowns = (n - 2) ** 2
    smoother = args.smoother or "gs4c"

    def make(precision):
        return mg.Solver(n, n, kx=kxt, ky=kyt, smoother=smoother, nu_pre=args.nu, nu_post=args.nu,
                         omega=args.omega, sor=args.sor, precision=precision, levels=args.levels, tune=args.tune)

    def run(s, steps, warmup):
        x = torch.zeros_like(rhs)
        for _ in range(warmup):
            x.zero_()
            s.solve(rhs, x, TOL, args.max_cycles, history=False)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = None
        for _ in range(steps):
            x.zero_()
            info = s.solve(rhs, x, TOL, args.max_cycles, history=False)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, info

    head = args.precision
    other = "fp64" if head == "mixed" else "mixed"
    w = 4 if head == "mixed" else 8
    s = make(head)
    wall_h, info_h = run(s, args.steps, args.warmup)
    if info_h.status != mg.MG_OK:
        raise SystemExit(f"solve did not converge: {mg.status_string(info_h.status)} rel_res {info_h.rel_res:.3e}")
    scratch = torch.zeros_like(rhs)
    if args.smoother:
        roofline = line_roofline(s, rhs, scratch, head, n, n, False, smoother, 1, cells=2)
    else:
        times = {which: s.profile_pass(rhs, scratch, 0, which, reps=20) for which in (0, 1)}
        dom = 1 if times[1] >= times[0] else 0
        kernel_name = s.pass_kernel_name(0, dom)
        bpn = pass_bytes_per_node(s, head, dom) + 2 * w  # + the two cell coefficients
        alg = bpn * n * n
        achieved = alg / (times[dom] * 1e-6) / 1e9
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic("sphere2049", kernel_name),
                    "kernel": kernel_name, "avg_us": times[dom], "bytes_per_launch": alg, "bytes_per_node": bpn,
                    "nodes": n * n, "other_pass_us": times[1 - dom]}
    s.close()
    s = make(other)
    steps_o = max(1, args.steps // 2)
    wall_o, info_o = run(s, steps_o, 1)
    s.close()
    if args.calibrate_copy:
        calibrate_copy()
    smoothing = SMOOTHER_NAMES[smoother] if args.smoother else "four-colour GS"
    if not args.smoother and args.sor != 1.0:
        smoothing = f"four-colour SOR (omega {args.sor:g})"
    out = {
        "metric": "unknowns/s to 1e-10 rel. residual",
        "value": unknowns * args.steps / wall_h,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall_h / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-inner/f64-outer" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "sphere2049: -Laplace(u) in spherical coordinates, r in [0.5,1], theta in "
                               "[0.1 pi,0.9 pi], weight r^2 sin(theta), mapped to the unit square, 2049x2049 "
                               f"nodes, Q1 with per-cell kx, ky, f = N(0,1), {smoothing} {args.nu}/{args.nu}, "
                               "F-cycle, x0=0, tol 1e-10", "precision": head},
        "roofline": roofline,
        "cycles": info_h.cycles,
        "rel_res": info_h.rel_res,
        "us_per_cycle": 1e6 * info_h.seconds / max(1, info_h.cycles),
        f"value_{other}": unknowns * steps_o / wall_o,
        f"cycles_{other}": info_o.cycles,
        "speedup_mixed_over_fp64": ((wall_o / steps_o) / (wall_h / args.steps)) if head == "mixed"
        else ((wall_h / args.steps) / (wall_o / steps_o)),
    }
    if rates is not None:
        out["cpu_baseline"] = cpu_baseline_from_rates(
            rates, info_h.cycles, f"rate per unknown-cycle applied to 2049^2 and the GPU's {info_h.cycles} cycles")
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.stats_summary:
        sys.stdout.write(stats_summary(args.stats_summary, args.command, args.trace))
        return
    if args.counters_summary:
        sys.stdout.write(counters_summary(args.counters_summary, args.durations, args.command))
        return
    if args.traffic_summary:
        sys.stdout.write(traffic_summary(*args.traffic_summary, args.command))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this library runs on one GPU only: collectives and multi-GPU sharding are not "
                                   "built; run with --gpus 1"}), flush=True)
        sys.exit(2)
    # the oracle's pools are forked before anything touches the GPU
    rates = None if args.no_cpu_baseline else oracle_rates(baseline_spec(args), args.cpu_seconds)
    if args.workload == "annulus4097":
        return annulus(args, rates)
    if args.workload == "batch256":
        return batch256(args, rates)
    if args.workload == "grf2049":
        return grf2049(args, rates)
    if args.workload == "sphere2049":
        return sphere2049(args, rates)
    return aniso1025(args, rates)


def aniso1025(args, rates=None):
    """Workload aniso1025: -(eps u_xx + u_yy) = f on the unit square, 1025 x
    1025 nodes, zero Dirichlet, 5-point finite differences, f = N(0, 1) (seed
    2), x0 = 0, red-black Gauss-Seidel 2/2, F-cycle over 10 levels down to
    3 x 3; one step solves the four problems eps in {1, 1e-1, 1e-2, 1e-3}.
    Its working set (8.4 MB per array) stays in the 256 MB last-level cache,
    so its bandwidth figures are L2-miss bandwidth rather than HBM."""
    import numpy as np
    import torch

    import workloads as W
    from paper_0805_3041_amd import mg

    n = 1025
    eps_list = list(W.ANISO_EPS) if args.eps is None else [args.eps]
    rhs = torch.tensor(W.aniso_rhs(n, 2), device="cuda")
    x0 = torch.tensor(W.aniso_x0(n, "zero" if args.x0 == "nested" else args.x0, 1), device="cuda")
    unknowns = (n - 2) ** 2

    smoother = args.smoother or "rbgs"

    def make(precision):
        return [mg.Solver(n, n, eps_x=e, smoother=smoother, nu_pre=args.nu, nu_post=args.nu, omega=args.omega,
                          sor=args.sor, precision=precision, levels=args.levels, tune=args.tune) for e in eps_list]

    def start(s, x):
        if args.x0 == "nested":
            s.nested_start(rhs, x)
        else:
            x.copy_(x0)

    def run(solvers, steps, warmup):
        xs = [x0.clone() for _ in solvers]
        for _ in range(warmup):
            for s, x in zip(solvers, xs):
                start(s, x)
                s.solve(rhs, x, TOL, args.max_cycles, history=False)
        torch.cuda.synchronize()
        infos = []
        t0 = time.perf_counter()
        for _ in range(steps):
            infos = []
            for s, x in zip(solvers, xs):
                start(s, x)
                infos.append(s.solve(rhs, x, TOL, args.max_cycles, history=False))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, infos

    head = args.precision
    other = "fp64" if head == "mixed" else "mixed"
    solvers = make(head)
    wall_h, infos_h = run(solvers, args.steps, args.warmup)
    for i in infos_h:
        if i.status != mg.MG_OK:
            raise SystemExit(f"solve did not converge: {mg.status_string(i.status)} rel_res {i.rel_res:.3e}")

    # roofline: finest-level post-pass of the headline precision, HIP events on the solver's stream
    scratch = x0.clone()
    s0 = solvers[0]
    if args.smoother:
        roofline = line_roofline(s0, rhs, scratch, head, n, n, False, smoother, 0, reps=100)
    else:
        times = {which: s0.profile_pass(rhs, scratch, 0, which, reps=100) for which in (0, 1)}
        dom = 1 if times[1] >= times[0] else 0
        kernel_name = s0.pass_kernel_name(0, dom)
        levels01 = fine_levels_roofline(s0, rhs, scratch, head, times, 100)
        nodes = n * n
        bpn = pass_bytes_per_node(s0, head, dom)
        alg_bytes = bpn * nodes
        achieved = alg_bytes / (times[dom] * 1e-6) / 1e9
        roofline = {"bound": "hbm", "measured": "L2-miss bandwidth: the 1025^2 working set stays in the 256 MB "
                                                "last-level cache",
                    "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": stored_traffic("aniso1025", kernel_name),
                    "kernel": kernel_name, "avg_us": times[dom], "bytes_per_launch": alg_bytes,
                    "bytes_per_node": bpn, "nodes": nodes,
                    "other_pass_us": times[1 - dom], "levels_0_1": levels01}
    for s in solvers:
        s.close()

    solvers_o = make(other)
    steps_o = max(1, args.steps // 2)
    wall_o, infos_o = run(solvers_o, steps_o, 1)
    for s in solvers_o:
        s.close()
    for i in infos_o:
        if i.status != mg.MG_OK:
            raise SystemExit(f"{other} solve did not converge: {mg.status_string(i.status)} rel_res {i.rel_res:.3e}")

    if args.calibrate_copy:
        calibrate_copy()

    total = unknowns * len(eps_list)
    smoothing = SMOOTHER_NAMES[smoother] if args.smoother else "red-black GS"
    if not args.smoother and args.sor != 1.0:
        smoothing = f"red-black SOR (omega {args.sor:g})"
    out = {
        "metric": "unknowns/s to 1e-10 rel. residual",
        "value": total * args.steps / wall_h,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall_h / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-inner/f64-outer" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"aniso1025: -(eps u_xx + u_yy) = N(0,1) on 1025x1025 nodes, eps in "
                               f"{{{','.join(f'{e:g}' for e in eps_list)}}}, 5-point FD, {smoothing} "
                               f"{args.nu}/{args.nu}, F-cycle to "
                               + (f"{args.levels} levels" if args.levels else "3x3")
                               + f", x0={args.x0}, tol 1e-10",
                   "precision": head},
        "roofline": roofline,
        "cycles": {f"{e:g}": i.cycles for e, i in zip(eps_list, infos_h)},
        "rel_res": {f"{e:g}": i.rel_res for e, i in zip(eps_list, infos_h)},
        "us_per_cycle": {f"{e:g}": 1e6 * i.seconds / max(1, i.cycles) for e, i in zip(eps_list, infos_h)},
        f"value_{other}": total * steps_o / wall_o,
        f"cycles_{other}": {f"{e:g}": i.cycles for e, i in zip(eps_list, infos_o)},
        "speedup_mixed_over_fp64": ((wall_o / steps_o) / (wall_h / args.steps)) if head == "mixed"
        else ((wall_h / args.steps) / (wall_o / steps_o)),
    }
    if rates is not None:
        total_cycles = sum(i.cycles for i in infos_h)
        out["cpu_baseline"] = cpu_baseline_from_rates(
            rates, total_cycles / len(eps_list),
            f"rate per unknown-cycle applied to the {total_cycles} cycles the {len(eps_list)} problems need")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
