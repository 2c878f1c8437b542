"""Throughput of the multigrid F-cycle solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload aniso1025]

A step solves every problem of the workload to a 1e-10 relative residual
(||b - A x_k|| <= 1e-10 ||b - A x_0||) from the stated start vector; inputs are
resident in device memory before the timed region.  `value` is unknowns solved
per second over the timed steps in the headline precision; the other
precision's figure is reported beside it.  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TOL = 1e-10


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="aniso1025", choices=["aniso1025"])
    ap.add_argument("--nu", type=int, default=2)
    ap.add_argument("--x0", default="zero", choices=["zero", "uniform"])
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--max-cycles", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eps", type=float, default=None, help="run one eps of the workload only (profiling)")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; use --gpus 1"}), flush=True)
        sys.exit(2)
    import numpy as np
    import torch

    import workloads as W
    from paper_0805_3041_amd import mg

    n = 1025
    eps_list = list(W.ANISO_EPS) if args.eps is None else [args.eps]
    rhs = torch.tensor(W.aniso_rhs(n, 2), device="cuda")
    x0 = torch.tensor(W.aniso_x0(n, args.x0, 1), device="cuda")
    unknowns = (n - 2) ** 2

    def run(precision, steps, warmup):
        solvers = [mg.Solver(n, n, eps_x=e, smoother="rbgs", nu_pre=args.nu, nu_post=args.nu,
                             precision=precision) for e in eps_list]
        xs = [x0.clone() for _ in eps_list]
        infos = []
        for _ in range(warmup):
            for s, x in zip(solvers, xs):
                x.copy_(x0)
                s.solve(rhs, x, TOL, args.max_cycles, history=False)
        torch.cuda.synchronize()
        dev_s = 0.0
        t0 = time.perf_counter()
        for _ in range(steps):
            infos = []
            for s, x in zip(solvers, xs):
                x.copy_(x0)
                info = s.solve(rhs, x, TOL, args.max_cycles, history=False)
                infos.append(info)
                dev_s += info.seconds
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        for s in solvers:
            s.close()
        return wall, dev_s, infos

    head = args.precision
    other = "fp64" if head == "mixed" else "mixed"
    wall_h, dev_h, infos_h = run(head, args.steps, args.warmup)
    wall_o, dev_o, infos_o = run(other, max(1, args.steps // 2), 1)
    steps_o = max(1, args.steps // 2)
    total = unknowns * len(eps_list)
    value = total * args.steps / wall_h
    out = {
        "metric": "unknowns/s to 1e-10 rel. residual",
        "value": value,
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
        "config": {"workload": "aniso1025: -(eps u_xx + u_yy) = N(0,1), 1025x1025, eps in {1,1e-1,1e-2,1e-3}, "
                               f"red-black GS {args.nu}/{args.nu}, F-cycle, x0={args.x0}",
                   "precision": head},
        "cycles": {f"{e:g}": i.cycles for e, i in zip(eps_list, infos_h)},
        "rel_res": {f"{e:g}": i.rel_res for e, i in zip(eps_list, infos_h)},
        f"value_{other}": total * steps_o / wall_o,
        f"cycles_{other}": {f"{e:g}": i.cycles for e, i in zip(eps_list, infos_o)},
        "speedup_mixed_over_fp64": (wall_o / steps_o) / (wall_h / args.steps) if head == "mixed"
        else (wall_h / args.steps) / (wall_o / steps_o),
        "us_per_cycle": {f"{e:g}": 1e6 * i.seconds / max(1, i.cycles) for e, i in zip(eps_list, infos_h)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
