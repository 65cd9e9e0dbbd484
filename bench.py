#!/usr/bin/env python3
"""Benchmark of the SAC MHD hot path on one MI355X.

Workload: Orszag-Tang vortex, 8000 x 8000 cells on [0, 2pi]^2, periodic, one
GPU's subdomain with 3-cell halos refilled through device pack/unpack
buffers before every stage (periodic self-exchange), hyper-diffusion on,
CFL 0.3, FP64 (default) or FP32 bulk arithmetic.  A step is one full RK4 step
(4 fused stage kernels + 4 halo exchanges + the device dt reduction).

Prints one JSON line: Mcell-updates/s over the timed steps, the roofline
position of the dominant kernel (the fused stage kernel, timed live with HIP
events on its stream) and the FP64 CPU oracle timed on a bounded sample of
the same workload (one RK4 step on a sub-block of the same state).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
METRIC = "Mcell-updates/s & % HBM roofline; plain vs FP32/batched/surrogate at equal error"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(prob, n_sample: int, cfl: float):
    """The oracle (test infrastructure) timed on one RK4 step of an
    n_sample x n_sample sub-block of the workload's own state."""
    import oracle
    oracle.build(force=False)
    cfg = oracle.make_cfg(prob, cfl=cfl)
    f = [prob.fields[k] for k in oracle.FIELDS]
    # global dt / c_max of the full state (needed by the step), not timed
    cx, cy, cmax, dt = oracle.wavespeed(cfg, f)
    m = 12
    idx = np.arange(-m, n_sample + m) % prob.nx
    patch = [a[np.ix_(idx, idx)] for a in f]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    oracle.step_patch(cfg, patch, None, dt, cmax)
    sec = time.perf_counter() - t0
    return {
        "value": n_sample * n_sample / sec / 1e6,
        "unit": "Mcell-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"one RK4 step (HD on) on a {n_sample}x{n_sample} sub-block of the OT {prob.nx}^2 "
                  f"initial state, 12-cell margin supplied; {sec:.2f} s",
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=8000, help="grid side")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--no-hd", action="store_true", help="the paper's 'without HD' column")
    ap.add_argument("--cpu-sample", type=int, default=3072, help="side of the oracle sub-block (0: skip)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs one GPU's subdomain only; --gpus {args.gpus} is not supported "
              f"(multi-GPU halo exchange is a design note, not part of this build).", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1710_06423_amd import FP32, FP64, Solver

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    n = args.n
    prec = FP64 if args.precision == "fp64" else FP32
    w = 8 if prec == FP64 else 4
    hd = not args.no_hd
    log(f"[bench] generating Orszag-Tang {n}x{n}")
    prob = W.orszag_tang(n)
    log("[bench] uploading and initialising")
    s = Solver.from_problem(prob, precision=prec, hd_on=hd, cfl=0.3)
    cpu = None
    if args.cpu_sample > 0:
        log(f"[bench] oracle baseline on a {args.cpu_sample}^2 sub-block")
        cpu = cpu_baseline(prob, min(args.cpu_sample, n), 0.3)
        log(f"[bench] oracle: {cpu['value']:.3f} Mcell-updates/s on {cpu['cores']} threads")
    del prob

    log(f"[bench] warmup {args.warmup} steps")
    if args.warmup:
        s.advance(args.warmup)
    torch.cuda.synchronize()

    stream = s.stream
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    s.profile_enable(True)
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    start.record(stream)
    s.advance(args.steps, sync=False)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    prof = s.profile_read()
    s.profile_enable(False)
    diag = s.diagnostics()
    if diag["nonphys"] or diag["steps"] != args.warmup + args.steps:
        log(f"[bench] run failed: {diag}")
        sys.exit(1)

    cells = n * n
    value = cells * args.steps / (ms / 1e3) / 1e6
    # dominant kernel: the fused stage kernel (four stage instantiations).
    # algorithmic bytes: 12 field accesses x 6 fields x w per cell and step,
    # i.e. 18 w bytes per cell per stage launch on average.
    n_launch = sum(prof["n_stage"])
    stage_ms = sum(prof["ms_stage"])
    avg_launch_s = stage_ms / n_launch / 1e3
    bytes_per_launch = 12 * 6 * w * cells / 4
    achieved = bytes_per_launch / avg_launch_s / 1e9
    per_stage = [prof["ms_stage"][k] / max(prof["n_stage"][k], 1) for k in range(4)]
    t_comp = stage_ms
    t_comm = prof["ms_halo"]
    log(f"[bench] {ms / args.steps:.3f} ms/step; stage launches avg {avg_launch_s * 1e3:.3f} ms "
        f"(per stage {['%.3f' % x for x in per_stage]}); halo {t_comm / max(prof['n_halo'], 1):.3f} ms/exchange; "
        f"tau = ln(T_comp/T_comm) = {math.log(t_comp / t_comm) if t_comm > 0 else float('inf'):.2f}")
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == FP64 else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"orszag_tang_{n}x{n}_{args.precision}_{'hd' if hd else 'nohd'}",
            "nx": n, "ny": n, "precision": args.precision, "hyper_diffusion": hd, "cfl": 0.3,
            "halo": "3-cell, device pack/unpack, periodic self-exchange",
            "bytes_per_cell_update": 12 * 6 * w,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None,
        },
        "cpu_baseline": cpu,
        "phases_ms": {"stage": [round(x, 3) for x in prof["ms_stage"]], "halo": round(t_comm, 3),
                      "scalar": round(prof["ms_scalar"], 3)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
