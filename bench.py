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
the same workload (one RK4 step on a sub-block of the same state, on all
host threads and, in a child process, on one).  The default run also carries
the metric's comparison under "compare": FP32 bulk arithmetic on the same
workload (error against the FP64 run), the batched launch of 64 mixed
instances (sampled instances against the oracle) and the learned coefficient
on Orszag-Tang 2048^2 (error against the plain FP64 path); --no-extras skips
them.

Other modes (one JSON line each):
  --mode batch      64 mixed Brio-Wu / Orszag-Tang instances in one persistent
                    launch (FP32, autotuned tiles) against the same instances
                    run one at a time;
  --mode surrogate  the learned hyper-diffusion coefficient: trained on
                    solver-generated Orszag-Tang data, evaluated on an
                    Orszag-Tang 2048^2 run at refresh intervals K = 1, 4, 16;
  --mode decomposed the same workload split into px x py subdomain contexts
                    on the one GPU (--split, default 2x2), stepped stage by
                    stage with a halo exchange between them before every
                    stage and a device max of the wave speeds per step,
                    beside the undivided run (the cost of the exchange path;
                    the results are compared bit for bit);
  --mode graph      an n x n Orszag-Tang grid (default 1024) stepped by eager
                    launches and by replays of a HIP graph of --graph-steps
                    captured steps (small grids are launch-bound); the two
                    runs end bit-identical;
  --mode 3d         the 3-D scheme: Orszag-Tang carried into z on an n^3
                    grid (default 512^3), FP64, hyper-diffusion on;
  --mode copy       a device copy of known size (calibrates the HBM byte
                    counters of a profiler run), and the streaming rate of a
                    plain elementwise kernel (b = a + 3c, 3 x 4 GiB).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from typing import Optional

import numpy as np

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "Mcell-updates/s & % HBM roofline; plain vs FP32/batched/surrogate at equal error"
# training data of the learned coefficient: seeded Orszag-Tang runs at 256^2
# to 1024^2, snapshots every SUR_EVERY[side] steps up to t = 3
SUR_SIDES = (256, 512, 1024)
SUR_EVERY = {256: 10, 512: 10, 1024: 40}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(prob, n_sample: int, cfl: float):
    """The oracle (test infrastructure) timed on one RK4 step of an
    n_sample x n_sample sub-block of the workload's own state (periodic
    images across periodic edges; with a background, interior rows only)."""
    import oracle
    oracle.build(force=False)
    cfg = oracle.make_cfg(prob, cfl=cfl)
    f = [prob.fields[k] for k in oracle.FIELDS]
    bg = None if prob.background is None else [prob.background[k] for k in oracle.BACKGROUND_FIELDS]
    # global dt / c_max of the full state (needed by the step), not timed
    cx, cy, cmax, dt = oracle.wavespeed(cfg, f, bg)
    m = 12
    ix = np.arange(-m, n_sample + m) % prob.nx
    if bg is None:
        iy = np.arange(-m, n_sample + m) % prob.ny
    else:
        n_sample = min(n_sample, prob.ny - 2 * m)
        y0 = (prob.ny - n_sample) // 2
        iy = np.arange(y0 - m, y0 + n_sample + m)
        ix = np.arange(-m, n_sample + m) % prob.nx
    patch = [a[np.ix_(iy, ix)] for a in f]
    bgp = None if bg is None else [a[np.ix_(iy, ix)] for a in bg]
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    oracle.step_patch(cfg, patch, bgp, dt, cmax)
    sec = time.perf_counter() - t0
    model = "unknown CPU"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": n_sample * n_sample / sec / 1e6,
        "unit": "Mcell-updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"one RK4 step (HD on) on a {n_sample}x{n_sample} sub-block of the {prob.name} "
                  f"initial state, 12-cell margin supplied; {sec:.2f} s on {threads} OpenMP threads of {model}",
    }


def traffic_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"k_stage_{workload}_traffic.md")


def rel_l2(a, b) -> float:
    import torch
    a = a.to(torch.float64)
    b = b.to(torch.float64)
    nb = float(torch.linalg.vector_norm(b))
    d = float(torch.linalg.vector_norm(a - b))
    return d / nb if nb > 0 else d


def base_record(args, metric_value, ms_step, dtype, config):
    return {
        "metric": METRIC,
        "value": round(metric_value, 3),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
    }


def oracle_one_thread(n_sample: int):
    """The oracle at one thread on an n_sample^2 sub-block of the headline
    state, in a child process (OMP_NUM_THREADS is read when the OpenMP
    runtime starts), started before this process touches the GPU."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--mode", "oracle-sample", "--n", "8000",
                        "--cpu-sample", str(n_sample)], capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr.strip()[-400:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


W2_SAMPLE_STEPS = 10


def run_oracle_workloads(args):
    """The oracle on the two smaller workloads: Brio-Wu 800 to t = 0.1 in
    full, and the first W2_SAMPLE_STEPS steps of Orszag-Tang 1024^2; on the
    threads OpenMP was started with."""
    import oracle
    import workloads as W
    out = {"threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)), "nproc": os.cpu_count(),
           "cpu": cpu_model()}
    bw = W.brio_wu(800)
    st = oracle.State(bw, form=oracle.LOWSTORE)
    t0 = time.perf_counter()
    done = st.run(100000, t_end=0.1)
    sec = time.perf_counter() - t0
    out["brio_wu_800"] = {"steps": done, "t": st.t, "seconds": round(sec, 3),
                          "mcell_updates_s": round(800 * done / sec / 1e6, 3)}
    ot = W.orszag_tang(1024)
    st = oracle.State(ot, form=oracle.LOWSTORE)
    t0 = time.perf_counter()
    done = st.run(W2_SAMPLE_STEPS)
    sec = time.perf_counter() - t0
    out["orszag_tang_1024"] = {"steps": done, "seconds": round(sec, 3),
                               "mcell_updates_s": round(1024 * 1024 * done / sec / 1e6, 3)}
    print(json.dumps(out), flush=True)


def oracle_workloads(threads: Optional[int]):
    """run_oracle_workloads in a child process (OpenMP reads its thread count
    when it starts), on `threads` threads or the inherited setting."""
    import subprocess
    env = dict(os.environ)
    if threads is not None:
        env["OMP_NUM_THREADS"] = str(threads)
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--mode", "oracle-workloads"],
                       capture_output=True, text=True, env=env, timeout=600)
    if r.returncode != 0:
        return {"error": r.stderr.strip()[-400:]}
    return json.loads(r.stdout.strip().splitlines()[-1])


def sub_workloads(args):
    """Brio-Wu 800 to t = 0.1 and Orszag-Tang 1024^2 (200 steps) on the GPU,
    FP64, beside the oracle's rates on the same workloads (all threads and one
    thread, timed before the GPU was touched)."""
    import workloads as W
    from paper_1710_06423_amd import FP64, Solver
    res = {}
    bw = Solver.from_problem(W.brio_wu(800), precision=FP64)
    bw.advance(2)
    bw.close()
    bw = Solver.from_problem(W.brio_wu(800), precision=FP64)
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done, t = bw.advance(100000, t_end=0.1)
    sec = time.perf_counter() - t0
    bw.close()
    res["brio_wu_800"] = {"steps": done, "t": t, "seconds": round(sec, 4),
                          "mcell_updates_s": round(800 * done / sec / 1e6, 3),
                          "note": "one 800-cell tube: launch-bound, timed on the host around the synchronising advance"}
    ot = Solver.from_problem(W.orszag_tang(1024), precision=FP64)
    ms = timed_advance(ot, 200, 2)
    ot.close()
    res["orszag_tang_1024"] = {"steps": 200, "ms_per_step": round(ms / 200, 4),
                               "mcell_updates_s": round(1024 * 1024 * 200 / (ms / 1e3) / 1e6, 1)}
    res["oracle_all_threads"] = args.cpu_workloads[0]
    res["oracle_1thread"] = args.cpu_workloads[1]
    res["oracle_note"] = (f"the oracle's Orszag-Tang 1024^2 rate is over its first {W2_SAMPLE_STEPS} steps; "
                          "Brio-Wu 800 is the full run to t = 0.1")
    return res


def run_oracle_sample(args):
    import workloads as W
    out = cpu_baseline(W.orszag_tang(args.n), args.cpu_sample, 0.3)
    out["nproc"] = os.cpu_count()
    print(json.dumps(out), flush=True)


def timed_advance(s, steps, warmup):
    import torch
    if warmup:
        s.advance(warmup)
    torch.cuda.synchronize()
    a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a0.record(s.stream)
    s.advance(steps, sync=False)
    a1.record(s.stream)
    torch.cuda.synchronize()
    return a0.elapsed_time(a1)


def sub_fp32(args, ref_fields, t_ref):
    """FP32 bulk arithmetic on the headline workload, same warm-up and timed
    steps; per-field relative L2 against the FP64 run's final state."""
    import torch
    import workloads as W
    from paper_1710_06423_amd import FP32, Solver
    s = Solver.from_problem(W.orszag_tang(args.n), precision=FP32, cfl=0.3)
    ms = timed_advance(s, args.steps, args.warmup)
    a = s.read_fields(torch.float64)
    t = s.diagnostics()["t"]
    s.close()
    names = ("rho", "mx", "my", "e", "bx", "by")
    return {"mcell_updates_s": round(args.n * args.n * args.steps / (ms / 1e3) / 1e6, 1),
            "ms_per_step": round(ms / args.steps, 4), "dtype": "f32 bulk, f64 dt and sums",
            "roofline_frac_algorithmic": round(288 * args.n * args.n * args.steps / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "rel_l2_vs_fp64": {names[k]: float("%.3e" % rel_l2(a[k], ref_fields[k])) for k in range(6)},
            "steps_compared": args.warmup + args.steps, "t": t, "t_fp64": t_ref}


def sub_batch(args):
    """64 mixed instances in one persistent launch (FP32, autotuned tiles),
    100 steps; beside it the same instances run one at a time in FP64 (rate,
    and every instance's error against its FP64 run), and sampled instances
    against the FP64 oracle."""
    import torch
    import oracle
    import workloads as W
    from paper_1710_06423_amd import FP32, FP64, Batch, Solver
    from paper_1710_06423_amd.autotune import tune_batch
    probs = W.batch_instances(seed=0)
    cells = sum(p.nx * p.ny for p in probs)
    b = Batch(probs, precision=FP32)
    t, r, _ = tune_batch(b, use_cache=False, log=lambda *a: None)
    b.close()
    b = Batch(probs, precision=FP32)
    b.set_tiles(t, [r] * len(probs))
    steps = 100
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.advance(steps, sync=False)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    value = cells * steps / (ms / 1e3) / 1e6
    # the same instances one at a time in FP64 (each its own context and launches)
    seq_ms, worst = 0.0, 0.0
    for i, p in enumerate(probs):
        s = Solver.from_problem(p, precision=FP64)
        torch.cuda.synchronize()
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record(s.stream)
        s.advance(steps, sync=False)
        a1.record(s.stream)
        torch.cuda.synchronize()
        seq_ms += a0.elapsed_time(a1)
        x, y = b[i].read_fields(torch.float64), s.read_fields(torch.float64)
        worst = max(worst, max(rel_l2(x[k], y[k]) for k in range(6)))
        s.close()
    seq = cells * steps / (seq_ms / 1e3) / 1e6
    # sampled against the oracle: the two smallest tubes and the two smallest boxes
    bw = sorted((i for i, p in enumerate(probs) if p.ny == 1), key=lambda i: probs[i].nx)[:2]
    ot = sorted((i for i, p in enumerate(probs) if p.ny > 1), key=lambda i: probs[i].nx * probs[i].ny)[:2]
    oracle.build(force=False)
    errs = {}
    for i in bw + ot:
        got = b[i].read_fields(torch.float64).cpu().numpy()
        ref = oracle.State(probs[i], form=oracle.LOWSTORE)
        ref.run(steps)
        want = ref.stacked()
        errs[f"{'briowu' if probs[i].ny == 1 else 'orszag_tang'}_{probs[i].nx}x{probs[i].ny}"] = float(
            "%.3e" % max(oracle.rel_l2(got[k], want[k]) for k in range(6)))
    b.close()
    return {"mcell_updates_s": round(value, 1), "ms_per_step": round(ms / steps, 4),
            "instances": len(probs), "cells": cells, "steps": steps, "tiles": {"threads": t, "rows2d": r},
            "dtype": "f32 bulk, f64 dt and sums",
            "one_at_a_time_fp64_mcell_updates_s": round(seq, 1), "speedup_vs_one_at_a_time_fp64": round(value / seq, 2),
            "max_rel_l2_vs_one_at_a_time_fp64": float("%.3e" % worst), "sampled_max_rel_l2_vs_oracle": errs}


def phase_profile(s, steps=32):
    """The library's own HIP-event timings (sacx_profile_*) over `steps` more
    steps of a context: per step its stage kernels and halo fills, per
    refresh of a learned coefficient the refresh (network inputs, network,
    check).  Taken after the timed region; the events cost a little time."""
    s.profile_enable(True)
    s.advance(steps)
    p = s.profile_read()
    s.profile_enable(False)
    return {"steps": steps, "stage_ms_per_step": round(sum(p["ms_stage"]) / steps, 4),
            "halo_ms_per_step": round(p["ms_halo"] / steps, 4),
            "refresh_ms": round(p["ms_surrogate"] / p["n_surrogate"], 4) if p["n_surrogate"] else None,
            "refreshes": p["n_surrogate"]}


def all_fallback_run(sur, prob, norm, K, tile, bound, steps, warmup=2):
    """Time a surrogate run whose network has zero weights, so that every
    check falls back everywhere: (ms, fallback tile fraction)."""
    import torch
    from paper_1710_06423_amd import FP64, Solver
    from paper_1710_06423_amd.sacx import CHECK_FLUX, CNN_NPARAM
    zero = sur.Network(torch.zeros(CNN_NPARAM, dtype=torch.float32))
    s = Solver.from_problem(prob, precision=FP64)
    s.set_surrogate(zero.packed, norm, refresh_every=K, tile=tile, bound=bound, metric=CHECK_FLUX)
    ms = timed_advance(s, steps, warmup)
    st = s.hd_stats()
    prof = phase_profile(s)
    s.close()
    return ms, round(st["tiles_fallback"] / max(st["tiles_checked"], 1), 4), prof


def sub_surrogate(args, log_every=1000):
    """The learned coefficient on Orszag-Tang 2048^2, 500 steps, refresh
    every 16 steps (and, briefer, every 1 and 4), flux bound 0.05: trained on
    solver-generated data by the library's own kernels, against the plain
    FP64 path."""
    import workloads as W
    from paper_1710_06423_amd import FP64, Solver
    from paper_1710_06423_amd import surrogate as sur
    from paper_1710_06423_amd.sacx import CHECK_FLUX
    t0 = time.time()
    data = sur.generate(sides=SUR_SIDES, seeds=tuple(range(1, 9)), snap_every=SUR_EVERY, t_end=3.0, log=lambda *a: None)
    gen_s = time.time() - t0
    net = sur.Network(seed=0)
    t1 = time.time()
    sur.train(net, data, iters=6000, batch_pixels=1 << 19, lr=2e-3, lr_end=1e-4, log=lambda *a: None,
              log_every=log_every)
    train_s = time.time() - t1
    n, steps, K, bound = 2048, 500, 16, 0.05
    prob = W.orszag_tang(n)
    plain = Solver.from_problem(prob, precision=FP64)
    ms_plain = timed_advance(plain, steps, 2)
    ref = plain.read_fields()
    plain.close()
    s = Solver.from_problem(prob, precision=FP64)
    s.set_surrogate(net.packed, data.norm, refresh_every=K, tile=16, bound=bound, metric=CHECK_FLUX)
    ms = timed_advance(s, steps, 2)
    st = s.hd_stats()
    a = s.read_fields()
    prof = phase_profile(s)
    s.close()
    names = ("rho", "mx", "my", "e", "bx", "by")
    # the other refresh intervals of the comparison
    other = {}
    for k in (1, 4):
        s = Solver.from_problem(prob, precision=FP64)
        s.set_surrogate(net.packed, data.norm, refresh_every=k, tile=16, bound=bound, metric=CHECK_FLUX)
        ms_k = timed_advance(s, steps, 2)
        st_k = s.hd_stats()
        a_k = s.read_fields()
        s.close()
        other[str(k)] = {"mcell_updates_s": round(n * n * steps / (ms_k / 1e3) / 1e6, 1),
                         "fallback_tile_fraction": round(st_k["tiles_fallback"] / max(st_k["tiles_checked"], 1), 4),
                         "max_rel_l2_vs_plain_fp64": float("%.3e" % max(rel_l2(a_k[f], ref[f]) for f in range(6)))}
    # the same run with a network that is never kept (zero weights predict 2
    # everywhere): what the refreshes and the check cost on their own
    ms0, fb0, prof0 = all_fallback_run(sur, prob, data.norm, K, 16, bound, steps)
    return {"workload": f"orszag_tang_{n}x{n}_fp64_hd_learned_coefficient", "steps": steps, "refresh_every": K,
            "bound": bound, "check": "flux, 16^2 tiles",
            "mcell_updates_s": round(n * n * steps / (ms / 1e3) / 1e6, 1),
            "plain_mcell_updates_s": round(n * n * steps / (ms_plain / 1e3) / 1e6, 1),
            "all_fallback_mcell_updates_s": round(n * n * steps / (ms0 / 1e3) / 1e6, 1),
            "all_fallback_tile_fraction": fb0,
            "all_fallback_phases": prof0,
            "fallback_tile_fraction": round(st["tiles_fallback"] / max(st["tiles_checked"], 1), 4),
            "phases": prof,
            "err_used": float("%.3e" % st["err_used"]),
            "rel_l2_vs_plain_fp64": {names[k]: float("%.3e" % rel_l2(a[k], ref[k])) for k in range(6)},
            "refresh_every_1_and_4": other,
            "training": {"sides": list(SUR_SIDES), "snap_every": {str(k): v for k, v in SUR_EVERY.items()},
                         "seeds": list(range(1, 9)), "snapshots": int(sum(v.shape[0] for v in data.x.values())),
                         "generate_s": round(gen_s, 1), "iterations": 6000, "train_s": round(train_s, 1)}}


def run_single(args):
    import torch
    import workloads as W
    from paper_1710_06423_amd import FP32, FP64, Solver
    from paper_1710_06423_amd.profiling import read_traffic

    n = args.n
    prec = FP64 if args.precision == "fp64" else FP32
    w = 8 if prec == FP64 else 4
    hd = not args.no_hd
    strat = args.problem == "stratified"
    workload = f"{args.problem}_{n}x{n}_{args.precision}_{'hd' if hd else 'nohd'}"
    log(f"[bench] generating {args.problem} {n}x{n}")
    prob = W.stratified_atmosphere(n, n, amp=0.05, b_b=(0.1, 0.4)) if strat else W.orszag_tang(n)
    log("[bench] uploading and initialising")
    s = Solver.from_problem(prob, precision=prec, hd_on=hd, cfl=0.3)
    ref = None
    if args.fp32_error and prec == FP32:
        ref = Solver.from_problem(prob, precision=FP64, hd_on=hd, cfl=0.3)
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
    # i.e. 18 w bytes per cell per stage launch on average; a background adds
    # its 4 fields, read once per stage launch.
    acc = 12 * 6 + (16 if strat else 0)
    n_launch = sum(prof["n_stage"])
    stage_ms = sum(prof["ms_stage"])
    avg_launch_s = stage_ms / n_launch / 1e3
    bytes_per_launch = acc * w * cells / 4
    achieved = bytes_per_launch / avg_launch_s / 1e9
    per_stage = [prof["ms_stage"][k] / max(prof["n_stage"][k], 1) for k in range(4)]
    t_comp = stage_ms
    t_comm = prof["ms_halo"]
    log(f"[bench] {ms / args.steps:.3f} ms/step; stage launches avg {avg_launch_s * 1e3:.3f} ms "
        f"(per stage {['%.3f' % x for x in per_stage]}); halo {t_comm / max(prof['n_halo'], 1):.3f} ms/exchange; "
        f"tau = ln(T_comp/T_comm) = {math.log(t_comp / t_comm) if t_comm > 0 else float('inf'):.2f}")
    tr = read_traffic(traffic_file(workload))
    traffic = None if tr is None else round(tr["traffic_bytes_per_launch"] / avg_launch_s / 1e9, 1)
    out = base_record(args, value, ms / args.steps, "f64" if prec == FP64 else "f32", {
        "workload": workload,
        "nx": n, "ny": n, "precision": args.precision, "hyper_diffusion": hd, "cfl": 0.3,
        "halo": ("3-cell; x periodic self-exchange, y open (zero-gradient fills)" if strat
                 else "3-cell, device pack/unpack, periodic self-exchange"),
        "bytes_per_cell_update": acc * w,
    })
    if strat:
        out["config"].update({"background": "isothermal hydrostatic, scale height 0.25, uniform field (0.1, 0.4)",
                              "gravity": [0.0, -1.0], "pulse_amplitude": 0.05})
    out["roofline"] = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
    }
    if tr is not None:
        out["roofline"]["traffic_over_algorithmic"] = round(tr["traffic_bytes_per_launch"] / bytes_per_launch, 3)
    if args.mode == "single":
        # beside the spec, what a plain streaming kernel reaches on this GPU
        # (measured after the timed region)
        stream_gbs = streaming_rate()
        log(f"[bench] streaming rate of a plain elementwise kernel: {stream_gbs:.1f} GB/s")
        out["roofline"]["achievable"] = round(stream_gbs, 1)
        out["roofline"]["frac_of_achievable"] = round(achieved / stream_gbs, 4)
        out["roofline"]["achievable_kernel"] = "b = a + 3c over three 4 GiB float64 arrays, best of 5"
    out["cpu_baseline"] = cpu
    out["phases_ms"] = {"stage": [round(x, 3) for x in prof["ms_stage"]], "halo": round(t_comm, 3),
                        "scalar": round(prof["ms_scalar"], 3)}
    if n == 8000 and hd and not strat:
        # the paper's own timing of this workload, on its hardware: context only
        out["paper_context"] = {"mcell_updates_s": 39.1, "hardware": "100x NVIDIA Tesla K20c (10x10 subdomains)",
                                "source": "Table 1, Orszag-Tang 8000^2 with hyper-diffusion, 163.6 s per 100 "
                                          "iterations; precision not stated"}
    extras = args.mode == "single" and not args.no_extras and n == 8000 and hd and not strat and prec == FP64
    if extras:
        # the metric's comparison: FP32, batched and learned forms beside the
        # plain FP64 path (each at its stated error), and the oracle at one thread
        t_ref = diag["t"]
        fields = s.read_fields()
        s.close()
        subs = {}
        subs_fns = [("fp32_8000", lambda: sub_fp32(args, fields, t_ref)), ("batch64", lambda: sub_batch(args)),
                    ("learned_coefficient_2048_k16", lambda: sub_surrogate(args)),
                    ("orszag_tang_3d_512", lambda: sub_3d(args))]
        if args.cpu_workloads is not None:
            subs_fns.append(("smaller_workloads", lambda: sub_workloads(args)))
        for name, fn in subs_fns:
            log(f"[bench] sub-record {name}")
            try:
                subs[name] = fn()
            except Exception as e:  # recorded, so the headline line still prints
                subs[name] = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] {name}: {subs[name]}")
        del fields
        out["compare"] = subs
        if args.one_thread is not None:
            out["cpu_baseline_1thread"] = args.one_thread
    if ref is not None:
        log("[bench] FP64 reference run for the FP32 error")
        ref.advance(args.warmup + args.steps)
        a, b = s.read_fields(torch.float64), ref.read_fields(torch.float64)
        names = ("rho", "mx", "my", "e", "bx", "by")
        out["error_vs_fp64"] = {names[k]: float("%.3e" % rel_l2(a[k], b[k])) for k in range(6)}
        out["error_vs_fp64"]["t"] = s.diagnostics()["t"]
        out["error_vs_fp64"]["t_fp64"] = ref.diagnostics()["t"]
    print(json.dumps(out), flush=True)


def run_decomposed(args):
    import torch
    import workloads as W
    from paper_1710_06423_amd import FP32, FP64, DecomposedSolver, Solver, even_cuts

    n = args.n
    px, py = (int(v) for v in args.split.lower().split("x"))
    prec = FP64 if args.precision == "fp64" else FP32
    log(f"[bench] generating orszag_tang {n}x{n}, split {px}x{py}")
    prob = W.orszag_tang(n)
    stream = torch.cuda.Stream()
    dec = DecomposedSolver(prob, even_cuts(n, px), even_cuts(n, py), precision=prec, stream=stream)
    one = Solver.from_problem(prob, precision=prec, stream=stream)
    del prob
    subs = [s for row in dec.subs for s in row]
    log(f"[bench] warmup {args.warmup} steps")
    dec.advance(args.warmup)
    one.advance(args.warmup)
    torch.cuda.synchronize()

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    log(f"[bench] timing {args.steps} decomposed steps")
    ms_dec = timed(lambda: dec.advance(args.steps))
    g = max(1, min(args.graph_steps, args.steps))
    reps = args.steps // g
    log(f"[bench] capturing {g} decomposed steps into a graph, timing {reps} replays")
    graph = dec.graph(g)
    ms_graph = timed(lambda: [graph.replay() for _ in range(reps)]) * args.steps / (reps * g)
    # the phase split from a separate profiled run (the events it records
    # around every launch group slow the run down)
    nprof = min(args.steps, 5)
    for s in subs:
        s.profile_enable(True)
    timed(lambda: dec.advance(nprof))
    profs = [s.profile_read() for s in subs]
    for s in subs:
        s.profile_enable(False)
    log(f"[bench] timing {args.steps} undivided steps")
    ms_one = timed(lambda: one.advance(args.steps, sync=False))
    one.advance(reps * g + nprof)
    diags = [s.diagnostics() for s in subs] + [one.diagnostics()]
    if any(d["nonphys"] or d["steps"] != args.warmup + args.steps + reps * g + nprof for d in diags):
        log(f"[bench] run failed: {diags}")
        sys.exit(1)
    same = bool(torch.equal(dec.read_fields(torch.float64), one.read_fields(torch.float64)))
    cells = n * n
    value = cells * args.steps / (ms_dec / 1e3) / 1e6
    stage_ms = sum(sum(p["ms_stage"]) for p in profs) / nprof
    halo_ms = sum(p["ms_halo"] for p in profs) / nprof
    log(f"[bench] decomposed {ms_dec / args.steps:.3f} ms/step (graph {ms_graph / args.steps:.3f}), undivided "
        f"{ms_one / args.steps:.3f}; profiled: stage kernels {stage_ms:.3f}, halo fills and exchange {halo_ms:.3f} "
        f"ms/step; bit-identical: {same}")
    out = base_record(args, value, ms_dec / args.steps, "f64" if prec == FP64 else "f32", {
        "workload": f"orszag_tang_{n}x{n}_{args.precision}_hd_decomposed_{px}x{py}",
        "nx": n, "ny": n, "precision": args.precision, "hyper_diffusion": True, "cfl": 0.3,
        "subdomains": [px, py],
        "halo": "3-cell; every side exchanged with a neighbour subdomain (periodic images included) "
                "through device pack/unpack buffers before every stage",
    })
    out["undivided"] = {"value": round(cells * args.steps / (ms_one / 1e3) / 1e6, 3),
                        "ms_per_step": round(ms_one / args.steps, 4)}
    out["overhead_vs_undivided"] = round(ms_dec / ms_one - 1.0, 4)
    out["graph"] = {"steps_per_graph": g, "ms_per_step": round(ms_graph / args.steps, 4),
                    "value": round(cells * args.steps / (ms_graph / 1e3) / 1e6, 3),
                    "overhead_vs_undivided": round(ms_graph / ms_one - 1.0, 4)}
    out["phases_ms_per_step"] = {"stage": round(stage_ms, 3), "halo": round(halo_ms, 3),
                                 "tau": round(math.log(stage_ms / halo_ms), 3) if halo_ms > 0 else None,
                                 "profiled_steps": nprof}
    out["bit_identical_to_undivided"] = same
    print(json.dumps(out), flush=True)


def run_graph(args):
    import torch
    import workloads as W
    from paper_1710_06423_amd import FP32, FP64, Solver

    n = args.n
    prec = FP64 if args.precision == "fp64" else FP32
    g = max(1, min(args.graph_steps, args.steps))
    reps = max(1, args.steps // g)
    steps = reps * g
    log(f"[bench] orszag_tang {n}x{n} {args.precision}: eager vs a graph of {g} steps x {reps}")
    prob = W.orszag_tang(n)
    stream = torch.cuda.Stream()
    eager = Solver.from_problem(prob, precision=prec, stream=stream)
    graphed = Solver.from_problem(prob, precision=prec, stream=stream)
    del prob
    eager.advance(args.warmup)
    graphed.advance(args.warmup)
    graph = graphed.graph(g)

    def timed(fn):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b)

    ms_eager = timed(lambda: eager.advance(steps, sync=False))
    ms_graph = timed(lambda: [graph.replay() for _ in range(reps)])
    de, dg = eager.diagnostics(), graphed.diagnostics()
    if de["nonphys"] or dg["nonphys"] or de["steps"] != dg["steps"] or de["steps"] != args.warmup + steps:
        log(f"[bench] run failed: {de} {dg}")
        sys.exit(1)
    same = bool(torch.equal(eager.read_fields(torch.float64), graphed.read_fields(torch.float64)))
    cells = n * n
    value = cells * steps / (ms_graph / 1e3) / 1e6
    log(f"[bench] eager {ms_eager / steps:.4f} ms/step, graph {ms_graph / steps:.4f} ms/step; bit-identical: {same}")
    out = base_record(args, value, ms_graph / steps, "f64" if prec == FP64 else "f32", {
        "workload": f"orszag_tang_{n}x{n}_{args.precision}_hd_graph{g}",
        "nx": n, "ny": n, "precision": args.precision, "hyper_diffusion": True, "cfl": 0.3,
        "steps_per_graph": g,
    })
    out["steps"] = steps
    out["eager"] = {"value": round(cells * steps / (ms_eager / 1e3) / 1e6, 3), "ms_per_step": round(ms_eager / steps, 4)}
    out["speedup_vs_eager"] = round(ms_eager / ms_graph, 4)
    out["bit_identical_to_eager"] = same
    print(json.dumps(out), flush=True)


def run_batch(args):
    import torch
    import workloads as W
    from paper_1710_06423_amd import FP32, FP64, Batch, Solver
    from paper_1710_06423_amd.autotune import tune_batch

    probs = W.batch_instances(seed=0)
    cells = sum(p.nx * p.ny for p in probs)
    log(f"[bench] batch of {len(probs)} instances, {cells} cells")
    b = Batch(probs, precision=FP32)
    t, r, trials = tune_batch(b, use_cache=False, log=log)
    log(f"[bench] tiles: {t} threads, {r} rows")
    b.close()
    b2 = Batch(probs, precision=FP32)
    b2.set_tiles(t, [r] * len(probs))
    if args.warmup:
        b2.advance(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(b2.stream)
    b2.advance(args.steps, sync=False)
    e1.record(b2.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    value = cells * args.steps / (ms / 1e3) / 1e6
    seq = {}
    errs = []
    for prec, name in ((FP32, "fp32"), (FP64, "fp64")):
        tot = 0.0
        for i, p in enumerate(probs):
            s = Solver.from_problem(p, precision=prec)
            if args.warmup:
                s.advance(args.warmup)
            torch.cuda.synchronize()
            a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a0.record(s.stream)
            s.advance(args.steps, sync=False)
            a1.record(s.stream)
            torch.cuda.synchronize()
            tot += a0.elapsed_time(a1)
            if prec == FP64:
                x, y = b2[i].read_fields(torch.float64), s.read_fields(torch.float64)
                errs.append(max(rel_l2(x[k], y[k]) for k in range(6)))
            s.close()
        seq[name] = cells * args.steps / (tot / 1e3) / 1e6
        log(f"[bench] one at a time, {name}: {tot / args.steps:.3f} ms/step -> {seq[name]:.1f} Mcell-updates/s")
    b2.close()
    out = base_record(args, value, ms / args.steps, "f32", {
        "workload": "batch64_briowu32_orszagtang32_fp32", "instances": len(probs), "cells": cells,
        "tiles": {"threads": t, "rows2d": r},
    })
    out["roofline"] = None
    out["cpu_baseline"] = None
    out["sequential_mcell_updates_s"] = {k: round(v, 1) for k, v in seq.items()}
    out["speedup_vs_sequential"] = {k: round(value / v, 2) for k, v in seq.items()}
    out["max_rel_l2_vs_fp64"] = float("%.3e" % max(errs))
    out["autotune_trials_ms"] = [[a, b_, round(c, 4)] for a, b_, c in trials]
    print(json.dumps(out), flush=True)


def run_surrogate(args):
    import torch
    import workloads as W
    from paper_1710_06423_amd import FP64, Solver
    from paper_1710_06423_amd import surrogate as sur
    from paper_1710_06423_amd.sacx import CHECK_FLUX

    t0 = time.time()
    data = sur.generate(sides=SUR_SIDES, seeds=tuple(range(1, 9)), snap_every=SUR_EVERY, t_end=3.0,
                        max_snaps=args.max_snaps, log=log)
    log(f"[bench] data: {sum(v.shape[0] for v in data.x.values())} snapshots in {time.time() - t0:.1f} s")
    net = sur.Network(seed=0)
    e0 = sur.evaluate(net, data)
    t1 = time.time()
    sur.train(net, data, iters=args.train_iters, batch_pixels=1 << 19, lr=2e-3, lr_end=1e-4, log=log,
              log_every=max(1, args.train_iters // 6))
    torch.cuda.synchronize()
    train_s = time.time() - t1
    e1 = sur.evaluate(net, data)
    log(f"[bench] trained {args.train_iters} iterations in {train_s:.1f} s; loss {e0:.3e} -> {e1:.3e}")

    n = args.n
    prob = W.orszag_tang(n)

    def timed(s):
        if args.warmup:
            s.advance(args.warmup)
        torch.cuda.synchronize()
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record(s.stream)
        s.advance(args.steps, sync=False)
        a1.record(s.stream)
        torch.cuda.synchronize()
        return a0.elapsed_time(a1)

    plain = Solver.from_problem(prob, precision=FP64)
    ms_plain = timed(plain)
    ref = plain.read_fields()
    prof_plain = phase_profile(plain)
    names = ("rho", "mx", "my", "e", "bx", "by")
    runs = {}
    for K in (1, 4, 16):
        s = Solver.from_problem(prob, precision=FP64)
        s.set_surrogate(net.packed, data.norm, refresh_every=K, tile=args.tile, bound=args.bound, metric=CHECK_FLUX)
        ms = timed(s)
        st = s.hd_stats()
        a = s.read_fields()
        runs[f"K{K}"] = {
            "mcell_updates_s": round(n * n * args.steps / (ms / 1e3) / 1e6, 1),
            "ms_per_step": round(ms / args.steps, 4),
            "kept_tile_fraction": round(1 - st["tiles_fallback"] / st["tiles_checked"], 4),
            "err_used": float("%.3e" % st["err_used"]),
            "rel_l2_vs_plain": {names[k]: float("%.3e" % rel_l2(a[k], ref[k])) for k in range(6)},
            "phases": phase_profile(s),
        }
        log(f"[bench] K={K}: {runs[f'K{K}']}")
        s.close()
        ms0, fb0, prof0 = all_fallback_run(sur, prob, data.norm, K, args.tile, args.bound, args.steps, args.warmup)
        runs[f"K{K}_all_fallback"] = {
            "mcell_updates_s": round(n * n * args.steps / (ms0 / 1e3) / 1e6, 1),
            "ms_per_step": round(ms0 / args.steps, 4),
            "fallback_tile_fraction": fb0,
            "phases": prof0,
        }
        log(f"[bench] K={K} zero network: {runs[f'K{K}_all_fallback']}")
    # the same with FP32 bulk arithmetic (the speed here comes from FP32; the
    # errors are against the FP64 plain run)
    from paper_1710_06423_amd import FP32
    p32 = Solver.from_problem(prob, precision=FP32)
    ms_p32 = timed(p32)
    b32 = p32.read_fields()
    runs["fp32_plain"] = {
        "mcell_updates_s": round(n * n * args.steps / (ms_p32 / 1e3) / 1e6, 1),
        "ms_per_step": round(ms_p32 / args.steps, 4),
        "rel_l2_vs_plain": {names[k]: float("%.3e" % rel_l2(b32[k], ref[k])) for k in range(6)},
    }
    p32.close()
    s = Solver.from_problem(prob, precision=FP32)
    s.set_surrogate(net.packed, data.norm, refresh_every=16, tile=args.tile, bound=args.bound, metric=CHECK_FLUX)
    ms = timed(s)
    st = s.hd_stats()
    a = s.read_fields()
    runs["fp32_K16"] = {
        "mcell_updates_s": round(n * n * args.steps / (ms / 1e3) / 1e6, 1),
        "ms_per_step": round(ms / args.steps, 4),
        "kept_tile_fraction": round(1 - st["tiles_fallback"] / st["tiles_checked"], 4),
        "err_used": float("%.3e" % st["err_used"]),
        "rel_l2_vs_plain": {names[k]: float("%.3e" % rel_l2(a[k], ref[k])) for k in range(6)},
    }
    log(f"[bench] fp32: {runs['fp32_plain']} / K=16: {runs['fp32_K16']}")
    s.close()
    best = max((runs[k] for k in ("K1", "K4", "K16")), key=lambda r: r["mcell_updates_s"])
    plain_v = n * n * args.steps / (ms_plain / 1e3) / 1e6
    out = base_record(args, best["mcell_updates_s"], best["ms_per_step"], "f64", {
        "workload": f"orszag_tang_{n}x{n}_fp64_hd_learned_coefficient", "nx": n, "ny": n,
        "check": {"metric": "flux", "bound": args.bound, "tile": args.tile},
        "training": {"sides": list(SUR_SIDES), "seeds": list(range(1, 9)),
                     "snap_every": {str(k): v for k, v in SUR_EVERY.items()}, "t_end": 3.0,
                     "iterations": args.train_iters, "seconds": round(train_s, 1),
                     "loss_before": float("%.3e" % e0), "loss_after": float("%.3e" % e1)},
    })
    out["roofline"] = None
    out["cpu_baseline"] = None
    out["plain_mcell_updates_s"] = round(plain_v, 1)
    out["plain_phases"] = prof_plain
    out["runs"] = runs
    print(json.dumps(out), flush=True)


def sub_3d(args, n=512, steps=5, warmup=2):
    """The 3-D scheme on Orszag-Tang carried into z at n^3, FP64, hyper-
    diffusion on: its rate and algorithmic HBM fraction over `steps` steps."""
    import torch
    import workloads as W
    from paper_1710_06423_amd.sacx3 import Solver3
    s = Solver3.from_problem(W.orszag_tang_3d(n), cfl=0.3)
    s.advance(warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.advance(steps, sync=False)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    d = s.diagnostics()
    s.close()
    if d["nonphys"] or d["steps"] != warmup + steps:
        raise RuntimeError(f"3-D run failed: {d}")
    alg = 12 * 8 * 8
    out = {"workload": f"orszag_tang_3d_{n}^3_fp64_hd", "steps": steps,
           "mcell_updates_s": round(n ** 3 * steps / (ms / 1e3) / 1e6, 1), "ms_per_step": round(ms / steps, 3),
           "roofline_frac_algorithmic": round(alg * n ** 3 / (ms / steps / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
           "parity": "bit-identical to the 3-D oracle (GPU tests)"}
    # the 3-D oracle beside it: one step of the same problem at a small size
    from oracle import oracle3d as O3
    O3.build(force=False)
    m = 64
    st = O3.State3(W.orszag_tang_3d(m), form=O3.LOWSTORE)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    st.run(1)
    sec = time.perf_counter() - t0
    out["oracle"] = {"mcell_updates_s": round(m ** 3 / sec / 1e6, 3), "threads": threads,
                     "sample": f"one RK4 step (HD on) of orszag_tang_3d at {m}^3: {sec:.2f} s"}
    return out


def run_3d(args):
    """The 3-D scheme: Orszag-Tang carried into z (eps = 0.2) on an n^3 grid,
    periodic, FP64, hyper-diffusion on, CFL 0.3.  A step is 4 stages, each a
    face-quantity launch and a fused stage launch after the ghost fills."""
    import torch
    import workloads as W
    from paper_1710_06423_amd.sacx3 import Solver3

    n = args.n
    log(f"[bench] generating orszag_tang_3d {n}^3")
    prob = W.orszag_tang_3d(n)
    s = Solver3.from_problem(prob, cfl=0.3)
    del prob
    cpu = None
    if args.cpu_sample > 0:
        from oracle import oracle3d as O3
        O3.build(force=False)
        m = min(args.cpu_sample, 128)
        sample = W.orszag_tang_3d(m)
        st = O3.State3(sample, form=O3.LOWSTORE)
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        t0 = time.perf_counter()
        st.run(1)
        sec = time.perf_counter() - t0
        cpu = {"value": m ** 3 / sec / 1e6, "unit": "Mcell-updates/s", "cores": threads, "kind": "oracle",
               "sample": f"one RK4 step (HD on) of orszag_tang_3d at {m}^3; {sec:.2f} s on {threads} OpenMP threads"}
        log(f"[bench] oracle: {cpu['value']:.3f} Mcell-updates/s")
    if args.warmup:
        s.advance(args.warmup)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s.stream)
    s.advance(args.steps, sync=False)
    e1.record(s.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    d = s.diagnostics()
    s.close()
    if d["nonphys"] or d["steps"] != args.warmup + args.steps:
        log(f"[bench] run failed: {d}")
        sys.exit(1)
    cells = n ** 3
    value = cells * args.steps / (ms / 1e3) / 1e6
    # algorithmic bytes: 12 field accesses x 8 fields x 8 B per cell and step
    alg = 12 * 8 * 8
    achieved = alg * cells / (ms / args.steps / 1e3) / 1e9
    log(f"[bench] 3-D {n}^3: {ms / args.steps:.3f} ms/step, {value:.1f} Mcell-updates/s, {achieved:.0f} GB/s algorithmic")
    out = base_record(args, value, ms / args.steps, "f64", {
        "workload": f"orszag_tang_3d_{n}^3_fp64_hd", "nx": n, "ny": n, "nz": n, "precision": "fp64",
        "hyper_diffusion": True, "cfl": 0.3, "bytes_per_cell_update": alg,
        "kernels": "per stage: k3_faces (face quantities to HBM) + k3_stage (fused RHS and combine)",
    })
    out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                       "scope": "whole step (both launches of every stage, ghost fills, dt)"}
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


def streaming_rate():
    """The HBM rate a plain elementwise kernel attains on this GPU: b = a + 3 c
    over three 4 GiB float64 arrays (2 reads, 1 write per element), best of 5
    timed launches after one untimed, in GB/s."""
    import torch
    n = 1 << 29
    a = torch.zeros(n, dtype=torch.float64, device="cuda")
    c = torch.zeros_like(a)
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(6):
        e0.record()
        torch.add(a, c, alpha=3.0, out=b)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b, c
    return 3 * 8 * n / (best / 1e3) / 1e9


def run_copy(args):
    """A 1 GiB device-to-device copy, five times: the dispatches a profiler run
    calibrates its byte counters with, and the achievable HBM bandwidth."""
    import torch
    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    gbs = 2 * nbytes / (ms / 1e3) / 1e9
    del src, dst
    tgbs = streaming_rate()
    print(json.dumps({"mode": "copy", "copy_bytes": nbytes, "dispatches": 5, "ms_per_copy": round(ms, 4),
                      "read_plus_write_gb_s": round(gbs, 1), "fraction_of_8tb_s": round(gbs / HBM_PEAK_GBS, 4),
                      "triad_gb_s": round(tgbs, 1), "triad_fraction_of_8tb_s": round(tgbs / HBM_PEAK_GBS, 4)}),
          flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 100, surrogate 500)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=["single", "batch", "surrogate", "decomposed", "graph", "copy", "3d",
                                       "oracle-sample", "oracle-workloads"],
                    default="single")
    ap.add_argument("--split", default="2x2", help="decomposed mode: subdomains along x and y, e.g. 2x2")
    ap.add_argument("--graph-steps", type=int, default=10, help="graph and decomposed modes: steps per captured graph")
    ap.add_argument("--n", type=int, default=None, help="grid side (default 8000, surrogate 2048, graph 1024)")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--problem", choices=["orszag_tang", "stratified"], default="orszag_tang",
                    help="single mode: Orszag-Tang, or a stratified atmosphere under gravity (background on)")
    ap.add_argument("--no-hd", action="store_true", help="the paper's 'without HD' column")
    ap.add_argument("--fp32-error", action="store_true", help="with --precision fp32: error against an FP64 run")
    ap.add_argument("--cpu-sample", type=int, default=8000, help="side of the oracle sub-block (0: skip)")
    ap.add_argument("--train-iters", type=int, default=6000)
    ap.add_argument("--max-snaps", type=int, default=0)
    ap.add_argument("--bound", type=float, default=0.05)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--no-extras", action="store_true",
                    help="single mode: only the headline (no FP32 / batch / learned-coefficient sub-records)")
    args = ap.parse_args()
    if args.mode == "oracle-sample":
        run_oracle_sample(args)
        return
    if args.mode == "oracle-workloads":
        run_oracle_workloads(args)
        return

    if args.gpus != 1:
        print(f"bench.py runs one GPU's subdomain only; --gpus {args.gpus} is not supported "
              f"(the halo exchange between GPUs is not implemented).", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = 500 if args.mode == "surrogate" else 100
    if args.n is None:
        args.n = {"surrogate": 2048, "graph": 1024, "3d": 512}.get(args.mode, 8000)

    args.one_thread = None
    args.cpu_workloads = None
    if args.mode == "single" and not args.no_extras and args.cpu_sample > 0 and args.n == 8000:
        # before anything initialises the GPU
        log("[bench] oracle at one thread on a 1000^2 sub-block")
        args.one_thread = oracle_one_thread(1000)
        log("[bench] oracle on Brio-Wu 800 and Orszag-Tang 1024^2, all threads and one thread")
        args.cpu_workloads = (oracle_workloads(None), oracle_workloads(1))
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    {"single": run_single, "batch": run_batch, "surrogate": run_surrogate, "decomposed": run_decomposed,
     "graph": run_graph, "copy": run_copy, "3d": run_3d}[args.mode](args)


if __name__ == "__main__":
    main()
