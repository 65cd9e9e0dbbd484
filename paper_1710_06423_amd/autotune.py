"""Tile autotuner for the batched launch (and the per-subdomain kernel).

Times a few steps of the real workload for each candidate tile shape and
keeps the fastest: threads per block for the launch, and output rows per tile
strip for each instance class (2-D boxes; 1-D tubes always use one-row
tiles).  Results depend only on speed, never on values (every shape gives the
same bits), so tuning on the live state is safe.  A JSON cache keyed by the
workload signature avoids re-tuning.
"""

from __future__ import annotations

import json
import os
import time
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import torch

from .sacx import FP32, FP64, Batch, Solver

CACHE = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")), "sacx", "autotune.json")


def _load_cache() -> Dict:
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save_cache(d: Dict):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(d, fh, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def _time(fn, reps: int) -> float:
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def batch_signature(batch: Batch) -> str:
    g = batch.grids
    return "batch:%d:%s:%s" % (batch.n, "fp64" if g[0].precision == FP64 else "fp32",
                               ",".join("%dx%d" % (g[i].nx, g[i].ny) for i in range(batch.n)))


def tune_batch(batch: Batch, threads: Sequence[int] = (128, 256), rows2d: Sequence[int] = (16, 32, 64, 128),
               steps: int = 2, use_cache: bool = True, log=None) -> Tuple[int, int, List[Tuple[int, int, float]]]:
    """Pick (threads, rows for 2-D instances) for a batch; advances the batch
    by (1 + steps) x number of candidates steps while measuring."""
    key = batch_signature(batch)
    cache = _load_cache() if use_cache else {}
    if key in cache:
        t, r = cache[key]["threads"], cache[key]["rows2d"]
        batch.set_tiles(t, [r] * batch.n)
        return t, r, []
    trials = []
    for t in threads:
        for r in rows2d:
            batch.set_tiles(t, [r] * batch.n)
            batch.advance(1, sync=True)                     # table build + warm-up
            ms = _time(lambda: batch.advance(steps, sync=False), 1) / steps
            trials.append((t, r, ms))
            if log:
                log(f"[autotune] threads={t} rows={r}: {ms:.3f} ms/step")
    t, r, _ = min(trials, key=lambda x: x[2])
    batch.set_tiles(t, [r] * batch.n)
    if use_cache:
        cache[key] = {"threads": t, "rows2d": r, "trials": trials}
        _save_cache(cache)
    return t, r, trials


def tune_solver(s: Solver, threads: Sequence[int] = (64, 128, 256), rows: Sequence[int] = (32, 64, 128, 256),
                log=None) -> Tuple[int, int]:
    """Pick the launch shape of one subdomain by timing single steps."""
    best = None
    for t in threads:
        for r in rows:
            try:
                s.set_launch(t, r)
            except Exception:
                continue
            s.advance(1)
            ms = _time(lambda: s.advance(1, sync=False), 2)
            if log:
                log(f"[autotune] threads={t} rows={r}: {ms:.3f} ms/step")
            if best is None or ms < best[2]:
                best = (t, r, ms)
    s.set_launch(best[0], best[1])
    return best[0], best[1]
