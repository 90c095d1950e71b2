"""Autotuner for the work decomposition of batched steps.

It times whole batch steps for candidate tile shapes and keeps the fastest, by
coordinate descent over the three parameters of ``pf_batch_tiles``: rows per
apply strip, vectors per CG-update work item and persistent blocks per compute
unit.  Because the state advances while it is timed and the number of CG
iterations changes from step to step, a candidate is scored by time per pass
of the persistent CG loop (the step time divided by one plus the largest
iteration count of any instance in that step).  Results are cached in a JSON file keyed by
GPU architecture, precision and a size class of the batch.
"""
from __future__ import annotations

import json
import math
import os
import time

APPLY_ROWS = (16, 32, 64, 128)
UPDATE_CHUNK = (1024, 4096, 8192, 16384)
BLOCKS_PER_CU = (1, 2, 3, 4)

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pfx_batch_tiles.json")


def _arch():
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def size_key(shapes, precision):
    cells = sum(ny * nx for ny, nx in shapes)
    return f"{_arch()}|dim2|{precision}|n{len(shapes)}|cells2^{int(round(math.log2(max(cells, 1))))}"


def _time_steps(batch, steps):
    """Mean seconds per CG-loop pass over `steps` single steps."""
    import torch
    total, passes = 0.0, 0
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = batch.step(1)
        torch.cuda.synchronize()
        total += time.perf_counter() - t0
        passes += 1 + max(s["cg_iters"] for s in st)
    return total / passes


def tune(batch, precision, steps=2, cache_path=DEFAULT_CACHE, log=None):
    """Tune `batch` in place (its state advances while it is timed) and return
    the chosen tiles.  A cached choice for the same key is applied directly."""
    key = size_key(batch.shapes, precision)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            cache = json.load(open(cache_path))
        except (OSError, ValueError):
            cache = {}
    if key in cache:
        t = cache[key]
        batch.set_tiles(t["apply_rows"], t["update_chunk"], t["blocks_per_cu"])
        return dict(t, cached=True)
    best = batch.tiles()
    trials = []

    def trial(**kw):
        try:
            batch.set_tiles(**kw)
        except Exception:            # e.g. more blocks per CU than can be resident
            return float("inf")
        batch.step(1)                # first replay of the new graphs
        t = _time_steps(batch, steps)
        trials.append((dict(kw), t))
        if log:
            log(f"[tune] {kw} -> {1e6 * t:.1f} us per CG pass")
        return t

    cur = {k: best[k] for k in ("apply_rows", "update_chunk", "blocks_per_cu")}
    best_t = trial(**cur)
    for name, choices in (("apply_rows", APPLY_ROWS), ("update_chunk", UPDATE_CHUNK), ("blocks_per_cu", BLOCKS_PER_CU)):
        for v in choices:
            if v == cur[name]:
                continue
            cand = dict(cur, **{name: v})
            t = trial(**cand)
            if t < best_t:
                best_t, cur = t, cand
    batch.set_tiles(**cur)
    result = dict(cur, us_per_pass=1e6 * best_t)
    if cache_path:
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            cache[key] = result
            json.dump(cache, open(cache_path, "w"), indent=1)
        except OSError:
            pass
    return dict(result, cached=False, trials=[(t, 1e6 * s) for t, s in trials])
