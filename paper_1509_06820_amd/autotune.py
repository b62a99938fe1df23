"""Autotuner of the batched TUXV engine: picks the block size b and the
output tile of the grouped products for a batch by timing every candidate
plan on the device, and caches the choice as JSON.

The key of a choice is the device name, k, p, the precision and a coarse
size signature of the batch (the number of matrices in each (log2 m,
log2 n) cell), so that batches with the same size mix reuse a choice.
Candidates: every b that divides k with b + p <= 64, from 8 up, and the
three tiles (64 x 64, 32 x 32, 128 x 64).  Timing: HIP events around
`reps` runs after one warm-up run, the median kept.

The cache is a JSON object {key: {"b": .., "tile": .., "ms": .., "candidates": [...]}};
`tune` reads it first (the file given, then the choices shipped with the
package for MI355X) and writes new choices to the file given.
"""

import json
import os

import numpy as np
import torch

from . import binding

SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch_tuning_mi355x.json")
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "rqrcp", "batch_tuning.json")
TILES = (binding.RQ_TILE_64x64, binding.RQ_TILE_32x32, binding.RQ_TILE_128x64)


def signature(shapes):
    """Counts of matrices per (floor(log2 m), floor(log2 n)) cell, as a string."""
    cells = {}
    for m, n in shapes:
        c = (int(np.log2(max(m, 1))), int(np.log2(max(n, 1))))
        cells[c] = cells.get(c, 0) + 1
    return ";".join(f"{a}x{b}:{cnt}" for (a, b), cnt in sorted(cells.items()))


def key(shapes, k, p, precision):
    dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    return f"{dev}|k={k}|p={p}|prec={int(binding._prec(precision))}|{signature(shapes)}"


def block_candidates(k, p):
    return [b for b in range(8, k + 1) if k % b == 0 and b + p <= 64 and (b & (b - 1)) == 0] or [k]


def _load(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def lookup(shapes, k, p, precision, cache_path=DEFAULT_CACHE):
    """The cached choice for this batch shape, or None."""
    kk = key(shapes, k, p, precision)
    for path in (cache_path, SHIPPED):
        c = _load(path)
        if kk in c:
            return c[kk]
    return None


def time_plan(bt, reps):
    """Median milliseconds of `reps` runs of a plan (after one warm-up run)."""
    bt.run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        bt.run()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def tune(mats, k, p, seeds, precision=binding.RQ_FP64, cache_path=DEFAULT_CACHE, reps=3, force=False, log=None):
    """Choose (b, tile) for this batch: the cached choice when there is one
    (unless force), else time every candidate plan and cache the fastest."""
    shapes = [tuple(A.shape) for A in mats]
    kk = key(shapes, k, p, precision)
    if not force:
        hit = lookup(shapes, k, p, precision, cache_path)
        if hit is not None:
            return hit
    results = []
    for b in block_candidates(k, p):
        for tile in TILES:
            bt = binding.BatchTUXV(mats, k, b, p, seeds, precision=precision, tile=tile)
            ms = time_plan(bt, reps)
            bt.close()
            del bt
            results.append({"b": b, "tile": tile, "ms": round(ms, 4)})
            if log:
                log(f"[autotune] b={b} tile={tile}: {ms:.3f} ms")
    best = min(results, key=lambda r: r["ms"])
    choice = {"b": best["b"], "tile": best["tile"], "ms": best["ms"], "candidates": results}
    if cache_path:
        cache = _load(cache_path)
        cache[kk] = choice
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return choice
