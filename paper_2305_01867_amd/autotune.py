"""Launch-parameter autotuner for the intersection kernels.

For a given workload it times every point of a grid of launch choices with
HIP events on the caller's stream, keeps the fastest, and caches the choice
in a JSON file keyed by a size class (mode, precision, number of meshes,
log2 of triangles and of segments), so later runs of the same class reuse it
without timing.  The default grid covers threads per workgroup, the LDS
stack depth (occupancy against how often a segment overflows to the
deep-stack pass), the resident waves per CU (fewer waves share a CU's L1
among fewer tree paths) and the segment processing order; MORTON_BITS can be added
for a `run` that rebuilds the tree (30-bit against 63-bit keys), NODE_WIDTHS
for a single-mesh `run` (4-wide against binary nodes).
"""
from __future__ import annotations

import itertools
import json
import math
import os

import torch

BLOCKS = (64, 128, 256, 512, 1024)
STACKS = (8, 12, 16, 20, 24, 32)
RAY_SORTS = (0, 1, 2)  # input order, midpoint Morton, octant + start Morton
WAVES_PER_CU = (0, 8, 12, 16, 24)  # 0: as many as registers and LDS allow
MORTON_BITS = (30, 63)
NODE_WIDTHS = (0, 2)  # the widest tree built (4-wide for one mesh) against binary nodes
SPACE = {"block": BLOCKS, "stack_depth": STACKS, "ray_sort": RAY_SORTS, "waves_per_cu": WAVES_PER_CU}


def size_class(mode: str, precision: str, n_meshes: int, n_triangles: int, n_rays: int) -> str:
    return (f"{mode}/{precision}/m{n_meshes}/t{int(math.log2(max(n_triangles, 1)))}"
            f"/r{int(math.log2(max(n_rays, 1)))}")


def tune(run, key: str, cache_path: str | None = None, space: dict | None = None, reps: int = 2):
    """run(**choice) must queue one intersection (and, if the grid holds
    morton_bits, the build it needs) on the current stream.  Returns (best
    choice with its "ms", all timings), or (cached choice, None)."""
    space = dict(SPACE if space is None else space)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            return cache[key], None
    stream = torch.cuda.current_stream()
    names = list(space)
    timings = []
    for values in itertools.product(*(space[k] for k in names)):
        choice = dict(zip(names, values))
        run(**choice)  # warm-up (also first-use costs)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            run(**choice)
        b.record(stream)
        b.synchronize()
        timings.append({**choice, "ms": a.elapsed_time(b) / reps})
    best = min(timings, key=lambda t: t["ms"])
    if cache_path:
        cache[key] = best
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return best, timings
