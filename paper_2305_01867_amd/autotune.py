"""Launch-parameter autotuner for the intersection kernels.

For a given workload it times every candidate (threads per workgroup x LDS
stack depth) with HIP events on the caller's stream, keeps the fastest, and
caches the choice in a JSON file keyed by a size class (mode, precision,
number of meshes, log2 of triangles and of segments), so later runs of the
same class reuse it without timing.  The stack depth trades LDS per workgroup
(occupancy) against how often a segment overflows to the deep-stack pass.
Segment order is always the input order (ray_sort 0 is the only value the
library offers).
"""
from __future__ import annotations

import json
import math
import os

import torch

BLOCKS = (64, 128, 256)
STACKS = (8, 12, 16, 20, 24, 32)


def size_class(mode: str, precision: str, n_meshes: int, n_triangles: int, n_rays: int) -> str:
    return (f"{mode}/{precision}/m{n_meshes}/t{int(math.log2(max(n_triangles, 1)))}"
            f"/r{int(math.log2(max(n_rays, 1)))}")


def tune(run, key: str, cache_path: str | None = None, blocks=BLOCKS, stacks=STACKS, reps: int = 2):
    """run(block, stack_depth) must queue one intersection on the current
    stream.  Returns (best {"block", "stack_depth", "ms"}, all timings)."""
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            cache = json.load(fh)
        if key in cache:
            return cache[key], None
    stream = torch.cuda.current_stream()
    timings = []
    for block in blocks:
        for stack in stacks:
            run(block, stack)  # warm-up (also first-use costs)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                run(block, stack)
            b.record(stream)
            b.synchronize()
            timings.append({"block": block, "stack_depth": stack, "ms": a.elapsed_time(b) / reps})
    best = min(timings, key=lambda t: t["ms"])
    if cache_path:
        cache[key] = best
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return best, timings
