"""The batched form: many meshes and segment batches in one build and one
persistent traversal; results per mesh equal single-mesh calls and the
oracle; the combined BVH keeps each mesh in one subtree; build + intersect
replay from a captured graph; the autotuner picks and caches a choice."""
import json
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
import paper_2305_01867_amd as rsi
from paper_2305_01867_amd import autotune, workloads
from gpu_helpers import dev, host, say

pytestmark = pytest.mark.gpu
MODES = ("boolean", "first_hit", "barycentric")


def small_batch():
    """Meshes of uneven size, with an empty mesh, a one-triangle mesh and a
    mesh without segments."""
    parts = []
    for m, (n, nr) in enumerate([(9, 700), (2, 300), (33, 2500), (0, 200), (17, 0), (1, 150), (24, 1900)]):
        if n == 0:
            V, F = np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32)
            O, E = workloads.rays_crossing_mix(nr, 50 + m)
        elif n == 1:
            V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
            F = np.array([[0, 1, 2]], np.int32)
            O, E = workloads.rays_crossing_mix(nr, 50 + m)
        else:
            V, F = workloads.heightfield(n, 60 + m)
            O, E = workloads.rays_in_box(nr, 70 + m, V.min(0), V.max(0))
        parts.append((V, F, O, E))
    off = lambda xs: np.concatenate([[0], np.cumsum([len(x) for x in xs])]).astype(np.int64)
    V = np.concatenate([p[0] for p in parts]).astype(np.float32)
    F = np.concatenate([p[1] for p in parts]).astype(np.int32)
    O = np.concatenate([p[2] for p in parts]).astype(np.float32)
    E = np.concatenate([p[3] for p in parts]).astype(np.float32)
    return parts, V, F, O, E, off([p[0] for p in parts]), off([p[1] for p in parts]), off([p[2] for p in parts])


def test_batch_equals_single_mesh_and_oracle():
    parts, V, F, O, E, vo, to, ro = small_batch()
    say(f"[batch] {len(parts)} meshes, {F.shape[0]} triangles, {O.shape[0]} segments")
    with rsi.rsi_batch_create(vo, to, ro) as b:
        rsi.rsi_batch_build(b, dev(V), dev(F))
        dO, dE = dev(O), dev(E)
        # 4-wide with each XCD group's top in LDS (1024-thread workgroups), 4-wide
        # with the combined top (256 threads: not every slot fits), binary nodes
        for mode, prec, width, block in [(m, p, w, bl) for m in MODES for p in ("certified", "plain")
                                         for w, bl in ((0, 0), (0, 256), (2, 0))]:
            if True:
                got = {k: host(v) for k, v in rsi.rsi_batch_intersect(b, dO, dE, mode=mode, precision=prec,
                                                                      node_width=width, block=block).items()}
                for m, (Vm, Fm, Om, Em) in enumerate(parts):
                    sl = slice(ro[m], ro[m + 1])
                    if len(Om) == 0:
                        continue
                    with rsi.rsi_build(dev(Vm), dev(Fm)) as mesh:
                        one = {k: host(v) for k, v in rsi.rsi_intersect(mesh, dev(Om), dev(Em), mode=mode,
                                                                        precision=prec).items()}
                    for k in one:
                        if k != "counters":
                            assert np.array_equal(got[k][sl], one[k], equal_nan=True), (mode, prec, width, block, m, k)
                    if prec == "certified":
                        hit, ids, uvt, _ = oracle.intersect(Vm, Fm, Om, Em) if len(Fm) else (
                            np.zeros(len(Om), np.uint8), np.full(len(Om), -1, np.int32), None, None)
                        key = "hit" if mode == "boolean" else "tri_id"
                        assert np.array_equal(got[key][sl], hit if mode == "boolean" else ids), (mode, m)


def test_combined_tree_keeps_each_mesh_in_one_subtree():
    parts, V, F, O, E, vo, to, ro = small_batch()
    with rsi.rsi_batch_create(vo, to, ro) as b:
        rsi.rsi_batch_build(b, dev(V), dev(F))
        keys = host(rsi.rsi_batch_export(b, "sorted_keys")).view(np.uint64)
        ids = host(rsi.rsi_batch_export(b, "sorted_ids"))
        nodes = host(rsi.rsi_batch_export(b, "nodes"))
        roots = host(rsi.rsi_batch_export(b, "mesh_roots"))
        counters = host(rsi.rsi_batch_export(b, "counters"))
    assert np.all(np.diff(keys.astype(np.float64)) >= 0)
    mesh_of_key = (keys >> np.uint64(30)).astype(np.int64)
    mesh_of_tri = np.searchsorted(to, np.arange(F.shape[0]), side="right") - 1
    assert np.array_equal(mesh_of_key, mesh_of_tri[ids])
    assert np.all(counters == 2)
    for m in range(len(parts)):
        n = to[m + 1] - to[m]
        if n == 0:
            assert roots[m] == -(2 ** 31)
            continue
        if n == 1:
            lo = hi = ~roots[m]
        else:
            lo, hi = nodes[roots[m], 14], nodes[roots[m], 15]
        assert np.array_equal(np.sort(ids[lo:hi + 1]), np.arange(to[m], to[m + 1]))


def test_batch_segment_orders_agree():
    """Each mesh's segments stay in their own position range under the
    mesh-prefixed segment keys, so every order gives the input-order results."""
    parts, V, F, O, E, vo, to, ro = small_batch()
    with rsi.rsi_batch_create(vo, to, ro) as b:
        rsi.rsi_batch_build(b, dev(V), dev(F))
        dO, dE = dev(O), dev(E)
        for mode in MODES:
            ref = {k: host(v) for k, v in rsi.rsi_batch_intersect(b, dO, dE, mode=mode, precision="certified").items()}
            for order in ("midpoint", "origin_octant"):
                got = rsi.rsi_batch_intersect(b, dO, dE, mode=mode, precision="certified", ray_sort=order)
                for k in ref:
                    if k != "counters":
                        assert np.array_equal(host(got[k]), ref[k], equal_nan=True), (mode, order, k)


def test_batch_intercept_count_equals_oracle():
    parts, V, F, O, E, vo, to, ro = small_batch()
    with rsi.rsi_batch_create(vo, to, ro) as b:
        rsi.rsi_batch_build(b, dev(V), dev(F))
        got = host(rsi.rsi_batch_intersect(b, dev(O), dev(E), mode="intercept_count",
                                           precision="certified")["count"])
        for m, (Vm, Fm, Om, Em) in enumerate(parts):
            if len(Om) == 0:
                continue
            want = oracle.intercept_count(Vm, Fm, Om, Em) if len(Fm) else np.zeros(len(Om), np.int32)
            assert np.array_equal(got[ro[m]:ro[m + 1]], want), m


def test_graph_capture_replays_build_and_intersect():
    parts, V, F, O, E, vo, to, ro = small_batch()
    dV, dF, dO, dE = dev(V), dev(F), dev(O), dev(E)
    with rsi.rsi_batch_create(vo, to, ro) as b:
        out = {"tri_id": torch.empty(O.shape[0], dtype=torch.int32, device="cuda"),
               "uvt": torch.empty((O.shape[0], 3), dtype=torch.float32, device="cuda"),
               "counters": torch.zeros(4, dtype=torch.int64, device="cuda")}
        rsi.rsi_batch_build(b, dV, dF)
        rsi.rsi_batch_intersect(b, dO, dE, mode="barycentric", precision="certified", out=out)
        want = {k: host(v).copy() for k, v in out.items()}
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
                rsi.rsi_batch_build(b, dV, dF)
                rsi.rsi_batch_intersect(b, dO, dE, mode="barycentric", precision="certified", out=out)
        torch.cuda.current_stream().wait_stream(s)
        for rep in range(4):
            out["tri_id"].fill_(-7)
            out["uvt"].fill_(5.0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            for k in want:
                assert np.array_equal(host(out[k]), want[k], equal_nan=True), (rep, k)
            # eager work between replays
            rsi.rsi_batch_intersect(b, dO, dE, mode="boolean")
            torch.cuda.synchronize()


def test_autotuner_picks_and_caches():
    parts, V, F, O, E, vo, to, ro = small_batch()
    dO, dE = dev(O), dev(E)
    with rsi.rsi_batch_create(vo, to, ro) as b, tempfile.TemporaryDirectory() as d:
        rsi.rsi_batch_build(b, dev(V), dev(F))
        path = os.path.join(d, "tune.json")
        key = autotune.size_class("boolean", "certified", len(parts), F.shape[0], O.shape[0])
        want = host(rsi.rsi_batch_intersect(b, dO, dE, mode="boolean", precision="certified")["hit"])

        def run(**choice):
            got = rsi.rsi_batch_intersect(b, dO, dE, mode="boolean", precision="certified", **choice)
            assert np.array_equal(host(got["hit"]), want), choice

        best, timings = autotune.tune(run, key, path, reps=1)
        assert best["block"] in autotune.BLOCKS and best["stack_depth"] in autotune.STACKS
        assert best["ray_sort"] in autotune.RAY_SORTS and best["waves_per_cu"] in autotune.WAVES_PER_CU
        assert len(timings) == (len(autotune.BLOCKS) * len(autotune.STACKS) * len(autotune.RAY_SORTS)
                                * len(autotune.WAVES_PER_CU))
        assert json.load(open(path))[key] == best
        again, t2 = autotune.tune(run, key, path)
        assert again == best and t2 is None


def test_batched_workload_sampled():
    """64 heightfields of log-uniform size with their own segment batches
    (~1.4e7 segments), on the 4-wide tree and on binary nodes: 1000 sampled
    segments of every mesh against the oracle in the boolean, first-hit and
    barycentric modes (u, v, t equal to the oracle's rounded once)."""
    V, F, O, E, vo, to, ro = workloads.batched_config()
    say(f"[batch] 64 meshes, {F.shape[0]} triangles, {O.shape[0]} segments")
    rng = np.random.default_rng(1)
    idx = [np.sort(rng.choice(np.arange(ro[m], ro[m + 1]), 1000, replace=False)) for m in range(64)]
    want = []
    for m in range(64):
        Vm, Fm = V[vo[m]:vo[m + 1]], F[to[m]:to[m + 1]]
        hit, ids, uvt, _ = oracle.intersect(Vm, Fm, O[idx[m]], E[idx[m]])
        # the oracle's ids are per mesh; the batch reports each mesh's own indices
        want.append((hit, ids, uvt.astype(np.float32)))
    with rsi.rsi_batch_create(vo, to, ro) as b:
        rsi.rsi_batch_build(b, dev(V), dev(F))
        dO, dE = dev(O), dev(E)
        for width in (0, 2):
            for mode in ("boolean", "first_hit", "barycentric"):
                r = rsi.rsi_batch_intersect(b, dO, dE, mode=mode, precision="certified", node_width=width)
                got = host(r["hit" if mode == "boolean" else "tri_id"])
                uvt = host(r["uvt"]) if mode == "barycentric" else None
                del r
                for m in range(64):
                    hit, ids, w_uvt = want[m]
                    assert np.array_equal(got[idx[m]], hit if mode == "boolean" else ids), (width, mode, m)
                    if uvt is not None:
                        g = uvt[idx[m]]
                        assert np.array_equal(np.isnan(g), np.isnan(w_uvt)), (width, m)
                        ok = ~np.isnan(w_uvt)
                        assert np.array_equal(g[ok], w_uvt[ok]), (width, m)
                say(f"  width {width or 'widest'}, {mode}: 64 x 1000 segments equal the oracle")
