"""Derived outputs of the barycentric mode (paper: Background; Performance
section steps 3a-3d) against the oracle's binary64 values: per-segment
distances and points, and the compacted (intersecting_rays, distances,
hit_triangles, hit_points) tuple -- same segments in the same order, same
triangles, distances and points within 1e-5 relative (|x - x_ref| <=
1e-5 max(1, |x_ref|)); the paper's printed hit points; tile-edge sizes and
the paper-scale configuration."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_01867_amd as rsi
from paper_2305_01867_amd import workloads
from gpu_helpers import dev, host, say

pytestmark = pytest.mark.gpu


def close(got, want, tol=1e-5):
    return np.all(np.abs(got.astype(np.float64) - want) <= tol * np.maximum(1.0, np.abs(want)))


def check(V, F, O, E, label):
    hit, ids, uvt, _ = oracle.intersect(V, F, O, E)
    w_idx, w_dist, w_tri, w_pts = oracle.derived(O, E, ids, uvt)
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        dO, dE = dev(O), dev(E)
        r = rsi.rsi_intersect(mesh, dO, dE, mode="barycentric", precision="certified")
        idx, dist, tri, pts = (host(x) for x in rsi.rsi_compact_hits(dO, dE, r))
        per = {k: host(v) for k, v in rsi.rsi_derive(dO, dE, r).items()}
    say(f"[derive] {label}: {len(idx)} of {O.shape[0]} segments hit")
    assert np.array_equal(idx, w_idx) and np.array_equal(tri, w_tri)
    assert close(dist, w_dist) and close(pts, w_pts)
    miss = ids < 0
    assert np.all(np.isnan(per["distance"][miss])) and np.all(np.isnan(per["point"][miss]))
    assert np.array_equal(per["distance"][~miss], dist) and np.array_equal(per["point"][~miss], pts)
    return idx, dist, tri, pts


def test_case_study_1_scene(golden_case_study_1):
    V, F, O, E = workloads.appendix_scene()
    idx, dist, tri, pts = check(V, F, O, E, "case study 1")
    rows = golden_case_study_1["hit"]
    assert idx.tolist() == [int(r[0]) for r in rows] and tri.tolist() == [int(r[1]) for r in rows]
    assert np.allclose(pts, np.array([[float(x) for x in r[2:5]] for r in rows]), atol=0.006)
    # the paper's one-call form, on numpy arrays
    got = rsi.rsi_test(V, F, O, E, mode="barycentric")
    assert np.array_equal(got[0], idx) and np.array_equal(got[3], pts)
    assert rsi.rsi_test(V, F, O, E, mode="boolean").tolist() == [int(x) for x in golden_case_study_1["boolean"][0]]


def test_tiny_config_and_tile_edges():
    V, F, O, E = workloads.tiny_config()
    check(V, F, O, E, "64x64 heightfield, 1e4 segments")
    V, F = workloads.heightfield(20, 3)
    for n in (1, 4095, 4096, 4097, 12289):
        O, E = workloads.rays_crossing_mix(n, n + 7)
        check(V, F, O, E, f"n={n}")


def test_empty_and_all_miss():
    V, F = workloads.heightfield(8, 1)
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        O = np.zeros((0, 3), np.float32)
        r = rsi.rsi_intersect(mesh, dev(O), dev(O), mode="barycentric")
        assert all(x.shape[0] == 0 for x in rsi.rsi_compact_hits(dev(O), dev(O), r))
        O = np.full((5000, 3), 7.0, np.float32)
        E = O + 1.0
        r = rsi.rsi_intersect(mesh, dev(O), dev(E), mode="barycentric")
        assert rsi.rsi_compact_hits(dev(O), dev(E), r)[0].shape[0] == 0


def test_paper_scale_sampled():
    V, F, O, E = workloads.paper_scale_config()
    with rsi.rsi_build(dev(V), dev(F), algorithm="restructured") as mesh:  # the benchmark's tree
        dO, dE = dev(O), dev(E)
        r = rsi.rsi_intersect(mesh, dO, dE, mode="barycentric", precision="certified")
        idx, dist, tri, pts = (host(x) for x in rsi.rsi_compact_hits(dO, dE, r))
        ids = host(r["tri_id"])
    assert np.array_equal(idx, np.nonzero(ids >= 0)[0]) and np.array_equal(tri, ids[idx])
    rng = np.random.default_rng(2)
    pick = np.sort(rng.choice(idx.size, 2000, replace=False))
    s = idx[pick]
    _, o_ids, o_uvt, _ = oracle.intersect(V, F, O[s], E[s])
    _, w_dist, w_tri, w_pts = oracle.derived(O[s], E[s], o_ids, o_uvt)
    assert np.array_equal(tri[pick], w_tri) and close(dist[pick], w_dist) and close(pts[pick], w_pts)
