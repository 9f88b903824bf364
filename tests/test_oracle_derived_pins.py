"""Pins of the oracle's derived outputs (paper: Background -- barycentric mode
returns the intersecting rays, triangles, distances and points; Performance
section, steps 3a-3d): a dyadic oblique segment whose distance and point are
exact, the paper's printed Case Study 1 hit points, and the compaction's
order and contents against the first-hit results."""
import numpy as np

import oracle
from paper_2305_01867_amd import workloads

UNIT_V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
UNIT_F = np.array([[0, 1, 2]], np.int32)


def test_dyadic_oblique_segment():
    # d = (0, 1, -0.75): |d| = 1.25; the plane z = 0 is reached at t = 0.5
    O = np.array([[0.25, -0.25, 0.375], [0.25, 0.25, 1.0], [5.0, 5.0, 1.0]], np.float32)
    E = np.array([[0.25, 0.75, -0.375], [0.25, 0.25, -1.0], [5.0, 5.0, -1.0]], np.float32)
    hit, ids, uvt, _ = oracle.intersect(UNIT_V, UNIT_F, O, E)
    idx, dist, tri, pts = oracle.derived(O, E, ids, uvt)
    assert idx.tolist() == [0, 1] and tri.tolist() == [0, 0]
    assert dist.tolist() == [0.625, 1.0]
    assert pts.tolist() == [[0.25, 0.25, 0.0], [0.25, 0.25, 0.0]]


def test_case_study_1_printed_points(golden_case_study_1):
    V, F, O, E = workloads.appendix_scene()
    hit, ids, uvt, _ = oracle.intersect(V, F, O, E)
    idx, dist, tri, pts = oracle.derived(O, E, ids, uvt)
    rows = golden_case_study_1["hit"]
    assert idx.tolist() == [int(r[0]) for r in rows]
    assert tri.tolist() == [int(r[1]) for r in rows]
    want = np.array([[float(x) for x in r[2:5]] for r in rows])
    assert np.allclose(pts, want, atol=0.006)
    length = np.linalg.norm(E[idx].astype(np.float64) - O[idx].astype(np.float64), axis=1)
    assert np.allclose(dist, np.linalg.norm(pts - O[idx], axis=1)) and np.all(dist <= length)


def test_compaction_matches_first_hits():
    V, F = workloads.heightfield(16, 9)
    O, E = workloads.rays_crossing_mix(500, 10)
    hit, ids, uvt, _ = oracle.intersect(V, F, O, E)
    idx, dist, tri, pts = oracle.derived(O, E, ids, uvt)
    assert np.array_equal(idx, np.nonzero(hit)[0]) and np.all(np.diff(idx) > 0)
    assert np.array_equal(tri, ids[hit == 1])
    # each point lies on its triangle's plane and at the stated distance from O
    Vd = V.astype(np.float64)
    A = Vd[F[tri, 0]]
    n = np.cross(Vd[F[tri, 1]] - A, Vd[F[tri, 2]] - A)
    assert np.all(np.abs(np.sum((pts - A) * n, axis=1)) <= 1e-12 * np.linalg.norm(n, axis=1))
    assert np.allclose(np.linalg.norm(pts - O[idx], axis=1), dist, rtol=1e-12)
