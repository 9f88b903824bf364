"""Pins of the oracle's intercept count (paper: Background -- the
intercept-count mode, unique intersections per ray), read as the number of
distinct binary64 t among the hits.  Closed forms where geometry fixes both
the number of triangles hit and the number of distinct points, with dyadic
inputs so that equal points give equal t in binary64 whatever triangle
produced them."""
import numpy as np

import oracle
from paper_2305_01867_amd import workloads

UNIT_V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)


def count1(V, F, o, e):
    O, E = np.array([o], np.float32), np.array([e], np.float32)
    _, _, _, nh = oracle.intersect(V, F, O, E)
    return int(oracle.intercept_count(V, F, O, E)[0]), int(nh[0])


def test_coincident_triangles_count_once():
    V = np.concatenate([UNIT_V, UNIT_V + np.float32([10, 10, 0])]).astype(np.float32)
    F = np.array([[3, 4, 5]] * 8, np.int32)
    F[3] = F[7] = (0, 1, 2)
    assert count1(V, F, (0.25, 0.25, 1.0), (0.25, 0.25, -1.0)) == (1, 2)
    assert count1(V, F, (5.0, 5.0, 1.0), (5.0, 5.0, -1.0)) == (0, 0)


def test_shared_edge_counts_once():
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], np.float32)
    F = np.array([[1, 3, 2], [0, 1, 2]], np.int32)
    assert count1(V, F, (0.5, 0.5, 1.0), (0.5, 0.5, -1.0)) == (1, 2)    # through the shared edge
    assert count1(V, F, (0.25, 0.5, 1.0), (0.25, 0.5, -1.0)) == (1, 1)  # inside one triangle


def test_stacked_split_layers():
    # k unit squares at z = 0..k-1, each split along its diagonal; a vertical
    # segment through the diagonal meets 2 triangles per layer at one point each
    for k in (1, 2, 5, 9):
        V, F = [], []
        for z in range(k):
            b = len(V)
            V += [(0, 0, z), (1, 0, z), (1, 1, z), (0, 1, z)]
            F += [(b, b + 1, b + 2), (b, b + 2, b + 3)]
        V, F = np.array(V, np.float32), np.array(F, np.int32)
        assert count1(V, F, (0.5, 0.5, k + 0.5), (0.5, 0.5, -0.5)) == (k, 2 * k)
        assert count1(V, F, (0.75, 0.25, k + 0.5), (0.75, 0.25, -0.5)) == (k, k)
        # a segment ending exactly on a layer counts that layer (closed segment)
        assert count1(V, F, (0.75, 0.25, -0.5), (0.75, 0.25, 0.0)) == (1, 1)


def test_flat_grid_vertex_and_edges():
    """Flat 5 x 5 grid of the heightfield triangulation at z = 0 (dyadic
    coordinates): through an interior vertex the segment meets the 6 triangles
    around it at one point; through an interior grid edge, 2; inside a
    triangle, 1."""
    n = 5
    xs = np.arange(n) / (n - 1)
    V = np.array([(xs[i], xs[j], 0.0) for j in range(n) for i in range(n)], np.float32)
    F = []
    for j in range(n - 1):
        for i in range(n - 1):
            v = lambda a, b: b * n + a
            F += [(v(i, j), v(i + 1, j), v(i + 1, j + 1)), (v(i, j), v(i + 1, j + 1), v(i, j + 1))]
    F = np.array(F, np.int32)
    assert count1(V, F, (0.5, 0.5, 1.0), (0.5, 0.5, -1.0)) == (1, 6)
    assert count1(V, F, (0.5, 0.375, 1.0), (0.5, 0.375, -1.0)) == (1, 2)      # vertical grid line
    assert count1(V, F, (0.625, 0.625, 1.0), (0.625, 0.625, -1.0)) == (1, 2)  # cell diagonal
    assert count1(V, F, (0.625, 0.5625, 1.0), (0.625, 0.5625, -1.0)) == (1, 1)


def test_counts_against_hits_on_a_heightfield():
    """Invariants on oblique segments over a random heightfield: 0 <= count
    <= number of triangles hit, count > 0 exactly for hitting segments, and
    count equals the number of hits whenever no two hits lie within 1e-9 in t
    (then they are distinct points)."""
    V, F = workloads.heightfield(16, 9)
    O, E = workloads.rays_crossing_mix(400, 10)
    hit, _, _, nh = oracle.intersect(V, F, O, E)
    cnt = oracle.intercept_count(V, F, O, E)
    assert np.all(cnt >= 0) and np.all(cnt <= nh)
    assert np.array_equal(cnt > 0, hit == 1)
    separated = 0
    for r in range(O.shape[0]):
        _, uvt = oracle.all_hits(V, F, O[r], E[r])
        t = np.sort(uvt[:, 2])
        if t.size < 2 or np.min(np.diff(t)) > 1e-9:
            assert cnt[r] == nh[r]
            separated += 1
    assert separated > 350
    assert np.any(nh >= 2)  # segments crossing the surface several times took part
