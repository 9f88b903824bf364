"""Pins of the binary64 intersection oracle to facts fixed by the paper and by
geometry, not by the oracle's own formula.

- closed forms with dyadic inputs (every intermediate exact in binary64);
- hand-worked boundary cases (edges, vertices, segment end points, parallel);
- the Case Study 1 scene: hit points and boolean vector printed in the paper;
- a heightfield closed form: a vertical segment crosses exactly one triangle,
  whose index follows from (x, y) alone;
- exact rational arithmetic with an independent formulation (signed volumes)
  on random and near-boundary pairs.
"""
import numpy as np
import pytest

import oracle
from paper_2305_01867_amd import workloads

UNIT_V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
UNIT_F = np.array([[0, 1, 2]], np.int32)


def run1(V, F, o, e):
    hit, ids, uvt, nh = oracle.intersect(V, F, np.array([o], np.float32), np.array([e], np.float32))
    return bool(hit[0]), int(ids[0]), uvt[0], int(nh[0])


@pytest.mark.parametrize("x,y,z0,z1", [
    (0.25, 0.25, 0.75, -0.25), (0.125, 0.5, 1.0, -1.0), (0.5, 0.375, 2.0, -2.0),
    (0.0625, 0.8125, 0.5, -1.5), (0.3, 0.2, 0.25, -0.75),
])
def test_closed_form_unit_triangle(x, y, z0, z1):
    # A=(0,0,0), B=(1,0,0), C=(0,1,0); the vertical segment through (x, y)
    # meets the plane at t = z0 / (z0 - z1) with barycentrics u = x, v = y.
    xf, yf = float(np.float32(x)), float(np.float32(y))
    hit, j, (u, v, t), n = run1(UNIT_V, UNIT_F, (x, y, z0), (x, y, z1))
    assert hit and j == 0 and n == 1
    assert u == xf and v == yf
    assert t == z0 / (z0 - z1)


def test_closed_form_oblique_dyadic():
    # General orientation: P = A + u (B-A) + v (C-A) with small dyadic data, the
    # segment passes P at parameter t0.  All values need few bits, so the
    # barycentrics and t come out exactly.
    rng = np.random.default_rng(7)
    for _ in range(200):
        A, B, C = (rng.integers(-16, 16, size=3) / 4.0 for _ in range(3))
        if np.linalg.norm(np.cross(B - A, C - A)) == 0:
            continue
        u = rng.integers(1, 8) / 32.0
        v = rng.integers(1, 8) / 32.0
        P = A + u * (B - A) + v * (C - A)
        d = rng.integers(-8, 9, size=3) / 8.0
        if abs(np.dot(d, np.cross(B - A, C - A))) == 0:
            continue
        t0 = rng.integers(1, 16) / 16.0
        O = P - t0 * d
        E = O + d
        V = np.array([A, B, C], np.float32)
        assert np.all(V.astype(np.float64) == np.array([A, B, C]))
        hit, j, uvt, _ = run1(V, UNIT_F, O, E)
        assert hit and j == 0
        assert tuple(uvt) == (u, v, t0)


@pytest.mark.parametrize("x,y,expect", [
    (0.25, 0.75, True),        # on the hypotenuse u + v = 1
    (0.5, 0.5, True),          # hypotenuse midpoint
    (0.0, 0.0, True),          # vertex A
    (1.0, 0.0, True),          # vertex B
    (0.0, 1.0, True),          # vertex C
    (0.5, 0.0, True),          # edge v = 0
    (0.0, 0.5, True),          # edge u = 0
    (1.0 + 2.0 ** -20, 0.0, False),
    (-(2.0 ** -20), 0.5, False),
    (0.5, -(2.0 ** -20), False),
    (0.5 + 2.0 ** -20, 0.5, False),  # just past the hypotenuse
])
def test_closed_triangle_boundary(x, y, expect):
    hit, j, uvt, _ = run1(UNIT_V, UNIT_F, (x, y, 1.0), (x, y, -1.0))
    assert hit == expect
    if expect:
        assert uvt[0] == x and uvt[1] == y and uvt[2] == 0.5


def test_segment_end_points():
    # start on the plane: t = 0; end on the plane: t = 1; both ends above: miss
    hit, _, uvt, _ = run1(UNIT_V, UNIT_F, (0.25, 0.25, 0.0), (0.25, 0.25, -1.0))
    assert hit and uvt[2] == 0.0
    hit, _, uvt, _ = run1(UNIT_V, UNIT_F, (0.25, 0.25, 1.0), (0.25, 0.25, 0.0))
    assert hit and uvt[2] == 1.0
    hit, *_ = run1(UNIT_V, UNIT_F, (0.25, 0.25, 1.0), (0.25, 0.25, 2.0 ** -30))
    assert not hit
    hit, *_ = run1(UNIT_V, UNIT_F, (0.25, 0.25, -(2.0 ** -30)), (0.25, 0.25, -1.0))
    assert not hit


def test_parallel_and_coplanar_are_misses():
    # d.z = 0: parallel above the plane, and coplanar straight across the triangle
    for o, e in [((0.1, 0.1, 0.5), (0.9, 0.05, 0.5)), ((-1.0, 0.25, 0.0), (2.0, 0.25, 0.0))]:
        hit, j, uvt, n = run1(UNIT_V, UNIT_F, o, e)
        assert not hit and j == -1 and n == 0 and np.all(np.isnan(uvt))


def test_zero_length_segment_is_a_miss():
    hit, *_ = run1(UNIT_V, UNIT_F, (0.25, 0.25, 0.0), (0.25, 0.25, 0.0))
    assert not hit


def test_first_hit_tie_breaks_to_lower_index():
    # coincident triangles 3 and 7 (the rest lie far away)
    V = np.concatenate([UNIT_V, UNIT_V + np.float32([10, 10, 0])]).astype(np.float32)
    F = np.array([[3, 4, 5]] * 8, np.int32)
    F[3] = F[7] = (0, 1, 2)
    hit, j, uvt, n = run1(V, F, (0.25, 0.25, 1.0), (0.25, 0.25, -1.0))
    assert hit and j == 3 and n == 2
    # two coplanar triangles sharing the edge x + y = 1; a segment through it
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], np.float32)
    F = np.array([[1, 3, 2], [0, 1, 2]], np.int32)
    hit, j, uvt, n = run1(V, F, (0.5, 0.5, 1.0), (0.5, 0.5, -1.0))
    assert hit and n == 2 and j == 0
    F = F[::-1].copy()
    hit, j, uvt, n = run1(V, F, (0.5, 0.5, 1.0), (0.5, 0.5, -1.0))
    assert hit and n == 2 and j == 0


def test_nearest_hit_among_stacked_layers():
    # layers at z = 0, 1, 2, 3 listed in scrambled order; a segment from z = 3.5
    # downward meets z = 3 first, one from -0.5 upward meets z = 0 first.
    layers = [2.0, 0.0, 3.0, 1.0]
    V = np.concatenate([UNIT_V + np.float32([0, 0, z]) for z in layers]).astype(np.float32)
    F = np.array([[3 * k, 3 * k + 1, 3 * k + 2] for k in range(4)], np.int32)
    hit, j, uvt, n = run1(V, F, (0.2, 0.3, 3.5), (0.2, 0.3, -0.5))
    assert hit and n == 4 and layers[j] == 3.0 and uvt[2] == 0.125
    hit, j, uvt, n = run1(V, F, (0.2, 0.3, -0.5), (0.2, 0.3, 3.5))
    assert hit and n == 4 and layers[j] == 0.0 and uvt[2] == 0.125


def test_case_study_1_scene(golden_case_study_1):
    """The paper's worked example: hit points (two decimals) and the printed
    boolean vector."""
    V, F, O, E = workloads.appendix_scene()
    hit, ids, uvt, _ = oracle.intersect(V, F, O, E)
    expect = [int(x) for x in golden_case_study_1["boolean"][0]]
    assert hit.tolist() == expect
    for ray, tri, x, y, z in golden_case_study_1["hit"]:
        r = int(ray)
        assert ids[r] == int(tri)
        p = O[r].astype(np.float64) + uvt[r, 2] * (E[r].astype(np.float64) - O[r].astype(np.float64))
        assert np.allclose(p, [float(x), float(y), float(z)], atol=0.005 + 1e-9)


def _heightfield_id(n, x, y):
    gx, gy = x * (n - 1), y * (n - 1)
    i, j = int(np.floor(gx)), int(np.floor(gy))
    fx, fy = gx - i, gy - j
    c = j * (n - 1) + i
    return 2 * c if fy < fx else 2 * c + 1, min(fx, fy, 1 - fx, 1 - fy, abs(fx - fy))


def test_heightfield_closed_form():
    """A vertical segment spanning the surface's z range crosses exactly one
    triangle; its index follows from the cell of (x, y) and the side of the
    cell diagonal, whatever the arithmetic of the test."""
    n = 24
    V, F = workloads.heightfield(n, 5)
    zlo, zhi = float(V[:, 2].min()), float(V[:, 2].max())
    rng = np.random.default_rng(3)
    O, E, want = [], [], []
    while len(want) < 400:
        x, y = rng.uniform(0.0, 1.0, 2)
        j, margin = _heightfield_id(n, x, y)
        if margin * 1.0 / (n - 1) < 1e-4:
            continue
        O.append((x, y, zhi + 1.0))
        E.append((x, y, zlo - 1.0))
        want.append(j)
    hit, ids, uvt, nh = oracle.intersect(V, F, np.array(O, np.float32), np.array(E, np.float32))
    assert np.all(hit == 1)
    assert np.all(nh == 1)
    assert ids.tolist() == want


def _random_pairs(rng, k):
    pts = rng.uniform(-1.0, 1.0, size=(k, 5, 3)).astype(np.float32)
    return pts


def _near_edge_pairs(rng, k):
    """Segments aimed at a point a hair away from a triangle edge or vertex."""
    out = []
    for _ in range(k):
        A, B, C = rng.uniform(-1.0, 1.0, size=(3, 3))
        lam = rng.uniform(0.0, 1.0)
        edge = rng.integers(0, 4)
        P = {0: A + lam * (B - A), 1: B + lam * (C - B), 2: C + lam * (A - C), 3: [A, B, C][rng.integers(0, 3)]}[int(edge)]
        P = P + rng.normal(size=3) * 10.0 ** rng.uniform(-9, -4)
        d = rng.normal(size=3)
        t0 = rng.uniform(0.0, 1.0)
        O = P - t0 * d
        out.append(np.array([A, B, C, O, O + d], np.float32))
    return out


def _check_against_exact(pairs, min_rel_margin=1e-9):
    V = np.concatenate([p[:3] for p in pairs]).astype(np.float32)
    checked = 0
    for k, p in enumerate(pairs):
        A, B, C, O, E = p
        hit, u, v, t, margin = oracle.exact(A, B, C, O, E)
        scale = max(1.0, float(np.abs(p).max())) ** 3
        if float(margin) < min_rel_margin * scale:
            continue
        F = np.array([[3 * k, 3 * k + 1, 3 * k + 2]], np.int32)
        h, j, uvt, _ = run1(V, F, O, E)
        assert h == hit, (k, p)
        if hit:
            assert abs(uvt[0] - float(u)) <= 1e-9 * max(1.0, abs(float(u)))
            assert abs(uvt[1] - float(v)) <= 1e-9 * max(1.0, abs(float(v)))
            assert abs(uvt[2] - float(t)) <= 1e-9 * max(1.0, abs(float(t)))
        checked += 1
    return checked


def test_exact_rationals_random_pairs():
    rng = np.random.default_rng(11)
    pairs = list(_random_pairs(rng, 3000))
    assert _check_against_exact(pairs) > 2900


def test_exact_rationals_near_boundary_pairs():
    rng = np.random.default_rng(12)
    pairs = _near_edge_pairs(rng, 3000)
    assert _check_against_exact(pairs) > 1500


def test_counts_and_first_hit_consistent_with_all_hits():
    V, F = workloads.heightfield(16, 9)
    O, E = workloads.rays_crossing_mix(300, 10)
    hit, ids, uvt, nh = oracle.intersect(V, F, O, E)
    for r in range(O.shape[0]):
        hid, huvt = oracle.all_hits(V, F, O[r], E[r])
        assert len(hid) == nh[r]
        assert bool(hit[r]) == (len(hid) > 0)
        if len(hid):
            k = np.lexsort((hid, huvt[:, 2]))[0]  # smallest t, then smallest index
            assert ids[r] == hid[k]
            assert np.array_equal(uvt[r], huvt[k])
        else:
            assert ids[r] == -1


def test_index_out_of_range_rejected():
    with pytest.raises(ValueError):
        oracle.intersect(UNIT_V, np.array([[0, 1, 3]], np.int32), np.zeros((1, 3)), np.ones((1, 3)))
    with pytest.raises(TypeError):
        oracle.intersect(UNIT_V, np.array([[0, 1, 2]], np.int64), np.zeros((1, 3)), np.ones((1, 3)))
