"""Intercept-count mode (paper: Background -- mode=intercept_count, the
number of unique intersections per ray) against the oracle's count of
distinct binary64 t, element by element: closed-form scenes, a heightfield
workload, segments with more distinct hits than a lane keeps (second pass),
forced stack overflow, sorted orders and the paper-scale configuration."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_01867_amd as rsi
from paper_2305_01867_amd import workloads
from gpu_helpers import dev, host, say

pytestmark = pytest.mark.gpu


def gpu_count(mesh, O, E, precision="certified", **kw):
    r = rsi.rsi_intersect(mesh, dev(O), dev(E), mode="intercept_count", precision=precision, **kw)
    return host(r["count"]), host(r["counters"])


def stacked(k):
    V, F = [], []
    for z in range(k):
        b = len(V)
        V += [(0, 0, z), (1, 0, z), (1, 1, z), (0, 1, z)]
        F += [(b, b + 1, b + 2), (b, b + 2, b + 3)]
    return np.array(V, np.float32), np.array(F, np.int32)


def test_closed_form_scenes():
    for k in (1, 3, 8, 11, 12, 13, 20, 40):  # more distinct hits than a lane keeps (certified 11, plain 12) go to the second pass
        V, F = stacked(k)
        O = np.array([[0.5, 0.5, k + 0.5], [0.75, 0.25, k + 0.5], [0.75, 0.25, -0.5], [2.0, 2.0, 1.0]], np.float32)
        E = np.array([[0.5, 0.5, -0.5], [0.75, 0.25, -0.5], [0.75, 0.25, 0.0], [2.0, 2.0, -1.0]], np.float32)
        want = oracle.intercept_count(V, F, O, E)
        assert want.tolist() == [k, k, 1, 0]
        with rsi.rsi_build(dev(V), dev(F)) as mesh:
            got, cnt = gpu_count(mesh, O, E)
            assert got.tolist() == want.tolist(), k
            # the segment on the layers' diagonal meets two triangles at one t
            # in every layer: overlapping intervals send it to the exact second
            # pass (counter 0) -- unless, past 12 layers, it fills the lane's
            # list first (counter 3); the other vertical one outgrows the list
            # past 12 distinct t
            if k <= 12:
                assert cnt[0] >= 1
            else:
                assert cnt[3] >= 1 and cnt[0] + cnt[3] >= 2
            plain, _ = gpu_count(mesh, O, E, "plain")
            assert plain.tolist() == want.tolist()
            hit = host(rsi.rsi_intersect(mesh, dev(O), dev(E), mode="intercept_count",
                                         out={"hit": torch.empty(4, dtype=torch.uint8, device="cuda")})["hit"])
            assert hit.tolist() == [1, 1, 1, 0]


@pytest.mark.parametrize("k", [200, 1100])
def test_more_hits_than_the_wave_list(k):
    """k stacked split layers: a vertical segment through the diagonals meets
    2k triangles at k points, one inside the triangles meets k.  The pass-2
    list holds 256 hits: at k = 200 the diagonal one (400 hits) is counted
    round by round and the other (200) from the list; at k = 1100 both take
    rounds."""
    V, F = stacked(k)
    O = np.array([[0.5, 0.5, k + 0.5], [0.75, 0.25, k + 0.5]], np.float32)
    E = np.array([[0.5, 0.5, -0.5], [0.75, 0.25, -0.5]], np.float32)
    want = oracle.intercept_count(V, F, O, E)
    assert want.tolist() == [k, k]
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        for prec in ("certified", "plain"):
            got, cnt = gpu_count(mesh, O, E, prec)
            assert got.tolist() == [k, k], prec
            assert cnt[3] == 2


def test_heightfield_counts_exact():
    V, F, O, E = workloads.tiny_config()
    want = oracle.intercept_count(V, F, O, E)
    _, _, _, nh = oracle.intersect(V, F, O, E)
    say(f"[count] tiny config: counts up to {want.max()}, {np.sum(want != nh)} segments with shared-point hits")
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        for stack, block in ((0, 0), (1, 64), (8, 128)):
            got, cnt = gpu_count(mesh, O, E, stack_depth=stack, block=block)
            bad = np.nonzero(got != want)[0]
            assert bad.size == 0, (stack, block, bad[:10], got[bad[:10]], want[bad[:10]])
            if stack == 1:
                assert cnt[1] > 0
        plain, _ = gpu_count(mesh, O, E, "plain")
        assert np.mean(plain == want) > 0.995
        for order in ("midpoint", "origin_octant"):
            got, _ = gpu_count(mesh, O, E, ray_sort=order)
            assert np.array_equal(got, want), order


def test_grid_vertices_and_edges():
    """Segments through the vertices and edges of a flat dyadic grid: the
    certified count merges the triangles met at one point."""
    n = 9
    xs = np.arange(n) / (n - 1)
    V = np.array([(xs[i], xs[j], 0.0) for j in range(n) for i in range(n)], np.float32)
    F = []
    for j in range(n - 1):
        for i in range(n - 1):
            v = lambda a, b: b * n + a
            F += [(v(i, j), v(i + 1, j), v(i + 1, j + 1)), (v(i, j), v(i + 1, j + 1), v(i, j + 1))]
    F = np.array(F, np.int32)
    rng = np.random.default_rng(4)
    pts = rng.integers(0, 4 * (n - 1) + 1, size=(3000, 2)) / (4 * (n - 1))  # on vertices, edges, inside
    O = np.concatenate([pts, np.ones((3000, 1))], 1).astype(np.float32)
    E = np.concatenate([pts, -np.ones((3000, 1))], 1).astype(np.float32)
    want = oracle.intercept_count(V, F, O, E)
    _, _, _, nh = oracle.intersect(V, F, O, E)
    assert np.all(want[nh > 0] == 1) and np.any(nh >= 6)
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        got, _ = gpu_count(mesh, O, E)
        assert np.array_equal(got, want)


def test_paper_scale_sampled():
    """1e7 segments on the benchmark's tree (restructured, 4-wide first pass),
    sampled against the oracle."""
    V, F, O, E = workloads.paper_scale_config()
    rng = np.random.default_rng(8)
    idx = rng.choice(O.shape[0], 2500, replace=False)
    want = oracle.intercept_count(V, F, O[idx], E[idx])
    with rsi.rsi_build(dev(V), dev(F), algorithm="restructured") as mesh:
        r = rsi.rsi_intersect(mesh, dev(O), dev(E), mode="intercept_count", precision="certified")
        got = host(r["count"])
        cnt = host(r["counters"])
        say(f"[count] paper scale: mean count {got.mean():.3f}, max {got.max()}, list overflow {cnt[3]}, "
            f"stack overflow {cnt[1]}")
        assert np.array_equal(got[idx], want)
        hit = host(rsi.rsi_intersect(mesh, dev(O), dev(E), mode="boolean", precision="certified")["hit"])
        assert np.array_equal(got > 0, hit == 1)
