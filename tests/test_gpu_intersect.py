"""GPU intersection vs the binary64 oracle, element by element.

CERTIFIED precision must reproduce the oracle exactly: hit flags and triangle
ids bit for bit, and (u, v, t) equal to the oracle's binary64 values rounded
to float32 (well inside the 1e-5 relative budget).  PLAIN precision is the
binary32 reference form: it may differ only on near-degenerate segments, and
such segments must be ones CERTIFIED re-decides in binary64."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_01867_amd as rsi
from paper_2305_01867_amd import workloads
from gpu_helpers import dev, host, intersect, say

pytestmark = pytest.mark.gpu
MODES = ("boolean", "first_hit", "barycentric")


def expect_exact(got, want_hit, want_id, want_uvt, mode):
    if mode == "boolean":
        bad = np.nonzero(got["hit"] != want_hit)[0]
        assert bad.size == 0, f"{bad.size} boolean mismatches, first rays {bad[:10]}"
        return
    bad = np.nonzero(got["tri_id"] != want_id)[0]
    assert bad.size == 0, f"{bad.size} id mismatches, first {bad[:10]} got {got['tri_id'][bad[:10]]} want {want_id[bad[:10]]}"
    if mode == "barycentric":
        g = got["uvt"]
        w = want_uvt.astype(np.float32)
        assert np.array_equal(np.isnan(g), np.isnan(w))
        m = ~np.isnan(w)
        assert np.all(g[m] == w[m]), "uvt differ from the rounded binary64 values"
        rel = np.abs(g[m].astype(np.float64) - want_uvt[m]) / np.maximum(1.0, np.abs(want_uvt[m]))
        assert rel.max(initial=0.0) <= 1e-5


def check_all_modes(V, F, O, E, label, plain_budget=None, **kw):
    say(f"[intersect] {label}: {F.shape[0]} triangles, {O.shape[0]} segments")
    hit, ids, uvt, _ = oracle.intersect(V, F, O, E)
    bkeys = ("morton_bits", "algorithm")
    with rsi.rsi_build(dev(V), dev(F), **{k: v for k, v in kw.items() if k in bkeys}) as mesh:
        ikw = {k: v for k, v in kw.items() if k not in bkeys}
        for mode in MODES:
            say(f"  mode={mode} certified")
            got = intersect(mesh, O, E, mode, "certified", **ikw)
            expect_exact(got, hit, ids, uvt, mode)
            say(f"  mode={mode} plain")
            plain = intersect(mesh, O, E, mode, "plain", **ikw)
            key = "hit" if mode == "boolean" else "tri_id"
            want = hit if mode == "boolean" else ids
            n_bad = int(np.sum(plain[key] != want))
            say(f"    plain mismatches: {n_bad}; certified re-decided: {int(got['counters'][0])}, "
                f"stack overflow: {int(got['counters'][1])}")
            if plain_budget is not None:
                assert n_bad <= plain_budget
            assert n_bad <= int(got["counters"][0]), "plain differs on segments certified did not re-decide"
    return hit, ids, uvt


def test_case_study_1_scene(golden_case_study_1):
    V, F, O, E = workloads.appendix_scene()
    hit, ids, uvt = check_all_modes(V, F, O, E, "case study 1")
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        got = intersect(mesh, O, E, "boolean")
        assert got["hit"].tolist() == [int(x) for x in golden_case_study_1["boolean"][0]]
        got = intersect(mesh, O, E, "barycentric")
        for ray, tri, x, y, z in golden_case_study_1["hit"]:
            r = int(ray)
            assert got["tri_id"][r] == int(tri)
            p = O[r] + got["uvt"][r, 2] * (E[r] - O[r])
            assert np.allclose(p, [float(x), float(y), float(z)], atol=0.006)


def test_tiny_heightfield_config():
    V, F, O, E = workloads.tiny_config()
    check_all_modes(V, F, O, E, "64x64 heightfield, 1e4 crossing-mix segments", plain_budget=20)
    check_all_modes(V, F, O, E, "same, agglomerative build", algorithm="agglomerative")
    check_all_modes(V, F, O, E, "same, restructured tree", algorithm="restructured")
    check_all_modes(V, F, O, E, "same, 63-bit keys, stack 8, block 64", morton_bits=63, stack_depth=8, block=64)


def test_heightfield_vertical_closed_form():
    n = 48
    V, F = workloads.heightfield(n, 4)
    rng = np.random.default_rng(8)
    xy = rng.uniform(0.0, 1.0, size=(5000, 2))
    gx, gy = xy[:, 0] * (n - 1), xy[:, 1] * (n - 1)
    fx, fy = gx - np.floor(gx), gy - np.floor(gy)
    margin = np.minimum.reduce([fx, fy, 1 - fx, 1 - fy, np.abs(fx - fy)])
    xy = xy[margin > 1e-3]
    gx, gy = xy[:, 0] * (n - 1), xy[:, 1] * (n - 1)
    c = np.floor(gy).astype(np.int64) * (n - 1) + np.floor(gx).astype(np.int64)
    want = np.where(gy - np.floor(gy) < gx - np.floor(gx), 2 * c, 2 * c + 1)
    O = np.concatenate([xy, np.full((len(xy), 1), 2.0)], axis=1).astype(np.float32)
    E = np.concatenate([xy, np.full((len(xy), 1), -2.0)], axis=1).astype(np.float32)
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        for prec in ("plain", "certified"):
            got = intersect(mesh, O, E, "first_hit", prec)
            assert np.array_equal(got["tri_id"], want)


def dyadic_grid(n=9, tilt=(0.25, 0.125)):
    """A tilted plane z = a x + b y triangulated on an integer grid, all
    coordinates small dyadic numbers: every edge, vertex and plane point a
    segment aims at is representable exactly."""
    g = np.arange(n, dtype=np.float64)
    x, y = np.meshgrid(g, g, indexing="xy")
    z = tilt[0] * x + tilt[1] * y
    V = np.stack([x.ravel(), y.ravel(), z.ravel()], 1).astype(np.float32)
    i, j = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="xy")
    i, j = i.ravel(), j.ravel()
    F = np.empty((2 * (n - 1) ** 2, 3), np.int64)
    F[0::2] = np.stack([j * n + i, j * n + i + 1, (j + 1) * n + i + 1], 1)
    F[1::2] = np.stack([j * n + i, (j + 1) * n + i + 1, (j + 1) * n + i], 1)
    return V, F.astype(np.int32), tilt


def adversarial_segments(n, tilt, k, seed):
    """Segments through grid vertices, edge points and cell diagonals, some
    with an end point exactly on the plane, some parallel to it (above or in
    it), some of zero length."""
    rng = np.random.default_rng(seed)
    P = []
    for _ in range(k):
        kind = rng.integers(0, 4)
        if kind == 0:
            x, y = rng.integers(0, n, 2).astype(float)
        elif kind == 1:
            x, y = float(rng.integers(0, n)), rng.integers(0, 8 * (n - 1)) / 8.0
            if rng.uniform() < 0.5:
                x, y = y, x
        elif kind == 2:
            t = rng.integers(0, 8 * (n - 1)) / 8.0
            x = y = t
            off = float(rng.integers(0, n - 2))
            x += off
            x = min(x, n - 1.0)
        else:
            x, y = rng.integers(0, 8 * (n - 1), 2) / 8.0
        P.append((x, y, tilt[0] * x + tilt[1] * y))
    P = np.array(P)
    O, E = [], []
    for p in P:
        kind = rng.integers(0, 6)
        d = rng.integers(-4, 5, 3) / 4.0
        if kind == 0:      # through p, interior
            O.append(p - 0.5 * d - [0, 0, 1]); E.append(p + 0.5 * d + [0, 0, 1])
        elif kind == 1:    # starts on the plane at p
            O.append(p); E.append(p + [d[0], d[1], 1.0 + abs(d[2])])
        elif kind == 2:    # ends on the plane at p
            O.append(p + [d[0], d[1], 1.0 + abs(d[2])]); E.append(p)
        elif kind == 3:    # in the plane through p
            v = np.array([1.0, 1.0, tilt[0] + tilt[1]]) * rng.integers(1, 4)
            O.append(p - v); E.append(p + v)
        elif kind == 4:    # parallel, above
            v = np.array([1.0, -1.0, tilt[0] - tilt[1]])
            O.append(p - v + [0, 0, 0.5]); E.append(p + v + [0, 0, 0.5])
        else:              # zero length on the plane
            O.append(p); E.append(p)
    return np.array(O, np.float32), np.array(E, np.float32)


def test_adversarial_edges_vertices_parallel():
    V, F, tilt = dyadic_grid()
    O, E = adversarial_segments(9, tilt, 3000, 5)
    check_all_modes(V, F, O, E, "dyadic grid adversarial")


def test_near_edge_and_near_parallel_segments():
    V, F = workloads.heightfield(40, 12)
    rng = np.random.default_rng(13)
    O, E = [], []
    for k in range(4000):
        t = int(rng.integers(0, F.shape[0]))
        A, B, C = V[F[t]].astype(np.float64)
        if k % 2 == 0:  # aimed within ~1e-7 (relative) of an edge or a vertex
            lam = rng.uniform(0.05, 0.95)
            p = [A + lam * (B - A), B + lam * (C - B), A, B][int(rng.integers(0, 4))]
            p = p + rng.normal(size=3) * 1e-7 * np.abs(p).max()
            d = rng.normal(size=3)
            d[2] = np.sign(d[2]) * max(abs(d[2]), 0.3)
            h = rng.uniform(0.05, 0.5)
            O.append(p - h * d); E.append(p + h * d)
        else:  # nearly parallel to the triangle's plane, through an interior point
            nrm = np.cross(B - A, C - A); nrm /= np.linalg.norm(nrm)
            u = rng.normal(size=3); u -= nrm * u.dot(nrm); u /= np.linalg.norm(u)
            th = rng.uniform(0.0, 1e-6)
            d = np.cos(th) * u + np.sin(th) * nrm
            p = A + 0.3 * (B - A) + 0.3 * (C - A) + nrm * rng.uniform(-1e-7, 1e-7)
            h = rng.uniform(0.01, 0.1)
            O.append(p - h * d); E.append(p + h * d)
    O, E = np.array(O, np.float32), np.array(E, np.float32)
    check_all_modes(V, F, O, E, "near-edge / near-parallel heightfield segments")


def test_stack_depth_one_and_block_sizes_stay_exact():
    V, F = workloads.heightfield(32, 21)
    O, E = workloads.rays_in_box(4000, 22, V.min(0), V.max(0))
    hit, ids, uvt, _ = oracle.intersect(V, F, O, E)
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        for stack in (1, 2, 5, 64):
            for block in (64, 128, 256, 512, 1024):  # 4-wide first pass; binary runs at most 256
                say(f"  stack={stack} block={block}")
                for mode in MODES:
                    got = intersect(mesh, O, E, mode, "certified", stack_depth=stack, block=block)
                    expect_exact(got, hit, ids, uvt, mode)
                    if stack == 1:
                        assert got["counters"][1] > 0


def test_segment_orders_exact_and_every_segment_once():
    """Sorted processing orders write every result at its input index: outputs
    prefilled with sentinels are all overwritten with the oracle's values, and
    every segment is traversed (its root fetched) exactly as in input order.
    (Per-segment node counts may differ between orders: a postponed leaf test
    tightens the nearest-hit limit at a moment that depends on the wave.)"""
    V, F = workloads.heightfield(32, 21)
    for n in (1, 65, 2049, 5000):
        O, E = workloads.rays_in_box(n, 30 + n, V.min(0), V.max(0))
        hit, ids, uvt, _ = oracle.intersect(V, F, O, E)
        with rsi.rsi_build(dev(V), dev(F)) as mesh:
            for order in ("midpoint", "origin_octant"):
                say(f"  n={n} order={order}")
                for mode in MODES:
                    out = {"hit": torch.full((n,), 7, dtype=torch.uint8, device="cuda"),
                           "tri_id": torch.full((n,), -7, dtype=torch.int32, device="cuda")}
                    if mode == "barycentric":
                        out["uvt"] = torch.full((n, 3), 5.0, dtype=torch.float32, device="cuda")
                    r = rsi.rsi_intersect(mesh, dev(O), dev(E), mode=mode, precision="certified", ray_sort=order,
                                          out=out)
                    got = {k: host(v) for k, v in r.items()}
                    assert np.array_equal(got["hit"], hit), (order, mode)
                    expect_exact(got, hit, ids, uvt, mode)
                plain_in = intersect(mesh, O, E, "first_hit", "plain")
                plain_sorted = intersect(mesh, O, E, "first_hit", "plain", ray_sort=order)
                assert np.array_equal(plain_in["tri_id"], plain_sorted["tri_id"])
                visits, _ = rsi.rsi_traversal_stats(mesh, dev(O), dev(E), mode="first_hit", ray_sort=order)
                assert host(visits).min() >= 1


def test_ragged_and_edge_sizes():
    V, F = workloads.heightfield(20, 3)
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        for n in (0, 1, 63, 64, 65, 255, 257, 1000):
            O, E = workloads.rays_crossing_mix(n, n + 1)
            hit, ids, uvt, _ = oracle.intersect(V, F, O, E)
            for mode in MODES:
                if n == 0:
                    r = rsi.rsi_intersect(mesh, dev(O.reshape(0, 3)), dev(E.reshape(0, 3)), mode=mode)
                    assert host(r["counters"]).tolist() == [0, 0, 0, 0]
                    continue
                expect_exact(intersect(mesh, O, E, mode), hit, ids, uvt, mode)


def test_single_triangle_and_empty_mesh():
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    F = np.array([[0, 1, 2]], np.int32)
    O, E = workloads.rays_crossing_mix(500, 9)
    O[:, :2] *= 0.8
    check_all_modes(V, F, O, E, "single triangle")
    with rsi.rsi_build(dev(V), dev(F[:0])) as mesh:
        assert rsi.rsi_mesh_info_get(mesh)["root"] == -(2 ** 31)
        for mode in MODES:
            got = intersect(mesh, O, E, mode)
            if mode == "boolean":
                assert np.all(got["hit"] == 0)
            else:
                assert np.all(got["tri_id"] == -1)
            if mode == "barycentric":
                assert np.all(np.isnan(got["uvt"]))


def test_unchecked_invalid_triangles_are_never_hit():
    V, F = workloads.heightfield(16, 2)
    bad = F.copy()
    bad[10] = (0, 1, V.shape[0] + 5)
    O, E = workloads.rays_crossing_mix(2000, 4)
    good_mask = np.ones(F.shape[0], bool)
    good_mask[10] = False
    # the oracle over the valid triangles only, ids mapped back
    keep = np.nonzero(good_mask)[0]
    hit, ids, uvt, _ = oracle.intersect(V, F[keep], O, E)
    ids = np.where(ids >= 0, keep[np.maximum(ids, 0)], -1)
    with rsi.rsi_build(dev(V), dev(bad)) as mesh:
        for mode in MODES:
            expect_exact(intersect(mesh, O, E, mode), hit, ids, uvt, mode)


def test_non_finite_segments_are_misses():
    V, F = workloads.heightfield(16, 2)
    O, E = workloads.rays_crossing_mix(256, 4)
    O[::3, 0] = np.nan
    E[1::5, 2] = 1e30  # finite but far: the widened boxes then admit everything
    hit, ids, uvt, _ = oracle.intersect(V, F, O, E)
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        for mode in MODES:
            expect_exact(intersect(mesh, O, E, mode, "certified"), hit, ids, uvt, mode)


def test_paper_scale_sampled():
    """128 x 128 heightfield (32,258 triangles), 1e7 segments, the launch
    configuration the benchmark times (restructured tree, 4-wide first pass,
    default launch).  Every segment where PLAIN and CERTIFIED disagree, plus a
    random sample, is checked against the oracle."""
    V, F, O, E = workloads.paper_scale_config()
    say(f"[intersect] paper scale: {F.shape[0]} triangles, {O.shape[0]} segments")
    rng = np.random.default_rng(0)
    sample = rng.choice(O.shape[0], 3000, replace=False)
    with rsi.rsi_build(dev(V), dev(F), algorithm="restructured") as mesh:
        assert rsi.rsi_mesh_info_get(mesh)["node_width"] == 4
        dO, dE = dev(O), dev(E)
        for mode in MODES:
            cert = rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision="certified")
            plain = rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision="plain")
            key = "hit" if mode == "boolean" else "tri_id"
            c, p = host(cert[key]), host(plain[key])
            diff = np.nonzero(c != p)[0]
            cnt = host(cert["counters"])
            say(f"  mode={mode}: plain/certified differ on {diff.size}; re-decided {cnt[0]}, overflow {cnt[1]}")
            idx = np.unique(np.concatenate([sample, diff[:2000]]))
            hit, ids, uvt, _ = oracle.intersect(V, F, O[idx], E[idx])
            sub = {k: host(v)[idx] for k, v in cert.items() if k != "counters"}
            expect_exact(sub, hit, ids, uvt, mode)
            if mode == "boolean":
                frac = float(c.mean())
                say(f"  hit fraction {frac:.4f}")
                with rsi.rsi_build(dev(V), dev(F)) as rmesh:  # the paper's radix tree
                    r = host(rsi.rsi_intersect(rmesh, dO, dE, mode=mode, precision="certified")["hit"])
                    assert np.array_equal(r, c), "radix tree"
                    r = host(rsi.rsi_intersect(rmesh, dO, dE, mode=mode, precision="certified",
                                               node_width=2)["hit"])
                    assert np.array_equal(r, c), "radix tree, binary nodes"
                    v0, _ = rsi.rsi_traversal_stats(rmesh, dO, dE, mode=mode, precision="certified")
                    v1, _ = rsi.rsi_traversal_stats(mesh, dO, dE, mode=mode, precision="certified")
                    m0, m1 = float(v0.double().mean()), float(v1.double().mean())
                    say(f"  mean 4-wide node fetches: radix tree {m0:.2f}, restructured {m1:.2f}")
                    assert m1 < m0
                for order in ("midpoint", "origin_octant"):  # the multi-block scan path of the sort
                    srt = host(rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision="certified",
                                                 ray_sort=order)["hit"])
                    assert np.array_equal(srt, c), order
            del cert, plain
            torch.cuda.empty_cache()
