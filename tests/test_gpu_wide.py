"""The 4-wide tree: structure against the binary tree it is collapsed from,
and the first pass over it against the binary first pass and the oracle,
element by element, in every mode and precision."""
import numpy as np
import pytest

import oracle
import paper_2305_01867_amd as rsi
from paper_2305_01867_amd import diagnostics, workloads
from gpu_helpers import dev, export, intersect, say

pytestmark = pytest.mark.gpu

MODES = ("boolean", "first_hit", "barycentric", "intercept_count")


def soup(n_tri, seed, n_vert=600, clustered=False):
    rng = np.random.default_rng(seed)
    V = rng.uniform(-1.0, 1.0, size=(n_vert, 3))
    if clustered:
        V = np.round(V * 4) / 4
    F = rng.integers(0, n_vert, size=(n_tri, 3))
    return V.astype(np.float32), F.astype(np.int32)


def mesh_case(case):
    if case == "scene":
        V, F, _, _ = workloads.appendix_scene()
    elif case.startswith("soup"):
        V, F = soup(int(case[4:]), int(case[4:]))
    elif case == "duplicates":
        V, F = soup(5000, 3, n_vert=300, clustered=True)
    else:
        V, F = workloads.heightfield(int(case[2:]), 21)
    return V, F


@pytest.mark.parametrize("algorithm", ["radix_tree", "restructured"])
@pytest.mark.parametrize("case", ["scene", "soup2", "soup3", "soup1023", "soup1024", "soup1025", "soup2049",
                                  "duplicates", "hf128", "hf401"])
def test_wide_tree_matches_the_binary_tree(case, algorithm):
    V, F = mesh_case(case)
    say(f"[wide] {case} {algorithm}: {F.shape[0]} triangles")
    with rsi.rsi_build(dev(V), dev(F), algorithm=algorithm) as mesh:
        assert rsi.rsi_mesh_info_get(mesh)["node_width"] == 4
        tree = diagnostics.export(mesh)
        wide = diagnostics.decode_wide(export(mesh, "wide_nodes"))
        top = diagnostics.decode_wide(export(mesh, "wide_top"))
    problems = diagnostics.check_wide(wide, top, tree)
    assert problems == [], problems[:5]


def test_width_of_other_builds():
    V, F = mesh_case("hf64")
    with rsi.rsi_build(dev(V), dev(F), algorithm="agglomerative") as mesh:
        assert rsi.rsi_mesh_info_get(mesh)["node_width"] == 2
        assert export(mesh, "wide_nodes").shape[0] == 0
        O, E = workloads.rays_in_box(100, 5, V.min(axis=0), V.max(axis=0))
        with pytest.raises(rsi.RSIError) as e:
            rsi.rsi_intersect(mesh, dev(O), dev(E), node_width=4)
        assert e.value.status == 1
    with rsi.rsi_build(dev(V[:3]), dev(np.array([[0, 1, 2]], np.int32))) as mesh:
        assert rsi.rsi_mesh_info_get(mesh)["node_width"] == 2  # one leaf: nothing to collapse
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        with pytest.raises(rsi.RSIError) as e:
            rsi.rsi_intersect(mesh, dev(O), dev(E), node_width=3)
        assert e.value.status == 1


def compare(mesh, O, E, mode, precision, **kw):
    a = intersect(mesh, O, E, mode, precision, node_width=4, **kw)
    b = intersect(mesh, O, E, mode, precision, node_width=2, **kw)
    for k in a:
        if k != "counters":  # uvt is NaN on a miss in both
            assert np.array_equal(a[k], b[k], equal_nan=(k == "uvt")), (mode, precision, k)
    return a


@pytest.mark.parametrize("algorithm", ["radix_tree", "restructured"])
def test_wide_equals_binary_and_oracle(algorithm):
    V, F = workloads.heightfield(48, 9)
    lo, hi = V.min(axis=0), V.max(axis=0)
    O, E = workloads.rays_in_box(20000, 31, lo, hi)
    o_hit, o_id, o_uvt, _ = oracle.intersect(V, F, O, E)
    o_cnt = oracle.intercept_count(V, F, O, E)
    with rsi.rsi_build(dev(V), dev(F), algorithm=algorithm) as mesh:
        for precision in ("plain", "certified"):
            for mode in MODES:
                say(f"[wide] {algorithm} {mode} {precision}")
                a = compare(mesh, O, E, mode, precision)
                if precision != "certified":
                    continue
                if mode == "boolean":
                    assert np.array_equal(a["hit"], o_hit)
                elif mode == "intercept_count":
                    assert np.array_equal(a["count"], o_cnt)
                else:
                    assert np.array_equal(a["tri_id"], o_id)
                    if mode == "barycentric":
                        h = o_id >= 0
                        assert np.allclose(a["uvt"][h], o_uvt[h], rtol=0, atol=1e-5)


def test_wide_with_a_tiny_stack_goes_through_the_second_pass():
    """Stack depth 1: most segments outgrow the 4-wide push and are finished
    by the deep-stack pass, results unchanged."""
    V, F = workloads.heightfield(32, 4)
    O, E = workloads.rays_in_box(5000, 8, V.min(axis=0), V.max(axis=0))
    o_hit, o_id, _, _ = oracle.intersect(V, F, O, E)
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        for mode in ("boolean", "first_hit"):
            a = compare(mesh, O, E, mode, "certified", stack_depth=1)
            assert a["counters"][1] > 0
            assert np.array_equal(a["hit"] if mode == "boolean" else a["tri_id"],
                                  o_hit if mode == "boolean" else o_id)


def test_wide_visits_fewer_nodes():
    V, F, O, E = workloads.paper_scale_config(200_000)
    with rsi.rsi_build(dev(V), dev(F), algorithm="restructured") as mesh:
        v4, t4 = rsi.rsi_traversal_stats(mesh, dev(O), dev(E), mode="boolean", precision="certified", node_width=4)
        v2, t2 = rsi.rsi_traversal_stats(mesh, dev(O), dev(E), mode="boolean", precision="certified", node_width=2)
        m4, m2 = float(v4.double().mean()), float(v2.double().mean())
        say(f"[wide] mean node fetches per segment: 4-wide {m4:.2f}, binary {m2:.2f}")
        assert m4 < 0.7 * m2
