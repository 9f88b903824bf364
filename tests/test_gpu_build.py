"""GPU build vs the oracle, bit for bit: Morton keys, stable sort order, radix
tree topology, child boxes, completion counters (the paper's Case Study 2
bar: every internal node reached twice), parents, leaf triangles, extent."""
import numpy as np
import pytest

import oracle
import paper_2305_01867_amd as rsi
from paper_2305_01867_amd import workloads
from gpu_helpers import decode_nodes, dev, export, say

pytestmark = pytest.mark.gpu


def triangle_soup(n_tri, seed, n_vert=600, clustered=False):
    rng = np.random.default_rng(seed)
    V = rng.uniform(-1.0, 1.0, size=(n_vert, 3))
    if clustered:
        V = np.round(V * 4) / 4  # many identical centroids -> duplicate keys
    F = rng.integers(0, n_vert, size=(n_tri, 3))
    return V.astype(np.float32), F.astype(np.int32)


def check_structure(V, F, bits):
    nt = F.shape[0]
    say(f"[build] n_tri={nt} n_vert={V.shape[0]} bits={bits}")
    want = oracle.build_structure(V, F, bits)
    with rsi.rsi_build(dev(V), dev(F), morton_bits=bits) as mesh:
        info = rsi.rsi_mesh_info_get(mesh)
        assert info["n_triangles"] == nt and info["morton_bits"] == bits
        keys = export(mesh, "sorted_keys").view(np.uint64)
        assert np.array_equal(keys, want["sorted_keys"]), "sorted keys differ"
        ids = export(mesh, "sorted_ids")
        assert np.array_equal(ids, want["order"]), "sort order differs"

        leaves = export(mesh, "leaves")
        lf = leaves.view(np.float32)
        order = want["order"].astype(np.int64)
        A = V[F[order, 0]]
        B = V[F[order, 1]]
        C = V[F[order, 2]]
        assert np.array_equal(lf[:, 0:3], A)
        assert np.array_equal(leaves[:, 3], want["order"])
        assert np.array_equal(lf[:, 4:7], B - A)
        assert np.array_equal(lf[:, 8:11], C - A)

        bounds = export(mesh, "bounds")
        lo, hi = oracle.mesh_bounds(V)
        assert np.array_equal(bounds[:3], lo) and np.array_equal(bounds[3:6], hi)
        assert bounds[6] == np.max(np.abs(np.concatenate([lo, hi])))

        if nt < 2:
            assert info["root"] == -1
            return
        assert info["root"] == 0
        words = export(mesh, "nodes")
        lref, rref, lbox, rbox = decode_nodes(words)
        t = want["tree"]
        want_l = np.where(t["left_leaf"] == 1, ~t["left"], t["left"])
        want_r = np.where(t["right_leaf"] == 1, ~t["right"], t["right"])
        assert np.array_equal(lref, want_l), "left children differ"
        assert np.array_equal(rref, want_r), "right children differ"
        assert np.array_equal(words[:, 14], t["first"]) and np.array_equal(words[:, 15], t["last"])

        def child_boxes(idx, is_leaf):
            return np.where(is_leaf[:, None] == 1, want["leaf_boxes"][idx], want["node_boxes"][np.minimum(idx, nt - 2)])

        assert np.array_equal(lbox, child_boxes(t["left"], t["left_leaf"])), "left boxes differ"
        assert np.array_equal(rbox, child_boxes(t["right"], t["right_leaf"])), "right boxes differ"

        counters = export(mesh, "counters")
        assert np.all(counters == 2), f"{np.sum(counters != 2)} internal nodes not completed"

        parents = export(mesh, "parents")
        want_par = np.full(2 * nt - 1, -7, np.int64)
        want_par[0] = -1
        for i in range(nt - 1):
            for c, leaf in ((t["left"][i], t["left_leaf"][i]), (t["right"][i], t["right_leaf"][i])):
                want_par[(nt - 1 + c) if leaf else c] = i
        assert np.array_equal(parents, want_par)


def test_case_study_1_scene_structure():
    V, F, _, _ = workloads.appendix_scene()
    for bits in (30, 63):
        check_structure(V, F, bits)


@pytest.mark.parametrize("n_tri", [1, 2, 3, 63, 64, 65, 1023, 1024, 1025, 2047, 2048, 2049, 29260])
def test_soup_sizes(n_tri):
    V, F = triangle_soup(n_tri, n_tri)
    check_structure(V, F, 30)
    check_structure(V, F, 63)


@pytest.mark.parametrize("n_side", [2, 3, 33, 64, 128, 256, 400, 401])  # 400+: multi-block histogram scan
def test_heightfields(n_side):
    V, F = workloads.heightfield(n_side, 100 + n_side)
    check_structure(V, F, 30 if n_side % 2 == 0 else 63)


def test_duplicate_keys_and_degenerate_triangles():
    V, F = triangle_soup(5000, 3, n_vert=300, clustered=True)
    F[::7, 1] = F[::7, 0]  # repeated index: zero-area triangle
    check_structure(V, F, 30)
    check_structure(V, F, 63)
    # every triangle with the same centroid: all keys equal
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 1]], np.float32)
    F = np.tile(np.array([[0, 1, 2]], np.int32), (777, 1))
    check_structure(V, F, 30)


def test_build_is_deterministic():
    V, F = workloads.heightfield(96, 7)
    outs = []
    for _ in range(3):
        with rsi.rsi_build(dev(V), dev(F)) as mesh:
            outs.append([export(mesh, w).tobytes() for w in ("sorted_keys", "sorted_ids", "nodes", "parents",
                                                              "counters", "leaves", "bounds")])
    assert outs[0] == outs[1] == outs[2]


def test_index_check_and_invalid_triangles():
    V, F = workloads.heightfield(8, 1)
    bad = F.copy()
    bad[5, 2] = V.shape[0]  # one past the end
    with pytest.raises(rsi.RSIError) as e:
        rsi.rsi_build(dev(V), dev(bad), check_indices=True)
    assert e.value.status == 2
    bad[6, 0] = -3
    with rsi.rsi_build(dev(V), dev(bad)) as mesh:  # unchecked: the bad triangles are never hit
        counters = export(mesh, "counters")
        assert np.all(counters == 2)


def test_host_pointer_rejected():
    import ctypes
    V = np.zeros((3, 3), np.float32)
    F = np.array([[0, 1, 2]], np.int32)
    h = ctypes.c_void_p()
    st = rsi.lib().rsi_build(V.ctypes.data_as(ctypes.c_void_p), 3, F.ctypes.data_as(ctypes.c_void_p), 1, None,
                             None, ctypes.byref(h))
    assert st == 1 and b"device pointer" in rsi.lib().rsi_last_error()


def test_diagnostics_on_the_device_tree():
    """The exported device tree decodes into the paper's Case Study 1 graph
    (root [0,3]; [0,1] and [2,3]; leaves [0] 0, [1] 3, [2] 1, [3] 2) and a
    large tree passes the structural checks."""
    from paper_2305_01867_amd import diagnostics
    V, F, _, _ = workloads.appendix_scene()
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        tree = diagnostics.export(mesh)
    assert diagnostics.check(tree, contiguous=True) == []
    dot = diagnostics.to_dot(tree)
    leaves = sorted(l.split('label="')[1].split('"')[0] for l in dot.splitlines() if "shape=box" in l)
    assert leaves == ["[0] 0", "[1] 3", "[2] 1", "[3] 2"]
    assert 'n0 [label="[0,3]", style=bold];' in dot
    V, F = workloads.heightfield(128, 21)
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        assert diagnostics.check(diagnostics.export(mesh)) == []


def canonical(words, n):
    """{(first, last): (left range, right range)} of a tree in the export layout."""
    rng = lambda r: (~r, ~r) if r < 0 else (int(words[r, 14]), int(words[r, 15]))
    return {(int(w[14]), int(w[15])): (rng(int(w[12])), rng(int(w[13]))) for w in words}


@pytest.mark.parametrize("case", ["scene", "heightfield", "duplicates"])
def test_agglomerative_build_is_the_same_tree(case):
    """The single-pass agglomerative build gives the radix tree's topology and
    boxes, numbered by split position: the paper's Case Study 1 dump has its
    root at internal index 1."""
    from paper_2305_01867_amd import diagnostics
    if case == "scene":
        V, F, _, _ = workloads.appendix_scene()
    elif case == "heightfield":
        V, F = workloads.heightfield(100, 4)
    else:
        V, F = triangle_soup(5000, 3, n_vert=300, clustered=True)
    for bits in (30, 63):
        with rsi.rsi_build(dev(V), dev(F), morton_bits=bits) as a, \
                rsi.rsi_build(dev(V), dev(F), morton_bits=bits, algorithm="agglomerative") as b:
            wa, wb = export(a, "nodes"), export(b, "nodes")
            assert canonical(wa, F.shape[0]) == canonical(wb, F.shape[0])
            ta, tb = diagnostics.export(a), diagnostics.export(b)
            assert diagnostics.check(tb) == []
            ka = {(f, l): tuple(bx) for f, l, bx in zip(ta["first"], ta["last"], ta["box"])}
            kb = {(f, l): tuple(bx) for f, l, bx in zip(tb["first"], tb["last"], tb["box"])}
            assert ka == kb
            assert np.array_equal(export(a, "leaves"), export(b, "leaves"))
            assert rsi.rsi_mesh_info_get(b)["root"] == tb["root"]
            if case == "scene":
                assert tb["root"] == 1 and "[1] x:[12,13], y:[2,3], z:[1,1.3]  ------ ROOT NODE" in diagnostics.listing(tb)


def sah_area(tree):
    """Sum of the internal boxes' half surface areas over the root's (the
    node-visit weight of random segments)."""
    b = tree["box"].astype(np.float64)
    d = b[:, 3:] - b[:, :3]
    a = d[:, 0] * d[:, 1] + d[:, 1] * d[:, 2] + d[:, 2] * d[:, 0]
    return float(a.sum() / a[tree["root"]])


@pytest.mark.parametrize("case", ["scene", "small", "paper_scale", "large", "duplicates"])
def test_restructured_build_is_a_valid_cheaper_tree(case):
    """Treelet restructuring keeps the leaves, gives a valid tree (every leaf
    once, boxes that contain their children, counters at 2), lowers the
    surface-area sum, and is deterministic."""
    from paper_2305_01867_amd import diagnostics
    if case == "scene":
        V, F, _, _ = workloads.appendix_scene()
    elif case == "small":
        V, F = workloads.heightfield(9, 5)
    elif case == "paper_scale":
        V, F = workloads.heightfield(128, 21)
    elif case == "large":
        V, F = workloads.heightfield(401, 8)  # 3.2e5 triangles: tiles and a top tree
    else:
        V, F = triangle_soup(5000, 3, n_vert=300, clustered=True)
    with rsi.rsi_build(dev(V), dev(F)) as a, rsi.rsi_build(dev(V), dev(F), algorithm="restructured") as b, \
            rsi.rsi_build(dev(V), dev(F), algorithm="restructured") as c:
        assert np.array_equal(export(a, "leaves"), export(b, "leaves"))
        ta, tb = diagnostics.export(a), diagnostics.export(b)
        assert diagnostics.check(tb) == [], diagnostics.check(tb)[:5]
        assert tb["root"] == 0 and tb["first"][0] == 0 and tb["last"][0] == F.shape[0] - 1
        assert np.array_equal(ta["box"][0], tb["box"][0])
        sa, sb = sah_area(ta), sah_area(tb)
        say(f"[restructure] {case}: {F.shape[0]} triangles, surface-area sum {sa:.2f} -> {sb:.2f}")
        if F.shape[0] >= 64:
            assert sb < 0.95 * sa
        for w in ("nodes", "parents", "counters"):
            assert np.array_equal(export(b, w), export(c, w)), w
        # parent links agree with the rewired children
        n_int = F.shape[0] - 1
        par = export(b, "parents")
        if n_int > 0:
            assert par[0] == -1
            for i in range(n_int):
                for r in (tb["left"][i], tb["right"][i]):
                    assert par[r if r >= 0 else n_int + ~r] == i
