"""BVH diagnostics on the CPU: decode a tree given in the export layout,
list it, draw it as DOT and check it.  The tree comes from the oracle's
definition-level construction of the paper's Case Study 1 scene, so the
expected labels are the paper's: root range [0,3], children [0,1] and [2,3],
leaves [0] 0, [1] 3, [2] 1, [3] 2 (Case Study 1 listing and its Graphviz
subsection)."""
import numpy as np

import oracle
from paper_2305_01867_amd import diagnostics, workloads


def export_layout(V, F, bits=30):
    """Arrays in the library's export layout, built from the oracle."""
    s = oracle.build_structure(V, F, bits)
    t, nb, lb = s["tree"], s["node_boxes"], s["leaf_boxes"]
    n = len(s["order"])
    left = np.where(t["left_leaf"] == 1, ~t["left"], t["left"]).astype(np.int32)
    right = np.where(t["right_leaf"] == 1, ~t["right"], t["right"]).astype(np.int32)
    box = lambda r: lb[~r] if r < 0 else nb[r]
    nodes = np.zeros((n - 1, 16), np.int32)
    f = nodes.view(np.float32)
    for i in range(n - 1):
        L, R = box(left[i]), box(right[i])
        f[i, 0:4] = (L[0], L[3], L[1], L[4])
        f[i, 4:8] = (R[0], R[3], R[1], R[4])
        f[i, 8:12] = (L[2], L[5], R[2], R[5])
    nodes[:, 12], nodes[:, 13], nodes[:, 14], nodes[:, 15] = left, right, t["first"], t["last"]
    leaves = np.zeros((n, 12), np.int32)
    lf = leaves.view(np.float32)
    order = s["order"]
    A, B, C = V[F[order, 0]], V[F[order, 1]], V[F[order, 2]]
    lf[:, 0:3], lf[:, 4:7], lf[:, 8:11] = A, B - A, C - A
    leaves[:, 3] = order
    parents = np.full(2 * n - 1, -1, np.int32)
    for i in range(n - 1):
        for r in (left[i], right[i]):
            parents[(n - 1 + ~r) if r < 0 else r] = i
    return nodes, leaves, parents, np.full(n - 1, 2, np.int32)


def test_case_study_1_graph_and_listing():
    V, F, _, _ = workloads.appendix_scene()
    tree = diagnostics.decode(*export_layout(V, F))
    assert diagnostics.check(tree, contiguous=True) == []
    dot = diagnostics.to_dot(tree)
    assert 'n0 [label="[0,3]", style=bold];' in dot
    labels = sorted(l.split('label="')[1].split('"')[0] for l in dot.splitlines() if "label=" in l and "shape=box" in l)
    assert labels == ["[0] 0", "[1] 3", "[2] 1", "[3] 2"]
    internal = sorted(l.split('label="')[1].split('"')[0] for l in dot.splitlines() if "label=" in l and "shape" not in l)
    assert internal == ["[0,1]", "[0,3]", "[2,3]"]
    assert dot.count("->") == 6
    text = diagnostics.listing(tree)
    assert "ROOT NODE" in text and text.count("triangleID:") == 4
    # the printed boxes of the paper's listing (two decimals)
    assert "[0] x:[12,13], y:[2,2.5], z:[1,1.2]" in text.replace("1.2000000476837158", "1.2")


def test_check_finds_planted_faults():
    V, F = workloads.heightfield(9, 2)
    nodes, leaves, parents, counters = export_layout(V, F)
    assert diagnostics.check(diagnostics.decode(nodes, leaves, parents, counters), contiguous=True) == []
    bad = nodes.copy()
    bad[3, 13] = bad[3, 12]  # a child listed twice, another lost
    assert diagnostics.check(diagnostics.decode(bad, leaves, parents, counters))
    c2 = counters.copy()
    c2[5] = 1  # an incomplete bottom-up pass (the paper's Case Study 2)
    assert any("counter" in p for p in diagnostics.check(diagnostics.decode(nodes, leaves, parents, c2)))
    shrunk = nodes.copy()
    shrunk.view(np.float32)[0, 1] -= 0.5  # a box that no longer holds its child
    assert any("box" in p for p in diagnostics.check(diagnostics.decode(shrunk, leaves, parents, counters)))
