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


def collapse_wide(tree):
    """A 4-wide collapse written here from its definition (each node takes
    its two children, then opens the largest-area internal child twice), in
    the export layout: the main array by binary index with references to
    internal children as binary index + 512, and the top array holding the
    first nodes in breadth-first order with references among them rewritten
    to their slots."""
    n_int = tree["left"].shape[0]
    T = diagnostics.TOP_SLOTS
    words = np.zeros((n_int, 32), np.int32)
    f = words.view(np.float32)
    box = lambda c: tree["leaf_box"][~c] if c < 0 else tree["box"][c]
    area = lambda b: (b[3] - b[0]) * (b[4] - b[1]) + (b[4] - b[1]) * (b[5] - b[2]) + (b[5] - b[2]) * (b[3] - b[0])
    kids_of = {}
    stack = [tree["root"]]
    while stack:
        r = stack.pop()
        kids = [int(tree["left"][r]), int(tree["right"][r])]
        for _ in range(2):
            inner = [c for c in kids if c >= 0]
            if not inner:
                break
            c = max(inner, key=lambda c: area(box(c)))
            kids[kids.index(c)] = int(tree["left"][c])
            kids.append(int(tree["right"][c]))
        kids_of[r] = kids
        for i in range(4):
            b = box(kids[i]) if i < len(kids) else np.full(6, np.inf, np.float32)
            for a in range(3):
                f[r, 8 * a + i], f[r, 8 * a + 4 + i] = b[a], b[3 + a]
            words[r, 24 + i] = (kids[i] + T if kids[i] >= 0 else kids[i]) if i < len(kids) else np.iinfo(np.int32).min
        words[r, 28] = len(kids)
        stack += [c for c in kids if c >= 0]
    order = [tree["root"]]
    for r in order:
        if len(order) >= T:
            break
        order += [c for c in kids_of[r] if c >= 0]
    order = order[:T]
    slot = {r: i for i, r in enumerate(order)}
    top = np.zeros((T, 32), np.int32)
    for i, r in enumerate(order):
        top[i] = words[r]
        for j in range(int(words[r, 28])):
            c = int(words[r, 24 + j])
            if c >= 0 and c - T in slot:
                top[i, 24 + j] = slot[c - T]
    return words, top, set(order)


def test_wide_checker_accepts_a_collapse_and_finds_planted_mistakes():
    V, F = workloads.heightfield(30, 3)
    tree = diagnostics.decode(*export_layout(V, F))
    words, top, cached = collapse_wide(tree)
    dw = diagnostics.decode_wide
    assert diagnostics.check_wide(dw(words), dw(top), tree) == []
    wide = dw(words)
    r = [q for q in np.nonzero(wide["n_children"] == 4)[0] if q not in cached][0]  # reached in the main array
    # a child dropped: its leaves are no longer reached
    bad = words.copy()
    bad[r, 28] = 3
    assert diagnostics.check_wide(dw(bad), dw(top), tree) != []
    # a box shrunk on one face, in the main array and in the top array
    bad = words.copy()
    bad.view(np.float32)[r, 0] += 1e-3
    assert any("box" in p for p in diagnostics.check_wide(dw(bad), dw(top), tree))
    badt = top.copy()
    badt.view(np.float32)[0, 0] += 1e-3
    assert any("box" in p for p in diagnostics.check_wide(dw(words), dw(badt), tree))
    # a top reference pointing one slot off
    badt = top.copy()
    j = int(np.nonzero((badt[0, 24:28] > 0) & (badt[0, 24:28] < diagnostics.TOP_SLOTS))[0][0])
    badt[0, 24 + j] += 1
    assert diagnostics.check_wide(dw(words), dw(badt), tree) != []
    # one leaf referenced twice
    bad = words.copy()
    leaf_slots = [(q, i) for q in range(bad.shape[0]) if q not in cached for i in range(int(bad[q, 28]))
                  if bad[q, 24 + i] < 0]
    (q0, i0), (q1, i1) = leaf_slots[-2], leaf_slots[-1]
    bad[q1, 24 + i1] = bad[q0, 24 + i0]
    assert diagnostics.check_wide(dw(bad), dw(top), tree) != []


def test_depth_of_chains_and_the_check():
    """A tree that is one chain (each internal node has a leaf and the next
    node as children) is as deep as it has internal nodes; the check names a
    depth past the exact second pass's stack, and a cycle."""
    def chain(n_int):
        left = np.array([~i for i in range(n_int)], np.int32)
        right = np.array(list(range(1, n_int)) + [~n_int], np.int32)
        return {"left": left, "right": right, "root": 0}

    assert diagnostics.max_depth(chain(1)) == 1
    assert diagnostics.max_depth(chain(97)) == 97
    # the paper's scene: root and two internal children
    V, F, _, _ = workloads.appendix_scene()
    tree = diagnostics.decode(*export_layout(V, F))
    assert diagnostics.max_depth(tree) == 2
    # a 64-triangle geometric chain with 63-bit keys: one internal node per level
    s = oracle.build_structure(*_geometric(64), 63)
    t = s["tree"]
    tree = {"left": np.where(t["left_leaf"] == 1, ~t["left"], t["left"]),
            "right": np.where(t["right_leaf"] == 1, ~t["right"], t["right"]), "root": 0}
    assert diagnostics.max_depth(tree) == 63
    # check() on a sound chain of 150 internal nodes: only the depth is named
    n_int = 150
    t = chain(n_int)
    leaf_box = np.array([[k, 0, 0, k + 1, 1, 1] for k in range(n_int + 1)], np.float32)
    box = np.array([[i, 0, 0, n_int + 1, 1, 1] for i in range(n_int)], np.float32)
    t.update({"first": np.arange(n_int, dtype=np.int32), "last": np.full(n_int, n_int, np.int32),
              "leaf_box": leaf_box, "box": box, "left_box": leaf_box[:n_int],
              "right_box": np.concatenate([box[1:], leaf_box[n_int:]]), "counter": np.full(n_int, 2, np.int32),
              "leaf_tri": np.arange(n_int + 1, dtype=np.int32)})
    assert diagnostics.check(t) == [f"depth {n_int} exceeds the second pass's stack of 128 entries"]
    t97 = chain(97)
    t97.update({k: (v[:97] if k not in ("leaf_box", "leaf_tri") else v[:98]) for k, v in t.items()
                if k not in ("left", "right", "root")})
    t97["last"] = np.full(97, 97, np.int32)
    t97["box"] = np.array([[i, 0, 0, 98, 1, 1] for i in range(97)], np.float32)
    t97["right_box"] = np.concatenate([t97["box"][1:], leaf_box[97:98]])
    assert diagnostics.check(t97) == []
    cyc = chain(5)
    cyc["right"] = cyc["right"].copy()
    cyc["right"][4] = 0
    assert diagnostics.max_depth(cyc) == -1


def _geometric(m):
    """m triangles shrinking by 2^(-1/3) towards a corner, plus one spanning the unit box."""
    V, F = [], []
    for k in range(m):
        c = 0.9 * np.array([2.0 ** -(k / 3.0), 2.0 ** -((k + 1) / 3.0), 2.0 ** -((k + 2) / 3.0)])
        s = 0.3 * 2.0 ** -(k / 3.0 + 2)
        b = len(V)
        V += [c + [-s, -s, 0], c + [s, -s, 0.1 * s], c + [0, s, -0.1 * s]]
        F.append([b, b + 1, b + 2])
    b = len(V)
    V += [[0, 0, 0], [1, 0, 0], [0, 1, 1]]
    F.append([b, b + 1, b + 2])
    return np.array(V, np.float32), np.array(F, np.int32)
