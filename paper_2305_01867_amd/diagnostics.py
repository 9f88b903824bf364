"""BVH diagnostics: decode the exported tree and print it as a node listing or
a Graphviz graph.

Paper: Case Study 1 (the BVH debugging strategy: copy the node arrays from
device memory, decode each node's fields, check connectivity) and its Test
code and Graphviz subsection (a DOT description of the binary radix tree,
internal nodes labelled with their leaf range [a,b], leaves drawn as boxes
labelled "[c] d" with the sorted leaf position c and triangle id d).

The exported layout differs from the paper's C struct: a node here holds both
children's boxes and the leaf range it covers (include/rsi.h,
RSI_EXPORT_NODES), numbered as in Karras 2012 (root = internal node 0).  The
decoder works on host numpy arrays, so it also serves trees built elsewhere.
"""
from __future__ import annotations

import numpy as np


def decode(nodes, leaves, parents=None, counters=None):
    """Decode exported arrays (int32 views, as copied from the device).

    nodes: int32 [N_t - 1, 16]; leaves: int32 [N_t, 12]; parents: int32
    [2 N_t - 1] or None; counters: int32 [N_t - 1] or None.  Returns a dict
    of numpy arrays:
      left, right      child reference (>= 0 internal node, < 0 leaf ~k)
      left_box, right_box, box   float [N_t - 1, 6] (lo.xyz, hi.xyz); box is
                       the union of the two children's boxes
      first, last      leaf range of each internal node
      leaf_box         float [N_t, 6]; leaf_tri int32 [N_t] (triangle index)
      parent, counter  as exported (None if not given)
      root             index of the internal node no other node points to
                       (0 in the radix-tree numbering, the split position of
                       the whole range in the agglomerative one), -1 if none
    """
    nodes = np.asarray(nodes, np.int32).reshape(-1, 16)
    leaves = np.asarray(leaves, np.int32).reshape(-1, 12)
    f = nodes.view(np.float32)
    left_box = np.stack([f[:, 0], f[:, 2], f[:, 8], f[:, 1], f[:, 3], f[:, 9]], axis=1)
    right_box = np.stack([f[:, 4], f[:, 6], f[:, 10], f[:, 5], f[:, 7], f[:, 11]], axis=1)
    box = np.concatenate([np.minimum(left_box[:, :3], right_box[:, :3]),
                          np.maximum(left_box[:, 3:], right_box[:, 3:])], axis=1)
    # a leaf's box is the one its parent stores for it; a lone leaf (one
    # triangle) has no parent, so its box is rebuilt from A and the edges
    lf = leaves.view(np.float32)
    A, e1, e2 = lf[:, 0:3], lf[:, 4:7], lf[:, 8:11]
    corners = np.stack([A, A + e1, A + e2])
    leaf_box = np.concatenate([corners.min(axis=0), corners.max(axis=0)], axis=1)
    for side_ref, side_box in ((nodes[:, 12], left_box), (nodes[:, 13], right_box)):
        is_leaf = side_ref < 0
        leaf_box[~side_ref[is_leaf]] = side_box[is_leaf]
    child = np.zeros(nodes.shape[0], bool)
    for side_ref in (nodes[:, 12], nodes[:, 13]):
        inner = side_ref[(side_ref >= 0) & (side_ref < nodes.shape[0])]
        child[inner] = True
    roots = np.nonzero(~child)[0]
    return {
        "root": int(roots[0]) if roots.size == 1 else -1,
        "left": nodes[:, 12].copy(), "right": nodes[:, 13].copy(),
        "left_box": left_box, "right_box": right_box, "box": box,
        "first": nodes[:, 14].copy(), "last": nodes[:, 15].copy(),
        "leaf_box": leaf_box, "leaf_tri": leaves[:, 3].copy(),
        "parent": None if parents is None else np.asarray(parents, np.int32).copy(),
        "counter": None if counters is None else np.asarray(counters, np.int32).copy(),
    }


def export(mesh) -> dict:
    """Decode a built mesh (rsi_build) or batch (rsi_batch_*)."""
    from . import Batch, rsi_batch_export, rsi_mesh_export

    get = (lambda w: rsi_batch_export(mesh, w)) if isinstance(mesh, Batch) else (lambda w: rsi_mesh_export(mesh, w))
    host = lambda w: get(w).cpu().numpy()
    return decode(host("nodes"), host("leaves"), host("parents"), host("counters"))


def _rng(b, k):
    return f"[{b[k]:.6g},{b[k + 3]:.6g}]"


def listing(tree: dict) -> str:
    """Text listing of every internal and leaf node: box, parent, children
    (leaf or internal), arrival counter and leaf range; leaves with their
    triangle index (the fields the paper's Case Study 1 listing shows)."""
    out = ["BVH tree structure", "---------------------------", "Internal nodes"]
    n_int = tree["left"].shape[0]
    par = tree["parent"]
    for i in range(n_int):
        b = tree["box"][i]
        tag = "  ------ ROOT NODE" if i == tree["root"] else ""
        out.append(f"[{i}] x:{_rng(b, 0)}, y:{_rng(b, 1)}, z:{_rng(b, 2)}{tag}")
        kind = lambda r: f"{~r}(leaf)" if r < 0 else f"{r}(internal)"
        p = "" if par is None or i == tree["root"] else f", parent: {par[i]}"
        out.append(f"self: {i}{p}")
        out.append(f"children: L {kind(tree['left'][i])}, R {kind(tree['right'][i])}")
        cnt = "" if tree["counter"] is None else f"atomic: {tree['counter'][i]}, "
        out.append(f"{cnt}range: {tree['first'][i]}..{tree['last'][i]}")
        out.append("")
    out += ["---------------------------", "Leaf nodes"]
    n_leaf = tree["leaf_tri"].shape[0]
    for k in range(n_leaf):
        b = tree["leaf_box"][k]
        out.append(f"[{k}] x:{_rng(b, 0)}, y:{_rng(b, 1)}, z:{_rng(b, 2)}")
        if par is not None and n_leaf > 1:
            out.append(f"parent: {par[n_int + k]}")
        out.append(f"triangleID: {tree['leaf_tri'][k]}")
        out.append("")
    return "\n".join(out)


def to_dot(tree: dict, name: str = "bvh") -> str:
    """Graphviz DOT description of the binary radix tree: internal node i as
    an ellipse labelled with its leaf range "[a,b]", leaf k as a box labelled
    "[k] d" with d its triangle index, and an edge from every node to each
    child."""
    lines = [f"digraph {name} {{", "  node [fontname=\"Helvetica\"];"]
    n_int = tree["left"].shape[0]
    for i in range(n_int):
        extra = ", style=bold" if i == tree["root"] else ""
        lines.append(f"  n{i} [label=\"[{tree['first'][i]},{tree['last'][i]}]\"{extra}];")
    for k, d in enumerate(tree["leaf_tri"]):
        lines.append(f"  l{k} [shape=box, label=\"[{k}] {d}\"];")
    ref = lambda r: f"l{~r}" if r < 0 else f"n{r}"
    for i in range(n_int):
        lines.append(f"  n{i} -> {ref(tree['left'][i])};")
        lines.append(f"  n{i} -> {ref(tree['right'][i])};")
    lines.append("}")
    return "\n".join(lines) + "\n"


SECOND_PASS_STACK = 128  # entries of a lane's private stack in the exact second pass


def max_depth(tree: dict) -> int:
    """Number of internal nodes on the longest root-to-leaf path (0 for a
    tree of one leaf), by a breadth-first walk from the root."""
    n_int = tree["left"].shape[0]
    if n_int == 0 or tree["root"] < 0:
        return 0
    level, depth, seen = [tree["root"]], 0, 0
    while level:
        depth += 1
        seen += len(level)
        if seen > n_int:
            return -1  # a cycle: not a tree
        nxt = []
        for i in level:
            for r in (tree["left"][i], tree["right"][i]):
                if 0 <= r < n_int:
                    nxt.append(int(r))
        level = nxt
    return depth


def check(tree: dict, contiguous: bool = False) -> list:
    """Structural checks of a decoded tree (the connectivity the paper's
    debugging looked for); returns a list of problems, empty when sound:
    every leaf and non-root internal node has exactly one parent, the
    children's leaf spans make up the parent's, each box contains its
    children's boxes, counters (if present) read 2, and the depth stays
    within the exact second pass's stack.  With contiguous=True
    (radix-tree numbering) the spans must also split the parent's range."""
    problems = []
    n_int = tree["left"].shape[0]
    n_leaf = tree["leaf_tri"].shape[0]
    if n_leaf <= 1:
        return problems
    seen = np.zeros(n_int + n_leaf, np.int32)
    for i in range(n_int):
        ranges = []
        for side, r in (("left", tree["left"][i]), ("right", tree["right"][i])):
            slot = n_int + ~r if r < 0 else r
            if not (0 <= slot < n_int + n_leaf):
                problems.append(f"node {i}: {side} child {r} out of range")
                continue
            seen[slot] += 1
            lo, hi = (~r, ~r) if r < 0 else (tree["first"][r], tree["last"][r])
            ranges.append((lo, hi))
            cb = tree["leaf_box"][~r] if r < 0 else tree["box"][r]
            pb = tree[side + "_box"][i]
            if not (np.all(pb[:3] <= cb[:3]) and np.all(pb[3:] >= cb[3:])):
                problems.append(f"node {i}: {side} box does not contain its child")
        # leaf spans: children's spans make up the parent's (a contiguous split
        # in the radix-tree numbering; after treelet restructuring the spans
        # are smallest / largest leaf and may interleave)
        if contiguous and len(ranges) == 2 and not (ranges[0][0] == tree["first"][i]
                                                    and ranges[0][1] + 1 == ranges[1][0]
                                                    and ranges[1][1] == tree["last"][i]):
            problems.append(f"node {i}: child ranges {ranges} do not split [{tree['first'][i]},{tree['last'][i]}]")
        if len(ranges) == 2 and (min(ranges[0][0], ranges[1][0]) != tree["first"][i]
                                 or max(ranges[0][1], ranges[1][1]) != tree["last"][i]):
            problems.append(f"node {i}: child spans {ranges} do not make up [{tree['first'][i]},{tree['last'][i]}]")
    root = tree["root"]
    if root < 0:
        problems.append("no single root")
    elif seen[root] != 0 or (tree["first"][root], tree["last"][root]) != (0, n_leaf - 1):
        problems.append("the root has a parent or does not cover every leaf")
    bad = np.array([j for j in np.nonzero(seen != 1)[0] if j != root])
    if bad.size:
        problems.append(f"{bad.size} nodes without exactly one parent")
    if tree["counter"] is not None and np.any(tree["counter"] != 2):
        problems.append(f"{int(np.sum(tree['counter'] != 2))} internal nodes not completed (counter != 2)")
    depth = max_depth(tree)
    if depth < 0:
        problems.append("the child references form a cycle")
    elif depth > SECOND_PASS_STACK:
        # still exact, but the second pass tests leaf spans where the stack runs out
        problems.append(f"depth {depth} exceeds the second pass's stack of {SECOND_PASS_STACK} entries")
    return problems


def decode_wide(words) -> dict:
    """Decode exported 4-wide nodes (int32 [m, 32], RSI_EXPORT_WIDE_NODES):
    lo / hi float [m, 4, 3] per child, child int32 [m, 4], n_children [m]."""
    w = np.asarray(words, np.int32).reshape(-1, 32)
    f = w.view(np.float32)
    lo = np.stack([f[:, 0:4], f[:, 8:12], f[:, 16:20]], axis=2)
    hi = np.stack([f[:, 4:8], f[:, 12:16], f[:, 20:24]], axis=2)
    return {"lo": lo, "hi": hi, "child": w[:, 24:28].copy(), "n_children": w[:, 28].copy()}


TOP_SLOTS = 512  # 4-wide references below this name top-array slots


def check_wide(wide: dict, top: dict, tree: dict) -> list:
    """The 4-wide tree (main array and top array, both decoded) against the
    binary tree it was collapsed from; returns a list of problems, empty when
    sound: walking from top slot 0 reaches every leaf exactly once and no
    node twice, every node has 2..4 children, each child's box equals the
    union of its own children's boxes (and, where the child is named by its
    binary index, the binary tree's box of that node; a leaf's box for a
    leaf), and unused slots hold INT32_MIN with boxes +inf on every face."""
    problems = []
    n_int = tree["left"].shape[0]
    n_leaf = tree["leaf_tri"].shape[0]
    if n_leaf <= 1:
        return problems
    empty = np.iinfo(np.int32).min
    seen_leaf = np.zeros(n_leaf, np.int64)
    seen = {"top": np.zeros(TOP_SLOTS, bool), "wide": np.zeros(n_int, bool)}
    arrays = {"top": top, "wide": wide}

    def node_of(r):
        return ("top", r) if r < TOP_SLOTS else ("wide", r - TOP_SLOTS)

    def union_of(arr, i):
        k = int(arr["n_children"][i])
        return np.concatenate([arr["lo"][i, :k].min(axis=0), arr["hi"][i, :k].max(axis=0)])

    stack = [("top", 0)]
    while stack and len(problems) < 20:
        which, i = stack.pop()
        arr = arrays[which]
        if not 0 <= i < seen[which].shape[0]:
            problems.append(f"{which} node {i} out of range")
            continue
        if seen[which][i]:
            problems.append(f"{which} node {i} reached twice")
            continue
        seen[which][i] = True
        k = int(arr["n_children"][i])
        if not 2 <= k <= 4:
            problems.append(f"{which} node {i}: {k} children")
            continue
        for j in range(4):
            c = int(arr["child"][i, j])
            box = np.concatenate([arr["lo"][i, j], arr["hi"][i, j]])
            if j >= k:
                if c != empty or not np.all(np.isposinf(box)):
                    problems.append(f"{which} node {i}: unused slot {j} is not empty")
                continue
            if c < 0:
                if not 0 <= ~c < n_leaf:
                    problems.append(f"{which} node {i}: leaf {~c} out of range")
                    continue
                seen_leaf[~c] += 1
                if not np.array_equal(box, tree["leaf_box"][~c]):
                    problems.append(f"{which} node {i}: child {j} box differs from the leaf's")
                continue
            cw, ci = node_of(c)
            if not 0 <= ci < seen[cw].shape[0]:
                problems.append(f"{which} node {i}: child {c} out of range")
                continue
            if not np.array_equal(box, union_of(arrays[cw], ci)):
                problems.append(f"{which} node {i}: child {j} box is not the union of its children's")
            if cw == "wide" and not np.array_equal(box, tree["box"][ci]):
                problems.append(f"{which} node {i}: child {j} box differs from the binary tree's")
            stack.append((cw, ci))
    if np.any(seen_leaf != 1):
        problems.append(f"{int(np.sum(seen_leaf != 1))} leaves not reached exactly once")
    return problems
