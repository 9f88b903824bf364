"""Plain, slow CPU oracle for the ray/surface-intersection path.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does, and
nothing here calls the GPU library.

Contents, each following the passage named in its docstring:
  intersect        exhaustive binary64 Moller-Trumbore over all pairs (C, OpenMP)
  all_hits         every hit of one segment (C)
  mesh_bounds      component-wise min / max of the vertices
  morton_keys      30- or 63-bit Morton keys of the triangle centroids (float32)
  sort_order       stable order of the keys
  radix_tree       Karras binary radix tree over the sorted keys (C)
  node_boxes       bounding box of every internal node (C)
  exact            exact rational segment/triangle classification (fractions)
"""
from __future__ import annotations

import ctypes
import os
from fractions import Fraction

import numpy as np

from . import build_oracle

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(build_oracle.LIB):
        build_oracle.build()
    lib = ctypes.CDLL(build_oracle.LIB)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    lib.rsi_oracle_intersect.argtypes = [P, I64, P, I64, P, P, I64, P, P, P, P, ctypes.c_int]
    lib.rsi_oracle_intersect.restype = ctypes.c_int
    lib.rsi_oracle_intercept_count.argtypes = [P, I64, P, I64, P, P, I64, P, ctypes.c_int]
    lib.rsi_oracle_intercept_count.restype = ctypes.c_int
    lib.rsi_oracle_all_hits.argtypes = [P, I64, P, I64, P, P, P, P, ctypes.c_int]
    lib.rsi_oracle_all_hits.restype = ctypes.c_int
    lib.rsi_oracle_radix_tree.argtypes = [P, I64, ctypes.c_int, P, P, P, P, P, P]
    lib.rsi_oracle_radix_tree.restype = None
    lib.rsi_oracle_node_boxes.argtypes = [P, P, P, I64, P, P, P]
    lib.rsi_oracle_node_boxes.restype = None
    lib.rsi_oracle_max_threads.argtypes = []
    lib.rsi_oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    a = np.asarray(a)
    if a.dtype != np.int32:
        raise TypeError("triangle indices must be int32")
    return np.ascontiguousarray(a)


def max_threads() -> int:
    return int(_load().rsi_oracle_max_threads())


def intersect(V, F, O, E, n_threads: int = 0):
    """Exhaustive binary64 search (paper: Background -- the exhaustive search
    over all triangle/ray pairs with the Moller-Trumbore test; the three
    operating modes).  Returns (hit uint8 [N], id int32 [N], uvt float64 [N,3],
    n_hits int32 [N])."""
    V, O, E = _f32(V), _f32(O), _f32(E)
    F = _i32(F)
    n = O.shape[0]
    hit = np.zeros(n, np.uint8)
    ids = np.zeros(n, np.int32)
    uvt = np.zeros((n, 3), np.float64)
    nh = np.zeros(n, np.int32)
    rc = _load().rsi_oracle_intersect(_ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(O), _ptr(E), n,
                                      _ptr(hit), _ptr(ids), _ptr(uvt), _ptr(nh), int(n_threads))
    if rc != 0:
        raise ValueError("triangle index out of range" if rc == -1 else "oracle allocation failed")
    return hit, ids, uvt, nh


def intercept_count(V, F, O, E, n_threads: int = 0):
    """Distinct intersections per segment (paper: Background -- the
    intercept-count mode): the number of distinct binary64 t among the hits
    of the exhaustive test.  int32 [N]."""
    V, O, E = _f32(V), _f32(O), _f32(E)
    F = _i32(F)
    n = O.shape[0]
    count = np.zeros(n, np.int32)
    rc = _load().rsi_oracle_intercept_count(_ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(O), _ptr(E), n,
                                            _ptr(count), int(n_threads))
    if rc != 0:
        raise ValueError("triangle index out of range" if rc == -1 else "oracle allocation failed")
    return count


def derived(O, E, ids, uvt):
    """The barycentric mode's result tuple (paper: Background -- the intersecting
    rays with the intersecting triangle, the distance to and the location of the
    nearest intersecting point; Performance section, steps 3a-3d): for every
    hitting segment, in ascending index, (index, distance, triangle, point)
    with distance = t ||E - O|| and point = O + t (E - O), in binary64 from the
    float32 end points and the binary64 t."""
    O = np.asarray(O, np.float32).astype(np.float64)
    E = np.asarray(E, np.float32).astype(np.float64)
    ids = np.asarray(ids)
    idx = np.nonzero(ids >= 0)[0]
    d = E[idx] - O[idx]
    t = np.asarray(uvt, np.float64)[idx, 2]
    length = np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2])
    return idx.astype(np.int64), t * length, ids[idx].astype(np.int32), O[idx] + t[:, None] * d


def all_hits(V, F, o, e, cap: int = 4096):
    """Every triangle one segment hits, ascending index: (ids, uvt)."""
    V = _f32(V)
    F = _i32(F)
    o = _f32(o).reshape(3)
    e = _f32(e).reshape(3)
    ids = np.zeros(cap, np.int32)
    uvt = np.zeros((cap, 3), np.float64)
    n = _load().rsi_oracle_all_hits(_ptr(V), V.shape[0], _ptr(F), F.shape[0], _ptr(o), _ptr(e),
                                    _ptr(ids), _ptr(uvt), cap)
    if n < 0:
        raise ValueError("triangle index out of range")
    n = min(n, cap)
    return ids[:n].copy(), uvt[:n].copy()


# --------------------------------------------------------------------------
# BVH structure (paper: Background -- Morton codes, sorting, binary radix tree
# of Karras 2012; Specific changes -- 64-bit Morton codes; Case Study 1 --
# sorted triangle ids as int32, leaf / internal node contents).
# --------------------------------------------------------------------------

def mesh_bounds(V):
    """Component-wise (lo, hi) over all vertices; NaN coordinates are ignored
    (an all-NaN axis gives NaN)."""
    V = _f32(V)
    return np.fmin.reduce(V, axis=0), np.fmax.reduce(V, axis=0)


def morton_keys(V, F, key_bits: int):
    """Morton key of every triangle, as uint64.

    The centroid c = ((A + B) + C) / 3 is formed in float32; each axis is
    normalised to the mesh box, n = (c - lo) / (hi - lo) (0 when hi == lo),
    quantised to b bits, q = floor(min(n 2^b, 2^b - 1)) (0 for n <= 0 or NaN),
    and the three b-bit integers are interleaved from the most significant bit
    down, z above y above x in every bit triple.  b = 10 gives 30-bit keys and
    b = 21 gives 63-bit keys.  Every float operation is a single IEEE float32
    operation (numpy evaluates them one at a time, no fused multiply-add)."""
    if key_bits not in (30, 63):
        raise ValueError("key_bits must be 30 or 63")
    b = key_bits // 3
    V = _f32(V)
    F = np.asarray(F, np.int64)
    lo, hi = mesh_bounds(V)
    A, B, C = V[F[:, 0]], V[F[:, 1]], V[F[:, 2]]
    with np.errstate(all="ignore"):
        c = ((A + B) + C) / np.float32(3.0)
        ext = hi - lo
        safe = np.where(ext > 0, ext, np.float32(1.0)).astype(np.float32)
        n = np.where(ext > 0, (c - lo) / safe, np.float32(0.0)).astype(np.float32)
        x = n * np.float32(2.0 ** b)
        top = np.float32(2 ** b - 1)
        q = np.where(x > 0, np.floor(np.minimum(x, top)), np.float32(0.0))
    q = q.astype(np.uint64)
    key = np.zeros(q.shape[0], np.uint64)
    for k in range(b - 1, -1, -1):
        bits = ((q[:, 2] >> np.uint64(k)) & np.uint64(1)) << np.uint64(2)
        bits |= ((q[:, 1] >> np.uint64(k)) & np.uint64(1)) << np.uint64(1)
        bits |= (q[:, 0] >> np.uint64(k)) & np.uint64(1)
        key = (key << np.uint64(3)) | bits
    return key


def sort_order(keys):
    """Positions of the keys in ascending order; equal keys keep their input
    order (so the triangle index breaks ties)."""
    return np.argsort(np.asarray(keys, np.uint64), kind="stable").astype(np.int32)


def radix_tree(sorted_keys, key_bits: int):
    """Binary radix tree over sorted keys (Karras 2012, section 3), as a dict of
    int32 arrays of length n-1: left, right (child index), left_leaf,
    right_leaf (1 if that child is a leaf), first, last (key range)."""
    k = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    n = k.shape[0]
    m = max(n - 1, 0)
    out = {name: np.zeros(m, np.int32) for name in ("left", "right", "first", "last")}
    ll = np.zeros(m, np.uint8)
    rl = np.zeros(m, np.uint8)
    if n >= 2:
        _load().rsi_oracle_radix_tree(_ptr(k), n, int(key_bits), _ptr(out["left"]), _ptr(out["right"]),
                                      _ptr(ll), _ptr(rl), _ptr(out["first"]), _ptr(out["last"]))
    out["left_leaf"] = ll
    out["right_leaf"] = rl
    return out


def node_boxes(V, F, order, tree):
    """float32 [n-1, 6] = lo.xyz, hi.xyz of every internal node: min / max over
    the corners of the triangles in its key range."""
    V = _f32(V)
    F = _i32(F)
    order = np.ascontiguousarray(order, np.int32)
    n = order.shape[0]
    boxes = np.zeros((max(n - 1, 0), 6), np.float32)
    if n >= 2:
        _load().rsi_oracle_node_boxes(_ptr(V), _ptr(F), _ptr(order), n,
                                      _ptr(np.ascontiguousarray(tree["first"])),
                                      _ptr(np.ascontiguousarray(tree["last"])), _ptr(boxes))
    return boxes


def leaf_boxes(V, F, order):
    """float32 [n, 6]: box of the triangle at every sorted position."""
    V = _f32(V)
    P = V[np.asarray(F, np.int64)[np.asarray(order, np.int64)]]  # [n, 3 corners, 3]
    return np.concatenate([P.min(axis=1), P.max(axis=1)], axis=1).astype(np.float32)


def build_structure(V, F, key_bits: int = 30):
    """The whole BVH description the build must reproduce, as a dict."""
    keys = morton_keys(V, F, key_bits)
    order = sort_order(keys)
    skeys = keys[order]
    tree = radix_tree(skeys, key_bits)
    return {
        "keys": keys,
        "order": order,
        "sorted_keys": skeys,
        "tree": tree,
        "node_boxes": node_boxes(V, F, order, tree),
        "leaf_boxes": leaf_boxes(V, F, order),
    }


# --------------------------------------------------------------------------
# Exact classification with rational arithmetic (independent of the
# Moller-Trumbore formulation above: signed volumes of tetrahedra).
# --------------------------------------------------------------------------

def _vol(a, b, c, d):
    """Six times the signed volume of tetrahedron (a, b, c, d), exactly."""
    b0, b1, b2 = b[0] - a[0], b[1] - a[1], b[2] - a[2]
    c0, c1, c2 = c[0] - a[0], c[1] - a[1], c[2] - a[2]
    d0, d1, d2 = d[0] - a[0], d[1] - a[1], d[2] - a[2]
    return b0 * (c1 * d2 - c2 * d1) - b1 * (c0 * d2 - c2 * d0) + b2 * (c0 * d1 - c1 * d0)


def exact(A, B, C, O, E):
    """Exact geometry of one segment against one triangle, from the float32
    inputs taken as rationals.

    The segment OE meets the closed triangle ABC, and is not parallel to its
    plane, iff the end points are not strictly on the same side of the plane
    (signed volumes s0 = vol(A,B,C,O), s1 = vol(A,B,C,E) with s0 != s1) and
    the line through O, E passes on the closed triangle (the three volumes
    vol(O,E,B,C), vol(O,E,C,A), vol(O,E,A,B) not of mixed strict signs).
    Returns (hit: bool, u, v, t as Fractions or None, margin) where u, v are the
    barycentric weights of B and C, t the segment parameter, and margin the
    smallest |signed volume| that took part in the decision (0 means a
    boundary case)."""
    A, B, C, O, E = ([Fraction(float(x)) for x in np.asarray(p, np.float32)] for p in (A, B, C, O, E))
    s0 = _vol(A, B, C, O)
    s1 = _vol(A, B, C, E)
    if s0 == s1:
        return False, None, None, None, Fraction(0)
    wa = _vol(O, E, B, C)
    wb = _vol(O, E, C, A)
    wc = _vol(O, E, A, B)
    sw = wa + wb + wc
    t = s0 / (s0 - s1)
    u = wb / sw if sw != 0 else None
    v = wc / sw if sw != 0 else None
    same_side = (s0 > 0 and s1 > 0) or (s0 < 0 and s1 < 0)
    mixed = (min(wa, wb, wc) < 0) and (max(wa, wb, wc) > 0)
    hit = (not same_side) and (not mixed) and sw != 0
    margin = min(abs(s0), abs(s1), abs(wa), abs(wb), abs(wc))
    return hit, u, v, t, margin
