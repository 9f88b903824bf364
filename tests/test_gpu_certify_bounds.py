"""The certified precision's error bounds, pinned by exact rational arithmetic.

For each (segment, triangle) pair the library returns its binary32 values of
det, U, W, T, their bounds B(X) and the classification (sure miss / sure hit
/ unsure).  Every float32 and float64 value is a dyadic rational, so scaled
to integers by 2^1104 all of them compare exactly.  Checked on adversarial
pairs (near edges and vertices, near-parallel, large offsets, tiny and huge
scales, degenerate triangles and segments):
  |X32 - X| <= B(X)    X the exact value from the float32 inputs
  |X32 - X64| <= B(X)  X64 evaluated in binary64 in the definition's order
  sure miss  => the oracle (binary64) and the exact decision both miss
  sure hit   => both hit, and [tlo, thi] holds the binary64 and the exact t
A plausible mistake in the bound (a factor, a dropped product, an absolute
value) fails the first two checks on these pairs."""
from fractions import Fraction

import numpy as np
import pytest
import torch

import oracle
import paper_2305_01867_amd as rsi
from gpu_helpers import say

pytestmark = pytest.mark.gpu
SHIFT = 1104  # 2^1104 * any finite float64 is an integer; inputs use 2^368 (3 * 368 = 1104)


def adversarial_pairs(n, seed):
    rng = np.random.default_rng(seed)
    kind = rng.integers(0, 9, n)
    A = rng.uniform(-1, 1, (n, 3))
    B = rng.uniform(-1, 1, (n, 3))
    C = rng.uniform(-1, 1, (n, 3))
    O = rng.uniform(-1.5, 1.5, (n, 3))
    E = rng.uniform(-1.5, 1.5, (n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    h = rng.uniform(0.05, 1.0, (n, 1))
    sign = rng.choice([-1.0, 1.0], (n, 1))
    # 1: through a point near an edge; 2: near a vertex
    lam = rng.uniform(0, 1, (n, 1))
    delta = sign * 10.0 ** rng.uniform(-9, -6, (n, 1))
    jitter = rng.normal(size=(n, 3))
    p_edge = A + lam * (B - A) + delta * jitter
    p_vert = A + delta * jitter
    for k, p in ((1, p_edge), (2, p_vert)):
        m = kind == k
        O[m] = p[m] - h[m] * d[m] * rng.uniform(0.1, 1, (m.sum(), 1))
        E[m] = p[m] + h[m] * d[m] * rng.uniform(0.1, 1, (m.sum(), 1))
    # 3: near-parallel, tilted out of the plane by 1e-12 .. 1e-4 rad, offset along the normal
    nrm = np.cross(B - A, C - A)
    nrm /= np.maximum(np.linalg.norm(nrm, axis=1, keepdims=True), 1e-300)
    u = B - A
    u /= np.maximum(np.linalg.norm(u, axis=1, keepdims=True), 1e-300)
    theta = 10.0 ** rng.uniform(-12, -4, (n, 1))
    dp = np.cos(theta) * u + sign * np.sin(theta) * nrm
    mid = (A + B + C) / 3 + nrm * sign * 10.0 ** rng.uniform(-10, -6, (n, 1))
    m = kind == 3
    O[m] = mid[m] - dp[m] * h[m]
    E[m] = mid[m] + dp[m] * h[m]
    # 4: large offset, small triangle and segment (cancellation in every difference)
    m = kind == 4
    off = 10.0 ** rng.uniform(1, 3.5, (m.sum(), 1)) * rng.choice([-1.0, 1.0], (m.sum(), 3))
    s = 10.0 ** rng.uniform(-3, 0, (m.sum(), 1))
    for X in (A, B, C, O, E):
        X[m] = off + s * X[m]
    # 5: tiny scales (products near and below the float32 normal range); 6: huge
    # scales (products overflow float32: must never be sure)
    for k, lo, hi in ((5, -15, -4), (6, 11, 14)):
        m = kind == k
        sc = 10.0 ** rng.uniform(lo, hi, (m.sum(), 1))
        for X in (A, B, C, O, E):
            X[m] = X[m] * sc
    # 7: degenerate: zero-area triangle or zero-length segment
    m = kind == 7
    half = rng.uniform(size=n) < 0.5
    B[m & half] = A[m & half]
    E[m & ~half] = O[m & ~half]
    # 8: exactly in-plane geometry: triangle in z = 0, segments with end points on
    # the plane or lying in it
    m = kind == 8
    for X in (A, B, C):
        X[m, 2] = 0.0
    which = rng.integers(0, 3, n)
    O[m & (which == 0), 2] = 0.0
    E[m & (which == 1), 2] = 0.0
    O[m & (which == 2), 2] = 0.0
    E[m & (which == 2), 2] = 0.0
    f = lambda X: X.astype(np.float32)
    return f(A), f(B), f(C), f(O), f(E), kind


def scaled(x, shift):
    """Exact integer x * 2^shift of float values (object array)."""
    def one(v):
        num, den = float(v).as_integer_ratio()
        return num * ((1 << shift) // den)
    return np.frompyfunc(one, 1, 1)(np.asarray(x, np.float64))


def cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def dot(a, b):
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]


def quantities(A, B, C, O, E):
    """det, U, W, T in the definition's operation order, from per-axis tuples
    (exact for Python integers, binary64 for float64 arrays)."""
    d = tuple(E[k] - O[k] for k in range(3))
    e1 = tuple(B[k] - A[k] for k in range(3))
    e2 = tuple(C[k] - A[k] for k in range(3))
    s = tuple(O[k] - A[k] for k in range(3))
    p = cross(d, e2)
    q = cross(s, e1)
    return dot(e1, p), dot(s, p), dot(d, q), dot(e2, q)


def decide(det, U, W, T):
    """The definition's predicates, vectorised; works on exact integers too."""
    pos = det > 0
    g = np.where(pos, 1, -1)
    a, b, tt, D = g * U, g * W, g * T, g * det
    return (det != 0) & (a >= 0) & (b >= 0) & (a + b <= D) & (tt >= 0) & (tt <= D)


def test_certified_bounds_against_exact_rationals():
    n = 200_000
    A, B, C, O, E, kind = adversarial_pairs(n, 77)
    dev = torch.device("cuda")
    corners = torch.from_numpy(np.stack([A, B, C], axis=1).copy()).to(dev)
    vals, cls = rsi.rsi_debug_certify(torch.from_numpy(O).to(dev), torch.from_numpy(E).to(dev), corners)
    vals = vals.cpu().numpy()
    cls = cls.cpu().numpy()
    say(f"[bounds] {n} pairs: sure miss {np.sum(cls == 0)}, sure hit {np.sum(cls == 1)}, unsure {np.sum(cls == 2)}")

    # every pair takes part: a bound that is finite must hold, and sure answers
    # must be right even where some binary32 quantity overflowed (a sure miss
    # may rest on one predicate whose sign is certain)
    idx = np.arange(n)
    axes = lambda X: tuple(scaled(X[:, k], 368) for k in range(3))
    exact = quantities(axes(A), axes(B), axes(C), axes(O), axes(E))
    f64 = lambda X: tuple(X[:, k].astype(np.float64) for k in range(3))
    x64 = quantities(f64(A), f64(B), f64(C), f64(O), f64(E))
    assert all(np.all(np.isfinite(x)) for x in x64)
    for j, name in enumerate(("det", "U", "W", "T")):
        fin_b = np.isfinite(vals[:, 4 + j])
        assert np.all(np.isfinite(vals[fin_b, j])), f"{name}: finite bound but non-finite binary32 value"
        k = np.nonzero(fin_b)[0]
        x32 = scaled(vals[k, j], SHIFT)
        bnd = scaled(vals[k, 4 + j], SHIFT)
        err_exact = np.abs(x32 - exact[j][k])
        err_64 = np.abs(x32 - scaled(x64[j][k], SHIFT))
        bad = np.nonzero(err_exact > bnd)[0]
        assert bad.size == 0, f"{name}: |X32 - X| > B(X) on {bad.size} pairs, kinds {np.bincount(kind[k[bad]]).tolist()}"
        bad = np.nonzero(err_64 > bnd)[0]
        assert bad.size == 0, f"{name}: |X32 - X64| > B(X) on {bad.size} pairs"
        # the bound is not vacuous: its slack over the worst error is modest
        ratio = max(float(Fraction(int(e), int(b))) for e, b in zip(err_exact[:5000], bnd[:5000]) if b > 0)
        say(f"  {name}: {np.sum(~fin_b)} infinite bounds; worst |X32 - X| / B(X) on 5000 pairs = {ratio:.3g}")
    nonfin = ~np.all(np.isfinite(vals[:, :8]), axis=1)
    say(f"  pairs with an overflowed binary32 quantity: {np.sum(nonfin)} (sure miss {np.sum(nonfin & (cls == 0))}, "
        f"sure hit {np.sum(nonfin & (cls == 1))})")

    hit_exact = decide(*exact)
    hit_64 = decide(*x64)
    c = cls
    assert not np.any((c == 0) & hit_exact), "sure miss but the exact segment hits"
    assert not np.any((c == 0) & hit_64), "sure miss but binary64 hits"
    assert not np.any((c == 1) & ~hit_exact), "sure hit but the exact segment misses"
    assert not np.any((c == 1) & ~hit_64), "sure hit but binary64 misses"
    # t intervals of sure hits hold the binary64 t and the exact t
    sure = np.nonzero(c == 1)[0]
    t64 = x64[3][sure] / x64[0][sure]
    assert np.all((vals[idx[sure], 8] <= t64) & (t64 <= vals[idx[sure], 9]))
    for k in sure[:3000]:
        te = Fraction(int(exact[3][k]), int(exact[0][k]))
        assert Fraction(float(vals[idx[k], 8])) <= te <= Fraction(float(vals[idx[k], 9]))
    # the binary64 decisions above are the oracle's: check them on a sample
    rng = np.random.default_rng(3)
    for k in rng.choice(idx.size, 4000, replace=False):
        i = idx[k]
        ids, _ = oracle.all_hits(np.stack([A[i], B[i], C[i]]), np.array([[0, 1, 2]], np.int32), O[i], E[i])
        assert (ids.size == 1) == bool(hit_64[k]), i
    say(f"  sure decisions agree with binary64 and exact arithmetic; unsure by kind "
        f"{np.bincount(kind[cls == 2], minlength=9).tolist()}")
