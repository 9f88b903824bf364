"""Segments that lie exactly in a triangle's plane, built from lattice points
of that plane, and the binary64 oracle's decisions on them.

For such a segment the exact Moller-Trumbore quantities det, U, W, T are all
zero (the segment is parallel to and inside the plane), so the exact reading
is a miss; the binary64 evaluation of det, however, is rounding noise and is
often non-zero, and then the binary64 test may report a hit although the
segment passes far from the triangle.  These helpers find such pairs so the
tests can state exactly what the library returns for them."""
import numpy as np

import oracle


def lattice_triangle(rng):
    """A triangle with float32 corners in [0.6, 0.9]^3 and edges of about
    0.01, and its lattice points A + i e1 + j e2 (|i|, |j| <= 6) that are
    float32 numbers inside [0.5, 1): in that range the differences and these
    sums are exact, so every lattice point lies exactly in the plane."""
    A = rng.uniform(0.6, 0.9, 3).astype(np.float32)
    B = (A + rng.normal(size=3) * 0.01).astype(np.float32)
    C = (A + rng.normal(size=3) * 0.01).astype(np.float32)
    E1, E2 = B.astype(np.float64) - A, C.astype(np.float64) - A
    pts = []
    for i in range(-6, 7):
        for j in range(-6, 7):
            P = A.astype(np.float64) + i * E1 + j * E2
            if np.all(P.astype(np.float32).astype(np.float64) == P) and np.all((P >= 0.5) & (P < 1.0)):
                pts.append(P.astype(np.float32))
    return A, B, C, np.array(pts, np.float32)


def box_distance(O, E, lo, hi):
    """Smallest distance from the segment O-E to the box [lo, hi] (the
    distance along the segment is convex: ternary search in binary64)."""
    O, E = O.astype(np.float64), E.astype(np.float64)
    lo, hi = lo.astype(np.float64), hi.astype(np.float64)

    def dist(t):
        P = O + t * (E - O)
        g = np.maximum(0.0, np.maximum(lo - P, P - hi))
        return float(np.sqrt(g @ g))

    a, b = 0.0, 1.0
    for _ in range(200):
        m1, m2 = a + (b - a) / 3, b - (b - a) / 3
        if dist(m1) <= dist(m2):
            b = m2
        else:
            a = m1
    return min(dist(0.0), dist(1.0), dist(0.5 * (a + b)))


def find_cases(seed=1, want=40, max_trials=200, per_trial=1500):
    """Pairs (triangle corners, segment) on which the binary64 oracle reports
    a hit and exact arithmetic a miss.  Returns a list of dicts with the
    corners A, B, C, the segment O, E, the distance from the segment to the
    triangle's box and the box-widening margin eta / 4 of the traversal
    (2^-22 of the largest coordinate magnitude)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(max_trials):
        A, B, C, pts = lattice_triangle(rng)
        if len(pts) < 2:
            continue
        k = rng.integers(0, len(pts), size=(per_trial, 2))
        k = k[k[:, 0] != k[:, 1]]
        O, E = pts[k[:, 0]], pts[k[:, 1]]
        V = np.stack([A, B, C])
        hit, _, _, _ = oracle.intersect(V, np.array([[0, 1, 2]], np.int32), O, E)
        lo, hi = V.min(axis=0), V.max(axis=0)
        for i in np.nonzero(hit)[0]:
            exact_hit = oracle.exact(A, B, C, O[i], E[i])[0]
            if exact_hit:
                continue
            eta4 = 2.0 ** -22 * max(np.abs(V).max(), np.abs(O[i]).max(), np.abs(E[i]).max())
            out.append({"A": A, "B": B, "C": C, "O": O[i], "E": E[i],
                        "distance": box_distance(O[i], E[i], lo, hi), "eta4": eta4})
            if len(out) >= want:
                return out
    return out
