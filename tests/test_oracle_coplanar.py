"""Binary64 decisions on segments lying exactly in a triangle's plane.

The reading the oracle takes is the binary64 evaluation of the
Moller-Trumbore predicates as written (det == 0 exactly is the only
parallel test; paper: Epilogue, binary64 intermediates for near-parallel
rays).  For a segment lying in the triangle's plane the exact predicates
all vanish; binary64 then evaluates det to rounding noise, and when that
noise is non-zero the oracle may report a hit although exact arithmetic says
miss -- also for segments that pass far from the triangle.  These pins show
the class exists and fix its description: exact det is 0 for every such
pair (so the binary32 bound of the certified test classifies it as unsure
whenever the pair is tested), and some of them lie much farther from the
triangle's box than the traversal's box-widening margin."""
from fractions import Fraction

import numpy as np

from coplanar_cases import find_cases


def _exact_det(A, B, C, O, E):
    q = lambda p: [Fraction(float(x)) for x in p]
    A, B, C, O, E = q(A), q(B), q(C), q(O), q(E)
    d = [E[k] - O[k] for k in range(3)]
    e1 = [B[k] - A[k] for k in range(3)]
    e2 = [C[k] - A[k] for k in range(3)]
    p = [d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]]
    return e1[0] * p[0] + e1[1] * p[1] + e1[2] * p[2]


def test_binary64_reports_hits_of_in_plane_segments_far_from_the_triangle():
    cases = find_cases()
    assert len(cases) >= 20
    for c in cases:
        assert _exact_det(c["A"], c["B"], c["C"], c["O"], c["E"]) == 0
    far = [c for c in cases if c["distance"] > 1000 * c["eta4"]]
    # many of them pass far outside the triangle's box
    assert len(far) >= len(cases) // 4
    assert max(c["distance"] for c in cases) > 1e-3
