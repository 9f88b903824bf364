"""Segments lying exactly in a triangle's plane (lattice points of the
plane), on which the binary64 oracle reports hits that exact arithmetic does
not (see tests/test_oracle_coplanar.py).  The certified path re-decides in
binary64 every pair whose triangle its conservative box test reaches, so it
returns the oracle's decision whenever the segment passes within the box
margin eta / 4 of the triangle's box; a segment farther away never reaches
that triangle, and there the certified answer is the exact one (no hit) while
the oracle's is the rounding artefact.  This is the one class of inputs on
which the certified path and the binary64 oracle may differ."""
import numpy as np
import pytest

import oracle
import paper_2305_01867_amd as rsi
from coplanar_cases import find_cases
from gpu_helpers import dev, intersect, say

pytestmark = pytest.mark.gpu


def test_in_plane_segments_near_and_far():
    cases = find_cases()
    near = far = 0
    for c in cases:
        A, B, C = c["A"], c["B"], c["C"]
        # a second triangle across the first one's box, so the tree has a root
        # node and box tests decide what the traversal reaches
        D = (A + np.float32(0.03)).astype(np.float32)
        V = np.stack([A, B, C, D, (D + [0.01, 0, 0]).astype(np.float32), (D + [0, 0.01, 0.002]).astype(np.float32)])
        F = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
        O, E = c["O"][None], c["E"][None]
        hit, ids, _, _ = oracle.intersect(V, F, O, E)
        hit2, ids2, _, _ = oracle.intersect(V, F[1:], O, E)  # the exact answer without the artefact
        with rsi.rsi_build(dev(V), dev(F)) as mesh:
            b = intersect(mesh, O, E, "boolean", "certified")["hit"]
            f = intersect(mesh, O, E, "first_hit", "certified")["tri_id"]
        if c["distance"] <= c["eta4"]:
            near += 1
            assert b[0] == hit[0] and f[0] == ids[0]
        else:
            far += 1
            assert b[0] == hit2[0] and f[0] == (ids2[0] + 1 if ids2[0] >= 0 else -1)
    say(f"  {len(cases)} in-plane segments with a binary64 hit and an exact miss: {near} within eta/4 of the "
        f"triangle's box (certified == oracle), {far} farther (certified == exact)")
    assert len(cases) >= 20
