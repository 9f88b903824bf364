"""Every segment of the paper-scale workload (128 x 128 heightfield, 32,258
triangles, 1e7 segments) and of the precision form (folded 256 x 256
heightfield, 130,050 triangles, 1e7 segments of which 25% aim at edges,
vertices or near-parallel planes) against the binary64 oracle's results, in
all four modes, on the benchmark's build and launch.

The oracle's outputs over 1e7 segments are stored as per-chunk digests by
tests/golden/make_full_fixtures.py (which calls only the oracle); a chunk
whose digest differs is re-run through the oracle here, so a failure names
the segments."""
import importlib.util
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2305_01867_amd as rsi
from gpu_helpers import dev, host, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location("full_fixtures", os.path.join(HERE, "golden", "make_full_fixtures.py"))
FIX = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(FIX)

# output array(s) of each mode and the fixture column(s) they are checked against
COLUMNS = {"boolean": (("hit", 0),), "first_hit": (("tri_id", 1),), "barycentric": (("tri_id", 1), ("uvt", 2)),
           "intercept_count": (("count", 3),)}


def _digest(key, a):
    if key == "hit":
        return FIX.digest(a.astype(np.uint8))
    if key == "uvt":
        return FIX.digest(FIX.uvt_f32(a))
    return FIX.digest(a.astype("<i4"))


def _bad_chunks(rows, key, col, arr):
    bad = []
    for c, (s, m, _, *dig) in sorted(rows.items()):
        if _digest(key, arr[s:s + m]) != dig[col]:
            bad.append(c)
    return bad


def _explain(V, F, O, E, rows, c, key, arr):
    """Oracle results of one chunk, and the segments that differ."""
    s, m = rows[c][0], rows[c][1]
    if key == "count":
        want = oracle.intercept_count(V, F, O[s:s + m], E[s:s + m])
    else:
        hit, ids, uvt, _ = oracle.intersect(V, F, O[s:s + m], E[s:s + m])
        want = {"hit": hit, "tri_id": ids, "uvt": FIX.uvt_f32(uvt)}[key]
    got = arr[s:s + m]
    if key == "uvt":
        got = FIX.uvt_f32(got)
        d = np.nonzero(np.any(got.view(np.uint32) != want.view(np.uint32), axis=1))[0]
    else:
        d = np.nonzero(got != want)[0]
    return [(int(s + i), got[i].tolist(), want[i].tolist()) for i in d[:8]], int(d.size)


def _check_all(name, builds):
    head, rows = FIX.read(name)
    V, F, O, E = FIX.workload(name)
    n = O.shape[0]
    n_chunks = (n + int(head["chunk"]) - 1) // int(head["chunk"])
    assert len(rows) == n_chunks, f"fixture for {name} holds {len(rows)} of {n_chunks} chunks"
    assert FIX.input_digest(V, F, O, E) == head["inputs"], "this host's inputs differ from the fixture's"
    n_hit = sum(r[2] for r in rows.values())
    say(f"[full size, {name}] {F.shape[0]} triangles, {n} segments, {n_hit} hit (oracle)")
    dO, dE = dev(O), dev(E)
    failures = []
    for algorithm, modes, node_width in builds:
        with rsi.rsi_build(dev(V), dev(F), algorithm=algorithm) as mesh:
            for mode in modes:
                for prec in ("certified", "plain"):
                    r = rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision=prec, node_width=node_width)
                    cnt = host(r["counters"])
                    for key, col in COLUMNS[mode]:
                        arr = host(r[key])
                        bad = _bad_chunks(rows, key, col, arr)
                        tag = f"{algorithm}, width {node_width or 'widest'}, {mode}, {prec}, {key}"
                        say(f"  {tag}: {n_chunks - len(bad)} of {n_chunks} chunks equal the oracle "
                            f"(re-decided in binary64 {int(cnt[0])}, second pass {int(cnt[1])})")
                        if bad and prec == "certified":
                            ex, k = _explain(V, F, O, E, rows, bad[0], key, arr)
                            failures.append((tag, bad[:10], k, ex))
                    del r
                    torch.cuda.empty_cache()
    assert not failures, failures


def test_paper_scale_every_segment():
    _check_all("paper_scale", [("restructured", ("boolean", "first_hit", "barycentric", "intercept_count"), 0),
                               ("radix_tree", ("boolean", "first_hit"), 0),
                               ("restructured", ("boolean", "first_hit"), 2)])


def test_precision_form_every_segment():
    _check_all("precision", [("restructured", ("boolean", "first_hit", "barycentric", "intercept_count"), 0),
                             ("radix_tree", ("boolean", "first_hit"), 0)])
