"""Deep trees and the exact second pass.

A mesh whose triangles shrink geometrically towards a corner gives a radix
tree that is one chain (63 levels for 64 triangles with 63-bit keys); treelet
restructuring may rewire it further.  Whatever the depth, the second pass
never drops a pending subtree: when its stack is full it tests that
subtree's leaves directly.  RSI_DEBUG_PASS2_STACK shrinks the second pass's
stacks to a few entries so that path runs on ordinary meshes too; with a
one-entry first-pass stack nearly every segment goes through it."""
import os

import numpy as np
import pytest

import oracle
import paper_2305_01867_amd as rsi
from paper_2305_01867_amd import diagnostics, workloads
from gpu_helpers import dev, host, intersect, say

pytestmark = pytest.mark.gpu


def chain_mesh(m):
    """m triangles around (0.9 2^(-k/3), 0.9 2^(-(k+1)/3), 0.9 2^(-(k+2)/3)),
    their size shrinking by 2^(-1/3) each, plus one triangle spanning the
    unit box (it fixes the extent)."""
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


def chain_segments(V, F, n, seed):
    """Vertical segments through the triangles' centroids (jittered) and
    random ones in the box."""
    rng = np.random.default_rng(seed)
    C = V[F].mean(axis=1).astype(np.float64)
    k = rng.integers(0, len(F), n // 2)
    P = C[k] + rng.normal(0, 1e-3, (k.size, 3)) * np.abs(C[k]).max(axis=1, keepdims=True)
    O = np.concatenate([P + [0, 0, 0.5], rng.uniform(-0.1, 1.1, (n - k.size, 3))]).astype(np.float32)
    E = np.concatenate([P - [0, 0, 0.5], rng.uniform(-0.1, 1.1, (n - k.size, 3))]).astype(np.float32)
    return O, E


@pytest.mark.parametrize("algorithm", ["radix_tree", "restructured"])
def test_chain_mesh_depth_and_results(algorithm):
    V, F = chain_mesh(200)
    O, E = chain_segments(V, F, 4000, 3)
    hit, ids, uvt, _ = oracle.intersect(V, F, O, E)
    count = oracle.intercept_count(V, F, O, E)
    with rsi.rsi_build(dev(V), dev(F), morton_bits=63, algorithm=algorithm) as mesh:
        tree = diagnostics.export(mesh)
        depth = diagnostics.max_depth(tree)
        say(f"  {algorithm}: {F.shape[0]} triangles, depth {depth}, {int(hit.sum())} of {len(O)} segments hit")
        # the radix tree is the chain; restructuring shortens it (to 39 levels
        # here), and either way the results below are exact
        assert depth >= (63 if algorithm == "radix_tree" else 1)
        assert diagnostics.check(tree) == []
        for mode in ("boolean", "first_hit", "barycentric", "intercept_count"):
            r = intersect(mesh, O, E, mode, "certified")
            if mode == "boolean":
                assert np.array_equal(r["hit"], hit)
            elif mode == "intercept_count":
                assert np.array_equal(r["count"], count)
            else:
                assert np.array_equal(r["tri_id"], ids)


@pytest.mark.parametrize("n", [3000, 30000])  # a wave per queued segment / a lane per queued segment
def test_second_pass_tests_leaf_spans_when_its_stacks_run_out(n):
    V, F = workloads.heightfield(40, 13)
    O, E = workloads.rays_in_box(n, 14, V.min(0), V.max(0))
    hit, ids, uvt, _ = oracle.intersect(V, F, O, E)
    count = oracle.intercept_count(V, F, O, E)
    with rsi.rsi_build(dev(V), dev(F), algorithm="restructured") as mesh:
        plain_ref = {m: intersect(mesh, O, E, m, "plain") for m in ("boolean", "first_hit", "barycentric",
                                                                   "intercept_count")}
        os.environ["RSI_DEBUG_PASS2_STACK"] = "2"
        try:
            for mode in ("boolean", "first_hit", "barycentric", "intercept_count"):
                for prec in ("certified", "plain"):
                    r = intersect(mesh, O, E, mode, prec, stack_depth=1)
                    say(f"  n={n} {mode} {prec}: second pass took {int(r['counters'][1])} segments")
                    if prec == "plain":
                        for k, v in plain_ref[mode].items():
                            if k != "counters":
                                assert np.array_equal(r[k], v, equal_nan=True), (mode, k)
                    elif mode == "boolean":
                        assert np.array_equal(r["hit"], hit)
                    elif mode == "intercept_count":
                        assert np.array_equal(r["count"], count)
                    else:
                        assert np.array_equal(r["tri_id"], ids)
                        if mode == "barycentric":
                            w = uvt.astype(np.float32)
                            m = ~np.isnan(w[:, 0])
                            assert np.array_equal(r["uvt"][m], w[m])
        finally:
            del os.environ["RSI_DEBUG_PASS2_STACK"]
