"""The precision form (folded 256 x 256 heightfield, 1e7 segments of which
20% aim within ~1e-7 of edges / vertices and 5% are within 1e-6 rad of
parallel) and the learned form (~5.26e5 triangles, proposal trained on
segments the method labels, 1e8 evaluation segments in 10 chunks) at full
size: sampled segments of every group, plus every segment where the binary32
and certified paths disagree, against the binary64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_01867_amd as rsi
from paper_2305_01867_amd import workloads
from gpu_helpers import dev, host, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("algorithm", ["radix_tree", "restructured"])
def test_precision_form_exact(algorithm):
    V, F, O, E, kind = workloads.precision_config()
    say(f"[precision form, {algorithm}] {F.shape[0]} triangles, {O.shape[0]} segments, "
        f"groups {np.bincount(kind).tolist()}")
    rng = np.random.default_rng(5)
    sample = np.concatenate([rng.choice(np.nonzero(kind == k)[0], c, replace=False)
                             for k, c in ((0, 600), (1, 1500), (2, 900))])
    with rsi.rsi_build(dev(V), dev(F), algorithm=algorithm) as mesh:
        assert rsi.rsi_mesh_info_get(mesh)["node_width"] == 4
        dO, dE = dev(O), dev(E)
        cnt = rsi.rsi_intersect(mesh, dO, dE, mode="intercept_count", precision="certified")
        got = host(cnt["count"])[sample]
        del cnt
        want = oracle.intercept_count(V, F, O[sample], E[sample])
        say(f"  intercept_count: {sample.size} sampled segments, {int(want.sum())} distinct hits")
        assert np.array_equal(got, want)
        for mode in ("boolean", "first_hit", "barycentric"):
            key = "hit" if mode == "boolean" else "tri_id"
            cert = rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision="certified")
            plain = rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision="plain")
            c, p = host(cert[key]), host(plain[key])
            diff = np.nonzero(c != p)[0]
            cnt = host(cert["counters"])
            say(f"  {mode}: re-decided in binary64 {cnt[0]}, binary32 differs on {diff.size} "
                f"(by group {np.bincount(kind[diff], minlength=3).tolist()})")
            idx = np.unique(np.concatenate([sample, diff[:2500]]))
            hit, ids, uvt, _ = oracle.intersect(V, F, O[idx], E[idx])
            if mode == "boolean":
                assert np.array_equal(c[idx], hit)
            else:
                assert np.array_equal(c[idx], ids)
            if mode == "barycentric":
                g = host(cert["uvt"])[idx]
                w = uvt.astype(np.float32)
                assert np.array_equal(np.isnan(g), np.isnan(w)) and np.all(g[~np.isnan(w)] == w[~np.isnan(w)])
            # the binary32 path is wrong only where the oracle agrees with the certified one
            bad_plain = np.sum(p[idx] != (hit if mode == "boolean" else ids))
            say(f"    oracle-checked {idx.size}: binary32 wrong on {bad_plain}, certified wrong on 0")
            del cert, plain
            torch.cuda.empty_cache()


def test_learned_form_exact_and_identical():
    V, F = workloads.learned_mesh()
    say(f"[learned form] {F.shape[0]} triangles")
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        Ot, Et = workloads.learned_rays(1_000_000, 5001)
        loss, n_lab = rsi.rsi_proposal_train(mesh, dev(Ot), dev(Et), epochs=2, batch=4096, lr=2e-3, seed=3)
        say(f"  trained on {n_lab} labelled segments, epoch loss {[round(x, 3) for x in loss.tolist()]}")
        rng = np.random.default_rng(9)
        tot = {"hits": 0, "late": 0, "segments": 0}
        for k in range(10):
            O, E = workloads.learned_rays(10_000_000, 5100 + k)
            dO, dE = dev(O), dev(E)
            a = rsi.rsi_intersect(mesh, dO, dE, mode="boolean", precision="certified")
            b = rsi.rsi_intersect(mesh, dO, dE, mode="boolean", precision="certified", proposal=True)
            ha, hb = host(a["hit"]), host(b["hit"])
            assert np.array_equal(ha, hb), f"chunk {k}: the proposal changed a result"
            tot["hits"] += int(hb.sum())
            tot["late"] += int(host(b["counters"])[2])
            tot["segments"] += O.shape[0]
            if k < 2:
                idx = rng.choice(O.shape[0], 700, replace=False)
                hit, _, _, _ = oracle.intersect(V, F, O[idx], E[idx])
                assert np.array_equal(hb[idx], hit), f"chunk {k}"
            del a, b, dO, dE
            torch.cuda.empty_cache()
        say(f"  1e8 segments: hit fraction {tot['hits'] / tot['segments']:.4f}, "
            f"proposal miss rate {tot['late'] / max(tot['hits'], 1):.4f}")
