"""The learned subtree proposal on the GPU: frontier vs the oracle tree,
features and gradients vs the binary64 CPU reference, the fused inference
kernel vs the training forward pass, training, and -- the property that
matters -- identical intersection results with and without the proposal."""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp_reference as ref
import paper_2305_01867_amd as rsi
from paper_2305_01867_amd import workloads
from gpu_helpers import dev, host, intersect, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tiny():
    V, F, O, E = workloads.tiny_config()
    mesh = rsi.rsi_build(dev(V), dev(F))
    yield V, F, O, E, mesh
    mesh.close()


def test_frontier_matches_oracle(tiny):
    V, F, O, E, mesh = tiny
    refs, first = rsi.rsi_proposal_frontier(mesh)
    s = oracle.build_structure(V, F, 30)
    want_refs, want_first = ref.frontier(s["tree"], F.shape[0])
    assert host(refs).tolist() == want_refs.tolist()
    assert host(first).tolist() == want_first.tolist()


def test_features_match_reference(tiny):
    V, F, O, E, mesh = tiny
    X = host(rsi.rsi_proposal_features(mesh, dev(O[:2000]), dev(E[:2000])).float())
    lo, hi = oracle.mesh_bounds(V)
    want = ref.bf16(ref.features(O[:2000], E[:2000], lo, hi))
    # bf16 of a float32 sinpi vs bf16 of a binary64 sin: at most one bf16 step
    diff = np.abs(X - want)
    assert np.all(diff <= np.maximum(np.abs(want), 1e-30) * 2.0 ** -7 + 1e-7)
    assert np.mean(diff > 0) < 0.01


def _random_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    P = np.zeros(rsi.MLP_PARAMS, np.float32)
    off = 0
    for o, i in ref.LAYER_SHAPES:
        fan = ref.FEAT if i == ref.INPUTS else i
        W = rng.uniform(-1, 1, (o, i)) * np.sqrt(6.0 / fan) * scale
        if i == ref.INPUTS:
            W[:, ref.FEAT:] = 0
        P[off:off + o * i] = W.ravel()
        off += o * i
    P[off:] = rng.normal(0, 0.05, 4 * ref.HIDDEN)
    return P


@pytest.mark.parametrize("rows", [250, 2900])
def test_gradient_matches_reference(tiny, rows):
    """250 rows: each weight gradient in one pass over the rows; 2900 rows:
    split over 12 row chunks of 256 (the last one ragged) and summed in order;
    both row counts end in a partial tile of the fused training pass."""
    V, F, O, E, mesh = tiny
    P = _random_params(3)
    rsi.rsi_proposal_params(mesh, dev(P))
    assert O.shape[0] >= rows
    nb = len(host(rsi.rsi_proposal_frontier(mesh)[0]))
    labels = np.random.default_rng(4).integers(0, nb, rows).astype(np.int32)
    dO, dE = dev(O[:rows]), dev(E[:rows])
    grad, logits, loss = rsi.rsi_proposal_gradient(mesh, dO, dE, dev(labels))
    X0 = host(rsi.rsi_proposal_features(mesh, dO, dE).float()).astype(np.float64)
    want_loss, want_logits, want_grad = ref.forward_backward(X0, labels, P.astype(np.float64), nb)
    g = host(grad).astype(np.float64)
    lg = host(logits).astype(np.float64)
    assert abs(float(host(loss)[0]) - want_loss) <= 1e-3 * abs(want_loss)
    assert np.linalg.norm(lg - want_logits) <= 1e-3 * np.linalg.norm(want_logits)
    off = 0
    blocks = [(o * i) for o, i in ref.LAYER_SHAPES] + [ref.HIDDEN] * 4
    for k, size in enumerate(blocks):
        a, b = g[off:off + size], want_grad[off:off + size]
        off += size
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
        say(f"  param block {k}: rel err {rel:.2e}, cosine {cos:.7f}")
        assert rel <= 1e-3 and cos >= 0.9999


def test_fused_inference_equals_forward_argmax(tiny):
    V, F, O, E, mesh = tiny
    rsi.rsi_proposal_params(mesh, dev(_random_params(5)))
    nb = len(host(rsi.rsi_proposal_frontier(mesh)[0]))
    rows = 4000  # not a multiple of the row tile
    dO, dE = dev(O[:rows]), dev(E[:rows])
    _, logits, _ = rsi.rsi_proposal_gradient(mesh, dO, dE, dev(np.zeros(rows, np.int32)))
    lg = host(logits)[:, :nb]
    want = np.argmax(lg, axis=1)  # first index on ties, as the kernel
    got = host(rsi.rsi_proposal_predict(mesh, dO, dE)).astype(np.int64)
    assert np.array_equal(got, want)


def test_inference_buckets_match_reference():
    """The fused inference kernel against the binary64 reference network
    (oracle/mlp_reference.py, same bf16 rounding points, features from the
    reference's own binary64 sin / cos) on trained weights, 6000 segments.
    The kernel accumulates in fp32, the reference in binary64, so a hidden
    activation may round to the neighbouring bf16 value on one side only; the
    bucket must equal the reference's argmax except where the reference's two
    largest logits lie within 2 s of each other, s = 2^-7 max_j sum_k
    |W4[j, k] h3[k]| -- every last-layer activation moved by two bf16 steps
    (earlier layers' rounding differences reach the logits through it)."""
    V, F = workloads.heightfield(64, 11)
    O, E = workloads.rays_in_box(60000, 33, V.min(0), V.max(0))
    Oe, Ee = workloads.rays_in_box(6000, 37, V.min(0), V.max(0))
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        rsi.rsi_proposal_train(mesh, dev(O), dev(E), epochs=2, batch=2048, lr=2e-3, seed=7)
        P = host(rsi.rsi_proposal_params(mesh)).astype(np.float64)
        nb = len(host(rsi.rsi_proposal_frontier(mesh)[0]))
        got = host(rsi.rsi_proposal_predict(mesh, dev(Oe), dev(Ee))).astype(np.int64)
    lo, hi = oracle.mesh_bounds(V)
    X0 = ref.bf16(ref.features(Oe, Ee, lo, hi))
    _, logits, _ = ref.forward_backward(X0, np.zeros(len(Oe), np.int64), P, nb)
    z = logits[:, :nb]
    want = np.argmax(z, axis=1)
    top2 = np.sort(z, axis=1)[:, -2:]
    gap = top2[:, 1] - top2[:, 0]
    # last hidden layer of the reference, recomputed from its parameters
    Ws, bs = ref.unpack(P)
    Wr = [ref.bf16(W) for W in Ws]
    h = X0
    for l in range(3):
        h = ref.bf16(np.maximum(h @ Wr[l].T + bs[l], 0.0))
    s = 2.0 ** -7 * (np.abs(h) @ np.abs(Wr[3][:nb]).T).max(axis=1)
    diff = got != want
    say(f"  {len(got)} segments, {nb} buckets: {int(diff.sum())} buckets differ from the reference argmax, "
        f"largest gap among them {gap[diff].max() if diff.any() else 0:.3g}, median gap {np.median(gap):.3g}")
    assert np.all(gap[diff] < 2 * s[diff])
    assert diff.mean() < 0.01


def test_training_lowers_loss_and_keeps_results_exact():
    V, F = workloads.heightfield(64, 11)
    O, E = workloads.rays_in_box(60000, 33, V.min(0), V.max(0))
    Ot, Et = workloads.rays_in_box(3000, 34, V.min(0), V.max(0))
    hit, ids, uvt, _ = oracle.intersect(V, F, Ot, Et)
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        loss, n_lab = rsi.rsi_proposal_train(mesh, dev(O), dev(E), epochs=4, batch=2048, lr=2e-3, seed=7)
        say(f"  labelled {n_lab}, epoch loss {loss.tolist()}")
        assert n_lab > 30000
        assert loss[0] < 1.2 * np.log(256) and loss[-1] < 0.8 * loss[0]
        dO, dE = dev(Ot), dev(Et)
        for width in (0, 2):  # the proposal order on its own 4-wide tree, and on binary nodes
            for mode in ("boolean", "first_hit", "barycentric"):
                for prec in ("plain", "certified"):
                    a = intersect(mesh, Ot, Et, mode, prec)
                    b = {k: host(v) for k, v in rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision=prec,
                                                                  proposal=True, node_width=width).items()}
                    for k in a:
                        if k != "counters":
                            assert np.array_equal(a[k], b[k], equal_nan=True), (width, mode, prec, k)
                    if prec == "certified":
                        key = "hit" if mode == "boolean" else "tri_id"
                        want = hit if mode == "boolean" else ids
                        assert np.array_equal(b[key], want)
        # the gain: work per segment with the trained, an untrained and no
        # proposal, on 4-wide nodes (node fetches) and on binary nodes
        visits = {}
        for width in (4, 2):
            visits["none", width] = rsi.rsi_traversal_stats(mesh, dO, dE, mode="boolean", node_width=width)[0]
            visits["trained", width] = rsi.rsi_traversal_stats(mesh, dO, dE, mode="boolean", proposal=True,
                                                               node_width=width)[0]
        got = rsi.rsi_intersect(mesh, dO, dE, mode="boolean", proposal=True)
        n_hit = int(host(got["hit"]).sum())
        miss_rate = float(host(got["counters"])[2]) / max(n_hit, 1)
        with tempfile.TemporaryDirectory() as d:
            path = os.path.join(d, "p.bin")
            rsi.rsi_proposal_save(mesh, path)
            P_trained = host(rsi.rsi_proposal_params(mesh))
            buckets = host(rsi.rsi_proposal_predict(mesh, dO, dE))
            rsi.rsi_proposal_train(mesh, dO[:64], dE[:64], epochs=1, reinit=True, seed=99)
            for width in (4, 2):
                visits["untrained", width] = rsi.rsi_traversal_stats(mesh, dO, dE, mode="boolean", proposal=True,
                                                                     node_width=width)[0]
            rsi.rsi_proposal_load(mesh, path)
            assert np.array_equal(host(rsi.rsi_proposal_params(mesh)), P_trained)
            assert np.array_equal(host(rsi.rsi_proposal_predict(mesh, dO, dE)), buckets)
        for width in (4, 2):
            m = [float(host(visits[k, width]).mean()) for k in ("none", "untrained", "trained")]
            say(f"  mean node visits ({width}-wide): none {m[0]:.2f}, untrained {m[1]:.2f}, trained {m[2]:.2f}; "
                f"proposal miss rate {miss_rate:.3f}")
            assert m[2] < m[1]
            assert m[2] < m[0]  # the trained proposal saves node visits over the plain order
        assert miss_rate < 0.95  # chance level is 1 - 1/(number of buckets) ~ 0.996


def test_proposal_on_a_restructured_tree():
    """Buckets are subtrees, not leaf ranges, once treelets are rewired: the
    labels come from each leaf's bucket, and proposal-first results stay the
    oracle's."""
    V, F = workloads.heightfield(48, 12)
    O, E = workloads.rays_in_box(40000, 35, V.min(0), V.max(0))
    Ot, Et = workloads.rays_in_box(2000, 36, V.min(0), V.max(0))
    hit, ids, _, _ = oracle.intersect(V, F, Ot, Et)
    with rsi.rsi_build(dev(V), dev(F), algorithm="restructured") as mesh:
        loss, n_lab = rsi.rsi_proposal_train(mesh, dev(O), dev(E), epochs=3, batch=2048, lr=2e-3, seed=8)
        say(f"  restructured tree: labelled {n_lab}, epoch loss {loss.tolist()}")
        assert n_lab > 20000 and loss[-1] < 0.8 * loss[0]
        for width in (0, 2):
            for mode, key, want in (("boolean", "hit", hit), ("first_hit", "tri_id", ids)):
                got = host(rsi.rsi_intersect(mesh, dev(Ot), dev(Et), mode=mode, precision="certified",
                                             proposal=True, node_width=width)[key])
                assert np.array_equal(got, want), (width, mode)


def test_training_is_deterministic():
    """The training list is compacted in segment order, the weight gradients
    and the loss are summed in fixed orders: two trainings from the same seed
    give bit-identical parameters and losses."""
    V, F = workloads.heightfield(64, 12)
    O, E = workloads.rays_in_box(40000, 35, V.min(0), V.max(0))
    runs = []
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        for _ in range(2):
            loss, n_lab = rsi.rsi_proposal_train(mesh, dev(O), dev(E), epochs=2, batch=2048, lr=2e-3, seed=9,
                                                 reinit=True)
            runs.append((loss.numpy().copy(), n_lab, host(rsi.rsi_proposal_params(mesh)).copy()))
    say(f"  labelled {runs[0][1]}, epoch loss {runs[0][0].tolist()}")
    assert runs[0][1] == runs[1][1] > 2048
    assert np.array_equal(runs[0][0], runs[1][0])
    assert np.array_equal(runs[0][2].view(np.uint32), runs[1][2].view(np.uint32))
