"""Pins of the CPU reference of the learned proposal: finite differences of
the binary64 network, bf16 rounding against torch's conversion, feature and
frontier closed forms."""
import math

import numpy as np
import torch

import oracle
from oracle import mlp_reference as ref
from paper_2305_01867_amd import workloads


def test_finite_differences_of_reference():
    rng = np.random.default_rng(0)
    shapes = [(6, 7), (6, 6), (6, 6), (5, 6)]
    n_params = sum(o * i for o, i in shapes) + sum(o for o, _ in shapes)
    params = rng.normal(0, 0.6, n_params)
    X = rng.normal(0, 1, (9, 7))
    y = rng.integers(0, 4, 9)
    loss, _, grad = ref.forward_backward(X, y, params, n_buckets=4, round_bf16=False, shapes=shapes)
    h = 1e-6
    for j in rng.choice(n_params, 60, replace=False):
        p1, p2 = params.copy(), params.copy()
        p1[j] += h
        p2[j] -= h
        l1 = ref.forward_backward(X, y, p1, 4, round_bf16=False, shapes=shapes)[0]
        l2 = ref.forward_backward(X, y, p2, 4, round_bf16=False, shapes=shapes)[0]
        fd = (l1 - l2) / (2 * h)
        assert abs(fd - grad[j]) <= 1e-6 * max(1.0, abs(grad[j])), (j, fd, grad[j])


def test_masked_buckets_get_no_gradient():
    rng = np.random.default_rng(1)
    shapes = [(6, 7), (6, 6), (6, 6), (5, 6)]
    n_params = sum(o * i for o, i in shapes) + sum(o for o, _ in shapes)
    params = rng.normal(0, 0.6, n_params)
    X = rng.normal(0, 1, (5, 7))
    _, _, grad = ref.forward_backward(X, rng.integers(0, 3, 5), params, n_buckets=3, round_bf16=False,
                                      shapes=shapes)
    Ws, bs = ref.unpack(grad, shapes)
    assert np.all(Ws[3][3:] == 0) and np.all(bs[3][3:] == 0)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.normal(0, 10, 20000), rng.normal(0, 1e-3, 1000),
                        # exact ties between two bf16 values
                        (np.arange(1000) * 2 + 1) * 2.0 ** -8 + 1.0]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).float().numpy()
    assert np.array_equal(ref.bf16(x).astype(np.float32), want)


def test_feature_closed_forms():
    lo, hi = np.float32([0, -1, 2]), np.float32([4, 1, 2])  # z is flat
    O = np.float32([[0, -1, 2], [4, 1, 2], [1, 0, 2]])
    E = np.float32([[2, 0.5, 2], [0, -1, 2], [3, 1, 2]])
    X = ref.features(O, E, lo, hi)
    assert X.shape == (3, 224)
    assert np.array_equal(X[:, :6], [[-1, -1, -1, 0, 0.5, -1], [1, 1, -1, -1, -1, -1], [-0.5, 0, -1, 0.5, 1, -1]])
    # band 0 of coordinate 0 is sin / cos(pi x)
    assert np.allclose(X[:, 6], np.sin(np.pi * X[:, 0])) and np.allclose(X[:, 7], np.cos(np.pi * X[:, 0]))
    # band 2 has frequency 2
    assert np.allclose(X[:, 10], np.sin(2 * np.pi * X[:, 0]), atol=1e-12)
    assert np.all(X[:, 198:] == 0)


def test_frontier_reference():
    V, F, _, _ = workloads.appendix_scene()
    s = oracle.build_structure(V, F, 30)
    refs, first = ref.frontier(s["tree"], 4)
    assert refs.tolist() == [~0, ~1, ~2, ~3] and first.tolist() == [0, 1, 2, 3]
    V, F = workloads.heightfield(64, 11)
    s = oracle.build_structure(V, F, 30)
    refs, first = ref.frontier(s["tree"], F.shape[0])
    # at most 2^8 buckets; fewer when some leaves sit above depth 8
    assert 128 < len(refs) <= 256
    assert first[0] == 0 and np.all(np.diff(first) > 0)
    # a bucket's first leaf is its subtree's leftmost leaf, and the subtree of
    # bucket b ends right before the first leaf of bucket b+1
    t = s["tree"]
    for b, r in enumerate(refs):
        last = ~r if r < 0 else t["last"][r]
        nxt = first[b + 1] if b + 1 < len(refs) else F.shape[0]
        assert last + 1 == nxt


def test_zero_network_loss_is_log_of_bucket_count_and_gradient_is_softmax_minus_onehot():
    """All weights and biases zero: every logit is 0, the softmax is uniform
    over the n unmasked buckets, so the loss is ln n for any labels, and
    dL/dz = (softmax - onehot) / rows gives the last bias gradient
    1/n - (share of rows with label k) in bucket k (0 for masked buckets);
    nothing reaches the other parameters, whose inputs or upstream gradients
    are all zero."""
    rng = np.random.default_rng(7)
    rows, nb = 37, 150
    X = rng.normal(0, 1, (rows, ref.INPUTS))
    y = rng.integers(0, nb, rows)
    for rnd in (False, True):
        loss, logits, grad = ref.forward_backward(X, y, np.zeros(ref.N_PARAMS), nb, round_bf16=rnd)
        assert np.all(logits == 0)
        assert abs(loss - np.log(nb)) <= 1e-15
        Ws, bs = ref.unpack(grad)
        want = np.zeros(ref.OUT)
        want[:nb] = 1.0 / nb
        np.subtract.at(want, y, 1.0 / rows)
        # with bf16 rounding each row's (p - y) / rows is rounded once (2^-9 relative)
        tol = 1e-15 if not rnd else rows * 2.0 ** -9 / rows
        assert np.allclose(bs[3], want, rtol=0, atol=tol)
        assert np.all(bs[3][nb:] == 0)
        for W in Ws:
            assert np.all(W == 0)
        for b in bs[:3]:
            assert np.all(b == 0)


def test_hand_computed_two_row_network():
    """A 2-2-2-2-3 network whose every value is worked out by hand:
    X = [[1, 2], [-1, 0.5]];  layer 1 identity, b1 = 0  -> relu [[1, 2], [0, 0.5]]
    layer 2 identity, b2 = (-0.5, 0)                    -> relu [[0.5, 2], [0, 0.5]]
    layer 3 [[1, 1], [0, 1]], b3 = 0                     -> [[2.5, 2], [0.5, 0.5]]
    layer 4 [[1, 0], [0, 1], [1, -1]], b4 = (0, 0, 0.25) -> logits [[2.5, 2, 0.75], [0.5, 0.5, 0.25]]
    labels (0, 2): loss = mean(log(e^2.5 + e^2 + e^0.75) - 2.5, log(2 e^0.5 + e^0.25) - 0.25).
    With only 2 buckets the third logit is masked: loss = mean(log(e^2.5 + e^2) - 2.5,
    log(2 e^0.5) - 0.5) for labels (0, 1)."""
    shapes = [(2, 2), (2, 2), (2, 2), (3, 2)]
    W1, W2, W3 = [1, 0, 0, 1], [1, 0, 0, 1], [1, 1, 0, 1]
    W4 = [1, 0, 0, 1, 1, -1]
    b = [0, 0, -0.5, 0, 0, 0, 0, 0, 0.25]
    params = np.array(W1 + W2 + W3 + W4 + b, np.float64)
    X = np.array([[1.0, 2.0], [-1.0, 0.5]])
    loss, logits, grad = ref.forward_backward(X, np.array([0, 2]), params, 3, round_bf16=False, shapes=shapes)
    assert np.array_equal(logits, [[2.5, 2.0, 0.75], [0.5, 0.5, 0.25]])
    e = math.exp
    want = 0.5 * ((math.log(e(2.5) + e(2.0) + e(0.75)) - 2.5) + (math.log(2 * e(0.5) + e(0.25)) - 0.25))
    assert abs(loss - want) <= 1e-15
    # dL/db4 = mean over rows of softmax - onehot
    p0 = np.array([e(2.5), e(2.0), e(0.75)]) / (e(2.5) + e(2.0) + e(0.75))
    p1 = np.array([e(0.5), e(0.5), e(0.25)]) / (2 * e(0.5) + e(0.25))
    want_b4 = 0.5 * ((p0 - [1, 0, 0]) + (p1 - [0, 0, 1]))
    _, bs = ref.unpack(grad, shapes)
    assert np.allclose(bs[3], want_b4, rtol=0, atol=1e-15)
    # dL/dW4 = dZ^T h3 with h3 = [[2.5, 2], [0.5, 0.5]]
    Ws, _ = ref.unpack(grad, shapes)
    dZ = 0.5 * np.stack([p0 - [1, 0, 0], p1 - [0, 0, 1]])
    assert np.allclose(Ws[3], dZ.T @ np.array([[2.5, 2.0], [0.5, 0.5]]), rtol=0, atol=1e-15)
    loss2, _, _ = ref.forward_backward(X, np.array([0, 1]), params, 2, round_bf16=False, shapes=shapes)
    want2 = 0.5 * ((math.log(e(2.5) + e(2.0)) - 2.5) + (math.log(2 * e(0.5)) - 0.5))
    assert abs(loss2 - want2) <= 1e-15
