"""CPU reference of the learned subtree proposal (TEST INFRASTRUCTURE ONLY).

What it follows: the proposal described for the learned form of the method --
inputs are the 6 end-point coordinates normalised to [-1, 1] over the mesh box
plus sin / cos(pi f_k x) for 16 bands f_k = 2^(k/2), three hidden ReLU layers
of 256, logits over the depth-8 frontier buckets of the BVH, cross-entropy
loss; buckets are the frontier subtrees in left-to-right order (the binary
radix tree of Karras 2012 walked top-down, as the paper's BVH is).

Arithmetic: binary64 throughout.  With round_bf16=True the operands are
rounded to bfloat16 (round to nearest even, via float32) at the points where
the GPU stores bfloat16: weights, hidden activations, and the gradients that
enter a matrix product -- so the comparison with the GPU measures only the
accumulation order.  With round_bf16=False it is a plain binary64 network,
used for the finite-difference pin.
"""
from __future__ import annotations

import numpy as np

BANDS = 16
FEAT = 6 + 6 * 2 * BANDS  # 198
INPUTS = 224
HIDDEN = 256
OUT = 256
LAYER_SHAPES = [(OUT, INPUTS), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN), (HIDDEN, HIDDEN)]  # [out][in]
N_WEIGHTS = sum(o * i for o, i in LAYER_SHAPES)
N_PARAMS = N_WEIGHTS + 4 * HIDDEN


def bf16(x):
    """Round to bfloat16 (nearest even) through float32; returns float64."""
    x32 = np.asarray(x, dtype=np.float64).astype(np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    r = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(x32), x32, out).astype(np.float64)


def band_freqs():
    """float32 values of 2^(k/2), k = 0..15."""
    s2 = np.float32(np.sqrt(2.0))
    return np.array([np.float32(2.0 ** (k // 2)) * (s2 if k % 2 else np.float32(1.0)) for k in range(BANDS)],
                    dtype=np.float32)


def features(O, E, lo, hi):
    """[n, 224] network inputs (float64 values of the float32 definition,
    before bf16 rounding): x = 2 (p - lo) / (hi - lo) - 1 per coordinate in
    float32, then sin / cos(pi * fl32(f_k x))."""
    P = np.concatenate([np.asarray(O, np.float32), np.asarray(E, np.float32)], axis=1)
    lo6 = np.tile(np.asarray(lo, np.float32), 2)
    hi6 = np.tile(np.asarray(hi, np.float32), 2)
    ext = (hi6 - lo6).astype(np.float32)
    with np.errstate(all="ignore"):
        n = np.where(ext > 0, (P - lo6) / np.where(ext > 0, ext, np.float32(1)), np.float32(0)).astype(np.float32)
    x = (n * np.float32(2.0) - np.float32(1.0)).astype(np.float32)
    X = np.zeros((P.shape[0], INPUTS), np.float64)
    X[:, :6] = x
    f = band_freqs()
    for c in range(6):
        a = (f[None, :] * x[:, c:c + 1]).astype(np.float32).astype(np.float64)
        X[:, 6 + c * 2 * BANDS + 0:6 + (c + 1) * 2 * BANDS:2] = np.sin(np.pi * a)
        X[:, 6 + c * 2 * BANDS + 1:6 + (c + 1) * 2 * BANDS:2] = np.cos(np.pi * a)
    return X


def unpack(params, shapes=LAYER_SHAPES, hidden_sizes=None):
    """Split the flat parameter vector into weight matrices [out][in] and biases."""
    params = np.asarray(params, np.float64)
    Ws, off = [], 0
    for o, i in shapes:
        Ws.append(params[off:off + o * i].reshape(o, i))
        off += o * i
    bs = []
    for o, _ in shapes:
        bs.append(params[off:off + o])
        off += o
    return Ws, bs


def forward_backward(X0, labels, params, n_buckets, round_bf16=True, shapes=LAYER_SHAPES):
    """Mean cross-entropy over the rows, logits, and the gradient (flat, same
    layout as params).  X0 [rows, in] are the inputs as the network sees them."""
    rnd = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    Ws, bs = unpack(params, shapes)
    Wr = [rnd(W) for W in Ws]
    rows = X0.shape[0]
    acts = [np.asarray(X0, np.float64)]
    for l in range(len(shapes)):
        Z = acts[-1] @ Wr[l].T + bs[l]
        if l < len(shapes) - 1:
            acts.append(rnd(np.maximum(Z, 0.0)))
        else:
            logits = Z
    z = logits[:, :n_buckets]
    zmax = z.max(axis=1, keepdims=True)
    ez = np.exp(z - zmax)
    s = ez.sum(axis=1, keepdims=True)
    p = ez / s
    y = np.asarray(labels, np.int64)
    loss = float(np.mean(np.log(s[:, 0]) + zmax[:, 0] - z[np.arange(rows), y]))
    dZ = np.zeros_like(logits)
    dZ[:, :n_buckets] = p
    dZ[np.arange(rows), y] -= 1.0
    dZ = rnd(dZ / rows)
    gW = [None] * len(shapes)
    gb = [None] * len(shapes)
    for l in range(len(shapes) - 1, -1, -1):
        gW[l] = dZ.T @ acts[l]
        gb[l] = dZ.sum(axis=0)
        if l > 0:
            dH = dZ @ Wr[l]
            dZ = rnd(dH * (acts[l] > 0))
    grad = np.concatenate([g.ravel() for g in gW] + [g.ravel() for g in gb])
    return loss, logits, grad


def frontier(tree, n_leaves, depth=8):
    """Left-to-right frontier at the given depth of the radix tree (oracle
    format: dict of left/right/left_leaf/right_leaf arrays).  Returns node
    references (>= 0 internal, < 0 leaf ~k) and each bucket's first leaf."""
    cur = [0] if n_leaves >= 2 else [~0]
    for _ in range(depth):
        nxt = []
        for r in cur:
            if r >= 0:
                nxt.append(~int(tree["left"][r]) if tree["left_leaf"][r] else int(tree["left"][r]))
                nxt.append(~int(tree["right"][r]) if tree["right_leaf"][r] else int(tree["right"][r]))
            else:
                nxt.append(r)
        cur = nxt
    first = []
    for r in cur:
        first.append(~r if r < 0 else int(tree["first"][r]))
    return np.array(cur, np.int64), np.array(first, np.int64)
