"""Helpers shared by the GPU tests: device transfer and decoding of the
library's exported arrays (layouts as documented in include/rsi.h)."""
import sys

import numpy as np
import torch

import paper_2305_01867_amd as rsi


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def export(mesh, what):
    return host(rsi.rsi_mesh_export(mesh, what))


def decode_nodes(words):
    """int32 [m, 16] -> (left ref, right ref, left box [m, 6], right box [m, 6])
    with boxes as lo.xyz, hi.xyz."""
    f = words.view(np.float32)
    left = np.stack([f[:, 0], f[:, 2], f[:, 8], f[:, 1], f[:, 3], f[:, 9]], axis=1)
    right = np.stack([f[:, 4], f[:, 6], f[:, 10], f[:, 5], f[:, 7], f[:, 11]], axis=1)
    return words[:, 12].copy(), words[:, 13].copy(), left, right


def intersect(mesh, O, E, mode, precision="certified", **kw):
    r = rsi.rsi_intersect(mesh, dev(O), dev(E), mode=mode, precision=precision, **kw)
    return {k: host(v) for k, v in r.items()}
