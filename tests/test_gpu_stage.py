"""Boolean results written a window at a time: every segment count around
the window size and the wave ranges, output buffers at 4-byte aligned and
unaligned offsets (unaligned ones are written byte by byte), and a mix of
fast and very slow segments (a window written before its slowest segment
finishes), all equal to the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_01867_amd as rsi
from paper_2305_01867_amd import workloads
from gpu_helpers import dev, host, say

pytestmark = pytest.mark.gpu


def _slow_and_fast(n, seed):
    """Segments along the plane of a flat grid (many candidates, slow) among
    short vertical ones (one candidate, fast)."""
    rng = np.random.default_rng(seed)
    O = np.empty((n, 3), np.float32)
    E = np.empty((n, 3), np.float32)
    slow = rng.random(n) < 0.02
    xy = rng.uniform(0.05, 0.95, (n, 2))
    O[:, :2] = xy
    E[:, :2] = xy
    O[:, 2], E[:, 2] = 0.5, -0.5
    # slow ones: long, nearly horizontal, just above the surface
    E[slow, 0] = 1.0 - xy[slow, 0]
    E[slow, 1] = 1.0 - xy[slow, 1]
    O[slow, 2] = 0.30
    E[slow, 2] = 0.29
    return O, E


@pytest.mark.parametrize("precision", ["certified", "plain"])
def test_staged_boolean_writes(precision):
    V, F = workloads.heightfield(80, 9)
    O, E = _slow_and_fast(200_000, 3)
    hit, _, _, _ = oracle.intersect(V, F, O, E)
    with rsi.rsi_build(dev(V), dev(F), algorithm="restructured") as mesh:
        for n in (1, 255, 256, 257, 4095, 70_001, 200_000):
            for offset in (0, 1, 4, 7):
                buf = torch.full((n + 16,), 9, dtype=torch.uint8, device="cuda")
                out = {"hit": buf[offset:offset + n]}
                for width in (0, 2):
                    buf.fill_(9)
                    rsi.rsi_intersect(mesh, dev(O[:n]), dev(E[:n]), mode="boolean", precision=precision,
                                      out=out, node_width=width)
                    b = host(buf)
                    assert np.array_equal(b[offset:offset + n], hit[:n]), (n, offset, width)
                    assert np.all(b[:offset] == 9) and np.all(b[offset + n:] == 9), (n, offset, width)
        say(f"  {precision}: staged and byte-wise boolean writes equal the oracle")
