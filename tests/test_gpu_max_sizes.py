"""The largest segment count the boundary accepts (2^31 - 1) at paper scale:
segments generated on the device, the benchmark's tree and launch; sampled
segments (including the first and the last 64 indices) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_01867_amd as rsi
from paper_2305_01867_amd import workloads
from gpu_helpers import dev, host, say

pytestmark = pytest.mark.gpu

N_MAX = (1 << 31) - 1


def test_largest_segment_count():
    V, F = workloads.heightfield(128, 21)
    lo, hi = V.min(axis=0), V.max(axis=0)
    c, h = (lo + hi) / 2, (hi - lo) / 2 * 1.1
    g = torch.Generator(device="cuda").manual_seed(5)
    dc, dh = torch.from_numpy(c).cuda(), torch.from_numpy(h).cuda()
    O = torch.rand((N_MAX, 3), generator=g, device="cuda").mul_(2).sub_(1).mul_(dh).add_(dc)  # in place: 26 GB each
    E = torch.rand((N_MAX, 3), generator=g, device="cuda").mul_(2).sub_(1).mul_(dh).add_(dc)
    rng = np.random.default_rng(6)
    idx = np.unique(np.concatenate([np.arange(64), np.arange(N_MAX - 64, N_MAX),
                                    rng.choice(N_MAX, 3000, replace=False)]))
    ti = torch.from_numpy(idx).cuda()
    Os, Es = host(O[ti]), host(E[ti])
    hit, ids, _, _ = oracle.intersect(V, F, Os, Es)
    with rsi.rsi_build(dev(V), dev(F), algorithm="restructured") as mesh:
        for mode in ("boolean", "first_hit"):
            say(f"[max] {N_MAX} segments, {mode}")
            r = rsi.rsi_intersect(mesh, O, E, mode=mode, precision="certified")
            key = "hit" if mode == "boolean" else "tri_id"
            got = host(r[key][ti])
            assert np.array_equal(got, hit if mode == "boolean" else ids), mode
            say(f"  counters {host(r['counters']).tolist()}")
            del r
            torch.cuda.empty_cache()
        # one segment more than the limit is refused before any GPU work
        import ctypes
        o = rsi._Outputs()
        st = rsi.lib().rsi_intersect(mesh.handle, ctypes.c_void_p(O.data_ptr()), ctypes.c_void_p(E.data_ptr()),
                                     N_MAX + 1, 0, None, ctypes.byref(o), None)
        assert st == 6 and b"n_rays" in rsi.lib().rsi_last_error()  # RSI_E_CAPACITY
