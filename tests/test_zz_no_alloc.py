"""The entry point that allocates no device memory (rsi_intersect_noalloc)
against rsi_intersect, through the C ABI: two calls in a row on the same
library array, the second with fewer segments, every mode and both
precisions, element by element; and a call past the array's size refused
before any GPU work."""
import numpy as np
import pytest
import torch

import paper_2305_01867_amd as rsi
from paper_2305_01867_amd import workloads
from gpu_helpers import dev, host, say

pytestmark = pytest.mark.gpu

KEYS = {"boolean": ("hit",), "first_hit": ("tri_id",), "barycentric": ("tri_id", "uvt"),
        "intercept_count": ("count",)}


def _outs(mode, n, fill):
    d = torch.device("cuda")
    o = {"counters": torch.full((4,), -1, dtype=torch.int64, device=d)}
    if mode == "boolean":
        o["hit"] = torch.full((n,), fill, dtype=torch.uint8, device=d)
    elif mode == "intercept_count":
        o["count"] = torch.full((n,), fill, dtype=torch.int32, device=d)
    else:
        o["tri_id"] = torch.full((n,), fill, dtype=torch.int32, device=d)
    if mode == "barycentric":
        o["uvt"] = torch.full((n, 3), float(fill), dtype=torch.float32, device=d)
    return o


def _same(a, b, key):
    x, y = host(a[key]), host(b[key])
    if key == "uvt":
        return np.array_equal(x.view(np.uint32), y.view(np.uint32))
    if key == "counters":
        # [2] and [3] follow from each segment's answer and hits; [0] (pairs
        # decided in binary64) and [1] (stack overflows) also depend on when a
        # wave's lanes reach their held leaves, and the last chunks of a
        # launch go to whichever waves are free first, so these two may differ
        # from call to call: both calls must have zeroed and counted them
        n_max = max(len(host(v)) for k, v in a.items() if k != "counters")
        return (np.array_equal(x[2:], y[2:]) and np.all((x[:2] >= 0) & (x[:2] <= n_max))
                and np.all((y[:2] >= 0) & (y[:2] <= n_max)))
    return np.array_equal(x, y)


@pytest.mark.parametrize("precision", ["certified", "plain"])
def test_noalloc_equals_intersect_two_calls(precision):
    V, F = workloads.heightfield(96, 3)
    with rsi.rsi_build(dev(V), dev(F), algorithm="restructured") as mesh:
        for n, seed in ((300_000, 41), (70_001, 42)):   # second call smaller, on the same array
            O, E = workloads.rays_crossing_mix(n, seed)
            dO, dE = dev(O), dev(E)
            for mode in KEYS:
                want = rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision=precision)
                got = rsi.rsi_intersect_noalloc(mesh, dO, dE, _outs(mode, n, 7), mode=mode, precision=precision)
                for key in KEYS[mode] + ("counters",):
                    assert _same(got, want, key), (n, mode, precision, key)
                say(f"  {precision} {mode} n={n}: equal, counters {host(got['counters']).tolist()}")


def test_noalloc_with_a_segment_order_and_the_refusal():
    V, F = workloads.heightfield(48, 5)
    with rsi.rsi_build(dev(V), dev(F)) as mesh:
        O, E = workloads.rays_crossing_mix(50_000, 7)
        dO, dE = dev(O), dev(E)
        want = rsi.rsi_intersect(mesh, dO, dE, mode="first_hit", precision="certified", ray_sort="midpoint")
        got = rsi.rsi_intersect_noalloc(mesh, dO, dE, _outs("first_hit", 50_000, 3), mode="first_hit",
                                        precision="certified", ray_sort="midpoint")
        assert _same(got, want, "tri_id")
        # 16,777,201 segments need more than the 64 MiB array (16,777,200 fit): refused before any GPU work
        n = 16_777_201
        big = torch.zeros((n, 3), dtype=torch.float32, device="cuda")
        out = _outs("boolean", n, 0)
        with pytest.raises(rsi.RSIError) as e:
            rsi.rsi_intersect_noalloc(mesh, big, big, out, mode="boolean")
        assert e.value.status == 6 and "scratch" in str(e.value)
        # certified precision needs no more scratch: refused at the same size
        with pytest.raises(rsi.RSIError) as e:
            rsi.rsi_intersect_noalloc(mesh, big, big, out, mode="boolean", precision="certified")
        assert e.value.status == 6
        # a segment order needs about 16 bytes more per segment: 4,000,000 do not fit
        k = 4_000_000
        with pytest.raises(rsi.RSIError) as e:
            rsi.rsi_intersect_noalloc(mesh, big[:k], big[:k], {"hit": out["hit"][:k], "counters": out["counters"]},
                                      mode="boolean", precision="certified", ray_sort="midpoint")
        assert e.value.status == 6
        assert int(host(out["hit"]).max()) == 0
