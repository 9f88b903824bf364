#!/usr/bin/env python3
"""Throughput of the segment / triangle-mesh intersection path on one GPU.

Workload: the paper-scale case -- a 128 x 128 heightfield (32,258 triangles,
seeded sinusoids + noise) and 1e7 segments with end points uniform in the mesh
box inflated by 10% (synthetic stand-in for the paper's 29,260-triangle /
1e7-ray data, which is not available).  One step = the whole path: build the
BVH (extent, Morton keys, LDS radix sort, radix tree, bottom-up boxes, and by
default two passes of treelet restructuring, which changes node visits but
never results, and the collapse into a 4-wide tree) and intersect every
segment (4-wide traversal with the tree's top in LDS, leaf tests, binary64
re-decisions), with the inputs already resident in GPU memory.  The metric is
Mrays/s.  --build radix_tree times the paper's own LBVH instead; the
variants record that step either way.

Printed: one JSON line (rank 0).  Besides the contract fields it carries
  roofline      the traversal launch, which is bound by vector-ALU issue:
                algorithmic fp32 FLOP (per node fetched and per triangle
                tested, counted by an instrumented run of the same traversal)
                over its average duration (HIP events on the launch stream),
                against the 157.3 TFLOP/s fp32 vector peak; beside it the
                VALU issue rate from the committed rocprofv3 counters, and the
                memory view: measured HBM traffic against the achievable
                bandwidth of the library's streaming copy kernel (measured in
                the same run), and the bytes the method touches
  cpu_baseline  the binary64 brute-force oracle timed on the host cores on a
                bounded sample of the same segments
  variants      Mrays/s of intersect alone per mode and precision
  learned_vs_plain  the learned subtree proposal (trained on 2e6 other
                segments the method labels) against the plain order:
                intersect Mrays/s, node visits, proposal miss rate, MLP cost
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X vendor HBM3E peak
FP32_PEAK_TFLOPS = 157.3       # MI355X fp32 vector peak (FMA = 2 FLOP)
VALU_ISSUE_PEAK = 256 * 2.4e9  # wave64 VALU instructions per second: one per CU per cycle
                               # (4 SIMD x 16 lanes, a wave64 instruction every 4 cycles each)
# fp32 operations of the method per step of the traversal, counted from the
# kernel source (FMA = 2, add / mul / min / max / compare / abs = 1):
#   segment set-up (direction, scale, widened reciprocal, slab offsets)  41
#   4-wide node: 4 children x (6 FMA + 3 max + 3 min + 1 compare)        76
#   binary node: 2 children x (6 FMA + 12 min/max + 1 compare)           50
#   leaf test, binary32 Moller-Trumbore (differences, two cross products,
#   four dot products)                                                   41
#     + plain decision (sign flips, five comparisons)                    12
#     + certified: magnitude sums of the bound (58) and classification (44)
FLOP_SETUP, FLOP_NODE4, FLOP_NODE2 = 41, 76, 50
FLOP_TEST = {"plain": 41 + 12, "certified": 41 + 58 + 44}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--rays", type=int, default=10_000_000)
    ap.add_argument("--mode", default="boolean", choices=["boolean", "first_hit", "barycentric", "intercept_count"])
    ap.add_argument("--precision", default="certified", choices=["plain", "certified"])
    ap.add_argument("--build", default="restructured", choices=["radix_tree", "restructured", "agglomerative"],
                    help="BVH build of the timed step")
    ap.add_argument("--cpu-seconds", type=float, default=24.0, help="target CPU time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="skip the learned form (5.26e5 triangles) leg")
    ap.add_argument("--no-configs", action="store_true", help="skip the tiny-case and precision-form leg")
    ap.add_argument("--c5-train-rays", type=int, default=10_000_000)
    ap.add_argument("--no-host", action="store_true", help="skip the host-resident (PCIe-inclusive) runs")
    ap.add_argument("--train-rays", type=int, default=2_000_000)
    ap.add_argument("--train-epochs", type=int, default=3)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB buffer 3 times (reference for the HBM byte counters)")
    return ap.parse_args()


def calibrate_copy():
    """The library's streaming copy of known size: 1 GiB read + 1 GiB written
    per launch.  Its FETCH_SIZE / WRITE_SIZE readings scale the counters of
    the other kernels to bytes."""
    import torch

    import paper_2305_01867_amd as rsi

    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        rsi.rsi_stream_copy(b, a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read_per_launch": a.numel() * 4, "copy_bytes_written_per_launch": b.numel() * 4,
                      "launches": 3}), flush=True)


def achievable_hbm(reps: int = 5):
    """Achievable HBM bandwidth: the library's streaming copy of 4 GiB into
    another 4 GiB buffer (8 GiB moved per launch), timed with HIP events on the
    launch stream.  Returns GB/s (and torch's own device copy beside it)."""
    import torch

    import paper_2305_01867_amd as rsi

    n = 1 << 30  # float32 elements: 4 GiB
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    stream = torch.cuda.current_stream()
    out = {}
    for name, fn in (("stream_copy", lambda: rsi.rsi_stream_copy(b, a)), ("torch_copy", lambda: b.copy_(a))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = round(2 * 4 * n / (ms * 1e-3) / 1e9, 1)
    ok = bool(torch.equal(a, b))
    del a, b
    torch.cuda.empty_cache()
    out["copy_verified"] = ok
    out["bytes_per_launch"] = 2 * 4 * n
    return out


def measured_traffic(mode, precision, build):
    """(HBM bytes per traversal launch, the counter view beside them) from the
    committed rocprofv3 counter summary, or (None, None) when the traversal
    source or the tree build differs from the one it was taken with (counters
    of another kernel say nothing about this one)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None, None
    rec = json.load(open(path)).get(f"{mode}_{precision}")
    if not rec or rec.get("build") != build:
        return None, None
    src = open(os.path.join(ROOT, "paper_2305_01867_amd", "csrc", "traverse.hip"), "rb").read()
    if hashlib.sha256(src).hexdigest() != rec["traverse_hip_sha256"]:
        return None, None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"], rec.get("counters")


def full_check(mode, out, n, workload="paper_scale"):
    """Compare the whole output of the timed path with the binary64 oracle's
    stored per-chunk digests of the same workload (tests/golden, written by
    the oracle alone).  None when no complete fixture covers this workload."""
    import importlib.util

    import numpy as np

    path = os.path.join(ROOT, "tests", "golden", "make_full_fixtures.py")
    if not os.path.exists(os.path.join(ROOT, "tests", "golden", f"full_{workload}.txt")):
        return None
    spec = importlib.util.spec_from_file_location("full_fixtures", path)
    fx = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(fx)
    head, rows = fx.read(workload)
    if int(head["n_segments"]) != n or len(rows) * int(head["chunk"]) < n:
        return None
    cols = {"boolean": [("hit", 0)], "first_hit": [("tri_id", 1)], "barycentric": [("tri_id", 1), ("uvt", 2)],
            "intercept_count": [("count", 3)]}[mode]
    res = {"segments": n, "chunks": len(rows), "source": f"tests/golden/full_{workload}.txt"}
    for key, col in cols:
        a = out[key].cpu().numpy()
        equal = 0
        for c, (s0, m, _, *dig) in rows.items():
            x = a[s0:s0 + m]
            d = fx.digest(x.astype(np.uint8)) if key == "hit" else (
                fx.digest(fx.uvt_f32(x)) if key == "uvt" else fx.digest(x.astype("<i4")))
            equal += d == dig[col]
        res[f"{key}_chunks_equal"] = equal
    return res


def host_cpu():
    """Model name and logical CPU count of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def other_configs(rsi, workloads, args, stream):
    """The tiny case and the precision form: intersect time of the binary32
    and the certified path (boolean and first hit, restructured tree, 4-wide
    first pass), segments re-decided in binary64, and mismatches against the
    oracle -- the tiny case in full, the precision form against the oracle's
    stored per-chunk digests of all 1e7 segments where they exist, else on a
    stratified sample."""
    import numpy as np
    import torch

    import oracle
    dev = torch.device("cuda:0")
    res = {}
    for name in ("tiny", "precision"):
        if name == "tiny":
            V, F, O, E = workloads.tiny_config()
            label = "64x64 heightfield (7,938 triangles), 1e4 crossing-mix segments"
        else:
            V, F, O, E, kind = workloads.precision_config()
            label = ("folded 256x256 heightfield (130,050 triangles), 1e7 segments: 75% in the box, 20% aimed "
                     "within 1e-7 of edges and vertices, 5% within 1e-6 rad of parallel")
        dO, dE = torch.from_numpy(O).to(dev), torch.from_numpy(E).to(dev)
        n = O.shape[0]
        r = {"workload": label, "n_triangles": int(F.shape[0]), "n_segments": int(n)}
        with rsi.rsi_build(torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev),
                           algorithm=args.build) as mesh:
            for mode, key in (("boolean", "hit"), ("first_hit", "tri_id")):
                got = {}
                for prec in ("plain", "certified"):
                    o = rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision=prec)
                    ms = _timed(lambda: rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision=prec, out=o), stream)
                    got[prec] = o[key].cpu().numpy()
                    r[f"{mode}/{prec}"] = {"ms": round(ms, 4), "mrays_s": round(n / (ms * 1e-3) / 1e6, 1),
                                           "redecided_fp64": int(o["counters"][0].item())}
                    if name == "precision" and prec == "certified":
                        full = full_check(mode, o, n, "precision")
                        if full:
                            r[f"{mode}/certified"]["every_segment_vs_oracle"] = full
                    del o
                if name == "tiny":
                    hit, ids, _, _ = oracle.intersect(V, F, O, E)
                    want = hit if mode == "boolean" else ids
                    r[f"{mode}/mismatches_vs_oracle"] = {p: int(np.sum(got[p] != want)) for p in got}
                    r[f"{mode}/oracle_segments"] = int(n)
                else:
                    # binary32 against the certified path (equal to the oracle where
                    # the digests say so), and a stratified oracle sample
                    r[f"{mode}/plain_differs_from_certified"] = int(np.sum(got["plain"] != got["certified"]))
                    if not args.no_cpu_baseline:
                        rng = np.random.default_rng(17)
                        idx = np.concatenate([rng.choice(np.nonzero(kind == k)[0], c, replace=False)
                                              for k, c in ((0, 300), (1, 800), (2, 400))])
                        hit, ids, _, _ = oracle.intersect(V, F, O[idx], E[idx])
                        want = hit if mode == "boolean" else ids
                        r[f"{mode}/sample_mismatches_vs_oracle"] = {
                            p: int(np.sum(got[p][idx] != want)) for p in got}
                        r[f"{mode}/sample_segments"] = int(idx.size)
        res[name] = r
        del dO, dE
        torch.cuda.empty_cache()
    return res


def _timed(fn, stream, reps=3):
    import torch
    fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn()
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def learned_leg(rsi, dV, dF, Ot, Et, dO, dE, o, mode, precision, build, epochs, stream):
    """Train the proposal on (Ot, Et), then time the intersection of (dO, dE)
    in the plain and the proposal order on the same mesh (4-wide trees and
    binary nodes), the inference alone, and count node fetches of both."""
    import torch
    n = dO.shape[0]
    dOt, dEt = torch.from_numpy(Ot).to(dO.device), torch.from_numpy(Et).to(dO.device)
    with rsi.rsi_build(dV, dF, algorithm=build) as mesh:
        torch.cuda.synchronize()
        t_tr = time.perf_counter()
        loss, n_lab = rsi.rsi_proposal_train(mesh, dOt, dEt, epochs=epochs, batch=4096, lr=2e-3, seed=1)
        t_tr = time.perf_counter() - t_tr
        del dOt, dEt
        run = lambda **kw: rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision=precision, out=o, **kw)
        ms = {}
        for width in (4, 2):
            ms["plain", width] = _timed(lambda: run(node_width=width), stream)
            ms["learned", width] = _timed(lambda: run(proposal=True, node_width=width), stream)
        late = int(o["counters"][2].item())
        n_hit = int(o["hit"].sum().item()) if mode == "boolean" else int((o["tri_id"] >= 0).sum().item())
        run(proposal=True)  # leave the default (4-wide) proposal order's results in o
        ms_mlp = _timed(lambda: rsi.rsi_proposal_predict(mesh, dO, dE), stream)
        visits = {}
        for width in (4, 2):
            for order, kw in (("plain", {}), ("learned", {"proposal": True})):
                v, _ = rsi.rsi_traversal_stats(mesh, dO, dE, mode=mode, precision=precision, node_width=width, **kw)
                visits[order, width] = round(float(v.double().mean().item()), 2)
                del v
    saved = ms["plain", 4] - (ms["learned", 4] - ms_mlp)
    return {
        "train_segments": int(Ot.shape[0]), "labelled": n_lab, "epochs": epochs,
        "train_s": round(t_tr, 2), "epoch_loss": [round(x, 4) for x in loss.tolist()],
        # GEMM work per labelled segment and epoch: forward 2 x 253,952, weight
        # gradients the same, input gradients 2 x 3 x 65,536 FLOP; over train_s,
        # which includes labelling the segments
        "train_tflops": round(epochs * n_lab * (4 * 253952 + 6 * 65536) / t_tr / 1e12, 2),
        "proposal_miss_rate": round(late / max(n_hit, 1), 4),
        "intersect_mrays_s_plain_order": round(n / (ms["plain", 4] * 1e-3) / 1e6, 1),
        "intersect_mrays_s_learned": round(n / (ms["learned", 4] * 1e-3) / 1e6, 1),
        "intersect_mrays_s_plain_order_binary_nodes": round(n / (ms["plain", 2] * 1e-3) / 1e6, 1),
        "intersect_mrays_s_learned_binary_nodes": round(n / (ms["learned", 2] * 1e-3) / 1e6, 1),
        "intersect_ms": {f"{k[0]}/{k[1]}-wide": round(v, 3) for k, v in ms.items()},
        "mlp_inference_ms": round(ms_mlp, 3),
        "mlp_tflops": round(n * 2 * 253952 / (ms_mlp * 1e-3) / 1e12, 1),
        "traversal_ms_saved_by_the_order": round(saved, 3),
        "break_even": "the learned order pays when the traversal time it saves exceeds the inference time",
        "mean_node_fetches": {f"{k[0]}/{k[1]}-wide": v for k, v in visits.items()},
        "mode": mode, "precision": precision, "_result": True,
    }


def learned_form(rsi, workloads, args, stream):
    """The learned-proposal form: a 512 x 512 heightfield with two folded
    sheets (about 5.26e5 triangles), the proposal trained on segments of the
    same distribution, evaluated on one chunk of 1e7 segments (boolean mode,
    early exit), against the plain order; a sample checked against the oracle."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    V, F = workloads.learned_mesh()
    print(f"[bench] learned form: {F.shape[0]} triangles, training on {args.c5_train_rays} segments",
          file=sys.stderr, flush=True)
    Ot, Et = workloads.learned_rays(args.c5_train_rays, 5001)
    O, E = workloads.learned_rays(10_000_000, 5100)
    dV, dF = torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev)
    dO, dE = torch.from_numpy(O).to(dev), torch.from_numpy(E).to(dev)
    o = {"hit": torch.empty(O.shape[0], dtype=torch.uint8, device=dev),
         "counters": torch.zeros(4, dtype=torch.int64, device=dev)}
    res = learned_leg(rsi, dV, dF, Ot, Et, dO, dE, o, "boolean", args.precision, args.build, 2, stream)
    res.pop("_result", None)
    got = o["hit"].cpu().numpy()
    res["hit_fraction"] = round(float(got.mean()), 4)
    res["workload"] = (f"learned form: 512x512 heightfield + two folded sheets ({F.shape[0]} triangles), "
                       f"evaluation chunk of {O.shape[0]} segments (seed 5100)")
    if not args.no_cpu_baseline:
        import oracle
        idx = np.random.default_rng(7).choice(O.shape[0], 2000, replace=False)
        want, _, _, _ = oracle.intersect(V, F, O[idx], E[idx])
        res["oracle_sample"] = {"segments": int(idx.size), "mismatches": int(np.sum(got[idx] != want))}
    del dV, dF, dO, dE, o
    torch.cuda.empty_cache()
    return res


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the path shards by segments with the BVH replicated; runs on more than one GPU are not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2305_01867_amd as rsi
    from paper_2305_01867_amd import workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    print(f"[bench] generating workload: 128x128 heightfield, {args.rays} segments", file=sys.stderr, flush=True)
    V, F, O, E = workloads.paper_scale_config(args.rays)
    dV = torch.from_numpy(V).to(dev)
    dF = torch.from_numpy(F).to(dev)
    dO = torch.from_numpy(O).to(dev)
    dE = torch.from_numpy(E).to(dev)
    n = O.shape[0]
    stream = torch.cuda.current_stream()

    out_keys = {"boolean": ("hit",), "first_hit": ("tri_id",), "barycentric": ("tri_id", "uvt"),
                "intercept_count": ("count",)}
    outs = {}
    for m, ks in out_keys.items():
        o = {"counters": torch.zeros(4, dtype=torch.int64, device=dev)}
        if "hit" in ks:
            o["hit"] = torch.empty(n, dtype=torch.uint8, device=dev)
        if "tri_id" in ks:
            o["tri_id"] = torch.empty(n, dtype=torch.int32, device=dev)
        if "uvt" in ks:
            o["uvt"] = torch.empty((n, 3), dtype=torch.float32, device=dev)
        if "count" in ks:
            o["count"] = torch.empty(n, dtype=torch.int32, device=dev)
        outs[m] = o

    def build(gV=None, gF=None, algorithm=args.build):
        return rsi.rsi_build(dV if gV is None else gV, dF if gF is None else gF, algorithm=algorithm)

    def step(mode=args.mode, precision=args.precision, ev=None, algorithm=args.build):
        mesh = build(algorithm=algorithm)
        if ev is not None:
            ev[0].record(stream)
        rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision=precision, out=outs[mode])
        if ev is not None:
            ev[1].record(stream)
        mesh.close()

    print("[bench] warmup", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # ---------------- timed region: exactly K steps
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(ev=evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    intersect_ms = sorted(a.elapsed_time(b) for a, b in evs)
    intersect_avg = sum(intersect_ms) / len(intersect_ms)
    value = n / (ms_per_step * 1e-3) / 1e6
    counters = outs[args.mode]["counters"].cpu().tolist()
    hit_frac = None
    if args.mode == "boolean":
        hit_frac = float(outs["boolean"]["hit"].float().mean().item())
    print(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step, intersect {intersect_avg:.3f} ms "
          f"-> {value:.1f} Mrays/s", file=sys.stderr, flush=True)
    # the whole timed output against the oracle's stored digests (every segment)
    full = full_check(args.mode, outs[args.mode], n) if n == 10_000_000 else None
    if full:
        print(f"[bench] every segment vs the oracle's digests: {full}", file=sys.stderr, flush=True)
    # results of each path on the leading segments, for the oracle comparison below
    key = {"boolean": "hit", "intercept_count": "count"}.get(args.mode, "tri_id")
    keep = min(n, 1 << 22)
    results = {f"{args.precision} (timed path)": outs[args.mode][key][:keep].cpu().numpy().copy()}

    # ---------------- algorithmic bytes of the traversal (instrumented, untimed)
    with build() as mesh:
        node_width = rsi.rsi_mesh_info_get(mesh)["node_width"]
        visits, tests = rsi.rsi_traversal_stats(mesh, dO, dE, mode=args.mode, precision=args.precision)
        torch.cuda.synchronize()
        mean_visits = float(visits.double().mean().item())
        mean_tests = float(tests.double().mean().item())
        p50_visits = float(visits.double().median().item())
        p99_visits = float(torch.quantile(visits[: min(n, 1 << 24)].double(), 0.99).item())
    out_bytes = {"boolean": 1, "first_hit": 4, "barycentric": 16, "intercept_count": 4}[args.mode]
    node_bytes = 112 if node_width == 4 else 64  # loaded per node fetch (7 or 4 16-byte loads)
    flop_node = FLOP_NODE4 if node_width == 4 else FLOP_NODE2
    flop_per_ray = FLOP_SETUP + flop_node * mean_visits + FLOP_TEST[args.precision] * mean_tests
    achieved_tflops = n * flop_per_ray / (intersect_avg * 1e-3) / 1e12
    bytes_per_ray = 24 + out_bytes + node_bytes * mean_visits + 48 * mean_tests
    traffic, counter_view = measured_traffic(args.mode, args.precision, args.build)
    print("[bench] achievable HBM: streaming copy of 4 GiB", file=sys.stderr, flush=True)
    hbm = achievable_hbm()
    hbm_gbs = hbm["stream_copy"]
    roofline = {
        "bound": "alu", "achieved": round(achieved_tflops, 3), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
        "frac": round(achieved_tflops / FP32_PEAK_TFLOPS, 4),
        "traffic": traffic,
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by the streaming copy's "
                        "readings)",
        "kernel": "k_traverse (+ k_reset, k_finish in the same event pair)", "node_width": node_width,
        "flop_per_segment": round(flop_per_ray, 1),
        "flop_counting": f"{FLOP_SETUP} per segment + {flop_node} per node fetch + {FLOP_TEST[args.precision]} per "
                         "leaf test (FMA = 2)",
        "mean_node_visits": round(mean_visits, 2), "p50_node_visits": p50_visits, "p99_node_visits": p99_visits,
        "mean_leaf_tests": round(mean_tests, 2), "avg_launch_ms": round(intersect_avg, 4),
        "reading": "the traversal is bound by VALU issue, not by HBM: divergent lanes (about half of a wave "
                   "active per instruction) and the control, stack and address work around the method's "
                   "arithmetic fill the issue slots; the tree lives in LDS (its top) and L2, so HBM carries "
                   "little more than the segment stream",
    }
    if counter_view:
        # issue-slot use of the same kernel, from the committed profile (its own launch time)
        insts = counter_view.get("sq_insts_valu_per_launch")
        us = counter_view.get("avg_launch_us_trace")
        if insts and us:
            roofline["valu_issue"] = {
                "insts_per_launch": insts, "rate_per_s": round(insts / (us * 1e-6), 1),
                "peak_per_s": VALU_ISSUE_PEAK, "frac": round(insts / (us * 1e-6) / VALU_ISSUE_PEAK, 4),
                "valu_busy_pct": counter_view.get("VALUBusy_pct"),
                "active_lanes_pct": counter_view.get("VALUUtilization_pct"),
                "source": "profiles/ counters of this kernel (SQ_INSTS_VALU over its traced launch time)"}
        roofline["counters_from_profile"] = counter_view
    roofline["hbm"] = {
        "achievable_gbs": hbm_gbs, "achievable_from": "rsi_stream_copy, 4 GiB -> 4 GiB, HIP events",
        "torch_copy_gbs": hbm["torch_copy"], "vendor_peak_gbs": HBM_PEAK_GBS,
        "achievable_over_vendor": round(hbm_gbs / HBM_PEAK_GBS, 4),
        "measured_gbs": round(traffic / (intersect_avg * 1e-3) / 1e9, 1) if traffic else None,
        "measured_frac": round(traffic / (intersect_avg * 1e-3) / 1e9 / hbm_gbs, 5) if traffic else None,
        "stream_bytes_per_segment": 24 + out_bytes,
        "stream_frac": round(n * (24 + out_bytes) / (intersect_avg * 1e-3) / 1e9 / hbm_gbs, 5),
        "touched_bytes_per_segment": round(bytes_per_ray, 1),
        "touched_gbs": round(n * bytes_per_ray / (intersect_avg * 1e-3) / 1e9, 1),
        "touched_note": f"{node_bytes} B per node fetch + 48 B per leaf test + the stream; served from LDS and L2 "
                        "(it exceeds what HBM could deliver), so it is no HBM fraction",
    }

    # ---------------- per-variant intersect throughput (untimed region)
    variants = {}
    if not args.no_variants:
        with build() as mesh:
            for mode in ("boolean", "first_hit", "barycentric", "intercept_count"):
                for prec in ("plain", "certified"):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision=prec, out=outs[mode])
                    reps = 3
                    a.record(stream)
                    for _ in range(reps):
                        rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision=prec, out=outs[mode])
                    b.record(stream)
                    torch.cuda.synchronize()
                    ms = a.elapsed_time(b) / reps
                    c = outs[mode]["counters"].cpu().tolist()
                    variants[f"{mode}/{prec}"] = {"mrays_s": round(n / (ms * 1e-3) / 1e6, 1),
                                                  "ms": round(ms, 3), "redecided_fp64": c[0],
                                                  "stack_overflow": c[1]}
                    if mode == args.mode and prec != args.precision:
                        results[prec] = outs[mode][key][:keep].cpu().numpy().copy()
            for mode in ("boolean", "first_hit"):  # the same first pass over binary nodes
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                run = lambda: rsi.rsi_intersect(mesh, dO, dE, mode=mode, precision=args.precision, out=outs[mode],
                                                node_width=2)
                run()
                a.record(stream)
                for _ in range(3):
                    run()
                b.record(stream)
                torch.cuda.synchronize()
                ms = a.elapsed_time(b) / 3
                variants[f"{mode}/{args.precision}/binary_nodes"] = {"mrays_s": round(n / (ms * 1e-3) / 1e6, 1),
                                                                     "ms": round(ms, 3)}
                if mode == args.mode:
                    results[f"{args.precision}, binary nodes"] = outs[mode][key][:keep].cpu().numpy().copy()
            for order in ("midpoint", "origin_octant"):  # segment processing orders (same results)
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                run = lambda: rsi.rsi_intersect(mesh, dO, dE, mode=args.mode, precision=args.precision,
                                                out=outs[args.mode], ray_sort=order)
                run()
                a.record(stream)
                for _ in range(3):
                    run()
                b.record(stream)
                torch.cuda.synchronize()
                ms = a.elapsed_time(b) / 3
                variants[f"{args.mode}/{args.precision}/order={order}"] = {
                    "mrays_s": round(n / (ms * 1e-3) / 1e6, 1), "ms": round(ms, 3)}
                results[f"{args.precision}, order={order}"] = outs[args.mode][key][:keep].cpu().numpy().copy()
            for alg in ("radix_tree", "restructured"):
                b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                build(algorithm=alg).close()
                b0.record(stream)
                for _ in range(5):
                    build(algorithm=alg).close()
                b1.record(stream)
                torch.cuda.synchronize()
                variants[f"build_ms_{alg}"] = round(b0.elapsed_time(b1) / 5, 4)
            build(algorithm="agglomerative").close()
            torch.cuda.synchronize()
            t_a = time.perf_counter()
            for _ in range(5):
                build(algorithm="agglomerative").close()  # waits once per build for the root
            torch.cuda.synchronize()
            variants["build_ms_agglomerative"] = round((time.perf_counter() - t_a) * 1e3 / 5, 4)
        # the whole step with each tree (same segments, same results)
        for alg in ("radix_tree", "restructured"):
            step(algorithm=alg)
            torch.cuda.synchronize()
            s0 = time.perf_counter()
            for _ in range(3):
                step(algorithm=alg)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - s0) * 1e3 / 3
            with build(algorithm=alg) as mesh:
                v_alg, _ = rsi.rsi_traversal_stats(mesh, dO, dE, mode=args.mode, precision=args.precision)
                mv = float(v_alg.double().mean().item())
            variants[f"step/{args.mode}/{args.precision}/build={alg}"] = {
                "mrays_s": round(n / (ms * 1e-3) / 1e6, 1), "ms": round(ms, 3), "mean_node_visits": round(mv, 2)}
            results[f"{args.precision}, build={alg}"] = outs[args.mode][key][:keep].cpu().numpy().copy()

    # ---------------- learned proposal vs plain order (BVH resident, untimed region)
    learned = None
    if not args.no_learned and args.mode != "intercept_count":
        lo, hi = V.min(axis=0), V.max(axis=0)
        Ot, Et = workloads.rays_in_box(args.train_rays, 23, lo, hi)  # training segments, own seed
        learned = learned_leg(rsi, dV, dF, Ot, Et, dO, dE, outs[args.mode], args.mode, args.precision, args.build,
                              args.train_epochs, stream)
        del Ot, Et
        if learned.pop("_result", None) is not None:
            results[f"{args.precision} + learned proposal"] = outs[args.mode][key][:keep].cpu().numpy().copy()
        learned["workload"] = "the headline mesh and segments; proposal trained on other segments of the same box"
        print(f"[bench] learned: {learned}", file=sys.stderr, flush=True)
    learned_c5 = None
    if not args.no_learned and not args.no_c5 and args.mode == "boolean":
        learned_c5 = learned_form(rsi, workloads, args, stream)
        print(f"[bench] learned form: {learned_c5}", file=sys.stderr, flush=True)

    # ---------------- the tiny case and the precision form (untimed region)
    configs = None
    if not args.no_configs:
        configs = other_configs(rsi, workloads, args, stream)
        print(f"[bench] configs: {configs}", file=sys.stderr, flush=True)

    # ---------------- host-resident runs: host arrays in, host results out (PCIe included)
    host = None
    if not args.no_host:
        pin = lambda a: torch.from_numpy(a).pin_memory()
        hV, hF, hO, hE = pin(V), pin(F), pin(O), pin(E)
        host = {"workload": "same mesh and segments, from pinned host memory to host results",
                "paper_ms_same_shape_other_gpu": {"boolean": 355.094, "barycentric": 456.346,
                                                  "intercept_count": 383.117}}
        for hmode in ("boolean", "barycentric", "intercept_count"):
            def job():
                gV, gF = hV.to(dev, non_blocking=True), hF.to(dev, non_blocking=True)
                gO, gE = hO.to(dev, non_blocking=True), hE.to(dev, non_blocking=True)
                with build(gV, gF) as mesh:
                    r = rsi.rsi_intersect(mesh, gO, gE, mode=hmode, precision=args.precision)
                    if hmode == "barycentric":
                        res = tuple(x.cpu() for x in rsi.rsi_compact_hits(gO, gE, r))
                    else:
                        res = r["hit" if hmode == "boolean" else "count"].cpu()
                torch.cuda.synchronize()
                return res
            job()
            t_h = []
            for _ in range(3):
                t0h = time.perf_counter()
                res = job()
                t_h.append((time.perf_counter() - t0h) * 1e3)
            host[hmode + "_ms"] = round(min(t_h), 2)
            if hmode == "barycentric":
                host["barycentric_hits"] = int(res[0].shape[0])
        print(f"[bench] host-resident: {host}", file=sys.stderr, flush=True)
        del hV, hF, hO, hE

    # ---------------- batched form: 64 meshes, build + intersect replayed from a graph
    batched = None
    if not args.no_batched:
        del outs
        torch.cuda.empty_cache()
        Vb, Fb, Ob, Eb, vo, to, ro = workloads.batched_config()
        dVb, dFb = torch.from_numpy(Vb).to(dev), torch.from_numpy(Fb).to(dev)
        dOb, dEb = torch.from_numpy(Ob).to(dev), torch.from_numpy(Eb).to(dev)
        nb = Ob.shape[0]
        bkey = "hit" if args.mode == "boolean" else ("count" if args.mode == "intercept_count" else "tri_id")
        bout = {bkey: torch.empty(nb, dtype=torch.uint8 if bkey == "hit" else torch.int32, device=dev),
                "counters": torch.zeros(4, dtype=torch.int64, device=dev)}
        if args.mode == "barycentric":
            bout["uvt"] = torch.empty((nb, 3), dtype=torch.float32, device=dev)
        with rsi.rsi_batch_create(vo, to, ro) as b:
            # launch choices tuned once for this size class (untimed), then captured
            rsi.rsi_batch_build(b, dVb, dFb)
            from paper_2305_01867_amd import autotune
            space = {"block": (256, 512, 1024), "stack_depth": (12, 16, 20, 24), "waves_per_cu": (0, 8, 16),
                     "ray_sort": (0, 1, 2), "node_width": (0, 2)}
            run = lambda **c: rsi.rsi_batch_intersect(b, dOb, dEb, mode=args.mode, precision=args.precision,
                                                      out=bout, **c)
            key = autotune.size_class(args.mode, args.precision, 64, Fb.shape[0], nb)
            choice, timings = autotune.tune(run, key, None, space=space, reps=2)
            choice = {k: v for k, v in choice.items() if k != "ms"}
            ms_default = min(t["ms"] for t in timings if t["block"] == 1024 and t["stack_depth"] == 20
                             and t["waves_per_cu"] == 0 and t["ray_sort"] == 0 and t["node_width"] == 0)
            ms_binary = min(t["ms"] for t in timings if t["node_width"] == 2)

            def bstep():
                rsi.rsi_batch_build(b, dVb, dFb)
                rsi.rsi_batch_intersect(b, dOb, dEb, mode=args.mode, precision=args.precision, out=bout, **choice)
            bstep()
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                with torch.cuda.graph(g, stream=side, capture_error_mode="thread_local"):
                    bstep()
            torch.cuda.current_stream().wait_stream(side)
            g.replay()
            torch.cuda.synchronize()
            reps = 5
            a, bb = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(reps):
                g.replay()
            bb.record(stream)
            torch.cuda.synchronize()
            ms_b = a.elapsed_time(bb) / reps
            batched = {"workload": f"64 heightfields, {Fb.shape[0]} triangles, {nb} segments",
                       "graph_replay_ms": round(ms_b, 3), "mrays_s": round(nb / (ms_b * 1e-3) / 1e6, 1),
                       "redecided_fp64": int(bout["counters"][0].item()), "mode": args.mode,
                       "precision": args.precision, "tuned_choice": choice,
                       "tuned_over": f"{len(timings)} launch choices, intersect only",
                       "intersect_ms_tuned": round(min(t["ms"] for t in timings), 3),
                       "intersect_ms_library_default": round(ms_default, 3),
                       "intersect_ms_best_binary_nodes": round(ms_binary, 3)}
        print(f"[bench] batched: {batched}", file=sys.stderr, flush=True)
        del dVb, dFb, dOb, dEb, bout

    # ---------------- CPU baseline: the oracle on a bounded sample
    cpu = None
    if not args.no_cpu_baseline:
        import oracle

        probe = 512
        s0 = time.perf_counter()
        oracle.intersect(V, F, O[:probe], E[:probe])
        dt = time.perf_counter() - s0
        m = int(min(n, keep, max(probe, probe * args.cpu_seconds / max(dt, 1e-6))))
        s0 = time.perf_counter()
        o_hit, o_id, _, _ = oracle.intersect(V, F, O[:m], E[:m])
        dt = time.perf_counter() - s0
        want = o_hit if args.mode == "boolean" else o_id
        if args.mode == "intercept_count":
            want = oracle.intercept_count(V, F, O[:m], E[:m])
        mismatches = {name: int(np.sum(r[:m] != want)) for name, r in results.items()}
        print(f"[bench] mismatches vs the oracle on {m} segments: {mismatches}", file=sys.stderr, flush=True)
        cpu = {"value": round(m / dt / 1e6, 6), "unit": "Mrays/s", "cores": oracle.max_threads(),
               "kind": "oracle",
               "sample": f"first {m} of the {n} segments x all {F.shape[0]} triangles "
                         f"(binary64 brute force, all three modes in one pass), {dt:.1f} s",
               "host": host_cpu(), "mismatches_vs_oracle": mismatches,
               "timed_path_every_segment_vs_oracle": full}
        print(f"[bench] cpu oracle: {cpu['value']} Mrays/s on {cpu['cores']} threads", file=sys.stderr,
              flush=True)

    line = {
        "metric": "Mrays/s at Nt~32k, Nr=1e7 (build + intersect, flags exact vs FP64 oracle)",
        "value": round(value, 2), "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "heightfield 128x128 (32,258 triangles), 1e7 segments in the 10%-inflated box",
                   "mode": args.mode, "precision": args.precision, "build": args.build,
                   "n_triangles": int(F.shape[0]),
                   "n_rays": int(n), "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "intersect_ms": {"avg": round(intersect_avg, 4), "min": round(intersect_ms[0], 4),
                         "median": round(intersect_ms[len(intersect_ms) // 2], 4)},
        "counters": {"redecided_fp64": counters[0], "stack_overflow": counters[1]},
        "every_segment_vs_oracle": full,
        "hit_fraction": hit_frac,
        "variants": variants,
        "learned_vs_plain": learned,
        "learned_form": learned_c5,
        "configs": configs,
        "batched": batched,
        "host_resident": host,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
