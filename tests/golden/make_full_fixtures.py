"""Write the full-size expected results of the paper-scale and precision
workloads, computed by the binary64 oracle alone.

The oracle is the exhaustive search of the paper's Background section (every
segment against every triangle, Moller-Trumbore in binary64) with its three
operating modes and the experimental intercept count.  At 1e7 segments the
outputs are too large to store, so each chunk of CHUNK segments is kept as
64-bit prefixes of SHA-256 digests of:
  hit     uint8  [n]        boolean mode
  id      int32  [n] (LE)   first-hit triangle index, -1 on a miss
  uvt     float32[n][3]     (u, v, t) of the first hit rounded once to float32
                            (NaN rows replaced by the canonical quiet NaN)
  count   int32  [n] (LE)   distinct binary64 t among the hits
plus the chunk's number of hitting segments.  The inputs' digest is stored
beside them so a test can tell an input that differs from an output that does.

Only `oracle` and the seeded input generators are called; nothing here loads
the GPU library.  The run is resumable: chunks already in the file are kept.

    python tests/golden/make_full_fixtures.py paper_scale
    python tests/golden/make_full_fixtures.py precision
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CHUNK = 1 << 17


def digest(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]


def input_digest(V, F, O, E) -> str:
    h = hashlib.sha256()
    for a, dt in ((V, "<f4"), (F, "<i4"), (O, "<f4"), (E, "<f4")):
        h.update(np.ascontiguousarray(a, dtype=dt).tobytes())
    return h.hexdigest()[:16]


def uvt_f32(uvt) -> np.ndarray:
    """float64 (u, v, t) rounded once to float32, NaN rows canonical."""
    out = np.asarray(uvt, np.float64).astype(np.float32)
    out[np.isnan(out)] = np.float32("nan")
    return out


def chunk_digests(hit, ids, uvt, count):
    return (digest(hit.astype(np.uint8)), digest(ids.astype("<i4")),
            digest(uvt_f32(uvt)), digest(count.astype("<i4")))


def workload(name: str):
    from paper_2305_01867_amd import workloads
    if name == "paper_scale":
        return workloads.paper_scale_config()
    if name == "precision":
        V, F, O, E, _ = workloads.precision_config()
        return V, F, O, E
    raise ValueError(name)


def path(name: str) -> str:
    return os.path.join(HERE, f"full_{name}.txt")


def read(name: str):
    """-> (header dict, {chunk index: (start, n, n_hit, hit, id, uvt, count)})."""
    head, rows = {}, {}
    with open(path(name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            f = line.split()
            if f[0] == "chunk_row":
                rows[int(f[1])] = (int(f[2]), int(f[3]), int(f[4]), *f[5:9])
            else:
                head[f[0]] = f[1]
    return head, rows


def main(name: str) -> None:
    import oracle

    V, F, O, E = workload(name)
    n = O.shape[0]
    dig = input_digest(V, F, O, E)
    p = path(name)
    done = {}
    if os.path.exists(p):
        head, done = read(name)
        if head.get("inputs") != dig or int(head.get("chunk", CHUNK)) != CHUNK:
            raise SystemExit(f"{p} was written for other inputs; remove it first")
    else:
        with open(p, "w") as fh:
            fh.write("# Expected results of the binary64 oracle (exhaustive search, paper:\n"
                     "# Background section: boolean, first-hit and barycentric modes, and the\n"
                     "# intercept count) for every segment of this workload.  Written by\n"
                     "# tests/golden/make_full_fixtures.py, which calls only the oracle.\n"
                     "# chunk_row <index> <first segment> <segments> <hitting segments>\n"
                     "#           <hit digest> <id digest> <uvt digest> <count digest>\n")
            fh.write(f"workload {name}\ninputs {dig}\nn_segments {n}\nn_triangles {F.shape[0]}\nchunk {CHUNK}\n")
    n_chunks = (n + CHUNK - 1) // CHUNK
    t0 = time.time()
    for c in range(n_chunks):
        if c in done:
            continue
        s, m = c * CHUNK, min(CHUNK, n - c * CHUNK)
        hit, ids, uvt, _ = oracle.intersect(V, F, O[s:s + m], E[s:s + m])
        count = oracle.intercept_count(V, F, O[s:s + m], E[s:s + m])
        d = chunk_digests(hit, ids, uvt, count)
        with open(p, "a") as fh:
            fh.write(f"chunk_row {c} {s} {m} {int(hit.sum())} {' '.join(d)}\n")
        print(f"[{name}] chunk {c + 1}/{n_chunks} ({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    for arg in sys.argv[1:]:
        main(arg)
