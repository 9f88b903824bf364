"""Python binding of librsi.so (include/rsi.h): segment / triangle-mesh
intersection on AMD gfx950.

Argument marshalling only: tensors must already be on the GPU, float32
coordinates and int32 indices (the paper's Case Study 1 is about a 64-bit
index array read as 32-bit; an int64 array is refused here, never converted).
Every step of the computation runs in the library's HIP kernels; this module
has no CPU fallback and raises if the library is not built.

Names follow the C ABI: rsi_build, rsi_intersect, rsi_destroy,
rsi_mesh_info_get, rsi_mesh_export, rsi_traversal_stats and the
rsi_proposal_* calls of the learned subtree proposal.
"""
from __future__ import annotations

import ctypes
import os

import torch  # imported first so the library binds to the HIP runtime torch loaded

__all__ = [
    "RSIError", "Mesh", "lib", "library_path", "rsi_build", "rsi_intersect", "rsi_destroy",
    "rsi_mesh_info_get", "rsi_mesh_export", "rsi_traversal_stats", "MODES", "PRECISIONS",
    "rsi_proposal_train", "rsi_proposal_predict", "rsi_proposal_params", "rsi_proposal_gradient",
    "rsi_proposal_features", "rsi_proposal_frontier", "rsi_proposal_save", "rsi_proposal_load",
    "MLP_PARAMS", "MLP_INPUTS", "MLP_BUCKETS",
    "Batch", "rsi_batch_create", "rsi_batch_build", "rsi_batch_intersect", "rsi_batch_export", "rsi_batch_destroy",
    "rsi_stream_copy", "rsi_intersect_noalloc",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "librsi.so")

ABI_VERSION = 7
MODES = {"boolean": 0, "first_hit": 1, "barycentric": 2, "intercept_count": 3}
PRECISIONS = {"plain": 0, "certified": 1}
EXPORTS = {"sorted_keys": 0, "sorted_ids": 1, "nodes": 2, "parents": 3, "counters": 4, "leaves": 5, "bounds": 6,
           "wide_nodes": 7, "wide_top": 8, "mesh_roots": 9}
STATUS = {0: "RSI_OK", 1: "RSI_E_ARG", 2: "RSI_E_RANGE", 3: "RSI_E_NOMEM", 4: "RSI_E_HIP",
          5: "RSI_E_STATE", 6: "RSI_E_CAPACITY"}


class RSIError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class _BuildOpts(ctypes.Structure):
    _fields_ = [("morton_bits", ctypes.c_int32), ("check_indices", ctypes.c_int32), ("algorithm", ctypes.c_int32)]


class _IntersectOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("block", ctypes.c_int32), ("stack_depth", ctypes.c_int32),
                ("ray_sort", ctypes.c_int32), ("proposal", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("node_width", ctypes.c_int32)]


class _Outputs(ctypes.Structure):
    _fields_ = [("hit", ctypes.c_void_p), ("tri_id", ctypes.c_void_p), ("uvt", ctypes.c_void_p),
                ("counters", ctypes.c_void_p), ("count", ctypes.c_void_p)]


class _TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("reinit", ctypes.c_int32), ("seed", ctypes.c_uint64)]


MLP_PARAMS = 254976
MLP_INPUTS = 224
MLP_BUCKETS = 256


class _MeshInfo(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int64), ("n_triangles", ctypes.c_int64), ("morton_bits", ctypes.c_int32),
                ("root", ctypes.c_int32), ("device_bytes", ctypes.c_int64), ("node_width", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None


def lib():
    """Load librsi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path):
        raise ImportError(f"{library_path} is missing: build it with paper_2305_01867_amd/build_lib.py "
                          "(or __graft_entry__.build())")
    L = ctypes.CDLL(library_path)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.rsi_build.argtypes = [P, I64, P, I64, ctypes.POINTER(_BuildOpts), P, ctypes.POINTER(P)]
    L.rsi_intersect.argtypes = [P, P, P, I64, I32, ctypes.POINTER(_IntersectOpts), ctypes.POINTER(_Outputs), P]
    L.rsi_intersect_noalloc.argtypes = [P, P, P, I64, I32, ctypes.POINTER(_IntersectOpts), ctypes.POINTER(_Outputs), P]
    L.rsi_destroy.argtypes = [P]
    L.rsi_mesh_info_get.argtypes = [P, ctypes.POINTER(_MeshInfo)]
    L.rsi_mesh_export.argtypes = [P, I32, P, I64, P]
    L.rsi_traversal_stats.argtypes = [P, P, P, I64, I32, ctypes.POINTER(_IntersectOpts), P, P, P]
    L.rsi_debug_certify.argtypes = [P, P, P, I64, P, P, P]
    L.rsi_derive.argtypes = [P, P, I64, P, P, P, P, P]
    L.rsi_compact_hits.argtypes = [P, P, I64, P, P, P, P, P, P, P, P]
    L.rsi_proposal_train.argtypes = [P, P, P, I64, ctypes.POINTER(_TrainOpts), P, ctypes.POINTER(I64), P]
    L.rsi_proposal_predict.argtypes = [P, P, P, I64, P, P]
    L.rsi_proposal_params.argtypes = [P, I32, P, P]
    L.rsi_proposal_gradient.argtypes = [P, P, P, P, I64, P, P, P, P]
    L.rsi_proposal_features.argtypes = [P, P, P, I64, P, P]
    L.rsi_proposal_frontier.argtypes = [P, P, P, ctypes.POINTER(I32), P]
    L.rsi_proposal_save.argtypes = [P, ctypes.c_char_p]
    L.rsi_proposal_load.argtypes = [P, ctypes.c_char_p]
    L.rsi_batch_create.argtypes = [I32, P, P, P, P, ctypes.POINTER(P)]
    L.rsi_batch_build.argtypes = [P, P, P, P]
    L.rsi_batch_intersect.argtypes = [P, P, P, I32, ctypes.POINTER(_IntersectOpts), ctypes.POINTER(_Outputs), P]
    L.rsi_batch_export.argtypes = [P, I32, P, I64, P]
    L.rsi_batch_destroy.argtypes = [P]
    L.rsi_stream_copy.argtypes = [P, P, I64, P]
    for f in ("rsi_batch_create", "rsi_batch_build", "rsi_batch_intersect", "rsi_batch_export", "rsi_batch_destroy"):
        getattr(L, f).restype = ctypes.c_int
    for f in ("rsi_build", "rsi_intersect", "rsi_destroy", "rsi_mesh_info_get", "rsi_mesh_export",
              "rsi_traversal_stats", "rsi_proposal_train", "rsi_proposal_predict", "rsi_proposal_params",
              "rsi_proposal_gradient", "rsi_proposal_features", "rsi_proposal_frontier", "rsi_proposal_save",
              "rsi_proposal_load", "rsi_debug_certify", "rsi_derive", "rsi_compact_hits", "rsi_stream_copy"):
        getattr(L, f).restype = ctypes.c_int
    L.rsi_status_string.argtypes = [ctypes.c_int]
    L.rsi_status_string.restype = ctypes.c_char_p
    L.rsi_last_error.argtypes = []
    L.rsi_last_error.restype = ctypes.c_char_p
    L.rsi_abi_version.argtypes = []
    L.rsi_abi_version.restype = ctypes.c_int32
    if L.rsi_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{library_path} has ABI {L.rsi_abi_version()}, this binding expects {ABI_VERSION}: "
                           "rebuild it with paper_2305_01867_amd/build_lib.py")
    _lib = L
    return L


def _check(status: int):
    if status != 0:
        raise RSIError(status, lib().rsi_last_error().decode(errors="replace"))


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _need(t: torch.Tensor, name: str, dtype, shape_tail=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_tail is not None and (t.dim() != 2 or t.shape[1] != shape_tail):
        raise ValueError(f"{name} must have shape [N, {shape_tail}]")
    return t


class Mesh:
    """A built BVH (owns the library handle)."""

    def __init__(self, handle, n_vertices, n_triangles, morton_bits, stream):
        self._h = handle
        self.n_vertices = n_vertices
        self.n_triangles = n_triangles
        self.morton_bits = morton_bits
        self._stream = stream

    @property
    def handle(self):
        if self._h is None:
            raise RSIError(5, "mesh destroyed")
        return self._h

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            _check(lib().rsi_destroy(h))

    def __del__(self):
        try:
            if self._h is not None and _lib is not None:
                _lib.rsi_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


BUILD_ALGORITHMS = {"radix_tree": 0, "agglomerative": 1, "restructured": 2}


def rsi_build(vertices: torch.Tensor, triangles: torch.Tensor, morton_bits: int = 30,
              check_indices: bool = False, stream=None, algorithm: str = "radix_tree") -> Mesh:
    """Build the BVH of a mesh: vertices float32 [N_v, 3], triangles int32 [N_t, 3].
    algorithm: "radix_tree" (default), "agglomerative" (single pass, nodes
    numbered by split position; waits once for the root) or "restructured"
    (radix tree + treelet restructuring: fewer node visits per query)."""
    if algorithm not in BUILD_ALGORITHMS:
        raise ValueError(f"algorithm must be one of {list(BUILD_ALGORITHMS)}")
    for t, name, dt in ((vertices, "vertices", torch.float32), (triangles, "triangles", torch.int32)):
        if isinstance(t, torch.Tensor) and t.dtype != dt:
            raise TypeError(f"{name} must be {dt}, got {t.dtype}")
    _need(vertices, "vertices", torch.float32, 3)
    _need(triangles, "triangles", torch.int32, 3)
    opts = _BuildOpts(int(morton_bits), int(bool(check_indices)), BUILD_ALGORITHMS[algorithm])
    h = ctypes.c_void_p()
    s = _stream_handle(stream)
    _check(lib().rsi_build(ctypes.c_void_p(vertices.data_ptr()), vertices.shape[0],
                           ctypes.c_void_p(triangles.data_ptr()), triangles.shape[0],
                           ctypes.byref(opts), s, ctypes.byref(h)))
    return Mesh(h, vertices.shape[0], triangles.shape[0], morton_bits, stream)


def rsi_destroy(mesh: Mesh):
    mesh.close()


RAY_ORDERS = {"input": 0, "midpoint": 1, "origin_octant": 2}


def _iopts(precision, block, stack_depth, proposal=False, ray_sort=0, waves_per_cu=0, node_width=0):
    if precision not in PRECISIONS:
        raise ValueError(f"precision must be one of {list(PRECISIONS)}")
    if isinstance(ray_sort, str):
        if ray_sort not in RAY_ORDERS:
            raise ValueError(f"ray_sort must be one of {list(RAY_ORDERS)}")
        ray_sort = RAY_ORDERS[ray_sort]
    return _IntersectOpts(PRECISIONS[precision], int(block), int(stack_depth), int(ray_sort), int(bool(proposal)),
                          int(waves_per_cu), int(node_width))


def rsi_intersect(mesh: Mesh, rays_from: torch.Tensor, rays_to: torch.Tensor, mode: str = "boolean",
                  precision: str = "plain", block: int = 0, stack_depth: int = 0, out: dict | None = None,
                  stream=None, proposal: bool = False, ray_sort=0, waves_per_cu: int = 0,
                  node_width: int = 0, _noalloc: bool = False) -> dict:
    """Test segments [N, 3] float32 against the mesh.  Returns a dict with the
    outputs of the mode ("hit" uint8, "tri_id" int32, "uvt" float32 [N, 3],
    "count" int32) and "counters" uint64 [4] (re-decided in binary64, past the
    LDS stack, proposal misses, count-mode list overflows).
    `out` may supply preallocated tensors under the same keys.  ray_sort:
    processing order ("input", "midpoint", "origin_octant" or 0 / 1 / 2);
    results are at input indices in every order.  node_width: tree the first
    pass walks (0 the widest built, 2 binary, 4 the 4-wide tree)."""
    if mode not in MODES:
        raise ValueError(f"mode must be one of {list(MODES)}")
    _need(rays_from, "rays_from", torch.float32, 3)
    _need(rays_to, "rays_to", torch.float32, 3)
    if rays_from.shape != rays_to.shape:
        raise ValueError("rays_from and rays_to must have the same shape")
    n = rays_from.shape[0]
    dev = rays_from.device
    out = dict(out or {})
    if mode == "boolean":
        if "hit" not in out:
            out["hit"] = torch.empty(n, dtype=torch.uint8, device=dev)
    elif mode == "intercept_count":
        if "count" not in out:
            out["count"] = torch.empty(n, dtype=torch.int32, device=dev)
    else:
        if "tri_id" not in out:
            out["tri_id"] = torch.empty(n, dtype=torch.int32, device=dev)
    if mode == "barycentric":
        if "uvt" not in out:
            out["uvt"] = torch.empty((n, 3), dtype=torch.float32, device=dev)
    if "counters" not in out:
        out["counters"] = torch.empty(4, dtype=torch.int64, device=dev)
    spec = {"hit": (torch.uint8, None), "tri_id": (torch.int32, None), "uvt": (torch.float32, 3),
            "count": (torch.int32, None), "counters": (torch.int64, None)}
    for k, t in out.items():
        if k not in spec:
            raise ValueError(f"unknown output {k}")
        _need(t, f"out[{k!r}]", spec[k][0], spec[k][1])
        if k != "counters" and t.shape[0] < n:
            raise ValueError(f"out[{k!r}] is too small")
        if k == "counters" and t.numel() < 4:
            raise ValueError("out['counters'] needs 4 entries")

    def ptr(k):
        return ctypes.c_void_p(out[k].data_ptr()) if k in out else ctypes.c_void_p()

    o = _Outputs(ptr("hit"), ptr("tri_id"), ptr("uvt"), ptr("counters"), ptr("count"))
    opts = _iopts(precision, block, stack_depth, proposal, ray_sort, waves_per_cu, node_width)
    fn = lib().rsi_intersect_noalloc if _noalloc else lib().rsi_intersect
    _check(fn(mesh.handle, ctypes.c_void_p(rays_from.data_ptr()), ctypes.c_void_p(rays_to.data_ptr()), n,
              MODES[mode], ctypes.byref(opts), ctypes.byref(o), _stream_handle(stream)))
    return out


def rsi_intersect_noalloc(mesh: Mesh, rays_from: torch.Tensor, rays_to: torch.Tensor, out: dict,
                          mode: str = "boolean", precision: str = "plain", stream=None, **opts) -> dict:
    """rsi_intersect through the entry point that allocates no device memory
    (its temporary memory is one fixed 64 MiB array of the library, shared by
    every call on the GPU).  `out` must hold every output tensor the mode
    needs and "counters"; options as rsi_intersect."""
    need = {"boolean": ("hit",), "first_hit": ("tri_id",), "barycentric": ("tri_id", "uvt"),
            "intercept_count": ("count",)}[mode] + ("counters",)
    missing = [k for k in need if k not in out]
    if missing:
        raise ValueError(f"rsi_intersect_noalloc allocates nothing: out needs {missing}")
    return rsi_intersect(mesh, rays_from, rays_to, mode=mode, precision=precision, out=out, stream=stream,
                         _noalloc=True, **opts)


def rsi_traversal_stats(mesh: Mesh, rays_from: torch.Tensor, rays_to: torch.Tensor, mode: str = "boolean",
                        precision: str = "plain", block: int = 0, stack_depth: int = 0, stream=None,
                        proposal: bool = False, ray_sort=0, waves_per_cu: int = 0, node_width: int = 0):
    """Per-segment (node visits, leaf tests) of the traversal (int32 tensors;
    visits count 4-wide nodes when the first pass walks them)."""
    _need(rays_from, "rays_from", torch.float32, 3)
    _need(rays_to, "rays_to", torch.float32, 3)
    n = rays_from.shape[0]
    visits = torch.zeros(n, dtype=torch.int32, device=rays_from.device)
    tests = torch.zeros(n, dtype=torch.int32, device=rays_from.device)
    opts = _iopts(precision, block, stack_depth, proposal, ray_sort, waves_per_cu, node_width)
    _check(lib().rsi_traversal_stats(mesh.handle, ctypes.c_void_p(rays_from.data_ptr()),
                                     ctypes.c_void_p(rays_to.data_ptr()), n, MODES[mode], ctypes.byref(opts),
                                     ctypes.c_void_p(visits.data_ptr()), ctypes.c_void_p(tests.data_ptr()),
                                     _stream_handle(stream)))
    return visits, tests


def rsi_debug_certify(rays_from: torch.Tensor, rays_to: torch.Tensor, corners: torch.Tensor, stream=None):
    """Binary32 predicates, their bounds and the certified classification for
    pairs (segment i, triangle with corners[i] [n, 3, 3]).  Returns (values
    float32 [n, 10], classes int32 [n]); see include/rsi.h."""
    n = _rays(rays_from, rays_to)
    _need(corners, "corners", torch.float32)
    if corners.shape != (n, 3, 3) or not corners.is_contiguous():
        raise ValueError("corners must be a contiguous [n, 3, 3] tensor")
    values = torch.empty((n, 10), dtype=torch.float32, device=rays_from.device)
    classes = torch.empty(n, dtype=torch.int32, device=rays_from.device)
    _check(lib().rsi_debug_certify(_p(rays_from), _p(rays_to), _p(corners), n, _p(values), _p(classes),
                                   _stream_handle(stream)))
    return values, classes


def _bary(rays_from, rays_to, result):
    n = _rays(rays_from, rays_to)
    if "tri_id" not in result or "uvt" not in result:
        raise ValueError("result must hold the barycentric outputs 'tri_id' and 'uvt'")
    _need(result["tri_id"], "result['tri_id']", torch.int32)
    _need(result["uvt"], "result['uvt']", torch.float32, 3)
    if result["tri_id"].shape[0] < n or result["uvt"].shape[0] < n:
        raise ValueError("result arrays are shorter than the segment arrays")
    return n


def rsi_derive(rays_from, rays_to, result: dict, stream=None) -> dict:
    """Distance t |E - O| and point O + t (E - O) of every segment from a
    barycentric result (NaN on a miss): {"distance": [N], "point": [N, 3]}."""
    n = _bary(rays_from, rays_to, result)
    dist = torch.empty(n, dtype=torch.float32, device=rays_from.device)
    point = torch.empty((n, 3), dtype=torch.float32, device=rays_from.device)
    _check(lib().rsi_derive(_p(rays_from), _p(rays_to), n, _p(result["tri_id"]), _p(result["uvt"]), _p(dist),
                            _p(point), _stream_handle(stream)))
    return {"distance": dist, "point": point}


def rsi_compact_hits(rays_from, rays_to, result: dict, stream=None):
    """The paper's barycentric tuple (intersecting_rays, distances,
    hit_triangles, hit_points) from a barycentric result, hitting segments in
    ascending index.  Waits for the stream once to learn the number of hits."""
    n = _bary(rays_from, rays_to, result)
    dev = rays_from.device
    idx = torch.empty(n, dtype=torch.int64, device=dev)
    dist = torch.empty(n, dtype=torch.float32, device=dev)
    tri = torch.empty(n, dtype=torch.int32, device=dev)
    point = torch.empty((n, 3), dtype=torch.float32, device=dev)
    count = torch.zeros(1, dtype=torch.int64, device=dev)
    _check(lib().rsi_compact_hits(_p(rays_from), _p(rays_to), n, _p(result["tri_id"]), _p(result["uvt"]), _p(idx),
                                  _p(dist), _p(tri), _p(point), _p(count), _stream_handle(stream)))
    k = int(count.item())
    return idx[:k], dist[:k], tri[:k], point[:k]


def rsi_test(vertices, triangles, rays_from, rays_to, mode: str = "boolean", precision: str = "certified", **opts):
    """The paper's one-call usage (Usage section: test(vertices, triangles,
    raysFrom, raysTo, cfg)): builds the mesh, intersects and returns, by mode,
    the hit flags (boolean), the compacted (intersecting_rays, distances,
    hit_triangles, hit_points) (barycentric), the number of distinct
    intersections (intercept_count) or the nearest triangle (first_hit).
    Arrays may be numpy or torch; numpy inputs are copied to the GPU and the
    results come back as numpy."""
    import numpy as _np
    as_numpy = isinstance(rays_from, _np.ndarray)
    dev = torch.device("cuda")
    t = lambda x, dt: (torch.from_numpy(_np.ascontiguousarray(x, dt)).to(dev) if isinstance(x, _np.ndarray)
                       else x)
    V, F = t(vertices, _np.float32), t(triangles, _np.int32)
    O, E = t(rays_from, _np.float32), t(rays_to, _np.float32)
    with rsi_build(V, F) as mesh:
        r = rsi_intersect(mesh, O, E, mode=mode, precision=precision, **opts)
        if mode == "barycentric":
            out = rsi_compact_hits(O, E, r)
        else:
            out = {"boolean": r.get("hit"), "first_hit": r.get("tri_id"), "intercept_count": r.get("count")}[mode]
    if as_numpy:
        out = tuple(x.cpu().numpy() for x in out) if isinstance(out, tuple) else out.cpu().numpy()
    return out


def rsi_mesh_info_get(mesh: Mesh) -> dict:
    info = _MeshInfo()
    _check(lib().rsi_mesh_info_get(mesh.handle, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in _MeshInfo._fields_}


def rsi_mesh_export(mesh: Mesh, what: str, stream=None) -> torch.Tensor:
    """Copy one internal array to a new GPU tensor (layouts in include/rsi.h)."""
    nt = mesh.n_triangles
    shapes = {
        "sorted_keys": ((nt,), torch.int64), "sorted_ids": ((nt,), torch.int32),
        "nodes": ((max(nt - 1, 0), 16), torch.int32), "parents": ((max(2 * nt - 1, 0),), torch.int32),
        "counters": ((max(nt - 1, 0),), torch.int32), "leaves": ((nt, 12), torch.int32),
        "bounds": ((8 if nt > 0 else 0,), torch.float32),
        "wide_nodes": ((max(nt - 1, 0) if rsi_mesh_info_get(mesh)["node_width"] == 4 else 0, 32), torch.int32),
        "wide_top": ((512 if rsi_mesh_info_get(mesh)["node_width"] == 4 else 0, 32), torch.int32),
    }
    if what not in shapes:
        raise ValueError(f"what must be one of {list(shapes)}")
    shape, dtype = shapes[what]
    dst = torch.empty(shape, dtype=dtype, device="cuda")
    _check(lib().rsi_mesh_export(mesh.handle, EXPORTS[what], ctypes.c_void_p(dst.data_ptr()),
                                 dst.numel() * dst.element_size(), _stream_handle(stream)))
    return dst


# --------------------------------------------------------------- learned proposal
def _rays(rays_from, rays_to):
    _need(rays_from, "rays_from", torch.float32, 3)
    _need(rays_to, "rays_to", torch.float32, 3)
    if rays_from.shape != rays_to.shape:
        raise ValueError("rays_from and rays_to must have the same shape")
    return rays_from.shape[0]


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def rsi_proposal_train(mesh: Mesh, rays_from, rays_to, epochs: int = 2, batch: int = 4096, lr: float = 1e-3,
                       seed: int = 1, reinit: bool = False, stream=None):
    """Train the proposal on segments labelled by the exact first-hit pass.
    Returns (mean loss per epoch as a CPU tensor, number of labelled segments)."""
    n = _rays(rays_from, rays_to)
    loss = torch.zeros(max(int(epochs), 1), dtype=torch.float32, device=rays_from.device)
    nl = ctypes.c_int64(0)
    opts = _TrainOpts(int(epochs), int(batch), float(lr), int(bool(reinit)), int(seed))
    _check(lib().rsi_proposal_train(mesh.handle, _p(rays_from), _p(rays_to), n, ctypes.byref(opts), _p(loss),
                                    ctypes.byref(nl), _stream_handle(stream)))
    torch.cuda.synchronize()
    return loss.cpu(), int(nl.value)


def rsi_proposal_predict(mesh: Mesh, rays_from, rays_to, stream=None) -> torch.Tensor:
    n = _rays(rays_from, rays_to)
    out = torch.empty(n, dtype=torch.uint8, device=rays_from.device)
    _check(lib().rsi_proposal_predict(mesh.handle, _p(rays_from), _p(rays_to), n, _p(out), _stream_handle(stream)))
    return out


def rsi_proposal_params(mesh: Mesh, new: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Get (new=None) or set the fp32 parameter vector [MLP_PARAMS]."""
    if new is None:
        buf = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
        _check(lib().rsi_proposal_params(mesh.handle, 0, _p(buf), _stream_handle(stream)))
        return buf
    _need(new, "params", torch.float32)
    if new.numel() != MLP_PARAMS:
        raise ValueError(f"params must have {MLP_PARAMS} entries")
    _check(lib().rsi_proposal_params(mesh.handle, 1, _p(new), _stream_handle(stream)))
    return new


def rsi_proposal_gradient(mesh: Mesh, rays_from, rays_to, labels: torch.Tensor, stream=None):
    """(gradient [MLP_PARAMS], logits [n, 256], mean loss [1]) of one batch."""
    n = _rays(rays_from, rays_to)
    _need(labels, "labels", torch.int32)
    if labels.numel() != n:
        raise ValueError("one label per segment")
    dev = rays_from.device
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=dev)
    logits = torch.empty((n, MLP_BUCKETS), dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    _check(lib().rsi_proposal_gradient(mesh.handle, _p(rays_from), _p(rays_to), _p(labels), n, _p(grad), _p(logits),
                                       _p(loss), _stream_handle(stream)))
    return grad, logits, loss


def rsi_proposal_features(mesh: Mesh, rays_from, rays_to, stream=None) -> torch.Tensor:
    """Network inputs [n, 224] as bfloat16."""
    n = _rays(rays_from, rays_to)
    X = torch.empty((n, MLP_INPUTS), dtype=torch.int16, device=rays_from.device)
    _check(lib().rsi_proposal_features(mesh.handle, _p(rays_from), _p(rays_to), n, _p(X), _stream_handle(stream)))
    return X.view(torch.bfloat16)


def rsi_proposal_frontier(mesh: Mesh, stream=None):
    """(bucket node references [nb], first sorted leaf of each bucket [nb])."""
    ref = torch.zeros(MLP_BUCKETS, dtype=torch.int32, device="cuda")
    first = torch.zeros(MLP_BUCKETS, dtype=torch.int32, device="cuda")
    nb = ctypes.c_int32(0)
    _check(lib().rsi_proposal_frontier(mesh.handle, _p(ref), _p(first), ctypes.byref(nb), _stream_handle(stream)))
    return ref[: nb.value], first[: nb.value]


def rsi_proposal_save(mesh: Mesh, path: str):
    _check(lib().rsi_proposal_save(mesh.handle, os.fsencode(path)))


def rsi_proposal_load(mesh: Mesh, path: str):
    _check(lib().rsi_proposal_load(mesh.handle, os.fsencode(path)))


# --------------------------------------------------------------- batched form
class Batch:
    """Many meshes and their segment batches (owns the library handle)."""

    def __init__(self, handle, v_off, t_off, r_off):
        self._h = handle
        self.vertex_offsets = list(v_off)
        self.triangle_offsets = list(t_off)
        self.ray_offsets = list(r_off)
        self.n_meshes = len(v_off) - 1

    @property
    def handle(self):
        if self._h is None:
            raise RSIError(5, "batch destroyed")
        return self._h

    @property
    def n_rays(self):
        return self.ray_offsets[-1]

    def close(self):
        if self._h is not None:
            h, self._h = self._h, None
            _check(lib().rsi_batch_destroy(h))

    def __del__(self):
        try:
            if self._h is not None and _lib is not None:
                _lib.rsi_batch_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def rsi_batch_create(vertex_offsets, triangle_offsets, ray_offsets, stream=None) -> Batch:
    """Offsets: sequences of n_meshes + 1 nondecreasing ints starting at 0."""
    import numpy as np

    offs = [np.ascontiguousarray(np.asarray(o, dtype=np.int64)) for o in (vertex_offsets, triangle_offsets, ray_offsets)]
    if not (len(offs[0]) == len(offs[1]) == len(offs[2]) >= 2):
        raise ValueError("three offset arrays of the same length n_meshes + 1 >= 2")
    h = ctypes.c_void_p()
    _check(lib().rsi_batch_create(len(offs[0]) - 1, *(o.ctypes.data_as(ctypes.c_void_p) for o in offs),
                                  _stream_handle(stream), ctypes.byref(h)))
    return Batch(h, *(o.tolist() for o in offs))


def rsi_batch_build(batch: Batch, vertices: torch.Tensor, triangles: torch.Tensor, stream=None):
    for t, name, dt in ((vertices, "vertices", torch.float32), (triangles, "triangles", torch.int32)):
        if isinstance(t, torch.Tensor) and t.dtype != dt:
            raise TypeError(f"{name} must be {dt}, got {t.dtype}")
    _need(vertices, "vertices", torch.float32, 3)
    _need(triangles, "triangles", torch.int32, 3)
    if vertices.shape[0] != batch.vertex_offsets[-1] or triangles.shape[0] != batch.triangle_offsets[-1]:
        raise ValueError("array sizes differ from the batch's offsets")
    _check(lib().rsi_batch_build(batch.handle, _p(vertices), _p(triangles), _stream_handle(stream)))


def rsi_batch_intersect(batch: Batch, rays_from, rays_to, mode: str = "boolean", precision: str = "plain",
                        block: int = 0, stack_depth: int = 0, out: dict | None = None, stream=None,
                        ray_sort=0, waves_per_cu: int = 0, node_width: int = 0) -> dict:
    """Outputs over all segments (triangle indices relative to each mesh).
    node_width: 0 the 4-wide tree (built for batches of more than one
    triangle), 2 binary nodes, 4 the 4-wide tree."""
    if mode not in MODES:
        raise ValueError(f"mode must be one of {list(MODES)}")
    n = _rays(rays_from, rays_to)
    if n != batch.n_rays:
        raise ValueError("segment count differs from the batch's ray offsets")
    dev = rays_from.device
    out = dict(out or {})
    if mode == "boolean":
        if "hit" not in out:
            out["hit"] = torch.empty(n, dtype=torch.uint8, device=dev)
    elif mode == "intercept_count":
        if "count" not in out:
            out["count"] = torch.empty(n, dtype=torch.int32, device=dev)
    else:
        if "tri_id" not in out:
            out["tri_id"] = torch.empty(n, dtype=torch.int32, device=dev)
    if mode == "barycentric":
        if "uvt" not in out:
            out["uvt"] = torch.empty((n, 3), dtype=torch.float32, device=dev)
    if "counters" not in out:
        out["counters"] = torch.empty(4, dtype=torch.int64, device=dev)

    def ptr(k):
        return ctypes.c_void_p(out[k].data_ptr()) if k in out else ctypes.c_void_p()

    o = _Outputs(ptr("hit"), ptr("tri_id"), ptr("uvt"), ptr("counters"), ptr("count"))
    opts = _iopts(precision, block, stack_depth, False, ray_sort, waves_per_cu, node_width)
    _check(lib().rsi_batch_intersect(batch.handle, _p(rays_from), _p(rays_to), MODES[mode], ctypes.byref(opts),
                                     ctypes.byref(o), _stream_handle(stream)))
    return out


def rsi_batch_export(batch: Batch, what: str, stream=None) -> torch.Tensor:
    """Arrays of the combined BVH (as rsi_mesh_export) or "mesh_roots"."""
    if what == "mesh_roots":
        dst = torch.empty(batch.n_meshes, dtype=torch.int32, device="cuda")
        _check(lib().rsi_batch_export(batch.handle, EXPORTS["mesh_roots"], _p(dst), dst.numel() * 4,
                                      _stream_handle(stream)))
        return dst
    view = Mesh(None, batch.vertex_offsets[-1], batch.triangle_offsets[-1], 63, stream)
    nt = view.n_triangles
    shapes = {
        "sorted_keys": ((nt,), torch.int64), "sorted_ids": ((nt,), torch.int32),
        "nodes": ((max(nt - 1, 0), 16), torch.int32), "parents": ((max(2 * nt - 1, 0),), torch.int32),
        "counters": ((max(nt - 1, 0),), torch.int32), "leaves": ((nt, 12), torch.int32),
        "bounds": ((8 if nt > 0 else 0,), torch.float32),
    }
    shape, dtype = shapes[what]
    dst = torch.empty(shape, dtype=dtype, device="cuda")
    _check(lib().rsi_batch_export(batch.handle, EXPORTS[what], _p(dst), dst.numel() * dst.element_size(),
                                  _stream_handle(stream)))
    return dst


def rsi_batch_destroy(batch: Batch):
    batch.close()


# --------------------------------------------------------------- measurement
def rsi_stream_copy(dst: torch.Tensor, src: torch.Tensor, stream=None):
    """Copy src into dst (contiguous GPU tensors of the same byte size, a
    multiple of 16) with the library's streaming copy kernel."""
    for t, name in ((dst, "dst"), (src, "src")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous GPU tensor")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("dst and src must have the same size in bytes")
    _check(lib().rsi_stream_copy(_p(dst), _p(src), nbytes, _stream_handle(stream)))
