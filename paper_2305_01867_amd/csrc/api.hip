// api.hip -- the C ABI declared in include/rsi.h: argument checks, device
// memory, stream-ordered launches and error reporting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>
#include <algorithm>
#include <mutex>

#include "rsi.h"
#include "rsi_internal.h"

struct rsi_mesh_s {
    uint32_t magic;
    rsi::MeshDev dev;
    hipStream_t stream;  // the stream the mesh was built on (used to free it)
    void *block;         // the one device allocation holding every array
};

struct rsi_batch_s {
    uint32_t magic;
    rsi::MeshDev dev;   // the combined BVH
    rsi::BatchDev b;
    hipStream_t stream;
    void *block;
    bool built;
};

namespace {

constexpr uint32_t kMagic = 0x52534931u;  // "RSI1"
constexpr uint32_t kDead = 0xdeadbeefu;

thread_local std::string g_error;

rsi_status fail(rsi_status st, const std::string &msg) {
    g_error = msg;
    return st;
}

rsi_status fail_hip(hipError_t e, const char *where) {
    return fail(RSI_E_HIP, std::string(where) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
}

bool aligned4(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 3u) == 0; }

// Is there a current device we were built for?  Checked once per device.
rsi_status check_device() {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RSI_E_STATE, std::string("no usable HIP device: ") + hipGetErrorString(e));
    }
    static thread_local int checked_dev = -1;
    if (checked_dev == dev)
        return RSI_OK;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RSI_E_STATE, std::string("hipGetDeviceProperties failed: ") + hipGetErrorString(e));
    }
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(RSI_E_STATE, std::string("library built for gfx950, device is ") + prop.gcnArchName);
    // keep freed stream-ordered memory in the pool instead of returning it to
    // the HIP runtime at every synchronisation
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
    checked_dev = dev;
    return RSI_OK;
}

// Inside stream capture only stream work may be queued; pointer queries are
// skipped there (the capture's first eager run has checked the same pointers).
thread_local bool g_capturing = false;

void note_capture(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    g_capturing = hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusActive;
    (void)hipGetLastError();
}

bool is_device_ptr(const void *p) {
    if (g_capturing)
        return true;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

rsi_status check_dev_ptr(const void *p, const char *name) {
    if (!is_device_ptr(p))
        return fail(RSI_E_ARG, std::string(name) + " is not a device pointer");
    return RSI_OK;
}

// Is there an error left by earlier asynchronous work?
rsi_status pending_error(const char *where) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail_hip(e, where);
    return RSI_OK;
}

size_t round_up(size_t x) { return (x + 255) & ~size_t(255); }

bool valid_mesh(rsi_mesh m) { return m != nullptr && m->magic == kMagic; }

rsi_status parse_intersect_opts(const rsi_intersect_opts *opts, int &precision, int &block, int &stack,
                                int &ray_sort, int &waves, int &width) {
    precision = RSI_PRECISION_PLAIN;
    block = 0;  // the library default of the first pass it runs
    stack = 20;
    ray_sort = RSI_RAY_ORDER_INPUT;
    waves = 0;
    width = 0;
    if (!opts)
        return RSI_OK;
    if (opts->precision != RSI_PRECISION_PLAIN && opts->precision != RSI_PRECISION_CERTIFIED)
        return fail(RSI_E_ARG, "precision must be RSI_PRECISION_PLAIN or RSI_PRECISION_CERTIFIED");
    precision = opts->precision;
    if (opts->block != 0) {
        if (opts->block != 64 && opts->block != 128 && opts->block != 256 && opts->block != 512 &&
            opts->block != 1024)
            return fail(RSI_E_ARG, "block must be 64, 128, 256, 512 or 1024");
        block = opts->block;
    }
    if (opts->stack_depth != 0) {
        if (opts->stack_depth < 1 || opts->stack_depth > 64)
            return fail(RSI_E_ARG, "stack_depth must be in 1..64");
        stack = opts->stack_depth;
    }
    if (opts->ray_sort != RSI_RAY_ORDER_INPUT && opts->ray_sort != RSI_RAY_ORDER_MIDPOINT &&
        opts->ray_sort != RSI_RAY_ORDER_ORIGIN_OCTANT)
        return fail(RSI_E_ARG, "ray_sort must be 0 (input order), 1 (midpoint Morton) or 2 (octant + start Morton)");
    ray_sort = opts->ray_sort;
    if (opts->proposal != 0 && opts->proposal != 1)
        return fail(RSI_E_ARG, "proposal must be 0 or 1");
    if (opts->waves_per_cu < 0 || opts->waves_per_cu > 32)
        return fail(RSI_E_ARG, "waves_per_cu must be in 0..32");
    waves = opts->waves_per_cu;
    if (opts->node_width != 0 && opts->node_width != 2 && opts->node_width != 4)
        return fail(RSI_E_ARG, "node_width must be 0 (widest built), 2 or 4");
    width = opts->node_width;
    return RSI_OK;
}

// Checks shared by rsi_intersect and rsi_traversal_stats that need no GPU.
rsi_status check_ray_args(rsi_mesh mesh, const float *from, const float *to, int64_t n, int32_t mode) {
    if (!valid_mesh(mesh))
        return fail(RSI_E_STATE, "invalid or destroyed mesh handle");
    if (n < 0)
        return fail(RSI_E_ARG, "n_rays must be >= 0");
    if (n >= (int64_t(1) << 31))
        return fail(RSI_E_CAPACITY, "n_rays must be < 2^31");
    if (mode != RSI_MODE_BOOLEAN && mode != RSI_MODE_FIRST_HIT && mode != RSI_MODE_BARYCENTRIC &&
        mode != RSI_MODE_INTERCEPT_COUNT)
        return fail(RSI_E_ARG, "unknown mode");
    if (n > 0 && (!from || !to))
        return fail(RSI_E_ARG, "rays_from / rays_to must not be NULL");
    if (n > 0 && (!aligned4(from) || !aligned4(to)))
        return fail(RSI_E_ARG, "rays_from / rays_to must be 4-byte aligned");
    return RSI_OK;
}

__global__ void k_widen_keys(const uint32_t *in, uint64_t *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = in[i];
}

}  // namespace

// Workspace of rsi_intersect_noalloc: the pass-2 queue and its counters, the
// proposal's buckets and the segment order, in one array that every GPU the
// library runs on holds until the process ends.  Host code never uses the
// array's name as an address (on the host it is only a stand-in for the
// symbol): each device's address comes from hipGetSymbolAddress.
static constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device with
// that device current.
rsi_status noalloc_scratch(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RSI_E_STATE, std::string("no usable HIP device: ") + hipGetErrorString(e));
    }
    if (dev < 0 || dev >= kMaxDevices)
        return fail(RSI_E_STATE, "device index beyond the library's per-device table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(RSI_E_HIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return RSI_OK;
}

}  // namespace

extern "C" {

rsi_status rsi_build(const float *vertices, int64_t n_vertices, const int32_t *triangles, int64_t n_triangles,
                     const rsi_build_opts *opts, void *stream, rsi_mesh *out) {
    g_error.clear();
    if (!out)
        return fail(RSI_E_ARG, "out must not be NULL");
    *out = nullptr;
    if (n_vertices < 0 || n_triangles < 0)
        return fail(RSI_E_ARG, "counts must be >= 0");
    if (n_triangles >= (int64_t(1) << 30))
        return fail(RSI_E_CAPACITY, "n_triangles must be < 2^30");
    if (n_vertices >= (int64_t(1) << 31))
        return fail(RSI_E_CAPACITY, "n_vertices must be < 2^31");
    if (n_triangles > 0 && (!triangles || !vertices))
        return fail(RSI_E_ARG, "vertices / triangles must not be NULL");
    if (n_vertices > 0 && !vertices)
        return fail(RSI_E_ARG, "vertices must not be NULL");
    if ((vertices && !aligned4(vertices)) || (triangles && !aligned4(triangles)))
        return fail(RSI_E_ARG, "vertices / triangles must be 4-byte aligned");
    int bits = 30, check = 0, algorithm = 0;
    if (opts) {
        if (opts->morton_bits != 0 && opts->morton_bits != 30 && opts->morton_bits != 63)
            return fail(RSI_E_ARG, "morton_bits must be 30 or 63");
        if (opts->morton_bits)
            bits = opts->morton_bits;
        check = opts->check_indices != 0;
        if (opts->algorithm < 0 || opts->algorithm > 2)
            return fail(RSI_E_ARG, "algorithm must be 0 (radix tree), 1 (agglomerative) or 2 (restructured)");
        algorithm = opts->algorithm;
    }
    rsi_status st = check_device();
    if (st != RSI_OK)
        return st;
    if (n_vertices > 0 && (st = check_dev_ptr(vertices, "vertices")) != RSI_OK)
        return st;
    if (n_triangles > 0 && (st = check_dev_ptr(triangles, "triangles")) != RSI_OK)
        return st;
    if ((st = pending_error("before rsi_build")) != RSI_OK)
        return st;

    hipStream_t s = static_cast<hipStream_t>(stream);
    rsi_mesh m = new (std::nothrow) rsi_mesh_s();
    if (!m)
        return fail(RSI_E_NOMEM, "host allocation failed");
    m->magic = kMagic;
    m->stream = s;
    m->block = nullptr;
    rsi::MeshDev &d = m->dev;
    d.nv = n_vertices;
    d.nt = n_triangles;
    d.morton_bits = bits;
    d.algorithm = algorithm;
    const int64_t nt = n_triangles;
    if (nt == 0) {
        d.root = INT32_MIN;
        *out = m;
        return RSI_OK;
    }
    d.root = nt >= 2 ? 0 : ~0;

    const size_t kb = bits > 32 ? 8 : 4;
    const size_t sz_V = round_up(12 * (size_t)n_vertices), sz_F = round_up(12 * (size_t)nt);
    const size_t sz_keys = round_up(kb * nt), sz_ids = round_up(4 * (size_t)nt);
    const size_t sz_nodes = round_up(64 * (size_t)(nt > 1 ? nt - 1 : 1));
    // the 4-wide tree (its top, then one 128-B slot per binary internal
    // node), for the builds whose tile list it is collapsed with
    const size_t sz_nodes4 = (algorithm != 1 && nt > 1) ? round_up(128 * (size_t)(nt - 1 + rsi::kTopSlots)) : 0;
    const size_t sz_par = round_up(4 * (size_t)(2 * nt - 1)), sz_cnt = round_up(4 * (size_t)(nt > 1 ? nt - 1 : 1));
    const size_t sz_tris = round_up(48 * (size_t)nt), sz_small = 256;
    const size_t sz_tmp = round_up(rsi::sort_tmp_bytes(nt, bits));
    const size_t total =
        sz_V + sz_F + sz_keys + sz_ids + sz_nodes + sz_nodes4 + sz_par + sz_cnt + sz_tris + sz_small + sz_tmp;
    hipError_t e = hipMallocAsync(&m->block, total, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        m->magic = kDead;
        delete m;
        return fail(e == hipErrorOutOfMemory ? RSI_E_NOMEM : RSI_E_HIP,
                    std::string("hipMallocAsync failed: ") + hipGetErrorString(e));
    }
    char *p = static_cast<char *>(m->block);
    auto take = [&](size_t bytes) {
        char *q = p;
        p += bytes;
        return q;
    };
    d.V = reinterpret_cast<float *>(take(sz_V));
    d.F = reinterpret_cast<int32_t *>(take(sz_F));
    d.keys = take(sz_keys);
    d.ids = reinterpret_cast<int32_t *>(take(sz_ids));
    d.nodes = reinterpret_cast<rsi::Node *>(take(sz_nodes));
    // top4 directly before nodes4, so a 4-wide reference r addresses top4[r] in both ranges
    d.top4 = sz_nodes4 ? reinterpret_cast<rsi::Node4 *>(take(sz_nodes4)) : nullptr;
    d.nodes4 = d.top4 ? d.top4 + rsi::kTopSlots : nullptr;
    d.parent = reinterpret_cast<int32_t *>(take(sz_par));
    d.counters = reinterpret_cast<int32_t *>(take(sz_cnt));
    d.tris = reinterpret_cast<rsi::Tri *>(take(sz_tris));
    char *small = take(sz_small);
    d.bounds = reinterpret_cast<float *>(small);
    d.flags = reinterpret_cast<int32_t *>(small + 64);
    d.sort_tmp = take(sz_tmp);
    d.bytes = (int64_t)total;

    // the build's first kernels copy the vertices and triangles into the mesh
    e = rsi::launch_build(d, vertices, triangles, s, sz_tmp);
    if (e != hipSuccess) {
        rsi_destroy(m);
        return fail_hip(e, "rsi_build launch");
    }
    if (algorithm == 1 && nt >= 2) {
        int32_t root = 0;
        e = hipMemcpyAsync(&root, d.flags + 1, sizeof(root), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            rsi_destroy(m);
            return fail_hip(e, "rsi_build (agglomerative root)");
        }
        if (root < 0 || root >= nt - 1) {
            rsi_destroy(m);
            return fail(RSI_E_HIP, "the agglomerative build did not reach a root");
        }
        d.root = root;
    }
    if (check) {
        int32_t flag = 0;
        e = hipMemcpyAsync(&flag, d.flags, sizeof(flag), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            rsi_destroy(m);
            return fail_hip(e, "rsi_build index check");
        }
        if (flag) {
            rsi_destroy(m);
            return fail(RSI_E_RANGE, "a triangle index lies outside [0, n_vertices)");
        }
    }
    *out = m;
    return RSI_OK;
}

rsi_status rsi_destroy(rsi_mesh mesh) {
    if (!mesh)
        return RSI_OK;
    if (mesh->magic != kMagic)
        return fail(RSI_E_STATE, "invalid or destroyed mesh handle");
    mesh->magic = kDead;
    hipError_t e = hipSuccess;
    if (mesh->dev.prop.block)
        e = hipFreeAsync(mesh->dev.prop.block, mesh->stream);
    if (mesh->block) {
        hipError_t e2 = hipFreeAsync(mesh->block, mesh->stream);
        if (e == hipSuccess)
            e = e2;
    }
    delete mesh;
    if (e != hipSuccess)
        return fail_hip(e, "rsi_destroy");
    return RSI_OK;
}

// scratch_ptr / scratch_cap: NULL -- the workspace is allocated and freed
// stream-ordered; otherwise it is this device buffer of scratch_cap bytes and
// nothing is allocated.
static rsi_status run_rays(rsi_mesh mesh, const float *from, const float *to, int64_t n, int32_t mode,
                           const rsi_intersect_opts *opts, const rsi_outputs *out, uint32_t *visits,
                           uint32_t *tests, void *stream, bool stats, void *scratch_ptr = nullptr,
                           size_t scratch_cap = 0) {
    g_error.clear();
    rsi_status st = check_ray_args(mesh, from, to, n, mode);
    if (st != RSI_OK)
        return st;
    int precision, block, stack, ray_sort, waves, width;
    if ((st = parse_intersect_opts(opts, precision, block, stack, ray_sort, waves, width)) != RSI_OK)
        return st;
    const bool use_prop = opts && opts->proposal == 1 && n > 0 && mesh->dev.nt > 0;
    if (use_prop && mode == RSI_MODE_INTERCEPT_COUNT)
        return fail(RSI_E_ARG, "intercept-count mode has no proposal order");
    if (use_prop && !mesh->dev.prop.ready)
        return fail(RSI_E_STATE, "proposal = 1 needs a trained or loaded proposal (rsi_proposal_train / _load)");
    if (width == 4 && mesh->dev.node_width != 4)
        return fail(RSI_E_ARG, "node_width = 4 needs a mesh built with algorithm 0 or 2 (more than one triangle)");
    if (!stats) {
        if (!out)
            return fail(RSI_E_ARG, "out must not be NULL");
        if (n > 0) {
            if (mode == RSI_MODE_BOOLEAN && !out->hit)
                return fail(RSI_E_ARG, "boolean mode needs out->hit");
            if ((mode == RSI_MODE_FIRST_HIT || mode == RSI_MODE_BARYCENTRIC) && !out->tri_id)
                return fail(RSI_E_ARG, "this mode needs out->tri_id");
            if (mode == RSI_MODE_INTERCEPT_COUNT && !out->count)
                return fail(RSI_E_ARG, "intercept-count mode needs out->count");
            if (mode == RSI_MODE_BARYCENTRIC && !out->uvt)
                return fail(RSI_E_ARG, "barycentric mode needs out->uvt");
        }
        if ((out->tri_id && !aligned4(out->tri_id)) || (out->uvt && !aligned4(out->uvt)) ||
            (out->count && !aligned4(out->count)) ||
            (out->counters && (reinterpret_cast<uintptr_t>(out->counters) & 7u)))
            return fail(RSI_E_ARG, "output buffers must be aligned to their element size");
    } else if (n > 0 && (!visits || !tests || !aligned4(visits) || !aligned4(tests))) {
        return fail(RSI_E_ARG, "node_visits / leaf_tests must be non-NULL and 4-byte aligned");
    }
    if ((st = check_device()) != RSI_OK)
        return st;
    if (n == 0 && !(out && out->counters))
        return RSI_OK;
    if (n > 0) {
        if ((st = check_dev_ptr(from, "rays_from")) != RSI_OK || (st = check_dev_ptr(to, "rays_to")) != RSI_OK)
            return st;
        if (!stats) {
            if (out->hit && (st = check_dev_ptr(out->hit, "out->hit")) != RSI_OK)
                return st;
            if (out->tri_id && (st = check_dev_ptr(out->tri_id, "out->tri_id")) != RSI_OK)
                return st;
            if (out->uvt && (st = check_dev_ptr(out->uvt, "out->uvt")) != RSI_OK)
                return st;
            if (out->count && (st = check_dev_ptr(out->count, "out->count")) != RSI_OK)
                return st;
        } else if ((st = check_dev_ptr(visits, "node_visits")) != RSI_OK ||
                   (st = check_dev_ptr(tests, "leaf_tests")) != RSI_OK) {
            return st;
        }
    }
    if (!stats && out->counters && (st = check_dev_ptr(out->counters, "out->counters")) != RSI_OK)
        return st;
    if ((st = pending_error("before rsi_intersect")) != RSI_OK)
        return st;

    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = nullptr;
    const size_t q_bytes = (4 * (size_t)n + 64 + 255) & ~size_t(255);
    const size_t b_bytes = use_prop ? ((size_t)n + 511) & ~size_t(255) : 0;
    const bool sorted = ray_sort != RSI_RAY_ORDER_INPUT && n > 1 && mesh->dev.nt > 0;
    const size_t ws_bytes = q_bytes + b_bytes + (sorted ? rsi::ray_sort_ws_bytes(n) : 0);
    const bool own_ws = scratch_ptr == nullptr;
    hipError_t e = hipSuccess;
    if (own_ws) {
        e = hipMallocAsync(&ws, ws_bytes, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(e == hipErrorOutOfMemory ? RSI_E_NOMEM : RSI_E_HIP,
                        std::string("hipMallocAsync failed: ") + hipGetErrorString(e));
        }
    } else {
        if (ws_bytes > scratch_cap)
            return fail(RSI_E_CAPACITY, "this call needs " + std::to_string(ws_bytes) +
                                            " bytes of scratch, more than the " + std::to_string(scratch_cap) +
                                            " the no-allocation entry point holds (4 bytes per segment, 1 more "
                                            "with the proposal and 16 more with a segment order)");
        ws = scratch_ptr;
    }
    rsi::TraverseArgs a;
    a.from = from;
    a.to = to;
    a.n = n;
    a.mode = mode;
    a.certified = precision == RSI_PRECISION_CERTIFIED;
    a.block = block;
    a.stack = stack;
    a.waves_per_cu = waves;
    a.node_width = width;
    uint64_t *ws_counters = reinterpret_cast<uint64_t *>(static_cast<char *>(ws));
    a.queue_len = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + 32);
    a.queue = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + 64);
    if (sorted) {
        a.ray_sort = ray_sort;
        a.key_bounds = mesh->dev.bounds;
        a.sort_ws = static_cast<char *>(ws) + q_bytes + b_bytes;
    }
    if (use_prop) {
        uint8_t *bucket = static_cast<uint8_t *>(ws) + q_bytes;
        e = rsi::proposal_predict(mesh->dev, mesh->dev.prop, from, to, n, mesh->dev.prop.n_buckets, bucket, s);
        if (e != hipSuccess) {
            if (own_ws)
                (void)hipFreeAsync(ws, s);
            return fail_hip(e, "proposal inference");
        }
        a.bucket = bucket;
        a.bucket_ref = mesh->dev.prop.bucket_ref;
    }
    if (stats) {
        a.visits = visits;
        a.tests = tests;
        a.counters = ws_counters;
        e = rsi::launch_stats(mesh->dev, a, s);
    } else {
        a.hit = out->hit;
        a.tri_id = out->tri_id;
        a.uvt = out->uvt;
        a.count = out->count;
        a.counters = out->counters ? out->counters : ws_counters;
        e = rsi::launch_intersect(mesh->dev, a, s);
    }
    const hipError_t e2 = own_ws ? hipFreeAsync(ws, s) : hipSuccess;
    if (e != hipSuccess)
        return fail_hip(e, stats ? "rsi_traversal_stats launch" : "rsi_intersect launch");
    if (e2 != hipSuccess)
        return fail_hip(e2, "hipFreeAsync");
    return RSI_OK;
}

rsi_status rsi_intersect(rsi_mesh mesh, const float *rays_from, const float *rays_to, int64_t n_rays, int32_t mode,
                         const rsi_intersect_opts *opts, const rsi_outputs *out, void *stream) {
    return run_rays(mesh, rays_from, rays_to, n_rays, mode, opts, out, nullptr, nullptr, stream, false);
}

rsi_status rsi_intersect_noalloc(rsi_mesh mesh, const float *rays_from, const float *rays_to, int64_t n_rays,
                                 int32_t mode, const rsi_intersect_opts *opts, const rsi_outputs *out,
                                 void *stream) {
    g_error.clear();
    // argument errors first, as rsi_intersect reports them
    rsi_status st = check_ray_args(mesh, rays_from, rays_to, n_rays, mode);
    if (st != RSI_OK)
        return st;
    if ((st = check_device()) != RSI_OK)
        return st;
    void *ptr = nullptr;
    if ((st = noalloc_scratch(&ptr)) != RSI_OK)
        return st;
    return run_rays(mesh, rays_from, rays_to, n_rays, mode, opts, out, nullptr, nullptr, stream, false, ptr,
                    kNoAllocScratchBytes);
}

rsi_status rsi_traversal_stats(rsi_mesh mesh, const float *rays_from, const float *rays_to, int64_t n_rays,
                               int32_t mode, const rsi_intersect_opts *opts, uint32_t *node_visits,
                               uint32_t *leaf_tests, void *stream) {
    return run_rays(mesh, rays_from, rays_to, n_rays, mode, opts, nullptr, node_visits, leaf_tests, stream, true);
}

// Checks shared by the derived-output entries: segments and barycentric results.
static rsi_status check_derive_args(const float *from, const float *to, int64_t n, const int32_t *tri_id,
                                    const float *uvt) {
    if (n < 0)
        return fail(RSI_E_ARG, "n_rays must be >= 0");
    if (n > 0 && (!from || !to || !tri_id || !uvt || !aligned4(from) || !aligned4(to) || !aligned4(tri_id) ||
                  !aligned4(uvt)))
        return fail(RSI_E_ARG, "rays_from, rays_to, tri_id and uvt must be non-NULL and 4-byte aligned");
    if (n > ((int64_t)1 << 31) - 1)
        return fail(RSI_E_CAPACITY, "at most 2^31 - 1 segments");
    rsi_status st = check_device();
    if (st != RSI_OK)
        return st;
    if (n > 0 && ((st = check_dev_ptr(from, "rays_from")) != RSI_OK || (st = check_dev_ptr(to, "rays_to")) != RSI_OK ||
                  (st = check_dev_ptr(tri_id, "tri_id")) != RSI_OK || (st = check_dev_ptr(uvt, "uvt")) != RSI_OK))
        return st;
    return pending_error("before a derived-output call");
}

rsi_status rsi_derive(const float *rays_from, const float *rays_to, int64_t n_rays, const int32_t *tri_id,
                      const float *uvt, float *distance, float *point, void *stream) {
    g_error.clear();
    rsi_status st = check_derive_args(rays_from, rays_to, n_rays, tri_id, uvt);
    if (st != RSI_OK)
        return st;
    if ((distance && !aligned4(distance)) || (point && !aligned4(point)))
        return fail(RSI_E_ARG, "distance / point must be 4-byte aligned");
    if (n_rays == 0 || (!distance && !point))
        return RSI_OK;
    if ((distance && (st = check_dev_ptr(distance, "distance")) != RSI_OK) ||
        (point && (st = check_dev_ptr(point, "point")) != RSI_OK))
        return st;
    const hipError_t e = rsi::launch_derive(rays_from, rays_to, n_rays, tri_id, uvt, distance, point,
                                            static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RSI_OK : fail_hip(e, "rsi_derive");
}

rsi_status rsi_compact_hits(const float *rays_from, const float *rays_to, int64_t n_rays, const int32_t *tri_id,
                            const float *uvt, int64_t *hit_index, float *distance, int32_t *hit_tri, float *point,
                            int64_t *n_hits, void *stream) {
    g_error.clear();
    rsi_status st = check_derive_args(rays_from, rays_to, n_rays, tri_id, uvt);
    if (st != RSI_OK)
        return st;
    if (!n_hits || (reinterpret_cast<uintptr_t>(n_hits) & 7u) ||
        (hit_index && (reinterpret_cast<uintptr_t>(hit_index) & 7u)) || (distance && !aligned4(distance)) ||
        (hit_tri && !aligned4(hit_tri)) || (point && !aligned4(point)))
        return fail(RSI_E_ARG, "n_hits must be non-NULL; outputs must be aligned to their element size");
    if ((st = check_dev_ptr(n_hits, "n_hits")) != RSI_OK ||
        (hit_index && (st = check_dev_ptr(hit_index, "hit_index")) != RSI_OK) ||
        (distance && (st = check_dev_ptr(distance, "distance")) != RSI_OK) ||
        (hit_tri && (st = check_dev_ptr(hit_tri, "hit_tri")) != RSI_OK) ||
        (point && (st = check_dev_ptr(point, "point")) != RSI_OK))
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, rsi::compact_ws_bytes(n_rays), s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? RSI_E_NOMEM : RSI_E_HIP,
                    std::string("hipMallocAsync failed: ") + hipGetErrorString(e));
    }
    e = rsi::launch_compact(rays_from, rays_to, n_rays, tri_id, uvt, hit_index, distance, hit_tri, point, n_hits, ws,
                            s);
    const hipError_t e2 = hipFreeAsync(ws, s);
    if (e != hipSuccess)
        return fail_hip(e, "rsi_compact_hits");
    return e2 == hipSuccess ? RSI_OK : fail_hip(e2, "hipFreeAsync");
}

rsi_status rsi_debug_certify(const float *rays_from, const float *rays_to, const float *corners, int64_t n,
                             float *values, int32_t *classes, void *stream) {
    g_error.clear();
    if (n < 0)
        return fail(RSI_E_ARG, "n must be >= 0");
    if (n == 0)
        return RSI_OK;
    if (!rays_from || !rays_to || !corners || !values || !classes || !aligned4(rays_from) || !aligned4(rays_to) ||
        !aligned4(corners) || !aligned4(values) || !aligned4(classes))
        return fail(RSI_E_ARG, "all arrays must be non-NULL and 4-byte aligned");
    rsi_status st = check_device();
    if (st != RSI_OK)
        return st;
    if ((st = check_dev_ptr(rays_from, "rays_from")) != RSI_OK || (st = check_dev_ptr(rays_to, "rays_to")) != RSI_OK ||
        (st = check_dev_ptr(corners, "corners")) != RSI_OK || (st = check_dev_ptr(values, "values")) != RSI_OK ||
        (st = check_dev_ptr(classes, "classes")) != RSI_OK)
        return st;
    if ((st = pending_error("before rsi_debug_certify")) != RSI_OK)
        return st;
    const hipError_t e = rsi::launch_debug_certify(rays_from, rays_to, corners, n, values, classes,
                                                   static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RSI_OK : fail_hip(e, "rsi_debug_certify");
}

rsi_status rsi_mesh_info_get(rsi_mesh mesh, rsi_mesh_info *info) {
    g_error.clear();
    if (!valid_mesh(mesh))
        return fail(RSI_E_STATE, "invalid or destroyed mesh handle");
    if (!info)
        return fail(RSI_E_ARG, "info must not be NULL");
    info->n_vertices = mesh->dev.nv;
    info->n_triangles = mesh->dev.nt;
    info->morton_bits = mesh->dev.morton_bits;
    info->root = mesh->dev.root;
    info->device_bytes = mesh->dev.bytes;
    info->node_width = mesh->dev.node_width;
    info->reserved = 0;
    return RSI_OK;
}

rsi_status rsi_mesh_export(rsi_mesh mesh, int32_t what, void *dst, int64_t dst_bytes, void *stream) {
    g_error.clear();
    if (!valid_mesh(mesh))
        return fail(RSI_E_STATE, "invalid or destroyed mesh handle");
    const rsi::MeshDev &d = mesh->dev;
    const int64_t nt = d.nt;
    const void *src = nullptr;
    int64_t bytes = 0;
    switch (what) {
    case RSI_EXPORT_SORTED_KEYS: bytes = 8 * nt; break;
    case RSI_EXPORT_SORTED_IDS: src = d.ids; bytes = 4 * nt; break;
    case RSI_EXPORT_NODES: src = d.nodes; bytes = nt > 1 ? 64 * (nt - 1) : 0; break;
    case RSI_EXPORT_PARENTS: src = d.parent; bytes = nt > 0 ? 4 * (2 * nt - 1) : 0; break;
    case RSI_EXPORT_COUNTERS: src = d.counters; bytes = nt > 1 ? 4 * (nt - 1) : 0; break;
    case RSI_EXPORT_LEAVES: src = d.tris; bytes = 48 * nt; break;
    case RSI_EXPORT_BOUNDS: src = d.bounds; bytes = nt > 0 ? 32 : 0; break;
    case RSI_EXPORT_WIDE_NODES: src = d.nodes4; bytes = d.node_width == 4 ? 128 * (nt - 1) : 0; break;
    case RSI_EXPORT_WIDE_TOP: src = d.top4; bytes = d.node_width == 4 ? 128 * rsi::kTopSlots : 0; break;
    default: return fail(RSI_E_ARG, "unknown export item");
    }
    if (!dst && bytes > 0)
        return fail(RSI_E_ARG, "dst must not be NULL");
    if (dst_bytes < bytes)
        return fail(RSI_E_ARG, "dst_bytes too small");
    if (bytes == 0)
        return RSI_OK;
    rsi_status st = check_device();
    if (st != RSI_OK)
        return st;
    if ((st = pending_error("before rsi_mesh_export")) != RSI_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool host_dst = !is_device_ptr(dst);
    hipError_t e = hipSuccess;
    void *tmp = nullptr;
    if (what == RSI_EXPORT_SORTED_KEYS) {
        if (d.morton_bits > 32) {
            src = d.keys;
        } else {
            e = hipMallocAsync(&tmp, 8 * nt, s);
            if (e == hipSuccess) {
                k_widen_keys<<<(int)((nt + 255) / 256), 256, 0, s>>>(static_cast<const uint32_t *>(d.keys),
                                                                    static_cast<uint64_t *>(tmp), nt);
                e = hipGetLastError();
                src = tmp;
            }
        }
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(dst, src, (size_t)bytes, hipMemcpyDefault, s);
    if (tmp)
        (void)hipFreeAsync(tmp, s);
    if (e == hipSuccess && host_dst)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail_hip(e, "rsi_mesh_export");
    return RSI_OK;
}

// ------------------------------------------------------------------ batch
constexpr uint32_t kBatchMagic = 0x52534942u;  // "RSIB"
// Segments per work item of the batched form: a wave spends about 0.35 ms on
// 512 of them, so the last items end close together (2048-segment items left
// the launch waiting on a few waves: 3.59 against 2.95 ms for 1.44e7
// segments; 256-segment items cost more in item changes than they balance).
constexpr int64_t kBatchChunk = 512;

static bool valid_batch(rsi_batch b) { return b != nullptr && b->magic == kBatchMagic; }

static bool offsets_ok(const int64_t *off, int M, int64_t limit) {
    if (!off || off[0] != 0)
        return false;
    for (int m = 0; m < M; ++m)
        if (off[m + 1] < off[m])
            return false;
    return off[M] < limit;
}

rsi_status rsi_batch_create(int32_t n_meshes, const int64_t *vertex_offsets, const int64_t *triangle_offsets,
                            const int64_t *ray_offsets, void *stream, rsi_batch *out) {
    g_error.clear();
    if (!out)
        return fail(RSI_E_ARG, "out must not be NULL");
    *out = nullptr;
    if (n_meshes < 1 || n_meshes > RSI_BATCH_MAX_MESHES)
        return fail(RSI_E_ARG, "n_meshes must be in 1..64");
    const int M = n_meshes;
    if (!offsets_ok(vertex_offsets, M, int64_t(1) << 31) || !offsets_ok(triangle_offsets, M, int64_t(1) << 30) ||
        !offsets_ok(ray_offsets, M, int64_t(1) << 31))
        return fail(RSI_E_ARG, "offsets must start at 0, not decrease, and stay below the size limits");
    rsi_status st = check_device();
    if (st != RSI_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rsi_batch bt = new (std::nothrow) rsi_batch_s();
    if (!bt)
        return fail(RSI_E_NOMEM, "host allocation failed");
    bt->magic = kBatchMagic;
    bt->stream = s;
    bt->block = nullptr;
    bt->built = false;
    rsi::MeshDev &d = bt->dev;
    rsi::BatchDev &b = bt->b;
    d.nv = vertex_offsets[M];
    d.nt = triangle_offsets[M];
    d.morton_bits = 63;
    d.root = d.nt >= 2 ? 0 : (d.nt == 1 ? ~0 : INT32_MIN);
    b.M = M;
    b.n_rays = ray_offsets[M];
    // work items of at most kBatchChunk segments, grouped per XCD: meshes go
    // to the group with the least estimated cost so far (largest first; cost
    // ~ segments x log2 triangles), each group's items mesh by mesh
    std::vector<int> order(M), group_of(M);
    std::vector<double> cost(M), load(rsi::kItemGroups, 0.0);
    for (int m = 0; m < M; ++m) {
        order[m] = m;
        cost[m] = (double)(ray_offsets[m + 1] - ray_offsets[m]) *
                  std::log2((double)(triangle_offsets[m + 1] - triangle_offsets[m]) + 2.0);
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    for (int m : order) {
        int g = 0;
        for (int h = 1; h < rsi::kItemGroups; ++h)
            g = load[h] < load[g] ? h : g;
        group_of[m] = g;
        load[g] += cost[m];
    }
    std::vector<int4> items;
    std::vector<int32_t> group_start(rsi::kItemGroups + 1, 0);
    for (int g = 0; g < rsi::kItemGroups; ++g) {
        group_start[g] = (int32_t)items.size();
        for (int m = 0; m < M; ++m)
            if (group_of[m] == g)
                for (int64_t a = ray_offsets[m]; a < ray_offsets[m + 1]; a += kBatchChunk)
                    items.push_back(make_int4(m, (int)a, (int)std::min(a + kBatchChunk, ray_offsets[m + 1]), 0));
    }
    group_start[rsi::kItemGroups] = (int32_t)items.size();
    b.n_items = (int)items.size();
    const int64_t nt = d.nt, nv = d.nv;
    const size_t sz_V = round_up(12 * (size_t)nv + 4), sz_F = round_up(12 * (size_t)nt + 4);
    const size_t sz_keys = round_up(8 * (size_t)nt + 8), sz_ids = round_up(4 * (size_t)nt + 4);
    const size_t sz_nodes = round_up(64 * (size_t)(nt > 1 ? nt - 1 : 1));
    // the 4-wide tree (top slots, then one slot per binary internal node)
    const size_t sz_nodes4 = nt > 1 ? round_up(128 * (size_t)(nt - 1 + rsi::kTopSlots)) : 0;
    const size_t sz_roots4 = round_up(4 * (size_t)M) + round_up(4 * (size_t)rsi::kTopSlots);
    // each XCD group's top and roots, and the mesh -> group map
    const size_t sz_groups = nt > 1 ? round_up(sizeof(rsi::Node4) * rsi::kItemGroups * rsi::kTopSlots) +
                                          round_up(4 * 64 * rsi::kItemGroups) + round_up(4 * (size_t)M)
                                    : 0;
    const size_t sz_par = round_up(4 * (size_t)(nt > 0 ? 2 * nt - 1 : 1)), sz_cnt = round_up(4 * (size_t)(nt > 1 ? nt - 1 : 1));
    const size_t sz_tris = round_up(48 * (size_t)nt + 48), sz_small = 256;
    const size_t sz_tmp = round_up(rsi::sort_tmp_bytes(nt, 63));
    const size_t sz_off = round_up(8 * (size_t)(M + 1)) * 2 + round_up(4 * (size_t)(M + 1)) + round_up(4 * (size_t)M) * 2;
    const size_t sz_tm = round_up(4 * (size_t)nt + 4), sz_mb = round_up(32 * (size_t)M);
    const size_t sz_items = round_up(16 * (size_t)(b.n_items + 1)) + round_up(4 * (rsi::kItemGroups + 1));
    const size_t sz_q = round_up(4 * (size_t)b.n_rays + 4) + 256;
    const size_t sz_order = round_up(rsi::ray_sort_ws_bytes(b.n_rays));
    const size_t total = sz_V + sz_F + sz_keys + sz_ids + sz_nodes + sz_nodes4 + sz_roots4 + sz_groups + sz_par + sz_cnt +
                         sz_tris + sz_small + sz_tmp + sz_off + sz_tm + sz_mb + sz_items + sz_q + sz_order;
    hipError_t e = hipMallocAsync(&bt->block, total, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        bt->magic = kDead;
        delete bt;
        return fail(RSI_E_NOMEM, std::string("hipMallocAsync failed: ") + hipGetErrorString(e));
    }
    char *p = static_cast<char *>(bt->block);
    auto take = [&](size_t bytes) {
        char *q = p;
        p += bytes;
        return q;
    };
    d.V = reinterpret_cast<float *>(take(sz_V));
    d.F = reinterpret_cast<int32_t *>(take(sz_F));
    d.keys = take(sz_keys);
    d.ids = reinterpret_cast<int32_t *>(take(sz_ids));
    d.nodes = reinterpret_cast<rsi::Node *>(take(sz_nodes));
    d.top4 = sz_nodes4 ? reinterpret_cast<rsi::Node4 *>(take(sz_nodes4)) : nullptr;
    d.nodes4 = d.top4 ? d.top4 + rsi::kTopSlots : nullptr;
    b.roots4 = reinterpret_cast<int32_t *>(take(round_up(4 * (size_t)M)));
    b.slot_bin = reinterpret_cast<int32_t *>(take(round_up(4 * (size_t)rsi::kTopSlots)));
    if (sz_groups) {
        b.top4g = reinterpret_cast<rsi::Node4 *>(take(round_up(sizeof(rsi::Node4) * rsi::kItemGroups * rsi::kTopSlots)));
        b.roots4g = reinterpret_cast<int32_t *>(take(round_up(4 * 64 * rsi::kItemGroups)));
        b.mesh_group = reinterpret_cast<int32_t *>(take(round_up(4 * (size_t)M)));
    }
    d.parent = reinterpret_cast<int32_t *>(take(sz_par));
    d.counters = reinterpret_cast<int32_t *>(take(sz_cnt));
    d.tris = reinterpret_cast<rsi::Tri *>(take(sz_tris));
    char *small = take(sz_small);
    d.bounds = reinterpret_cast<float *>(small);
    d.flags = reinterpret_cast<int32_t *>(small + 64);
    d.sort_tmp = take(sz_tmp);
    b.v_off = reinterpret_cast<int64_t *>(take(round_up(8 * (size_t)(M + 1))));
    b.t_off = reinterpret_cast<int64_t *>(take(round_up(8 * (size_t)(M + 1))));
    b.r_off = reinterpret_cast<int32_t *>(take(round_up(4 * (size_t)(M + 1))));
    b.mesh_toff = reinterpret_cast<int32_t *>(take(round_up(4 * (size_t)M)));
    b.roots = reinterpret_cast<int32_t *>(take(round_up(4 * (size_t)M)));
    b.tri_mesh = reinterpret_cast<int32_t *>(take(sz_tm));
    b.mesh_bounds = reinterpret_cast<float *>(take(sz_mb));
    b.items = reinterpret_cast<int4 *>(take(round_up(16 * (size_t)(b.n_items + 1))));
    b.group_start = reinterpret_cast<int32_t *>(take(round_up(4 * (rsi::kItemGroups + 1))));
    char *q = take(sz_q);
    b.counters = reinterpret_cast<uint64_t *>(q);
    b.queue_len = reinterpret_cast<uint32_t *>(q + 32);
    b.queue = reinterpret_cast<int32_t *>(q + 256);
    b.sort_ws = take(sz_order);
    d.bytes = (int64_t)total;
    std::vector<int32_t> r32(M + 1), toff(M);
    for (int m = 0; m <= M; ++m)
        r32[m] = (int32_t)ray_offsets[m];
    for (int m = 0; m < M; ++m)
        toff[m] = (int32_t)triangle_offsets[m];
    e = hipMemcpyAsync(b.v_off, vertex_offsets, 8 * (size_t)(M + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.t_off, triangle_offsets, 8 * (size_t)(M + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.r_off, r32.data(), 4 * (size_t)(M + 1), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.mesh_toff, toff.data(), 4 * (size_t)M, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && b.n_items > 0)
        e = hipMemcpyAsync(b.items, items.data(), 16 * (size_t)b.n_items, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b.group_start, group_start.data(), 4 * (size_t)(rsi::kItemGroups + 1),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && b.mesh_group)
        e = hipMemcpyAsync(b.mesh_group, group_of.data(), 4 * (size_t)M, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);  // the host vectors go out of scope
    if (e != hipSuccess) {
        rsi_batch_destroy(bt);
        return fail_hip(e, "rsi_batch_create");
    }
    *out = bt;
    return RSI_OK;
}

rsi_status rsi_batch_build(rsi_batch batch, const float *vertices, const int32_t *triangles, void *stream) {
    g_error.clear();
    if (!valid_batch(batch))
        return fail(RSI_E_STATE, "invalid or destroyed batch handle");
    rsi::MeshDev &d = batch->dev;
    if ((d.nv > 0 && (!vertices || !aligned4(vertices))) || (d.nt > 0 && (!triangles || !aligned4(triangles))))
        return fail(RSI_E_ARG, "vertices / triangles must be non-NULL and 4-byte aligned");
    rsi_status st = check_device();
    if (st != RSI_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    note_capture(s);
    if ((d.nv > 0 && (st = check_dev_ptr(vertices, "vertices")) != RSI_OK) ||
        (d.nt > 0 && (st = check_dev_ptr(triangles, "triangles")) != RSI_OK))
        return st;
    if ((st = pending_error("before rsi_batch_build")) != RSI_OK)
        return st;
    hipError_t e = rsi::launch_batch_build(d, batch->b, vertices, triangles, s);
    if (e != hipSuccess)
        return fail_hip(e, "rsi_batch_build");
    batch->built = true;
    return RSI_OK;
}

rsi_status rsi_batch_intersect(rsi_batch batch, const float *rays_from, const float *rays_to, int32_t mode,
                               const rsi_intersect_opts *opts, const rsi_outputs *out, void *stream) {
    g_error.clear();
    if (!valid_batch(batch))
        return fail(RSI_E_STATE, "invalid or destroyed batch handle");
    if (!batch->built)
        return fail(RSI_E_STATE, "rsi_batch_build has not been called");
    rsi::BatchDev &b = batch->b;
    const int64_t n = b.n_rays;
    if (mode != RSI_MODE_BOOLEAN && mode != RSI_MODE_FIRST_HIT && mode != RSI_MODE_BARYCENTRIC &&
        mode != RSI_MODE_INTERCEPT_COUNT)
        return fail(RSI_E_ARG, "unknown mode");
    int precision, block, stack, ray_sort, waves, width;
    rsi_status st = parse_intersect_opts(opts, precision, block, stack, ray_sort, waves, width);
    if (st != RSI_OK)
        return st;
    if (opts && opts->proposal)
        return fail(RSI_E_ARG, "the batched form has no learned proposal");
    if (width == 4 && batch->dev.node_width != 4)
        return fail(RSI_E_ARG, "node_width = 4 needs a batch of more than one triangle");
    if (!out)
        return fail(RSI_E_ARG, "out must not be NULL");
    if (n > 0 && (!rays_from || !rays_to || !aligned4(rays_from) || !aligned4(rays_to)))
        return fail(RSI_E_ARG, "rays_from / rays_to must be non-NULL and 4-byte aligned");
    if (n > 0 && ((mode == RSI_MODE_BOOLEAN && !out->hit) ||
                  ((mode == RSI_MODE_FIRST_HIT || mode == RSI_MODE_BARYCENTRIC) && !out->tri_id) ||
                  (mode == RSI_MODE_BARYCENTRIC && !out->uvt) || (mode == RSI_MODE_INTERCEPT_COUNT && !out->count)))
        return fail(RSI_E_ARG, "missing output buffer for this mode");
    if ((st = check_device()) != RSI_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    note_capture(s);
    if (n > 0 && ((st = check_dev_ptr(rays_from, "rays_from")) != RSI_OK ||
                  (st = check_dev_ptr(rays_to, "rays_to")) != RSI_OK))
        return st;
    if ((st = pending_error("before rsi_batch_intersect")) != RSI_OK)
        return st;
    rsi::TraverseArgs a;
    a.from = rays_from;
    a.to = rays_to;
    a.n = n;
    a.mode = mode;
    a.certified = precision == RSI_PRECISION_CERTIFIED;
    a.block = block;
    a.stack = stack;
    a.waves_per_cu = waves;
    a.node_width = width;
    a.hit = out->hit;
    a.tri_id = out->tri_id;
    a.uvt = out->uvt;
    a.count = out->count;
    a.counters = out->counters ? out->counters : b.counters;
    a.queue = b.queue;
    a.queue_len = b.queue_len;
    a.items = b.items;
    a.n_items = b.n_items;
    a.group_start = b.group_start;
    a.n_groups = rsi::kItemGroups;
    a.n_meshes = b.M;
    a.mesh_root = b.roots;
    a.mesh_root4 = batch->dev.node_width == 4 ? b.roots4 : nullptr;
    a.top4g = batch->dev.node_width == 4 ? b.top4g : nullptr;
    a.roots4g = b.roots4g;
    a.mesh_toff = b.mesh_toff;
    a.ray_off = b.r_off;
    if (ray_sort != RSI_RAY_ORDER_INPUT) {
        a.ray_sort = ray_sort;
        a.key_bounds = b.mesh_bounds;
        a.sort_ws = b.sort_ws;
    }
    hipError_t e = rsi::launch_intersect(batch->dev, a, s);
    return e == hipSuccess ? RSI_OK : fail_hip(e, "rsi_batch_intersect");
}

rsi_status rsi_batch_export(rsi_batch batch, int32_t what, void *dst, int64_t dst_bytes, void *stream) {
    g_error.clear();
    if (!valid_batch(batch))
        return fail(RSI_E_STATE, "invalid or destroyed batch handle");
    if (what == RSI_EXPORT_MESH_ROOTS) {
        const int64_t bytes = 4 * (int64_t)batch->b.M;
        if (!dst || dst_bytes < bytes)
            return fail(RSI_E_ARG, "dst too small");
        rsi_status st = check_device();
        if (st != RSI_OK)
            return st;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const bool host_dst = !is_device_ptr(dst);
        hipError_t e = hipMemcpyAsync(dst, batch->b.roots, (size_t)bytes, hipMemcpyDefault, s);
        if (e == hipSuccess && host_dst)
            e = hipStreamSynchronize(s);
        return e == hipSuccess ? RSI_OK : fail_hip(e, "rsi_batch_export");
    }
    // the other items come from the combined BVH, exported like a mesh
    rsi_mesh_s view;
    view.magic = kMagic;
    view.dev = batch->dev;
    view.stream = batch->stream;
    view.block = nullptr;
    rsi_status st = rsi_mesh_export(&view, what, dst, dst_bytes, stream);
    view.magic = kDead;
    return st;
}

rsi_status rsi_batch_destroy(rsi_batch batch) {
    if (!batch)
        return RSI_OK;
    if (batch->magic != kBatchMagic)
        return fail(RSI_E_STATE, "invalid or destroyed batch handle");
    batch->magic = kDead;
    hipError_t e = hipSuccess;
    if (batch->block)
        e = hipFreeAsync(batch->block, batch->stream);
    delete batch;
    return e == hipSuccess ? RSI_OK : fail_hip(e, "rsi_batch_destroy");
}

// ------------------------------------------------------------------ proposal
static rsi_status ensure_proposal(rsi_mesh mesh, hipStream_t s, uint64_t seed, bool reinit) {
    rsi::MeshDev &d = mesh->dev;
    rsi::Proposal &pr = d.prop;
    if (d.nt < 1)
        return fail(RSI_E_STATE, "the proposal needs a mesh with at least one triangle");
    if (!pr.block) {
        const size_t f = round_up(4 * (size_t)rsi::kMlpParams);
        const size_t wb = round_up(2 * (size_t)rsi::kMlpWeights);
        const size_t wbt = round_up(2 * 3 * (size_t)rsi::kMlpHidden * rsi::kMlpHidden);
        const size_t small = round_up(4 * 256) * 2 + 256;
        const size_t rk = round_up(4 * (size_t)d.nt), lbk = round_up((size_t)d.nt);
        // the proposal order's 4-wide tree, where the mesh has one
        const bool wide = d.node_width == 4 && d.nt > 1;
        const size_t w4 = wide ? sizeof(rsi::Node4) * (size_t)(rsi::kTopSlots + d.nt - 1) : 0;
        const size_t wsmall = wide ? round_up(4 * 256) + round_up(4 * rsi::kTopSlots) + 2 * rk : 0;
        hipError_t e = hipMallocAsync(&pr.block, 4 * f + wb + wbt + small + rk + lbk + w4 + wsmall, s);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            pr.block = nullptr;
            return fail(RSI_E_NOMEM, std::string("proposal allocation: ") + hipGetErrorString(e));
        }
        char *p = static_cast<char *>(pr.block);
        pr.P = reinterpret_cast<float *>(p); p += f;
        pr.G = reinterpret_cast<float *>(p); p += f;
        pr.m1 = reinterpret_cast<float *>(p); p += f;
        pr.m2 = reinterpret_cast<float *>(p); p += f;
        pr.Wb = reinterpret_cast<__bf16 *>(p); p += wb;
        pr.WbT = reinterpret_cast<__bf16 *>(p); p += wbt;
        pr.bucket_ref = reinterpret_cast<int32_t *>(p); p += round_up(4 * 256);
        pr.bucket_first = reinterpret_cast<int32_t *>(p); p += round_up(4 * 256);
        pr.dev_n_buckets = reinterpret_cast<int32_t *>(p); p += 256;
        pr.rank = reinterpret_cast<int32_t *>(p); p += rk;
        pr.leaf_bucket = reinterpret_cast<uint8_t *>(p); p += lbk;
        if (wide) {
            pr.top4 = reinterpret_cast<rsi::Node4 *>(p); p += w4;
            pr.bucket_ref4 = reinterpret_cast<int32_t *>(p); p += round_up(4 * 256);
            pr.slot_bin = reinterpret_cast<int32_t *>(p); p += round_up(4 * rsi::kTopSlots);
            pr.wide_flag = reinterpret_cast<int32_t *>(p); p += rk;
            pr.wide_queue = reinterpret_cast<int32_t *>(p);
        }
        e = rsi::proposal_frontier(d, pr, s);
        if (e == hipSuccess && wide)
            e = rsi::launch_collapse_proposal(d, pr, s);
        int32_t nb = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&nb, pr.dev_n_buckets, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            return fail_hip(e, "proposal frontier");
        pr.n_buckets = nb;
    }
    if (!pr.ready || reinit) {
        hipError_t e = rsi::proposal_init(pr, seed, s);
        if (e != hipSuccess)
            return fail_hip(e, "proposal init");
        pr.ready = true;
        pr.step = 0;
    }
    return RSI_OK;
}

static rsi_status prop_args(rsi_mesh mesh, const float *from, const float *to, int64_t n) {
    if (!valid_mesh(mesh))
        return fail(RSI_E_STATE, "invalid or destroyed mesh handle");
    if (mesh->dev.nt < 1)
        return fail(RSI_E_STATE, "the proposal needs a mesh with at least one triangle");
    if (n < 0)
        return fail(RSI_E_ARG, "n_rays must be >= 0");
    if (n >= (int64_t(1) << 31))
        return fail(RSI_E_CAPACITY, "n_rays must be < 2^31");
    if (n > 0 && (!from || !to || !aligned4(from) || !aligned4(to)))
        return fail(RSI_E_ARG, "rays_from / rays_to must be non-NULL and 4-byte aligned");
    rsi_status st = check_device();
    if (st != RSI_OK)
        return st;
    if (n > 0 && ((st = check_dev_ptr(from, "rays_from")) != RSI_OK || (st = check_dev_ptr(to, "rays_to")) != RSI_OK))
        return st;
    return pending_error("before a proposal call");
}

rsi_status rsi_proposal_train(rsi_mesh mesh, const float *rays_from, const float *rays_to, int64_t n_rays,
                              const rsi_train_opts *opts, float *epoch_loss, int64_t *n_labelled, void *stream) {
    g_error.clear();
    rsi_status st = prop_args(mesh, rays_from, rays_to, n_rays);
    if (st != RSI_OK)
        return st;
    int epochs = 2, batch = 4096, reinit = 0;
    float lr = 1e-3f;
    uint64_t seed = 1;
    if (opts) {
        if (opts->epochs < 0 || opts->batch < 0 || opts->lr < 0.0f)
            return fail(RSI_E_ARG, "epochs, batch and lr must be >= 0");
        if (opts->batch != 0 && (opts->batch < 64 || opts->batch > 65536))
            return fail(RSI_E_ARG, "batch must be in 64..65536");
        if (opts->epochs)
            epochs = opts->epochs;
        if (opts->batch)
            batch = opts->batch;
        if (opts->lr > 0.0f)
            lr = opts->lr;
        reinit = opts->reinit;
        seed = opts->seed;
    }
    if (epoch_loss && (st = check_dev_ptr(epoch_loss, "epoch_loss")) != RSI_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = ensure_proposal(mesh, s, seed, reinit != 0)) != RSI_OK)
        return st;
    rsi::Proposal &pr = mesh->dev.prop;
    // labels from the exact first-hit pass
    void *tmp = nullptr;
    const size_t scratch = rsi::proposal_batch_scratch(batch);
    const size_t lab_bytes = round_up(rsi::proposal_label_scratch(n_rays));
    const size_t tmp_bytes = round_up(12 * (size_t)n_rays + 64) + scratch + round_up(4 * (size_t)epochs + 4) + lab_bytes;
    hipError_t e = hipMallocAsync(&tmp, tmp_bytes, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RSI_E_NOMEM, std::string("training scratch: ") + hipGetErrorString(e));
    }
    char *t = static_cast<char *>(tmp);
    int32_t *tri = reinterpret_cast<int32_t *>(t);
    int32_t *seg = tri + n_rays;
    int32_t *lab = seg + n_rays;
    uint32_t *count = reinterpret_cast<uint32_t *>(lab + n_rays);
    char *ws = t + round_up(12 * (size_t)n_rays + 64);
    float *loss_sink = reinterpret_cast<float *>(ws + scratch);
    int32_t *lab_blk = reinterpret_cast<int32_t *>(ws + scratch + round_up(4 * (size_t)epochs + 4));
    auto bail = [&](rsi_status code) {
        (void)hipFreeAsync(tmp, s);
        return code;
    };
    rsi_intersect_opts io{RSI_PRECISION_CERTIFIED, 0, 0, 0, 0};
    rsi_outputs out{nullptr, tri, nullptr, nullptr};
    if ((st = rsi_intersect(mesh, rays_from, rays_to, n_rays, RSI_MODE_FIRST_HIT, &io, &out, stream)) != RSI_OK)
        return bail(st);
    uint32_t n_lab = 0;
    e = hipMemsetAsync(count, 0, 4, s);
    if (e == hipSuccess && n_rays > 0)
        e = rsi::proposal_labels(mesh->dev, pr, tri, n_rays, seg, lab, count, lab_blk, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(&n_lab, count, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        bail(RSI_OK);
        return fail_hip(e, "proposal labels");
    }
    if (n_labelled)
        *n_labelled = n_lab;
    if (epoch_loss)
        e = hipMemsetAsync(epoch_loss, 0, 4 * (size_t)epochs, s);
    for (int ep = 0; ep < epochs && e == hipSuccess; ++ep) {
        const int64_t nbatches = (n_lab + batch - 1) / batch;
        for (int64_t b = 0; b < nbatches && e == hipSuccess; ++b) {
            const int64_t r0 = b * batch;
            const int rows = (int)(n_lab - r0 < batch ? n_lab - r0 : batch);
            // each batch adds (its mean loss) * rows / n_lab: the epoch's mean loss
            const rsi::AdamStep step{lr, (int)(++pr.step)};
            e = rsi::proposal_batch_grad(mesh->dev, pr, rays_from, rays_to, seg, lab, r0, rows, pr.n_buckets,
                                         epoch_loss ? epoch_loss + ep : loss_sink, 1.0f / (float)n_lab, ws, s,
                                         nullptr, &step);
        }
    }
    if (e != hipSuccess) {
        bail(RSI_OK);
        return fail_hip(e, "proposal training");
    }
    (void)hipFreeAsync(tmp, s);
    return RSI_OK;
}

rsi_status rsi_proposal_predict(rsi_mesh mesh, const float *rays_from, const float *rays_to, int64_t n_rays,
                                uint8_t *bucket, void *stream) {
    g_error.clear();
    rsi_status st = prop_args(mesh, rays_from, rays_to, n_rays);
    if (st != RSI_OK)
        return st;
    if (!mesh->dev.prop.ready)
        return fail(RSI_E_STATE, "no trained or loaded proposal");
    if (n_rays > 0 && (!bucket || (st = check_dev_ptr(bucket, "bucket")) != RSI_OK))
        return bucket ? st : fail(RSI_E_ARG, "bucket must not be NULL");
    hipError_t e = rsi::proposal_predict(mesh->dev, mesh->dev.prop, rays_from, rays_to, n_rays,
                                         mesh->dev.prop.n_buckets, bucket, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RSI_OK : fail_hip(e, "rsi_proposal_predict");
}

rsi_status rsi_proposal_params(rsi_mesh mesh, int32_t what, float *buf, void *stream) {
    g_error.clear();
    rsi_status st = prop_args(mesh, nullptr, nullptr, 0);
    if (st != RSI_OK)
        return st;
    if (what != 0 && what != 1)
        return fail(RSI_E_ARG, "what must be 0 (get) or 1 (set)");
    if (!buf || (st = check_dev_ptr(buf, "buf")) != RSI_OK)
        return buf ? st : fail(RSI_E_ARG, "buf must not be NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (what == 0 && !mesh->dev.prop.ready)
        return fail(RSI_E_STATE, "no trained or loaded proposal");
    if ((st = ensure_proposal(mesh, s, 1, false)) != RSI_OK)
        return st;
    rsi::Proposal &pr = mesh->dev.prop;
    const size_t bytes = 4 * (size_t)rsi::kMlpParams;
    hipError_t e;
    if (what == 0) {
        e = hipMemcpyAsync(buf, pr.P, bytes, hipMemcpyDeviceToDevice, s);
    } else {
        e = hipMemcpyAsync(pr.P, buf, bytes, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemsetAsync(pr.m1, 0, bytes, s);
        if (e == hipSuccess)
            e = hipMemsetAsync(pr.m2, 0, bytes, s);
        if (e == hipSuccess)
            e = rsi::proposal_set_params(pr, s);
        pr.step = 0;
        pr.ready = true;
    }
    return e == hipSuccess ? RSI_OK : fail_hip(e, "rsi_proposal_params");
}

rsi_status rsi_proposal_gradient(rsi_mesh mesh, const float *rays_from, const float *rays_to, const int32_t *labels,
                                 int64_t n_rays, float *grad, float *logits, float *loss, void *stream) {
    g_error.clear();
    rsi_status st = prop_args(mesh, rays_from, rays_to, n_rays);
    if (st != RSI_OK)
        return st;
    if (n_rays < 1 || n_rays > 65536)
        return fail(RSI_E_ARG, "n_rays must be in 1..65536");
    if (!mesh->dev.prop.ready)
        return fail(RSI_E_STATE, "no trained or loaded proposal");
    if (!labels || !grad || !logits || !loss)
        return fail(RSI_E_ARG, "labels, grad, logits and loss must not be NULL");
    if ((st = check_dev_ptr(labels, "labels")) != RSI_OK || (st = check_dev_ptr(grad, "grad")) != RSI_OK ||
        (st = check_dev_ptr(logits, "logits")) != RSI_OK || (st = check_dev_ptr(loss, "loss")) != RSI_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rsi::Proposal &pr = mesh->dev.prop;
    void *ws = nullptr;
    hipError_t e = hipMallocAsync(&ws, rsi::proposal_batch_scratch((int)n_rays), s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(RSI_E_NOMEM, "gradient scratch");
    }
    e = hipMemsetAsync(loss, 0, 4, s);
    if (e == hipSuccess)
        e = rsi::proposal_batch_grad(mesh->dev, pr, rays_from, rays_to, nullptr, labels, 0, (int)n_rays,
                                     pr.n_buckets, loss, 0.0f, static_cast<char *>(ws), s, logits, nullptr);
    if (e == hipSuccess)
        e = hipMemcpyAsync(grad, pr.G, 4 * (size_t)rsi::kMlpParams, hipMemcpyDeviceToDevice, s);
    (void)hipFreeAsync(ws, s);
    return e == hipSuccess ? RSI_OK : fail_hip(e, "rsi_proposal_gradient");
}

rsi_status rsi_proposal_features(rsi_mesh mesh, const float *rays_from, const float *rays_to, int64_t n_rays,
                                 uint16_t *features, void *stream) {
    g_error.clear();
    rsi_status st = prop_args(mesh, rays_from, rays_to, n_rays);
    if (st != RSI_OK)
        return st;
    if (n_rays > 0 && (!features || (st = check_dev_ptr(features, "features")) != RSI_OK))
        return features ? st : fail(RSI_E_ARG, "features must not be NULL");
    hipError_t e = rsi::proposal_features(mesh->dev, rays_from, rays_to, n_rays, reinterpret_cast<__bf16 *>(features),
                                          static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RSI_OK : fail_hip(e, "rsi_proposal_features");
}

rsi_status rsi_proposal_frontier(rsi_mesh mesh, int32_t *bucket_ref, int32_t *bucket_first, int32_t *n_buckets,
                                 void *stream) {
    g_error.clear();
    rsi_status st = prop_args(mesh, nullptr, nullptr, 0);
    if (st != RSI_OK)
        return st;
    if (!bucket_ref || !bucket_first || !n_buckets)
        return fail(RSI_E_ARG, "outputs must not be NULL");
    if ((st = check_dev_ptr(bucket_ref, "bucket_ref")) != RSI_OK ||
        (st = check_dev_ptr(bucket_first, "bucket_first")) != RSI_OK)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rsi::Proposal &pr = mesh->dev.prop;
    const bool had = pr.ready;
    if ((st = ensure_proposal(mesh, s, 1, false)) != RSI_OK)
        return st;
    pr.ready = had || pr.ready;
    hipError_t e = hipMemcpyAsync(bucket_ref, pr.bucket_ref, 4 * 256, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bucket_first, pr.bucket_first, 4 * 256, hipMemcpyDeviceToDevice, s);
    *n_buckets = pr.n_buckets;
    return e == hipSuccess ? RSI_OK : fail_hip(e, "rsi_proposal_frontier");
}

namespace {
struct PropHeader {
    char magic[8];
    int32_t inputs, hidden, outputs, layers;
    int64_t params, step, n_triangles;
    int32_t n_buckets, reserved;
};
}  // namespace

rsi_status rsi_proposal_save(rsi_mesh mesh, const char *path) {
    g_error.clear();
    rsi_status st = prop_args(mesh, nullptr, nullptr, 0);
    if (st != RSI_OK)
        return st;
    if (!path)
        return fail(RSI_E_ARG, "path must not be NULL");
    rsi::Proposal &pr = mesh->dev.prop;
    if (!pr.ready)
        return fail(RSI_E_STATE, "no trained or loaded proposal");
    const size_t np = (size_t)rsi::kMlpParams;
    std::string buf(3 * 4 * np, '\0');
    hipError_t e = hipStreamSynchronize(mesh->stream);
    if (e == hipSuccess)
        e = hipMemcpy(&buf[0], pr.P, 4 * np, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(&buf[4 * np], pr.m1, 4 * np, hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(&buf[8 * np], pr.m2, 4 * np, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return fail_hip(e, "rsi_proposal_save");
    PropHeader h{{'R', 'S', 'I', 'M', 'L', 'P', '0', '1'}, rsi::kMlpIn, rsi::kMlpHidden, rsi::kMlpOut, 4,
                 rsi::kMlpParams, pr.step, mesh->dev.nt, pr.n_buckets, 0};
    FILE *f = std::fopen(path, "wb");
    if (!f)
        return fail(RSI_E_ARG, std::string("cannot open ") + path);
    const bool ok = std::fwrite(&h, sizeof h, 1, f) == 1 && std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
    std::fclose(f);
    return ok ? RSI_OK : fail(RSI_E_ARG, std::string("short write to ") + path);
}

rsi_status rsi_proposal_load(rsi_mesh mesh, const char *path) {
    g_error.clear();
    rsi_status st = prop_args(mesh, nullptr, nullptr, 0);
    if (st != RSI_OK)
        return st;
    if (!path)
        return fail(RSI_E_ARG, "path must not be NULL");
    FILE *f = std::fopen(path, "rb");
    if (!f)
        return fail(RSI_E_ARG, std::string("cannot open ") + path);
    PropHeader h;
    const size_t np = (size_t)rsi::kMlpParams;
    std::string buf(3 * 4 * np, '\0');
    const bool ok = std::fread(&h, sizeof h, 1, f) == 1 && std::fread(&buf[0], 1, buf.size(), f) == buf.size();
    std::fclose(f);
    if (!ok || std::memcmp(h.magic, "RSIMLP01", 8) != 0 || h.inputs != rsi::kMlpIn || h.hidden != rsi::kMlpHidden ||
        h.outputs != rsi::kMlpOut || h.params != rsi::kMlpParams)
        return fail(RSI_E_ARG, std::string(path) + " is not a proposal file of this network");
    hipStream_t s = mesh->stream;
    if ((st = ensure_proposal(mesh, s, 1, false)) != RSI_OK)
        return st;
    rsi::Proposal &pr = mesh->dev.prop;
    if (h.n_triangles != mesh->dev.nt || h.n_buckets != pr.n_buckets)
        return fail(RSI_E_ARG, "proposal file was trained on a different mesh");
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = hipMemcpy(pr.P, &buf[0], 4 * np, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(pr.m1, &buf[4 * np], 4 * np, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(pr.m2, &buf[8 * np], 4 * np, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = rsi::proposal_set_params(pr, s);
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return fail_hip(e, "rsi_proposal_load");
    pr.step = h.step;
    pr.ready = true;
    return RSI_OK;
}

rsi_status rsi_stream_copy(void *dst, const void *src, int64_t bytes, void *stream) {
    g_error.clear();
    if (bytes < 0 || (bytes & 15) != 0)
        return fail(RSI_E_ARG, "bytes must be a non-negative multiple of 16");
    if (bytes == 0)
        return RSI_OK;
    if (!dst || !src || (reinterpret_cast<uintptr_t>(dst) & 15u) || (reinterpret_cast<uintptr_t>(src) & 15u))
        return fail(RSI_E_ARG, "dst / src must be non-NULL and 16-byte aligned");
    rsi_status st = check_device();
    if (st != RSI_OK)
        return st;
    if ((st = check_dev_ptr(dst, "dst")) != RSI_OK || (st = check_dev_ptr(src, "src")) != RSI_OK)
        return st;
    if ((st = pending_error("before rsi_stream_copy")) != RSI_OK)
        return st;
    const hipError_t e = rsi::launch_stream_copy(dst, src, bytes / 16, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? RSI_OK : fail_hip(e, "rsi_stream_copy launch");
}

const char *rsi_status_string(rsi_status status) {
    switch (status) {
    case RSI_OK: return "RSI_OK";
    case RSI_E_ARG: return "RSI_E_ARG: invalid argument";
    case RSI_E_RANGE: return "RSI_E_RANGE: triangle index out of range";
    case RSI_E_NOMEM: return "RSI_E_NOMEM: device memory exhausted";
    case RSI_E_HIP: return "RSI_E_HIP: HIP runtime error";
    case RSI_E_STATE: return "RSI_E_STATE: no usable device or invalid handle";
    case RSI_E_CAPACITY: return "RSI_E_CAPACITY: size beyond the supported limit";
    }
    return "unknown rsi_status";
}

const char *rsi_last_error(void) { return g_error.c_str(); }

int32_t rsi_abi_version(void) { return RSI_ABI_VERSION; }

}  // extern "C"
