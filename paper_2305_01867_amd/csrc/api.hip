// api.hip -- the C ABI declared in include/rsi.h: argument checks, device
// memory, stream-ordered launches and error reporting.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "rsi.h"
#include "rsi_internal.h"

struct rsi_mesh_s {
    uint32_t magic;
    rsi::MeshDev dev;
    hipStream_t stream;  // the stream the mesh was built on (used to free it)
    void *block;         // the one device allocation holding every array
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
    // the driver at every synchronisation
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t keep = UINT64_MAX;
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
    checked_dev = dev;
    return RSI_OK;
}

bool is_device_ptr(const void *p) {
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

rsi_status parse_intersect_opts(const rsi_intersect_opts *opts, int &precision, int &block, int &stack) {
    precision = RSI_PRECISION_PLAIN;
    block = 256;
    stack = 20;
    if (!opts)
        return RSI_OK;
    if (opts->precision != RSI_PRECISION_PLAIN && opts->precision != RSI_PRECISION_CERTIFIED)
        return fail(RSI_E_ARG, "precision must be RSI_PRECISION_PLAIN or RSI_PRECISION_CERTIFIED");
    precision = opts->precision;
    if (opts->block != 0) {
        if (opts->block != 64 && opts->block != 128 && opts->block != 256)
            return fail(RSI_E_ARG, "block must be 64, 128 or 256");
        block = opts->block;
    }
    if (opts->stack_depth != 0) {
        if (opts->stack_depth < 1 || opts->stack_depth > 64)
            return fail(RSI_E_ARG, "stack_depth must be in 1..64");
        stack = opts->stack_depth;
    }
    if (opts->ray_sort != 0)
        return fail(RSI_E_ARG, "ray_sort: only 0 (input order) is available");
    if (opts->proposal != 0)
        return fail(RSI_E_ARG, "proposal: only 0 (none) is available");
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
    if (mode != RSI_MODE_BOOLEAN && mode != RSI_MODE_FIRST_HIT && mode != RSI_MODE_BARYCENTRIC)
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
    int bits = 30, check = 0;
    if (opts) {
        if (opts->morton_bits != 0 && opts->morton_bits != 30 && opts->morton_bits != 63)
            return fail(RSI_E_ARG, "morton_bits must be 30 or 63");
        if (opts->morton_bits)
            bits = opts->morton_bits;
        check = opts->check_indices != 0;
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
    const size_t sz_par = round_up(4 * (size_t)(2 * nt - 1)), sz_cnt = round_up(4 * (size_t)(nt > 1 ? nt - 1 : 1));
    const size_t sz_tris = round_up(48 * (size_t)nt), sz_small = 256;
    const size_t sz_tmp = round_up(rsi::sort_tmp_bytes(nt, bits));
    const size_t total = sz_V + sz_F + sz_keys + sz_ids + sz_nodes + sz_par + sz_cnt + sz_tris + sz_small + sz_tmp;
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
    d.parent = reinterpret_cast<int32_t *>(take(sz_par));
    d.counters = reinterpret_cast<int32_t *>(take(sz_cnt));
    d.tris = reinterpret_cast<rsi::Tri *>(take(sz_tris));
    char *small = take(sz_small);
    d.bounds = reinterpret_cast<float *>(small);
    d.flags = reinterpret_cast<int32_t *>(small + 64);
    d.sort_tmp = take(sz_tmp);
    d.bytes = (int64_t)total;

    if (n_vertices > 0)
        e = hipMemcpyAsync(d.V, vertices, 12 * (size_t)n_vertices, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d.F, triangles, 12 * (size_t)nt, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess)
        e = rsi::launch_build(d, vertices, triangles, s, sz_tmp);
    if (e != hipSuccess) {
        rsi_destroy(m);
        return fail_hip(e, "rsi_build launch");
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
    if (mesh->block)
        e = hipFreeAsync(mesh->block, mesh->stream);
    delete mesh;
    if (e != hipSuccess)
        return fail_hip(e, "rsi_destroy");
    return RSI_OK;
}

static rsi_status run_rays(rsi_mesh mesh, const float *from, const float *to, int64_t n, int32_t mode,
                           const rsi_intersect_opts *opts, const rsi_outputs *out, uint32_t *visits,
                           uint32_t *tests, void *stream, bool stats) {
    g_error.clear();
    rsi_status st = check_ray_args(mesh, from, to, n, mode);
    if (st != RSI_OK)
        return st;
    int precision, block, stack;
    if ((st = parse_intersect_opts(opts, precision, block, stack)) != RSI_OK)
        return st;
    if (!stats) {
        if (!out)
            return fail(RSI_E_ARG, "out must not be NULL");
        if (n > 0) {
            if (mode == RSI_MODE_BOOLEAN && !out->hit)
                return fail(RSI_E_ARG, "boolean mode needs out->hit");
            if (mode != RSI_MODE_BOOLEAN && !out->tri_id)
                return fail(RSI_E_ARG, "this mode needs out->tri_id");
            if (mode == RSI_MODE_BARYCENTRIC && !out->uvt)
                return fail(RSI_E_ARG, "barycentric mode needs out->uvt");
        }
        if ((out->tri_id && !aligned4(out->tri_id)) || (out->uvt && !aligned4(out->uvt)) ||
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
    const size_t ws_bytes = 4 * (size_t)n + 64;
    hipError_t e = hipMallocAsync(&ws, ws_bytes, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(e == hipErrorOutOfMemory ? RSI_E_NOMEM : RSI_E_HIP,
                    std::string("hipMallocAsync failed: ") + hipGetErrorString(e));
    }
    rsi::TraverseArgs a;
    a.from = from;
    a.to = to;
    a.n = n;
    a.mode = mode;
    a.certified = precision == RSI_PRECISION_CERTIFIED;
    a.block = block;
    a.stack = stack;
    uint64_t *ws_counters = reinterpret_cast<uint64_t *>(static_cast<char *>(ws));
    a.queue_len = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + 32);
    a.queue = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + 64);
    if (stats) {
        a.visits = visits;
        a.tests = tests;
        a.counters = ws_counters;
        e = rsi::launch_stats(mesh->dev, a, s);
    } else {
        a.hit = out->hit;
        a.tri_id = out->tri_id;
        a.uvt = out->uvt;
        a.counters = out->counters ? out->counters : ws_counters;
        e = rsi::launch_intersect(mesh->dev, a, s);
    }
    hipError_t e2 = hipFreeAsync(ws, s);
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

rsi_status rsi_traversal_stats(rsi_mesh mesh, const float *rays_from, const float *rays_to, int64_t n_rays,
                               int32_t mode, const rsi_intersect_opts *opts, uint32_t *node_visits,
                               uint32_t *leaf_tests, void *stream) {
    return run_rays(mesh, rays_from, rays_to, n_rays, mode, opts, nullptr, node_visits, leaf_tests, stream, true);
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
