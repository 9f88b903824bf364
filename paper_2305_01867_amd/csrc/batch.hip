// batch.hip -- many meshes in one BVH build and one persistent traversal.
//
// Keys are mesh id (6 bits) above a 57-bit Morton code, so after the one
// sort each mesh's triangles are contiguous and, by the prefix property of
// the binary radix tree (Karras 2012), form exactly one subtree: one sort, one
// tree build and one bottom-up pass cover every mesh.  The traversal then
// takes (mesh, segment range) items from a queue and starts each segment at
// its mesh's subtree root.  Every step here is a kernel on the caller's
// stream, with no allocation and no host synchronisation, so build and
// intersect can be captured in a graph and replayed.
#include "rsi_internal.h"

namespace rsi {
namespace {

__device__ __forceinline__ int mesh_of(const int64_t *__restrict__ off, int M, int64_t x) {
    int lo = 0, hi = M - 1;  // last mesh whose first element is <= x
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// Copy the vertices, turn per-mesh vertex indices into global ones, and note
// each triangle's mesh.  A triangle with an index outside its mesh gets -1 in
// all three slots: it is never hit and widens no box.
__global__ void k_batch_prepare(const float *__restrict__ Vin, int64_t nv, const int32_t *__restrict__ Fin,
                                int64_t nt, const int64_t *__restrict__ v_off, const int64_t *__restrict__ t_off,
                                int M, float *__restrict__ V, int32_t *__restrict__ F,
                                int32_t *__restrict__ tri_mesh) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * nv; i += stride)
        V[i] = Vin[i];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += stride) {
        const int m = mesh_of(t_off, M, t);
        const int64_t base = v_off[m], nvm = v_off[m + 1] - base;
        bool ok = true;
        int32_t g[3];
        for (int c = 0; c < 3; ++c) {
            const int32_t idx = Fin[3 * t + c];
            ok = ok && idx >= 0 && idx < nvm;
            g[c] = (int32_t)(base + idx);
        }
        for (int c = 0; c < 3; ++c)
            F[3 * t + c] = ok ? g[c] : -1;
        tri_mesh[t] = m;
    }
}

// Extent of each mesh (one workgroup per mesh), as the extent kernels of the single-mesh build do.
__global__ __launch_bounds__(256) void k_batch_bounds(const float *__restrict__ V, const int64_t *__restrict__ v_off,
                                                      float *__restrict__ mesh_bounds) {
    const int m = blockIdx.x;
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = v_off[m] + threadIdx.x; i < v_off[m + 1]; i += blockDim.x)
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], V[3 * i + a]);
            hi[a] = fmaxf(hi[a], V[3 * i + a]);
        }
    for (int off = 32; off > 0; off >>= 1)
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], off));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off));
        }
    __shared__ float red[4][6];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int a = 0; a < 3; ++a) {
            red[w][a] = lo[a];
            red[w][3 + a] = hi[a];
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        float scale = 0.0f;
        for (int a = 0; a < 3; ++a) {
            for (int k = 1; k < 4; ++k) {
                lo[a] = fminf(lo[a], red[k][a]);
                hi[a] = fmaxf(hi[a], red[k][3 + a]);
            }
            mesh_bounds[8 * m + a] = lo[a];
            mesh_bounds[8 * m + 3 + a] = hi[a];
            if (lo[a] <= hi[a])  // an empty mesh (lo = +inf, hi = -inf) adds no scale
                scale = fmaxf(scale, fmaxf(fabsf(lo[a]), fabsf(hi[a])));
        }
        mesh_bounds[8 * m + 6] = scale;
        mesh_bounds[8 * m + 7] = 0.0f;
    }
}

// The union box and the largest coordinate magnitude of all meshes (the
// traversal widens boxes relative to it).
__global__ void k_batch_global(const float *__restrict__ mesh_bounds, int M, float *__restrict__ bounds) {
    if (threadIdx.x != 0)
        return;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, scale = 0.0f;
    for (int m = 0; m < M; ++m) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], mesh_bounds[8 * m + a]);
            hi[a] = fmaxf(hi[a], mesh_bounds[8 * m + 3 + a]);
        }
        scale = fmaxf(scale, mesh_bounds[8 * m + 6]);
    }
    for (int a = 0; a < 3; ++a) {
        bounds[a] = lo[a];
        bounds[3 + a] = hi[a];
    }
    bounds[6] = scale;
    bounds[7] = 0.0f;
}

__global__ void k_roots_init(int32_t *__restrict__ roots, int M) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < M)
        roots[m] = INT32_MIN;
}

// The subtree root of each mesh: the internal node whose key range is exactly
// the mesh's keys, or the leaf of a one-triangle mesh.
__global__ void k_mesh_roots(const Node *__restrict__ nodes, const uint64_t *__restrict__ keys, int64_t nt,
                             int32_t *__restrict__ roots) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt)
        return;
    auto mesh = [&](int64_t k) { return (int)(keys[k] >> 57); };
    int64_t lo = i, hi = i;
    if (i < nt - 1) {
        lo = nodes[i].refs.z;
        hi = nodes[i].refs.w;
        const int m = mesh(lo);
        if (mesh(hi) == m && (lo == 0 || mesh(lo - 1) != m) && (hi == nt - 1 || mesh(hi + 1) != m))
            roots[m] = (int32_t)i;
    }
    // leaf i alone
    const int m = mesh(i);
    if ((i == 0 || mesh(i - 1) != m) && (i == nt - 1 || mesh(i + 1) != m))
        roots[m] = ~(int32_t)i;
}

inline int blocks(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

hipError_t launch_batch_build(MeshDev &m, BatchDev &b, const float *V, const int32_t *F, hipStream_t s) {
    const int64_t work = 3 * m.nv > m.nt ? 3 * m.nv : m.nt;
    const int grid = work > 0 ? (blocks(work, 256) < 4096 ? blocks(work, 256) : 4096) : 1;
    k_batch_prepare<<<grid, 256, 0, s>>>(V, m.nv, F, m.nt, b.v_off, b.t_off, b.M, m.V, m.F, b.tri_mesh);
    k_batch_bounds<<<b.M, 256, 0, s>>>(m.V, b.v_off, b.mesh_bounds);
    k_batch_global<<<1, 64, 0, s>>>(b.mesh_bounds, b.M, m.bounds);
    k_roots_init<<<blocks(b.M, 64), 64, 0, s>>>(b.roots, b.M);
    if (m.nt == 0)
        return hipGetLastError();
    hipError_t e = launch_morton_batch(m, b.tri_mesh, b.mesh_bounds, s);
    if (e == hipSuccess)
        e = build_from_keys64(m, 63, s);
    if (e != hipSuccess)
        return e;
    k_mesh_roots<<<blocks(m.nt, 256), 256, 0, s>>>(m.nodes, static_cast<const uint64_t *>(m.keys), m.nt, b.roots);
    e = hipGetLastError();
    return e == hipSuccess ? launch_collapse_batch(m, b, s) : e;
}

}  // namespace rsi
