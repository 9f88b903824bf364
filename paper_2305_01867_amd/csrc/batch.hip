// batch.hip -- many meshes in one BVH build and one persistent traversal.
//
// Keys are mesh id (6 bits) above a 30-bit Morton code, so after the one
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

// Extent of each mesh: kBoundSlices workgroups per mesh, each over a slice of
// its vertex floats read in order (coalesced), merged with atomic min / max
// on an order-preserving integer form of the floats.  A slice is a whole
// number of 768-float steps, so a thread's three loads per step always fall
// on the same axes: load k of thread t is axis (t + k) mod 3.  NaN
// coordinates are skipped, as fminf / fmaxf skip them.
constexpr int kBoundSlices = 16;
constexpr int kBoundStep = 768;  // floats per workgroup step: 256 threads x 3 loads

__device__ __forceinline__ uint32_t order_key(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u >> 31) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float order_value(uint32_t k) {
    return __uint_as_float((k >> 31) ? (k & 0x7fffffffu) : ~k);
}

// keys of the per-mesh minima at their identity (all ones), of the maxima at 0
__global__ void k_batch_init(uint32_t *__restrict__ key_bounds, int32_t *__restrict__ roots, int M) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < M) {
        roots[m] = INT32_MIN;
        for (int a = 0; a < 3; ++a) {
            key_bounds[8 * m + a] = 0xffffffffu;
            key_bounds[8 * m + 3 + a] = 0u;
        }
    }
}

__global__ __launch_bounds__(256) void k_batch_bounds(const float *__restrict__ V, const int64_t *__restrict__ v_off,
                                                      uint32_t *__restrict__ key_bounds) {
    const int m = blockIdx.x / kBoundSlices, part = blockIdx.x % kBoundSlices;
    const int t = threadIdx.x;
    const int64_t first = 3 * v_off[m], n = 3 * v_off[m + 1] - first;
    const int64_t per = (n + (int64_t)kBoundSlices * kBoundStep - 1) / ((int64_t)kBoundSlices * kBoundStep) * kBoundStep;
    const int64_t s0 = part * per, s1 = s0 + per < n ? s0 + per : n;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};  // per load slot
    for (int64_t j = s0 + t; j < s1; j += kBoundStep) {
        float v[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
            v[k] = j + 256 * k < s1 ? V[first + j + 256 * k] : NAN;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            lo[k] = fminf(lo[k], v[k]);
            hi[k] = fmaxf(hi[k], v[k]);
        }
    }
    // load slot k -> axis (t + k) mod 3
    float L[3], H[3];
    const int r = t % 3;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int k = (a - r + 3) % 3;
        L[a] = k == 0 ? lo[0] : (k == 1 ? lo[1] : lo[2]);
        H[a] = k == 0 ? hi[0] : (k == 1 ? hi[1] : hi[2]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            L[a] = fminf(L[a], __shfl_xor(L[a], off));
            H[a] = fmaxf(H[a], __shfl_xor(H[a], off));
        }
    __shared__ float red[4][6];
    const int w = t >> 6;
    if ((t & 63) == 0)
        for (int a = 0; a < 3; ++a) {
            red[w][a] = L[a];
            red[w][3 + a] = H[a];
        }
    __syncthreads();
    if (t < 6) {
        const bool is_lo = t < 3;
        float x = red[0][t];
        for (int k = 1; k < 4; ++k)
            x = is_lo ? fminf(x, red[k][t]) : fmaxf(x, red[k][t]);
        if (is_lo)
            atomicMin(key_bounds + 8 * m + t, order_key(x));
        else
            atomicMax(key_bounds + 8 * m + t, order_key(x));
    }
}

// The union box and the largest coordinate magnitude of all meshes (the
// traversal widens boxes relative to it).
__global__ void k_batch_global(float *__restrict__ mesh_bounds, int M, float *__restrict__ bounds) {
    if (threadIdx.x != 0)
        return;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, scale = 0.0f;
    uint32_t *key_bounds = reinterpret_cast<uint32_t *>(mesh_bounds);
    for (int m = 0; m < M; ++m) {
        float ms = 0.0f;  // an empty mesh (lo = +inf, hi = -inf) adds no scale
        for (int a = 0; a < 3; ++a) {
            const float l = order_value(key_bounds[8 * m + a]), h = order_value(key_bounds[8 * m + 3 + a]);
            mesh_bounds[8 * m + a] = l;
            mesh_bounds[8 * m + 3 + a] = h;
            if (l <= h)
                ms = fmaxf(ms, fmaxf(fabsf(l), fabsf(h)));
            lo[a] = fminf(lo[a], l);
            hi[a] = fmaxf(hi[a], h);
        }
        mesh_bounds[8 * m + 6] = ms;
        mesh_bounds[8 * m + 7] = 0.0f;
        scale = fmaxf(scale, ms);
    }
    for (int a = 0; a < 3; ++a) {
        bounds[a] = lo[a];
        bounds[3 + a] = hi[a];
    }
    bounds[6] = scale;
    bounds[7] = 0.0f;
}

// The subtree root of each mesh: the internal node whose key range is exactly
// the mesh's keys, or the leaf of a one-triangle mesh.
__global__ void k_mesh_roots(const Node *__restrict__ nodes, const uint64_t *__restrict__ keys, int64_t nt,
                             int32_t *__restrict__ roots) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nt)
        return;
    auto mesh = [&](int64_t k) { return (int)(keys[k] >> kBatchMortonBits); };
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
    uint32_t *key_bounds = reinterpret_cast<uint32_t *>(b.mesh_bounds);
    k_batch_init<<<1, 64, 0, s>>>(key_bounds, b.roots, b.M);
    k_batch_bounds<<<b.M * kBoundSlices, 256, 0, s>>>(m.V, b.v_off, key_bounds);
    k_batch_global<<<1, 64, 0, s>>>(b.mesh_bounds, b.M, m.bounds);
    if (m.nt == 0)
        return hipGetLastError();
    hipError_t e = launch_morton_batch(m, b.tri_mesh, b.mesh_bounds, s);
    if (e == hipSuccess)
        e = build_from_keys64(m, kBatchMortonBits + 6, s);  // five 8-bit sort passes
    if (e != hipSuccess)
        return e;
    k_mesh_roots<<<blocks(m.nt, 256), 256, 0, s>>>(m.nodes, static_cast<const uint64_t *>(m.keys), m.nt, b.roots);
    e = hipGetLastError();
    return e == hipSuccess ? launch_collapse_batch(m, b, s) : e;
}

}  // namespace rsi
