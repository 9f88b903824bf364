// build.hip -- bounding volume hierarchy construction on gfx950.
//
// Steps (paper: Background -- Morton codes, spatial sort, binary radix tree of
// Karras 2012; Specific changes -- Morton kernel, 64-bit codes; Case Studies
// 1-2 -- sorted int32 triangle ids, bottom-up node filling with one atomic
// counter per internal node, N_t - 1 internal nodes, a launch sized by N_t):
//   1. mesh extent            one workgroup, min / max over all vertices
//   2. Morton keys            one lane per triangle
//   3. LDS radix sort         stable LSD, 8-bit digits: tile histograms,
//                             one device-wide scan, stable tile scatter
//   4. radix tree             one lane per internal node (Karras section 3)
//   5. leaves + bottom-up     one lane per leaf, arrival counters in LDS
//                             inside subtrees of <= 1024 leaves; one
//                             workgroup finishes the nodes above them
#include "rsi_internal.h"

namespace rsi {
namespace {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;  // 2048 keys per tile
constexpr int kRadix = 256;
// Up to this many tiles (131,072 keys) a pass is one launch: every scatter
// workgroup derives its own offsets from the whole (small) histogram and adds
// its keys to the next pass's histogram as it places them.
constexpr int kSmallSortTiles = 64;
constexpr int kBoxTile = 1024;  // leaves per bottom-up workgroup (one per lane)
constexpr int kNoTile = INT32_MIN;  // never a child reference (leaves are ~k with k < 2^30)
constexpr int kRestructureRounds = 2;  // treelet restructuring passes of algorithm 2

// ---------------------------------------------------------------- 1. extent
// Min / max are exact in any order, so the extent is reduced in two steps:
// up to kBoundsParts workgroups each reduce a strided share of the vertices,
// then one workgroup combines their partial boxes and the coordinate scale.
constexpr int kBoundsParts = 256;

// Block-wide min / max of six values (lo xyz, hi xyz); the result is valid in
// thread 0.
__device__ __forceinline__ void block_minmax(float lo[3], float hi[3]) {
    for (int off = 32; off > 0; off >>= 1)
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], __shfl_xor(lo[a], off));
            hi[a] = fmaxf(hi[a], __shfl_xor(hi[a], off));
        }
    __shared__ float red[16][6];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int a = 0; a < 3; ++a) {
            red[w][a] = lo[a];
            red[w][3 + a] = hi[a];
        }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int k = 1; k < nw; ++k)
            for (int a = 0; a < 3; ++a) {
                lo[a] = fminf(lo[a], red[k][a]);
                hi[a] = fmaxf(hi[a], red[k][3 + a]);
            }
    }
}

// (also copies the caller's vertices into the mesh's own array, and clears
// the build flags)
__global__ __launch_bounds__(1024) void k_mesh_bounds_part(const float *__restrict__ V, int64_t nv,
                                                           float *__restrict__ partial, float *__restrict__ V_copy,
                                                           int32_t *__restrict__ flags) {
    if (blockIdx.x == 0 && threadIdx.x < 4)
        flags[threadIdx.x] = 0;
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x)
        for (int a = 0; a < 3; ++a) {
            const float x = V[3 * i + a];
            V_copy[3 * i + a] = x;
            lo[a] = fminf(lo[a], x);
            hi[a] = fmaxf(hi[a], x);
        }
    block_minmax(lo, hi);
    if (threadIdx.x == 0)
        for (int a = 0; a < 3; ++a) {
            partial[6 * blockIdx.x + a] = lo[a];
            partial[6 * blockIdx.x + 3 + a] = hi[a];
        }
}

__global__ __launch_bounds__(kBoundsParts) void k_mesh_bounds_final(const float *__restrict__ partial, int parts,
                                                                    float *__restrict__ bounds) {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if ((int)threadIdx.x < parts)
        for (int a = 0; a < 3; ++a) {
            lo[a] = partial[6 * threadIdx.x + a];
            hi[a] = partial[6 * threadIdx.x + 3 + a];
        }
    block_minmax(lo, hi);
    if (threadIdx.x == 0) {
        float scale = 0.0f;
        for (int a = 0; a < 3; ++a) {
            bounds[a] = lo[a];
            bounds[3 + a] = hi[a];
            if (lo[a] <= hi[a])  // no vertices: no scale
                scale = fmaxf(scale, fmaxf(fabsf(lo[a]), fabsf(hi[a])));
        }
        bounds[6] = scale;
        bounds[7] = 0.0f;
    }
}

// ---------------------------------------------------------- 2. Morton keys
// Spread the low 10 (or 21) bits of x so that bit k lands on bit 3k.
__device__ __forceinline__ uint32_t spread3(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}
__device__ __forceinline__ uint64_t spread3(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// Quantise one centroid coordinate: n = (c - lo) / ext (0 for a flat axis),
// q = floor(min(n 2^b, 2^b - 1)), 0 for n <= 0 or NaN.  Single float32 ops,
// no contraction.
__device__ __forceinline__ uint32_t quantise(float c, float lo, float ext, float two_b, float top) {
#pragma clang fp contract(off)
    float n = ext > 0.0f ? (c - lo) / ext : 0.0f;
    float x = n * two_b;
    return x > 0.0f ? (uint32_t)floorf(fminf(x, top)) : 0u;
}

// (also copies the caller's triangles into the mesh's own array)
template <typename K>
__global__ __launch_bounds__(256) void k_morton(const float *__restrict__ V, int64_t nv,
                                                const int32_t *__restrict__ F, int64_t nt,
                                                const float *__restrict__ bounds, K *__restrict__ keys,
                                                int32_t *__restrict__ ids, int32_t *__restrict__ flags,
                                                int32_t *__restrict__ F_copy) {
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt)
        return;
    constexpr int b = sizeof(K) == 4 ? 10 : 21;
    const int32_t i0 = F[3 * t], i1 = F[3 * t + 1], i2 = F[3 * t + 2];
    F_copy[3 * t] = i0;
    F_copy[3 * t + 1] = i1;
    F_copy[3 * t + 2] = i2;
    ids[t] = (int32_t)t;
    if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= nv || i1 >= nv || i2 >= nv) {
        atomicOr(flags, 1);
        keys[t] = (K)0;
        return;
    }
    float c[3];
    for (int a = 0; a < 3; ++a)
        c[a] = ((V[3 * (int64_t)i0 + a] + V[3 * (int64_t)i1 + a]) + V[3 * (int64_t)i2 + a]) / 3.0f;
    const float two_b = (float)(1u << b), top = (float)((1u << b) - 1u);
    K key = 0;
    for (int a = 2; a >= 0; --a) {  // z, then y, then x: z lands on the top bit of each triple
        const float lo = bounds[a], ext = bounds[3 + a] - bounds[a];
        key = (K)(key << 1) | spread3((K)quantise(c[a], lo, ext, two_b, top));
    }
    keys[t] = key;
}

// Batched form: the key of a triangle of mesh m is m (6 bits) above a 30-bit
// Morton code (10 bits per axis) of its centroid normalised to mesh m's box,
// so each mesh's triangles are contiguous after the sort and form one subtree.
__global__ __launch_bounds__(256) void k_morton_batch(const float *__restrict__ V, const int32_t *__restrict__ F,
                                                      const int32_t *__restrict__ tri_mesh, int64_t nt,
                                                      const float *__restrict__ mesh_bounds,
                                                      uint64_t *__restrict__ keys, int32_t *__restrict__ ids) {
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nt)
        return;
    ids[t] = (int32_t)t;
    const int m = tri_mesh[t];
    const int32_t i0 = F[3 * t], i1 = F[3 * t + 1], i2 = F[3 * t + 2];
    if (i0 < 0 || i1 < 0 || i2 < 0) {  // marked invalid while copying
        keys[t] = (uint64_t)m << kBatchMortonBits;
        return;
    }
    const float *bb = mesh_bounds + 8 * m;
    // 10 bits per axis of the mesh's own box, as the single-mesh 30-bit codes
    const float two_b = (float)(1u << 10), top = (float)((1u << 10) - 1u);
    uint64_t key = 0;
    for (int a = 2; a >= 0; --a) {
        const float c = ((V[3 * (int64_t)i0 + a] + V[3 * (int64_t)i1 + a]) + V[3 * (int64_t)i2 + a]) / 3.0f;
        key = (key << 1) | spread3((uint64_t)quantise(c, bb[a], bb[3 + a] - bb[a], two_b, top));
    }
    keys[t] = ((uint64_t)m << kBatchMortonBits) | key;
}

// ---------------------------------------------------------- 3. radix sort
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_sort_hist(const K *__restrict__ keys, int64_t n, int shift,
                                                            int ntiles, uint32_t *__restrict__ hist,
                                                            uint32_t *__restrict__ clear) {
    __shared__ uint32_t h[kRadix];
    const int tid = threadIdx.x, tile = blockIdx.x;
    h[tid] = 0;
    if (clear)  // one-launch passes: the histogram the first pass adds to
        clear[(int64_t)tid * ntiles + tile] = 0u;
    __syncthreads();
    const int64_t base = (int64_t)tile * kSortTile;
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = base + r * kSortThreads + tid;
        if (idx < n)
            atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    hist[(int64_t)tid * ntiles + tile] = h[tid];
}

// Exclusive scan of hist[0..len) in place, one workgroup of 1024 lanes.
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t *__restrict__ hist, int64_t len) {
    __shared__ uint32_t part[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (len + 1023) / 1024;
    const int64_t beg = tid * chunk, end = beg + chunk < len ? beg + chunk : len;
    uint32_t s = 0;
    for (int64_t i = beg; i < end; ++i)
        s += hist[i];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = tid >= off ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t run = part[tid] - s;  // exclusive prefix of this chunk
    for (int64_t i = beg; i < end; ++i) {
        uint32_t v = hist[i];
        hist[i] = run;
        run += v;
    }
}

// Large histograms: per-block sums, a scan of those (k_sort_scan), then each
// block scans its own segment from its offset.  Reads are coalesced rounds of
// 1024 entries; seg is a multiple of 1024.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *wsum, uint32_t &total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    uint32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off)
            x += y;
    }
    if (lane == 63)
        wsum[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int k = 0; k < nw; ++k) {
        const uint32_t t = wsum[k];
        before += k < w ? t : 0u;
        all += t;
    }
    __syncthreads();  // wsum is reused by the next round
    total = all;
    return before + x - v;
}

__global__ __launch_bounds__(1024) void k_scan_partials(const uint32_t *__restrict__ hist, int64_t len, int64_t seg,
                                                        uint32_t *__restrict__ partial) {
    __shared__ uint32_t wsum[16];
    const int64_t beg = (int64_t)blockIdx.x * seg, end = beg + seg < len ? beg + seg : len;
    uint32_t s = 0;
    for (int64_t i = beg + threadIdx.x; i < end; i += blockDim.x)
        s += hist[i];
    uint32_t total;
    (void)block_excl_scan(s, wsum, total);
    if (threadIdx.x == 0)
        partial[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void k_scan_apply(uint32_t *__restrict__ hist, int64_t len, int64_t seg,
                                                     const uint32_t *__restrict__ partial) {
    __shared__ uint32_t wsum[16];
    const int64_t beg = (int64_t)blockIdx.x * seg, end = beg + seg < len ? beg + seg : len;
    uint32_t run = partial[blockIdx.x];
    for (int64_t r = beg; r < end; r += blockDim.x) {
        const int64_t i = r + threadIdx.x;
        const uint32_t v = i < end ? hist[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan(v, wsum, total);
        if (i < end)
            hist[i] = run + ex;
        run += total;
    }
}

// The tile histograms of a large sort, one row of ntiles per digit: workgroup
// d scans row d in place (exclusive) and writes its total to totals[d]; the
// scatter adds the digits below from those totals.  One launch instead of
// a three-step scan of the whole histogram.
__global__ __launch_bounds__(1024) void k_scan_rows(uint32_t *__restrict__ hist, int64_t ntiles,
                                                    uint32_t *__restrict__ totals) {
    __shared__ uint32_t wsum[16];
    uint32_t *row = hist + (int64_t)blockIdx.x * ntiles;
    uint32_t run = 0;
    for (int64_t r = 0; r < ntiles; r += blockDim.x) {
        const int64_t i = r + threadIdx.x;
        const uint32_t v = i < ntiles ? row[i] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan(v, wsum, total);
        if (i < ntiles)
            row[i] = run + ex;
        run += total;
    }
    if (threadIdx.x == 0)
        totals[blockIdx.x] = run;
}

// Exclusive scan of hist[0..len); partial holds 1024 entries.
void scan_hist(uint32_t *hist, int64_t len, uint32_t *partial, hipStream_t s) {
    if (len <= 32768) {
        k_sort_scan<<<1, 1024, 0, s>>>(hist, len);
        return;
    }
    const int64_t per = (len + 1023) / 1024;
    const int64_t seg = (per + 1023) / 1024 * 1024;
    const int g = (int)((len + seg - 1) / seg);
    k_scan_partials<<<g, 1024, 0, s>>>(hist, len, seg, partial);
    k_sort_scan<<<1, 1024, 0, s>>>(partial, g);
    k_scan_apply<<<g, 1024, 0, s>>>(hist, len, seg, partial);
}

// Stable scatter of one tile.  Its keys are loaded at once (eight per
// lane), then ranked in rounds of 256 consecutive keys: inside a wave by
// matching the 8 digit bits with ballots, across the four waves and earlier
// rounds through per-digit LDS counts.  base[d] is where the tile's keys of
// digit d start; run and wcnt start at zero.  With hist_next, each placed
// key's next digit is counted at the tile its new position falls in.
template <typename K>
__device__ __forceinline__ void scatter_tile(const K *__restrict__ kin, const int32_t *__restrict__ iin,
                                             K *__restrict__ kout, int32_t *__restrict__ iout, int64_t n,
                                             int shift, int tile, uint32_t *run, const uint32_t *base,
                                             uint32_t (*wcnt)[kRadix], uint32_t *__restrict__ hist_next,
                                             int ntiles) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t t0 = (int64_t)tile * kSortTile;
    K key[kSortItems];
    int32_t id[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t idx = t0 + r * kSortThreads + tid;
        key[r] = idx < n ? kin[idx] : K(0);
        id[r] = idx < n ? iin[idx] : 0;
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const bool valid = t0 + r * kSortThreads + tid < n;
        const uint32_t digit = valid ? (uint32_t)(key[r] >> shift) & 0xffu : 0u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool set = (digit >> bit) & 1u;
            const uint64_t m = __ballot(set);
            peers &= set ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & lt_mask);
        if (valid && rank == 0)
            wcnt[wave][digit] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = base[digit] + run[digit] + rank;
            for (int w = 0; w < wave; ++w)
                pos += wcnt[w][digit];
            kout[pos] = key[r];
            iout[pos] = id[r];
            if (hist_next)
                atomicAdd(hist_next + (int64_t)((uint32_t)(key[r] >> (shift + 8)) & 0xffu) * ntiles + pos / kSortTile,
                          1u);
        }
        __syncthreads();
        uint32_t add = 0;
        for (int w = 0; w < kSortThreads / 64; ++w) {
            add += wcnt[w][tid];
            wcnt[w][tid] = 0;
        }
        run[tid] += add;
        __syncthreads();
    }
}

// One scatter pass over tile histograms scanned per digit (offs: digit-major,
// exclusive within each digit's row; totals: each digit's count).
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(const K *__restrict__ kin,
                                                               const int32_t *__restrict__ iin,
                                                               K *__restrict__ kout, int32_t *__restrict__ iout,
                                                               int64_t n, int shift, int ntiles,
                                                               const uint32_t *__restrict__ offs,
                                                               const uint32_t *__restrict__ totals) {
    __shared__ uint32_t run[kRadix];
    __shared__ uint32_t base[kRadix];
    __shared__ uint32_t wcnt[kSortThreads / 64][kRadix];
    __shared__ uint32_t wsum[kSortThreads / 64];
    const int tid = threadIdx.x, tile = blockIdx.x;
    uint32_t all;
    const uint32_t below = block_excl_scan(totals[tid], wsum, all);  // keys of the digits below
    run[tid] = 0;
    base[tid] = below + offs[(int64_t)tid * ntiles + tile];
    for (int w = 0; w < kSortThreads / 64; ++w)
        wcnt[w][tid] = 0;
    __syncthreads();
    scatter_tile<K>(kin, iin, kout, iout, n, shift, tile, run, base, wcnt, nullptr, ntiles);
}

// One pass of a small sort in one launch.  hist holds this pass's per-tile
// digit counts (digit-major); each workgroup sums them into its own offsets
// (digits below, then earlier tiles of its digit) and scatters its tile,
// counting the next digit into hist_next (null after the last pass).
// hist_clear (the histogram two passes on) is zeroed here: nothing reads or
// adds to it during this pass.
template <typename K>
__global__ __launch_bounds__(kSortThreads) void k_sort_pass_small(const K *__restrict__ kin,
                                                                  const int32_t *__restrict__ iin,
                                                                  K *__restrict__ kout, int32_t *__restrict__ iout,
                                                                  int64_t n, int shift, int ntiles,
                                                                  const uint32_t *__restrict__ hist,
                                                                  uint32_t *__restrict__ hist_next,
                                                                  uint32_t *__restrict__ hist_clear) {
    __shared__ uint32_t run[kRadix];
    __shared__ uint32_t base[kRadix];
    __shared__ uint32_t wcnt[kSortThreads / 64][kRadix];
    __shared__ uint32_t wsum[kSortThreads / 64];
    const int tid = threadIdx.x, tile = blockIdx.x;
    uint32_t earlier = 0, total = 0;
    const uint32_t *h = hist + (int64_t)tid * ntiles;
    for (int t = 0; t < ntiles; ++t) {
        const uint32_t v = h[t];
        earlier += t < tile ? v : 0u;
        total += v;
    }
    uint32_t all;
    base[tid] = block_excl_scan(total, wsum, all) + earlier;
    hist_clear[(int64_t)tid * ntiles + tile] = 0u;
    run[tid] = 0;
    for (int w = 0; w < kSortThreads / 64; ++w)
        wcnt[w][tid] = 0;
    __syncthreads();
    scatter_tile<K>(kin, iin, kout, iout, n, shift, tile, run, base, wcnt, hist_next, ntiles);
}

// ---------------------------------------------------------- 4. radix tree
// Length of the common prefix of key_i || i and key_j || j; -1 outside [0, n).
template <typename K>
__device__ __forceinline__ int prefix(const K *__restrict__ k, int n, int i, K ki, int j) {
    if (j < 0 || j >= n)
        return -1;
    const K kj = k[j];
    if (ki != kj) {
        if constexpr (sizeof(K) == 8)
            return __builtin_clzll((unsigned long long)(ki ^ kj));
        else
            return __builtin_clz((unsigned)(ki ^ kj));
    }
    return (int)(8 * sizeof(K)) + __builtin_clz((unsigned)(i ^ j));
}

// Also lists the bottom-up tiles: the largest subtrees with at most kBoxTile
// leaves (children of larger nodes, or the root itself), wave-aggregated into
// tiles[0 .. *n_tiles); and flags each internal node of at most kBoxTile
// leaves with kTileRootFlag (the 4-wide collapse above the tiles stops at the
// first flagged nodes from the root, which are the tiles).
template <typename K>
__global__ __launch_bounds__(256) void k_radix_tree(const K *__restrict__ keys, int n, Node *__restrict__ nodes,
                                                    int32_t *__restrict__ parent, int32_t *__restrict__ counters,
                                                    int32_t *__restrict__ tiles, int32_t *__restrict__ n_tiles,
                                                    int32_t *__restrict__ tile_flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1)
        return;
    const K ki = keys[i];
    const int d = prefix(keys, n, i, ki, i + 1) > prefix(keys, n, i, ki, i - 1) ? 1 : -1;
    const int below = prefix(keys, n, i, ki, i - d);
    int len_max = 2;
    while (prefix(keys, n, i, ki, i + len_max * d) > below)
        len_max <<= 1;
    int len = 0;
    for (int step = len_max >> 1; step >= 1; step >>= 1)
        if (prefix(keys, n, i, ki, i + (len + step) * d) > below)
            len += step;
    const int j = i + len * d;
    const int node_prefix = prefix(keys, n, i, ki, j);
    int s = 0;
    for (int div = 2;; div <<= 1) {
        const int step = (len + div - 1) / div;
        if (prefix(keys, n, i, ki, i + (s + step) * d) > node_prefix)
            s += step;
        if (step <= 1)
            break;
    }
    const int split = i + s * d + (d < 0 ? -1 : 0);
    const int lo = min(i, j), hi = max(i, j);
    const int left = (lo == split) ? ~split : split;
    const int right = (hi == split + 1) ? ~(split + 1) : split + 1;
    nodes[i].refs = make_int4(left, right, lo, hi);
    parent[left >= 0 ? left : (n - 1) + ~left] = i;
    parent[right >= 0 ? right : (n - 1) + ~right] = i;
    counters[i] = 0;
    tile_flag[i] = hi - lo + 1 <= kBoxTile ? kTileRootFlag : 0;
    if (i == 0)
        parent[0] = -1;

    int emit0 = kNoTile, emit1 = kNoTile;
    if (hi - lo + 1 > kBoxTile) {
        if (split - lo + 1 <= kBoxTile)
            emit0 = left;
        if (hi - split <= kBoxTile)
            emit1 = right;
    } else if (i == 0) {
        emit0 = 0;  // the whole tree is one tile
    }
    const uint64_t m1 = __ballot(emit0 != kNoTile || emit1 != kNoTile);
    const uint64_t m2 = __ballot(emit0 != kNoTile && emit1 != kNoTile);
    if (m1) {
        const int lane = threadIdx.x & 63;
        const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
        const int leader = __ffsll((unsigned long long)m1) - 1;
        int base = 0;
        if (lane == leader)
            base = atomicAdd(n_tiles, __popcll(m1) + __popcll(m2));
        base = __shfl(base, leader);
        int o = base + __popcll(m1 & lt) + __popcll(m2 & lt);
        if (emit0 != kNoTile)
            tiles[o++] = emit0;
        if (emit1 != kNoTile)
            tiles[o] = emit1;
    }
}

__global__ void k_single_tile(int32_t *tiles, int32_t *n_tiles) {
    tiles[0] = ~0;  // one triangle: the leaf is the whole tree
    *n_tiles = 1;
}

// ------------------------------------------------- 5. leaves and bottom-up
// Boxes are merged bottom-up, each internal node by the second of its two
// children to finish (the paper's Case Study 2: one arrival counter per
// internal node).  The tree is cut into tiles, the largest subtrees with at
// most kBoxTile leaves (listed by k_radix_tree), and nodes above them:
//   k_leaves_subtree  one workgroup per tile: counters and child boxes in LDS,
//                     no cross-workgroup synchronisation at all;
//   k_boxes_top       one workgroup climbs the nodes above the tiles (about
//                     log2(N_t / kBoxTile) levels) with workgroup-scope atomics.
// Cross-XCD agent-scope atomics, which cost an L2 write-back each on gfx950,
// are not needed.  Every child box lands in its parent node in HBM; a
// finished internal node's counter reads 2.
// Leaf k (sorted position): write its triangle (A, B - A, C - A, input index)
// and return its box.  An invalid triangle is never hit and widens no box.
__device__ __forceinline__ void make_leaf(const float *__restrict__ V, int64_t nv, const int32_t *__restrict__ F,
                                          const int32_t *__restrict__ ids, int n, int k, Tri *__restrict__ tris,
                                          float *lo, float *hi) {
    int t = ids[k];
    const bool t_ok = t >= 0 && t < n;  // always true for a correct sort; guards the loads below
    if (!t_ok)
        t = 0;
    const int32_t i0 = F[3 * (int64_t)t], i1 = F[3 * (int64_t)t + 1], i2 = F[3 * (int64_t)t + 2];
    Tri tri;
    if (!t_ok || i0 < 0 || i1 < 0 || i2 < 0 || i0 >= nv || i1 >= nv || i2 >= nv) {
        tri.a = make_float4(NAN, NAN, NAN, __int_as_float(t));
        tri.e1 = make_float4(NAN, NAN, NAN, 0.0f);
        tri.e2 = make_float4(NAN, NAN, NAN, 0.0f);
        for (int d = 0; d < 3; ++d) {
            lo[d] = INFINITY;
            hi[d] = -INFINITY;
        }
    } else {
        float A[3], B[3], C[3];
        for (int d = 0; d < 3; ++d) {
            A[d] = V[3 * (int64_t)i0 + d];
            B[d] = V[3 * (int64_t)i1 + d];
            C[d] = V[3 * (int64_t)i2 + d];
            lo[d] = fminf(A[d], fminf(B[d], C[d]));
            hi[d] = fmaxf(A[d], fmaxf(B[d], C[d]));
        }
        tri.a = make_float4(A[0], A[1], A[2], __int_as_float(t));
        tri.e1 = make_float4(B[0] - A[0], B[1] - A[1], B[2] - A[2], 0.0f);
        tri.e2 = make_float4(C[0] - A[0], C[1] - A[1], C[2] - A[2], 0.0f);
    }
    tris[k] = tri;
}

__device__ __forceinline__ void store_child_box(Node *node, bool is_left, const float *lo, const float *hi) {
    if (is_left) {
        node->xy_left = make_float4(lo[0], hi[0], lo[1], hi[1]);
        *reinterpret_cast<float2 *>(&node->z_both.x) = make_float2(lo[2], hi[2]);
    } else {
        node->xy_right = make_float4(lo[0], hi[0], lo[1], hi[1]);
        *reinterpret_cast<float2 *>(&node->z_both.z) = make_float2(lo[2], hi[2]);
    }
}

// Phase 1: one workgroup per listed tile (a subtree of at most kBoxTile
// leaves, sorted positions [a, b]).  Lane j takes leaf a + j, writes its
// triangle and climbs; every internal node of the tile lies in [a, b], so
// arrival counters and child boxes live in LDS at p - a.  The lane completing
// the tile root hands its box to the root's parent.
__global__ __launch_bounds__(kBoxTile) void k_leaves_subtree(const float *__restrict__ V, int64_t nv,
                                                            const int32_t *__restrict__ F,
                                                            const int32_t *__restrict__ ids, int n,
                                                            Tri *__restrict__ tris, Node *nodes,
                                                            const int32_t *__restrict__ parent, int32_t *counters,
                                                            const int32_t *__restrict__ tiles,
                                                            const int32_t *__restrict__ n_tiles) {
    __shared__ int arrived[kBoxTile];
    __shared__ float box[kBoxTile][2][6];
    const int total = *n_tiles;
    for (int e = blockIdx.x; e < total; e += gridDim.x) {
        const int c = tiles[e];
        int a, b;
        if (c < 0) {
            a = b = ~c;
        } else {
            const int4 r = nodes[c].refs;
            a = r.z;
            b = r.w;
        }
        arrived[threadIdx.x] = 0;
        __syncthreads();
        const int k = a + (int)threadIdx.x;
        if (a >= 0 && k <= b && b < n && b - a < kBoxTile) {
            float lo[3], hi[3];
            make_leaf(V, nv, F, ids, n, k, tris, lo, hi);
            int self = ~k;
            int p = n >= 2 ? parent[(n - 1) + k] : -1;
            if (self == c) {
                // a one-leaf tile: its box goes straight to the parent
                if (p >= 0 && p < n - 1)
                    store_child_box(nodes + p, nodes[p].refs.x == self, lo, hi);
            } else {
                // a radix tree is at most 97 levels deep; the bound only guards the loop
                for (int level = 0; p >= a && p <= b && p < n - 1 && level < kDeepStack; ++level) {
                    Node *node = nodes + p;
                    const bool is_left = node->refs.x == self;
                    store_child_box(node, is_left, lo, hi);
                    float *mine = box[p - a][is_left ? 0 : 1];
                    for (int d = 0; d < 3; ++d) {
                        mine[d] = lo[d];
                        mine[3 + d] = hi[d];
                    }
                    __threadfence_block();
                    if (atomicAdd(&arrived[p - a], 1) == 0)
                        break;  // the sibling subtree is not finished; its last lane continues
                    __threadfence_block();
                    const float *other = box[p - a][is_left ? 1 : 0];
                    for (int d = 0; d < 3; ++d) {
                        lo[d] = fminf(lo[d], other[d]);
                        hi[d] = fmaxf(hi[d], other[3 + d]);
                    }
                    counters[p] = 2;
                    if (p == c) {
                        const int q = parent[p];
                        if (q >= 0 && q < n - 1)
                            store_child_box(nodes + q, nodes[q].refs.x == p, lo, hi);
                        break;
                    }
                    self = p;
                    p = parent[p];
                }
            }
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

// Phase 2: one workgroup finishes the nodes above the tiles (every node with
// more than kBoxTile leaves).  Each listed tile is an arrival at its parent;
// the second arrival merges the two child boxes (written by phase 1, or by
// this workgroup before its release) and climbs on.
__global__ __launch_bounds__(1024) void k_boxes_top(Node *nodes, const int32_t *__restrict__ parent,
                                                    int32_t *counters, const int32_t *__restrict__ tiles,
                                                    const int32_t *__restrict__ n_tiles, int n) {
    const int total = *n_tiles;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int c = tiles[e];
        int p = c < 0 ? parent[(n - 1) + ~c] : parent[c];
        for (int level = 0; p >= 0 && p < n - 1 && level < kDeepStack; ++level) {
            if (__hip_atomic_fetch_add(counters + p, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == 0)
                break;
            const Node *node = nodes + p;
            const float4 L = node->xy_left, R = node->xy_right, Z = node->z_both;
            const float lo[3] = {fminf(L.x, R.x), fminf(L.z, R.z), fminf(Z.x, Z.z)};
            const float hi[3] = {fmaxf(L.y, R.y), fmaxf(L.w, R.w), fmaxf(Z.y, Z.w)};
            const int q = parent[p];
            if (q < 0 || q >= n - 1)
                break;  // p is the root
            store_child_box(nodes + q, nodes[q].refs.x == p, lo, hi);
            p = q;
        }
    }
}

// ------------------------------------------ 5'. agglomerative single pass
// The same binary radix tree, built bottom-up in one pass (Apetrei 2014,
// "Fast and simple agglomerative LBVH construction"; the numbering the paper's
// Case Study 1 dump shows): a lane per leaf climbs; a node covering [l, r]
// joins the neighbour across the boundary with the longer common prefix, so
// its parent is internal node r (it is the left child) or l - 1 (the right
// child) -- internal nodes are numbered by their split position.  The first
// child to reach a parent leaves its far bound in other[p] and stops; the
// second learns the parent's range from the exchange, merges the boxes and
// climbs on.  Every step is a cross-workgroup exchange at agent scope.
template <typename K>
__global__ __launch_bounds__(256) void k_agglomerate(const K *__restrict__ keys, const float *__restrict__ V,
                                                     int64_t nv, const int32_t *__restrict__ F,
                                                     const int32_t *__restrict__ ids, int n, Tri *__restrict__ tris,
                                                     Node *nodes, int32_t *__restrict__ parent, int32_t *counters,
                                                     int32_t *other, int32_t *__restrict__ root_out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n)
        return;
    float lo[3], hi[3];
    make_leaf(V, nv, F, ids, n, k, tris, lo, hi);
    if (n < 2) {
        *root_out = ~0;
        return;
    }
    auto delta = [&](int i) { return prefix(keys, n, i, keys[i], i + 1); };  // boundary between i and i + 1
    int l = k, r = k, self = ~k;
    for (int level = 0; level < kDeepStack; ++level) {
        const bool left_child = l == 0 || (r != n - 1 && delta(r) > delta(l - 1));
        const int p = left_child ? r : l - 1;
        Node *node = nodes + p;
        store_child_box(node, left_child, lo, hi);
        if (left_child)
            node->refs.x = self;
        else
            node->refs.y = self;
        parent[self >= 0 ? self : (n - 1) + ~self] = p;
        const int prev = __hip_atomic_exchange(other + p, left_child ? l : r, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
        if (prev < 0)
            return;  // the sibling is not finished; its lane continues
        const int pl = left_child ? l : prev, pr = left_child ? prev : r;
        const float4 xy = left_child ? node->xy_right : node->xy_left;
        const float2 z = left_child ? *reinterpret_cast<const float2 *>(&node->z_both.z)
                                    : *reinterpret_cast<const float2 *>(&node->z_both.x);
        lo[0] = fminf(lo[0], xy.x);
        hi[0] = fmaxf(hi[0], xy.y);
        lo[1] = fminf(lo[1], xy.z);
        hi[1] = fmaxf(hi[1], xy.w);
        lo[2] = fminf(lo[2], z.x);
        hi[2] = fmaxf(hi[2], z.y);
        node->refs.z = pl;
        node->refs.w = pr;
        counters[p] = 2;
        l = pl;
        r = pr;
        self = p;
        if (l == 0 && r == n - 1) {
            parent[p] = -1;
            *root_out = p;
            return;
        }
    }
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = v;
}

__global__ void k_zero_i32(int32_t *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = 0;
}

inline int blocks_for(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

// After an odd number of sort passes the sorted pairs sit in the scratch
// buffers: copy them back.
template <typename K>
__global__ void k_copy_pairs(const K *__restrict__ k_in, const int32_t *__restrict__ i_in, K *__restrict__ k_out,
                             int32_t *__restrict__ i_out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        k_out[i] = k_in[i];
        i_out[i] = i_in[i];
    }
}

// Stable LSD passes over (keys, ids) with 8-bit digits; tmp holds the
// ping-pong copies, the tile histograms and the scan partials.  Up to
// kSmallSortTiles tiles a pass is one launch; above that, a histogram, a scan
// of each digit's row and a scatter.  An even number of passes (key_bits 30 or 63 rounded up to
// 32 or 64) leaves the result in (keys, ids); an odd one (the batched form's
// 36-bit keys) ends with a copy back.
template <typename K>
void sort_passes(K *keys, int32_t *ids, void *tmp, int64_t n, int key_bits, hipStream_t s) {
    K *keys_tmp = static_cast<K *>(tmp);
    int32_t *ids_tmp = reinterpret_cast<int32_t *>(keys_tmp + n);
    const int ntiles = blocks_for(n, kSortTile);
    uint32_t *hist = reinterpret_cast<uint32_t *>(ids_tmp + n);
    uint32_t *partial = hist + (int64_t)kRadix * ntiles;
    K *src_k = keys, *dst_k = keys_tmp;
    int32_t *src_i = ids, *dst_i = ids_tmp;
    if (n <= 1)
        return;  // nothing to order
    if (ntiles <= kSmallSortTiles) {
        // three histograms in turn: read by this pass, added to for the next,
        // cleared for the one after
        const int64_t hl = (int64_t)kRadix * ntiles;
        uint32_t *H[3] = {hist, hist + hl, hist + 2 * hl};
        k_sort_hist<K><<<ntiles, kSortThreads, 0, s>>>(src_k, n, 0, ntiles, H[0], H[1]);
        for (int shift = 0, pass = 0; shift < key_bits; shift += 8, ++pass) {
            k_sort_pass_small<K><<<ntiles, kSortThreads, 0, s>>>(src_k, src_i, dst_k, dst_i, n, shift, ntiles,
                                                                  H[pass % 3], shift + 8 < key_bits ? H[(pass + 1) % 3] : nullptr,
                                                                  H[(pass + 2) % 3]);
            K *tk = src_k; src_k = dst_k; dst_k = tk;
            int32_t *ti = src_i; src_i = dst_i; dst_i = ti;
        }
    } else {
        for (int shift = 0; shift < key_bits; shift += 8) {
            k_sort_hist<K><<<ntiles, kSortThreads, 0, s>>>(src_k, n, shift, ntiles, hist, nullptr);
            k_scan_rows<<<kRadix, 1024, 0, s>>>(hist, ntiles, partial);
            k_sort_scatter<K><<<ntiles, kSortThreads, 0, s>>>(src_k, src_i, dst_k, dst_i, n, shift, ntiles, hist,
                                                               partial);
            K *tk = src_k; src_k = dst_k; dst_k = tk;
            int32_t *ti = src_i; src_i = dst_i; dst_i = ti;
        }
    }
    if (src_k != keys && n > 0)
        k_copy_pairs<K><<<blocks_for(n, 256), 256, 0, s>>>(src_k, src_i, keys, ids, n);
}

size_t pass_tmp_bytes(int64_t n, size_t key_bytes) {
    const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    const int64_t hists = ntiles <= kSmallSortTiles ? 3 : 1;  // one-launch passes keep three
    return key_bytes * n + 4 * n + 4 * (size_t)kRadix * ntiles * hists + 4 * 1024 + 256;
}

// Sort (key, id), build the radix tree and fill the boxes bottom-up, for keys
// already in m.keys and ids in m.ids.
template <typename K>
hipError_t build_from_keys(MeshDev &m, int key_bits, hipStream_t s) {
    const int64_t nt = m.nt;
    K *keys = static_cast<K *>(m.keys);
    sort_passes<K>(keys, m.ids, m.sort_tmp, nt, key_bits, s);  // sorted pairs back in (keys, ids)
    if (m.algorithm == 1) {
        // the sort's scratch is free again: the exchange slots
        int32_t *other = static_cast<int32_t *>(m.sort_tmp);
        if (nt >= 2) {
            k_fill_i32<<<blocks_for(nt - 1, 256), 256, 0, s>>>(other, nt - 1, -1);
            k_zero_i32<<<blocks_for(nt - 1, 256), 256, 0, s>>>(m.counters, (int)(nt - 1));
        }
        k_agglomerate<K><<<blocks_for(nt, 256), 256, 0, s>>>(keys, m.V, m.nv, m.F, m.ids, (int)nt, m.tris, m.nodes,
                                                            m.parent, m.counters, other, m.flags + 1);
        return hipGetLastError();
    }
    // the sort's scratch is free again: the list of bottom-up tiles
    const BuildLists L = build_lists(m.sort_tmp, nt);
    int32_t *n_tiles = L.n_tiles;
    int32_t *tiles = L.tiles;
    if (nt >= 2) {
        k_zero_i32<<<1, 64, 0, s>>>(n_tiles, 1);
        k_radix_tree<K><<<blocks_for(nt - 1, 256), 256, 0, s>>>(keys, (int)nt, m.nodes, m.parent, m.counters, tiles,
                                                                n_tiles, L.tile_flag);
    } else {
        k_single_tile<<<1, 1, 0, s>>>(tiles, n_tiles);
    }
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t grid = nt < 2 * (int64_t)cus ? nt : 2 * (int64_t)cus;  // tiles are taken in a loop
    k_leaves_subtree<<<(int)grid, kBoxTile, 0, s>>>(m.V, m.nv, m.F, m.ids, (int)nt, m.tris, m.nodes, m.parent,
                                                    m.counters, tiles, n_tiles);
    if (nt > kBoxTile)
        k_boxes_top<<<1, 1024, 0, s>>>(m.nodes, m.parent, m.counters, tiles, n_tiles, (int)nt);
    return hipGetLastError();
}

template <typename K>
hipError_t build_typed(MeshDev &m, const int32_t *F_in, hipStream_t s) {
    const int64_t nt = m.nt;
    k_morton<K><<<blocks_for(nt, 256), 256, 0, s>>>(m.V, m.nv, F_in, nt, m.bounds, static_cast<K *>(m.keys), m.ids,
                                                    m.flags, m.F);
    return build_from_keys<K>(m, m.morton_bits, s);
}

}  // namespace

hipError_t launch_morton_batch(MeshDev &m, const int32_t *tri_mesh, const float *mesh_bounds, hipStream_t s) {
    if (m.nt > 0)
        k_morton_batch<<<blocks_for(m.nt, 256), 256, 0, s>>>(m.V, m.F, tri_mesh, m.nt, mesh_bounds,
                                                            static_cast<uint64_t *>(m.keys), m.ids);
    return hipGetLastError();
}

size_t sort_tmp_bytes(int64_t nt, int morton_bits) {
    const size_t kb = morton_bits > 32 ? 8 : 4;
    const size_t sort = pass_tmp_bytes(nt, kb);
    const size_t lists = build_lists_bytes(nt);  // lists kept after the sort
    const size_t parts = 6 * sizeof(float) * kBoundsParts;  // extent partials before the sort
    const size_t most = sort > lists ? sort : lists;
    return most > parts ? most : parts;
}

size_t sort_u32_tmp_bytes(int64_t n) { return pass_tmp_bytes(n, 4); }

hipError_t scan_u32_exclusive(uint32_t *a, int64_t len, uint32_t *partial, hipStream_t s) {
    if (len > 0)
        scan_hist(a, len, partial, s);
    return hipGetLastError();
}

hipError_t sort_u32_pairs(uint32_t *keys, int32_t *ids, void *tmp, int64_t n, hipStream_t s) {
    if (n > 1)
        sort_passes<uint32_t>(keys, ids, tmp, n, 32, s);  // four passes
    return hipGetLastError();
}

hipError_t build_from_keys64(MeshDev &m, int key_bits, hipStream_t s) { return build_from_keys<uint64_t>(m, key_bits, s); }

hipError_t launch_build(MeshDev &m, const float *V_in, const int32_t *F_in, hipStream_t s, size_t) {
    // the sort scratch is free until the keys are sorted; the first kernels
    // also copy the caller's vertices and triangles into the mesh
    const int64_t want = (m.nv + 1023) / 1024;
    const int parts = (int)(want < 1 ? 1 : (want < kBoundsParts ? want : kBoundsParts));
    float *partial = static_cast<float *>(m.sort_tmp);
    k_mesh_bounds_part<<<parts, 1024, 0, s>>>(V_in, m.nv, partial, m.V, m.flags);
    k_mesh_bounds_final<<<1, kBoundsParts, 0, s>>>(partial, parts, m.bounds);
    hipError_t e = m.morton_bits > 32 ? build_typed<uint64_t>(m, F_in, s) : build_typed<uint32_t>(m, F_in, s);
    if (e == hipSuccess && m.algorithm == 2)
        e = launch_restructure(m, kRestructureRounds, s);
    if (e == hipSuccess && m.algorithm != 1 && m.nodes4)
        e = launch_collapse(m, s);
    return e;
}

}  // namespace rsi
