// derive.hip -- the barycentric mode's derived outputs on gfx950.
//
// Paper: Background (barycentric mode: the intersecting rays, the hit
// triangle, the distance to and the location of the nearest intersecting
// point) and the Performance section (steps 3a-3d: identify the intersecting
// rays, compute distances, keep the hit triangles, compute points -- moved
// from host numpy to the GPU there).  Here:
//   k_derive      per segment: distance t |E - O| and point O + t (E - O)
//                 (NaN on a miss), evaluated in binary64 from the float32 end
//                 points and t, rounded once to float32;
//   k_hit_counts  hits per tile of kCompactTile segments;
//   (scan of the tile counts)
//   k_compact     ordered stream compaction of the hitting segments into
//                 (index, distance, triangle, point), ascending index.
// All HBM-bound streams: coalesced segment / result reads, one write each.
#include "rsi_internal.h"

namespace rsi {
namespace {

constexpr int kCompactThreads = 1024;
constexpr int kCompactItems = 4;
constexpr int kCompactTile = kCompactThreads * kCompactItems;

__device__ __forceinline__ void derive_one(const float *__restrict__ from, const float *__restrict__ to, int64_t i,
                                           float t32, float &dist, float &px, float &py, float &pz) {
    const double ox = from[3 * i], oy = from[3 * i + 1], oz = from[3 * i + 2];
    const double dx = (double)to[3 * i] - ox, dy = (double)to[3 * i + 1] - oy, dz = (double)to[3 * i + 2] - oz;
    const double t = t32;
    dist = (float)(t * sqrt(dx * dx + dy * dy + dz * dz));
    px = (float)(ox + t * dx);
    py = (float)(oy + t * dy);
    pz = (float)(oz + t * dz);
}

__global__ void k_derive(const float *__restrict__ from, const float *__restrict__ to, int64_t n,
                         const int32_t *__restrict__ tri_id, const float *__restrict__ uvt, float *__restrict__ dist,
                         float *__restrict__ point) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    float d = NAN, px = NAN, py = NAN, pz = NAN;
    if (tri_id[i] >= 0)
        derive_one(from, to, i, uvt[3 * i + 2], d, px, py, pz);
    if (dist)
        dist[i] = d;
    if (point) {
        point[3 * i] = px;
        point[3 * i + 1] = py;
        point[3 * i + 2] = pz;
    }
}

__global__ __launch_bounds__(kCompactThreads) void k_hit_counts(const int32_t *__restrict__ tri_id, int64_t n,
                                                                uint32_t *__restrict__ counts) {
    __shared__ uint32_t wsum[kCompactThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kCompactTile;
    uint32_t c = 0;
    for (int r = 0; r < kCompactItems; ++r) {
        const int64_t i = base + r * kCompactThreads + threadIdx.x;
        c += (i < n && tri_id[i] >= 0) ? 1u : 0u;
    }
    for (int off = 32; off > 0; off >>= 1)
        c += __shfl_xor(c, off);
    if ((threadIdx.x & 63) == 0)
        wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < kCompactThreads / 64; ++w)
            t += wsum[w];
        counts[blockIdx.x] = t;
    }
}

// offs holds each tile's first output slot (exclusive scan of the counts).
__global__ __launch_bounds__(kCompactThreads) void k_compact(const float *__restrict__ from,
                                                             const float *__restrict__ to, int64_t n,
                                                             const int32_t *__restrict__ tri_id,
                                                             const float *__restrict__ uvt,
                                                             const uint32_t *__restrict__ offs, int n_tiles,
                                                             int64_t *__restrict__ hit_index,
                                                             float *__restrict__ dist, int32_t *__restrict__ hit_tri,
                                                             float *__restrict__ point, int64_t *__restrict__ n_hits) {
    __shared__ uint32_t wcount[kCompactThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int64_t base = (int64_t)blockIdx.x * kCompactTile;
    int64_t out = offs[blockIdx.x];
    for (int r = 0; r < kCompactItems; ++r) {
        const int64_t i = base + r * kCompactThreads + threadIdx.x;
        const int32_t tri = i < n ? tri_id[i] : -1;
        const bool hit = tri >= 0;
        const uint64_t m = __ballot(hit);
        if (lane == 0)
            wcount[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int w = 0; w < kCompactThreads / 64; ++w) {
            const uint32_t c = wcount[w];
            before += w < wave ? c : 0u;
            all += c;
        }
        if (hit) {
            const int64_t o = out + before + (uint32_t)__popcll(m & lt);
            float d, px, py, pz;
            derive_one(from, to, i, uvt[3 * i + 2], d, px, py, pz);
            if (hit_index)
                hit_index[o] = i;
            if (dist)
                dist[o] = d;
            if (hit_tri)
                hit_tri[o] = tri;
            if (point) {
                point[3 * o] = px;
                point[3 * o + 1] = py;
                point[3 * o + 2] = pz;
            }
        }
        out += all;
        __syncthreads();  // wcount is rewritten by the next round
    }
    if (blockIdx.x == n_tiles - 1 && threadIdx.x == 0)
        *n_hits = out;  // the last tile ends where the hits end
}

__global__ void k_zero_count(int64_t *n_hits) { *n_hits = 0; }

}  // namespace

hipError_t launch_derive(const float *from, const float *to, int64_t n, const int32_t *tri_id, const float *uvt,
                         float *dist, float *point, hipStream_t s) {
    if (n > 0)
        k_derive<<<(int)((n + 255) / 256), 256, 0, s>>>(from, to, n, tri_id, uvt, dist, point);
    return hipGetLastError();
}

size_t compact_ws_bytes(int64_t n) {
    const int64_t tiles = (n + kCompactTile - 1) / kCompactTile;
    return 4 * (size_t)(tiles > 0 ? tiles : 1) + 4 * 1024 + 256;
}

hipError_t launch_compact(const float *from, const float *to, int64_t n, const int32_t *tri_id, const float *uvt,
                          int64_t *hit_index, float *dist, int32_t *hit_tri, float *point, int64_t *n_hits,
                          void *ws, hipStream_t s) {
    if (n == 0) {
        k_zero_count<<<1, 1, 0, s>>>(n_hits);
        return hipGetLastError();
    }
    const int64_t tiles = (n + kCompactTile - 1) / kCompactTile;
    uint32_t *counts = static_cast<uint32_t *>(ws);
    uint32_t *partial = counts + ((tiles + 63) & ~int64_t(63));
    k_hit_counts<<<(int)tiles, kCompactThreads, 0, s>>>(tri_id, n, counts);
    hipError_t e = scan_u32_exclusive(counts, tiles, partial, s);
    if (e != hipSuccess)
        return e;
    k_compact<<<(int)tiles, kCompactThreads, 0, s>>>(from, to, n, tri_id, uvt, counts, (int)tiles, hit_index, dist,
                                                     hit_tri, point, n_hits);
    return hipGetLastError();
}

}  // namespace rsi
