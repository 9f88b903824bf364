// wide.hip -- collapse of the binary BVH into a 4-wide one on gfx950.
//
// The traversal's cost per node is one dependent fetch from L2 plus the box
// arithmetic; a 4-wide node halves the number of dependent fetches per
// segment (each tests four children at once) and fits one 128-byte L2 line.
// The collapse keeps the binary tree's boxes and leaves: a 4-wide node starts
// at a binary internal node r and takes its two children, then opens the
// child of largest surface area twice (greedy, as in the usual collapse of
// binary BVHs into wide ones), so it covers exactly the leaves of r.  It is
// stored at index r of the 4-wide array, so no renumbering is needed.
//
// Work split as in the bottom-up pass: one workgroup per tile (a subtree of
// at most 1024 leaves listed by the radix-tree kernel), breadth-first from
// the tile root with the queue in LDS; one more workgroup of the same launch
// for the nodes above the tiles, which never opens a tile root (every tile
// root starts a 4-wide node of its own).  Treelet restructuring keeps every tile root and its leaves,
// so the same tile list serves both builds.
#include "rsi_internal.h"

namespace rsi {
namespace {

constexpr int kTileQueue = 1024;  // a tile of <= 1024 leaves has <= 1023 internal nodes

__device__ __forceinline__ float half_area6(const float *b) {
    const float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return dx * dy + dy * dz + dz * dx;
}

// The two children of binary node r: references and boxes (lo xyz, hi xyz).
__device__ __forceinline__ void children_of(const Node *__restrict__ nodes, int r, int &l, int &rr, float lb[6],
                                            float rb[6]) {
    const Node *nd = nodes + r;
    const float4 L = nd->xy_left, R = nd->xy_right, Z = nd->z_both;
    const int4 refs = nd->refs;
    l = refs.x;
    rr = refs.y;
    lb[0] = L.x, lb[1] = L.z, lb[2] = Z.x, lb[3] = L.y, lb[4] = L.w, lb[5] = Z.y;
    rb[0] = R.x, rb[1] = R.z, rb[2] = Z.z, rb[3] = R.y, rb[4] = R.w, rb[5] = Z.w;
}

// Collapse the binary subtree at r into nodes4[r]; returns the internal
// children that start 4-wide nodes below.  flag (may be NULL) marks nodes:
// one whose flag shares a bit with no_open is never opened (it starts a
// 4-wide node of its own); one whose flag shares a bit with no_start is not
// returned either (another workgroup starts it).
__device__ __forceinline__ int collapse_node(const Node *__restrict__ nodes, Node4 *__restrict__ nodes4, int r,
                                             const int32_t *__restrict__ flag, int no_open, int no_start,
                                             int kids[4]) {
    int ref[4] = {0, 0, kEmptyChild, kEmptyChild};
    float b[4][6];
#pragma unroll
    for (int i = 2; i < 4; ++i)
#pragma unroll
        for (int a = 0; a < 6; ++a)
            b[i][a] = INFINITY;
    children_of(nodes, r, ref[0], ref[1], b[0], b[1]);
    int m = 2;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        int best = -1;
        float best_a = -1.0f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const bool open = i < m && ref[i] >= 0 && !(flag && (flag[ref[i]] & no_open));
            const float a = half_area6(b[i]);
            if (open && a > best_a) {
                best_a = a;
                best = i;
            }
        }
        if (best < 0)
            break;
        int c = ref[0];
#pragma unroll
        for (int i = 1; i < 4; ++i)
            c = best == i ? ref[i] : c;
        int l, rr;
        float lb[6], rb[6];
        children_of(nodes, c, l, rr, lb, rb);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i == best) {
                ref[i] = l;
#pragma unroll
                for (int a = 0; a < 6; ++a)
                    b[i][a] = lb[a];
            }
            if (i == m) {
                ref[i] = rr;
#pragma unroll
                for (int a = 0; a < 6; ++a)
                    b[i][a] = rb[a];
            }
        }
        ++m;
    }
    Node4 o;
    o.lox = make_float4(b[0][0], b[1][0], b[2][0], b[3][0]);
    o.loy = make_float4(b[0][1], b[1][1], b[2][1], b[3][1]);
    o.loz = make_float4(b[0][2], b[1][2], b[2][2], b[3][2]);
    o.hix = make_float4(b[0][3], b[1][3], b[2][3], b[3][3]);
    o.hiy = make_float4(b[0][4], b[1][4], b[2][4], b[3][4]);
    o.hiz = make_float4(b[0][5], b[1][5], b[2][5], b[3][5]);
    // internal children are named by binary index + kTopSlots (the top slots
    // are assigned afterwards by k_top_cache)
    auto enc = [](int c) { return c >= 0 ? c + kTopSlots : c; };
    o.child = make_int4(enc(ref[0]), enc(ref[1]), enc(ref[2]), enc(ref[3]));
    o.spare = make_int4(m, 0, 0, 0);
    nodes4[r] = o;
    int nk = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool go = ref[i] >= 0 && !(flag && (flag[ref[i]] & no_start));
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (go && k == nk)
                kids[k] = ref[i];
        nk += go ? 1 : 0;
    }
    return nk;
}

__global__ void k_clear_flags(int32_t *flag, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        flag[i] = 0;
}


// One workgroup's tile: breadth-first from the tile root c, a lane per 4-wide
// node of the current level, the queue in LDS.
__device__ void collapse_tile(const Node *__restrict__ nodes, Node4 *__restrict__ nodes4, int c,
                              const int32_t *__restrict__ flag, int no_open, int *q, int &qn) {
    if (threadIdx.x == 0) {
        q[0] = c;
        qn = 1;
    }
    __syncthreads();
    int b0 = 0, b1 = 1;
    while (b0 < b1) {
        for (int i = b0 + (int)threadIdx.x; i < b1; i += blockDim.x) {
            int kids[4];
            const int nk = collapse_node(nodes, nodes4, q[i], flag, no_open, 0, kids);
            for (int k = 0; k < nk; ++k) {
                const int slot = atomicAdd(&qn, 1);
                if (slot < kTileQueue)
                    q[slot] = kids[k];
            }
        }
        __syncthreads();
        b0 = b1;
        b1 = qn < kTileQueue ? qn : kTileQueue;
        __syncthreads();  // every lane has read qn before the next level appends
    }
}

// One workgroup: breadth-first from the root with the queue in global
// scratch.  The nodes above the tiles (tile roots flagged kTileRoot: never
// opened, started by the tile workgroups), or the whole tree with the
// frontier of the learned proposal flagged kFrontier (each frontier node
// starts a 4-wide node, so the proposal order can start and skip it).
constexpr int kTileRoot = kTileRootFlag, kFrontier = 2, kMeshRoot = 4;
__device__ void collapse_from_root(const Node *__restrict__ nodes, Node4 *__restrict__ nodes4,
                                   const int32_t *__restrict__ flag, int no_open, int no_start, int32_t *queue,
                                   int64_t n_internal, int &qn) {
    if (flag[0] & no_start)
        return;  // the whole tree is one tile
    if (threadIdx.x == 0) {
        queue[0] = 0;
        qn = 1;
    }
    __syncthreads();
    int b0 = 0, b1 = 1;
    while (b0 < b1) {
        for (int i = b0 + (int)threadIdx.x; i < b1; i += blockDim.x) {
            int kids[4];
            const int nk = collapse_node(nodes, nodes4, queue[i], flag, no_open, no_start, kids);
            for (int k = 0; k < nk; ++k) {
                const int slot = atomicAdd(&qn, 1);
                if (slot < n_internal)
                    queue[slot] = kids[k];
            }
        }
        __syncthreads();
        b0 = b1;
        b1 = qn < n_internal ? qn : (int)n_internal;
        __syncthreads();
    }
}

// The tiles and the nodes above them in one launch: the last workgroup takes
// the nodes above the tiles, the others the tiles in turn.  The two parts
// write disjoint nodes (a tile root is never opened from above).  tile_no_open
// marks the nodes a tile never opens (0: none).
__global__ __launch_bounds__(256) void k_collapse(const Node *__restrict__ nodes, Node4 *__restrict__ nodes4,
                                                  const int32_t *__restrict__ tiles,
                                                  const int32_t *__restrict__ n_tiles,
                                                  const int32_t *__restrict__ flag, int tile_no_open,
                                                  int top_no_open, int32_t *queue, int64_t n_internal) {
    __shared__ int q[kTileQueue];
    __shared__ int qn;
    if (blockIdx.x == gridDim.x - 1) {
        collapse_from_root(nodes, nodes4, flag, top_no_open, kTileRoot, queue, n_internal, qn);
        return;
    }
    const int32_t *tile_flag = tile_no_open ? flag : nullptr;
    const int total = *n_tiles;
    for (int e = blockIdx.x; e < total; e += gridDim.x - 1) {
        const int c = tiles[e];
        if (c < 0)
            continue;  // a one-leaf tile: no internal node
        collapse_tile(nodes, nodes4, c, tile_flag, tile_no_open, q, qn);
    }
}

// The whole tree from the root in one workgroup (the learned proposal's
// collapse: a one-off set-up, not on the hot path).
__global__ __launch_bounds__(1024) void k_collapse_top(const Node *__restrict__ nodes, Node4 *__restrict__ nodes4,
                                                       const int32_t *__restrict__ flag, int no_open, int no_start,
                                                       int32_t *queue, int64_t n_internal) {
    __shared__ int qn;
    collapse_from_root(nodes, nodes4, flag, no_open, no_start, queue, n_internal, qn);
}

// One workgroup: the first kTopSlots 4-wide nodes in breadth-first order from
// the root, copied into top4 with the references of children that also got a
// slot rewritten to that slot.  Slots follow a block-wide prefix sum over each
// level, so the layout does not depend on thread timing.
// slot_bin (may be NULL) receives the binary index of the node in each slot,
// -1 for unused slots.
__global__ __launch_bounds__(kTopSlots) void k_top_cache(const Node4 *__restrict__ nodes4, Node4 *__restrict__ top4,
                                                         int32_t *__restrict__ slot_bin) {
    constexpr int kWaves = kTopSlots / 64;
    __shared__ int bidx[kTopSlots];  // binary index of the node in each slot
    __shared__ int wave_sum[kWaves];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0)
        bidx[0] = 0;
    __syncthreads();
    int b0 = 0, b1 = 1;
    while (b0 < b1) {
        const int i = b0 + tid;  // a level has at most kTopSlots = blockDim nodes
        Node4 nd;
        int cnt = 0;
        if (i < b1) {
            nd = nodes4[bidx[i]];
            cnt = (nd.child.x >= 0) + (nd.child.y >= 0) + (nd.child.z >= 0) + (nd.child.w >= 0);
        }
        // inclusive prefix sum of cnt: within the wave by shuffles, then across waves
        int incl = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off);
            incl += lane >= off ? t : 0;
        }
        if (lane == 63)
            wave_sum[w] = incl;
        __syncthreads();
        int total = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
            const int x = wave_sum[k];
            incl += k < w ? x : 0;
            total += x;
        }
        if (i < b1) {
            int slot = b1 + incl - cnt;
            int c[4] = {nd.child.x, nd.child.y, nd.child.z, nd.child.w};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (c[k] >= 0) {
                    if (slot < kTopSlots) {
                        bidx[slot] = c[k] - kTopSlots;
                        c[k] = slot;
                    }
                    ++slot;
                }
            nd.child = make_int4(c[0], c[1], c[2], c[3]);
            top4[i] = nd;
        }
        __syncthreads();  // bidx of the next level written, wave_sum read
        b0 = b1;
        b1 = b1 + total < kTopSlots ? b1 + total : kTopSlots;
    }
    if (slot_bin)
        slot_bin[tid] = tid < b1 ? bidx[tid] : -1;
}

// Batched form: the top of each XCD group's meshes, breadth-first from their
// roots (group g = blockIdx.x), laid out as k_top_cache lays out one tree's
// top, and each mesh's root as a reference in it (a slot for the group's own
// meshes, the node index + kTopSlots or a leaf reference for the others).
__global__ __launch_bounds__(kTopSlots) void k_top_cache_group(const Node4 *__restrict__ nodes4,
                                                               const int32_t *__restrict__ roots,
                                                               const int32_t *__restrict__ mesh_group, int M,
                                                               Node4 *__restrict__ top4g,
                                                               int32_t *__restrict__ roots4g) {
    constexpr int kWaves = kTopSlots / 64;
    __shared__ int bidx[kTopSlots];
    __shared__ int wave_sum[kWaves];
    __shared__ int root_slot[64];
    const int g = blockIdx.x, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    Node4 *top4 = top4g + (int64_t)g * kTopSlots;
    // the group's internal roots in mesh order take the first slots
    if (w == 0) {
        const bool mine = tid < M && mesh_group[tid] == g && roots[tid] >= 0;
        const uint64_t all = __ballot(mine);  // the whole wave votes: not inside a lane branch
        const int k = __popcll(all & (lane ? (~0ull >> (64 - lane)) : 0ull));
        root_slot[tid] = mine ? k : -1;
        if (mine)
            bidx[k] = roots[tid];
        if (lane == 0)
            wave_sum[0] = __popcll(all);
    }
    __syncthreads();
    int b0 = 0, b1 = wave_sum[0];
    __syncthreads();
    while (b0 < b1) {
        const int i = b0 + tid;
        Node4 nd;
        int cnt = 0;
        if (i < b1) {
            nd = nodes4[bidx[i]];
            cnt = (nd.child.x >= 0) + (nd.child.y >= 0) + (nd.child.z >= 0) + (nd.child.w >= 0);
        }
        int incl = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off);
            incl += lane >= off ? t : 0;
        }
        if (lane == 63)
            wave_sum[w] = incl;
        __syncthreads();
        int total = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
            const int x = wave_sum[k];
            incl += k < w ? x : 0;
            total += x;
        }
        if (i < b1) {
            int slot = b1 + incl - cnt;
            int c[4] = {nd.child.x, nd.child.y, nd.child.z, nd.child.w};
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (c[k] >= 0) {
                    if (slot < kTopSlots) {
                        bidx[slot] = c[k] - kTopSlots;
                        c[k] = slot;
                    }
                    ++slot;
                }
            nd.child = make_int4(c[0], c[1], c[2], c[3]);
            top4[i] = nd;
        }
        __syncthreads();  // bidx of the next level written, wave_sum read
        b0 = b1;
        b1 = b1 + total < kTopSlots ? b1 + total : kTopSlots;
    }
    if (tid < M) {
        const int r = roots[tid];
        const int sl = tid < 64 ? root_slot[tid] : -1;
        roots4g[(int64_t)g * 64 + tid] = sl >= 0 ? sl : (r >= 0 ? r + kTopSlots : r);
    }
}

__global__ void k_mark_frontier(const int32_t *__restrict__ bucket_ref, const int32_t *__restrict__ n_buckets,
                                int32_t *flag, int64_t n_internal) {
    const int b = threadIdx.x;
    if (b < *n_buckets) {
        const int c = bucket_ref[b];
        if (c >= 0 && c < n_internal)
            flag[c] |= kFrontier;
    }
}

__global__ void k_mark_mesh_roots(const int32_t *__restrict__ roots, int M, int32_t *flag, int64_t n_internal) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < M) {
        const int c = roots[m];
        if (c >= 0 && c < n_internal)
            flag[c] |= kMeshRoot;
    }
}

// The reference under which each bucket's frontier node appears in the
// 4-wide tree: its top slot if it has one, else binary index + kTopSlots;
// a leaf keeps its leaf reference.
// (The same for each mesh root of the batched form, n_buckets = NULL: count M.)
// One workgroup of kTopSlots threads: the buckets' references are staged in
// LDS, then each slot claims the buckets whose node it holds (at most
// kTopSlots buckets or meshes).
__global__ __launch_bounds__(kTopSlots) void k_bucket_ref4(const int32_t *__restrict__ bucket_ref,
                                                           const int32_t *__restrict__ n_buckets, int M,
                                                           const int32_t *__restrict__ slot_bin,
                                                           int32_t *__restrict__ ref4) {
    __shared__ int ref[kTopSlots];  // each bucket's binary reference
    const int t = threadIdx.x;
    const int n_raw = n_buckets ? *n_buckets : M;
    const int n = n_raw < kTopSlots ? n_raw : kTopSlots;
    const int c = t < n ? bucket_ref[t] : -1;
    ref[t] = c;
    if (t < n)
        ref4[t] = c >= 0 ? c + kTopSlots : c;  // by default the node itself (not in the top)
    __syncthreads();  // the defaults are written before any slot claims a bucket
    // slot t claims the buckets whose node it holds (each slot holds one node)
    const int mine = slot_bin[t];
    if (mine >= 0)
        for (int b = 0; b < n; ++b)
            if (ref[b] == mine)
                ref4[b] = t;
}

}  // namespace

hipError_t launch_collapse(MeshDev &m, hipStream_t s) {
    if (m.nt < 2)
        return hipSuccess;  // one leaf: nothing to collapse
    const int64_t n_internal = m.nt - 1;
    const BuildLists L = build_lists(m.sort_tmp, m.nt);
    // (the radix-tree kernel flagged the tiles' nodes)
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t want = (m.nt + 1023) / 1024 * 2;  // tiles hold up to 1024 leaves, usually fewer
    const int grid = (int)(want < 4 * cus ? want : 4 * cus) + 1;  // + the nodes above the tiles
    k_collapse<<<grid, 256, 0, s>>>(m.nodes, m.nodes4, L.tiles, L.n_tiles, L.tile_flag, 0, kTileRoot, L.queue,
                                    n_internal);
    k_top_cache<<<1, kTopSlots, 0, s>>>(m.nodes4, m.top4, nullptr);
    const hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        m.node_width = 4;
    return e;
}

hipError_t launch_collapse_proposal(const MeshDev &m, Proposal &pr, hipStream_t s) {
    if (m.nt < 2 || m.node_width != 4 || !pr.top4)
        return hipSuccess;
    const int64_t n_internal = m.nt - 1;
    const int blocks = (int)((n_internal + 255) / 256);
    k_clear_flags<<<blocks, 256, 0, s>>>(pr.wide_flag, n_internal);
    k_mark_frontier<<<1, kMlpOut, 0, s>>>(pr.bucket_ref, pr.dev_n_buckets, pr.wide_flag, n_internal);
    // one workgroup over the whole tree: a one-off set-up, not on the hot path
    k_collapse_top<<<1, 1024, 0, s>>>(m.nodes, pr.top4 + kTopSlots, pr.wide_flag, kFrontier, 0, pr.wide_queue,
                                      n_internal);
    k_top_cache<<<1, kTopSlots, 0, s>>>(pr.top4 + kTopSlots, pr.top4, pr.slot_bin);
    k_bucket_ref4<<<1, kTopSlots, 0, s>>>(pr.bucket_ref, pr.dev_n_buckets, 0, pr.slot_bin, pr.bucket_ref4);
    return hipGetLastError();
}

// Batched form: the collapse of the combined tree with every mesh's subtree
// root starting a 4-wide node (never opened from above), so a segment starts
// at its mesh root's 4-wide node.
hipError_t launch_collapse_batch(MeshDev &m, BatchDev &b, hipStream_t s) {
    if (m.nt < 2 || !m.nodes4 || !b.roots4) {
        m.node_width = 2;
        return hipSuccess;
    }
    const int64_t n_internal = m.nt - 1;
    const BuildLists L = build_lists(m.sort_tmp, m.nt);
    // (the radix-tree kernel flagged the tiles' nodes)
    k_mark_mesh_roots<<<1, 64, 0, s>>>(b.roots, b.M, L.tile_flag, n_internal);
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t want = (m.nt + 1023) / 1024 * 2;
    const int grid = (int)(want < 4 * cus ? want : 4 * cus) + 1;  // + the nodes above the tiles
    k_collapse<<<grid, 256, 0, s>>>(m.nodes, m.nodes4, L.tiles, L.n_tiles, L.tile_flag, kMeshRoot,
                                    kTileRoot | kMeshRoot, L.queue, n_internal);
    k_top_cache<<<1, kTopSlots, 0, s>>>(m.nodes4, m.top4, b.slot_bin);
    k_bucket_ref4<<<1, kTopSlots, 0, s>>>(b.roots, nullptr, b.M, b.slot_bin, b.roots4);
    if (b.top4g)
        k_top_cache_group<<<kItemGroups, kTopSlots, 0, s>>>(m.nodes4, b.roots, b.mesh_group, b.M, b.top4g,
                                                            b.roots4g);
    const hipError_t e = hipGetLastError();
    m.node_width = e == hipSuccess ? 4 : 2;
    return e;
}

}  // namespace rsi
