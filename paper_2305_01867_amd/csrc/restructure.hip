// restructure.hip -- treelet restructuring of the BVH on gfx950.
//
// The radix tree over Morton codes splits space at fixed midpoints; for
// segments that cross a surface, the total surface area of its boxes (which
// is what a random segment's node visits follow) is well above what a
// surface-area-heuristic tree reaches.  Treelet restructuring (Karras & Aila
// 2013, "Fast parallel construction of high-quality bounding volume
// hierarchies") improves it in place: bottom-up, each node with enough leaves
// becomes the root of a treelet of up to 7 leaves (grown by opening the
// largest-area internal leaf), and the treelet's internal nodes are rebuilt
// in the topology of least SAH cost, found by dynamic programming over the
// 127 subsets of its leaves.  The leaves (sorted triangles) do not move; only
// internal nodes are rewired, so every query result stays the same.
//
// On gfx950 the work is kept inside workgroups: one workgroup loads a whole
// tile (a subtree of at most 1024 leaves, listed by the radix-tree kernel)
// into LDS, restructures it level by level (treelets of one level have
// disjoint subtrees, a wave per treelet), and writes it back; one workgroup
// then does the same for the nodes above the tiles, with the tiles as fixed
// leaves.  No cross-workgroup synchronisation at all.
//
// After restructuring, an internal node's leaves are no longer a contiguous
// range of sorted positions: words 14 / 15 of a node then hold the smallest
// and largest sorted leaf below it (the root still spans every leaf).
#include "rsi_internal.h"

namespace rsi {
namespace {

constexpr int kTile = 1024;            // leaves per tile (= lanes per workgroup)
constexpr int kTreelet = 7;            // leaves per treelet
constexpr int kSubsets = 1 << kTreelet;
constexpr int kWaves = kTile / 64;
constexpr int kMaxLevels = 130;        // > deepest radix tree (97) + treelet growth
constexpr float kCostNode = 1.2f;      // SAH weight of a node visit (one 64-B node, two box tests)
constexpr float kCostTri = 1.0f;       // SAH weight of a triangle test

// LDS image of one (sub)tree.  Local internal node 0 is the root.  A local
// child reference is >= 0 for a local internal node and ~j for local leaf j.
struct TileLds {
    int in_child[2][kTile];
    int in_slot[kTile];        // global internal node index
    float in_box[6][kTile];    // own box: lo xyz, hi xyz
    float in_cost[kTile];      // SAH cost of the subtree
    int in_count[kTile];       // leaves below
    int in_lo[kTile], in_hi[kTile];  // smallest / largest sorted leaf below
    int order[kTile];          // internal nodes by level
    int lf_ref[kTile];         // global reference of local leaf j (a leaf ~k, or a fixed subtree)
    float lf_box[6][kTile];
    float lf_cost[kTile];
    int lf_count[kTile];
    int lf_lo[kTile], lf_hi[kTile];
    int lvl_start[kMaxLevels + 2];
    int n_in, n_lf, n_levels, overflow;
    // per-wave scratch of the treelet optimisation
    float w_area[kWaves][kSubsets];
    float w_cost[kWaves][kSubsets];
    unsigned char w_split[kWaves][kSubsets];
    int w_leaf[kWaves][8];     // treelet leaves (local references)
    int w_int[kWaves][8];      // treelet internal nodes (local ids), [0] = root
    int w_m[kWaves];
};

__device__ __forceinline__ float half_area(float x0, float y0, float z0, float x1, float y1, float z1) {
    const float dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
    return dx * dy + dy * dz + dz * dx;  // half the surface area; the common factor 2 cancels in comparisons
}

__device__ __forceinline__ void lds_sync_wave() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Box / cost / count / leaf span of a local reference.
__device__ __forceinline__ float ref_box(const TileLds &T, int r, int a) {
    return r >= 0 ? T.in_box[a][r] : T.lf_box[a][~r];
}
__device__ __forceinline__ float ref_cost(const TileLds &T, int r) { return r >= 0 ? T.in_cost[r] : T.lf_cost[~r]; }
__device__ __forceinline__ int ref_count(const TileLds &T, int r) { return r >= 0 ? T.in_count[r] : T.lf_count[~r]; }
__device__ __forceinline__ int ref_lo(const TileLds &T, int r) { return r >= 0 ? T.in_lo[r] : T.lf_lo[~r]; }
__device__ __forceinline__ int ref_hi(const TileLds &T, int r) { return r >= 0 ? T.in_hi[r] : T.lf_hi[~r]; }

// Levels of the local tree, top down, into T.order / T.lvl_start.  Block-wide.
__device__ void compute_levels(TileLds &T) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        T.order[0] = 0;
        T.lvl_start[0] = 0;
        T.lvl_start[1] = 1;
        T.n_levels = 1;
    }
    __syncthreads();
    for (int lv = 0; lv < kMaxLevels; ++lv) {
        const int b0 = T.lvl_start[lv], b1 = T.lvl_start[lv + 1];
        if (b0 == b1)
            break;
        __shared__ int next;
        if (tid == 0)
            next = b1;
        __syncthreads();
        for (int i = b0 + tid; i < b1; i += blockDim.x) {
            const int j = T.order[i];
            for (int side = 0; side < 2; ++side) {
                const int c = T.in_child[side][j];
                if (c >= 0 && c < kTile) {
                    const int slot = atomicAdd(&next, 1);
                    if (slot < kTile)
                        T.order[slot] = c;
                }
            }
        }
        __syncthreads();
        if (tid == 0) {
            T.lvl_start[lv + 2] = next < kTile ? next : kTile;
            if (next > b1)
                T.n_levels = lv + 2;
        }
        __syncthreads();
    }
}

// Cost, count and leaf span of internal node j from its children.
__device__ __forceinline__ float node_cost(const TileLds &T, int j) {
    return kCostNode * half_area(T.in_box[0][j], T.in_box[1][j], T.in_box[2][j], T.in_box[3][j], T.in_box[4][j],
                                 T.in_box[5][j]) +
           ref_cost(T, T.in_child[0][j]) + ref_cost(T, T.in_child[1][j]);
}

__device__ void refresh_level(TileLds &T, int lv) {
    for (int i = T.lvl_start[lv] + threadIdx.x; i < T.lvl_start[lv + 1]; i += blockDim.x) {
        const int j = T.order[i];
        const int c0 = T.in_child[0][j], c1 = T.in_child[1][j];
        T.in_cost[j] = node_cost(T, j);
        T.in_count[j] = ref_count(T, c0) + ref_count(T, c1);
        T.in_lo[j] = min(ref_lo(T, c0), ref_lo(T, c1));
        T.in_hi[j] = max(ref_hi(T, c0), ref_hi(T, c1));
    }
}

// Every internal node from its children, deepest level first.  Block-wide.
__device__ void refresh_bottom_up(TileLds &T) {
    for (int lv = T.n_levels - 1; lv >= 0; --lv) {
        refresh_level(T, lv);
        __syncthreads();
    }
}

// One wave restructures the treelet rooted at local node p (wave-uniform call).
__device__ void optimize_treelet(TileLds &T, int p, int w) {
    const int lane = threadIdx.x & 63;
    float *area = T.w_area[w];
    float *cost = T.w_cost[w];
    unsigned char *split = T.w_split[w];
    if (lane == 0) {
        int leaf[kTreelet], inner[kTreelet];
        leaf[0] = T.in_child[0][p];
        leaf[1] = T.in_child[1][p];
        inner[0] = p;
        int m = 2;
        while (m < kTreelet) {
            int best = -1;
            float best_a = -1.0f;
            for (int i = 0; i < m; ++i) {
                const int r = leaf[i];
                if (r >= 0) {
                    const float a = half_area(T.in_box[0][r], T.in_box[1][r], T.in_box[2][r], T.in_box[3][r],
                                              T.in_box[4][r], T.in_box[5][r]);
                    if (a > best_a) {
                        best_a = a;
                        best = i;
                    }
                }
            }
            if (best < 0)
                break;
            const int r = leaf[best];
            inner[m - 1] = r;
            leaf[best] = T.in_child[0][r];
            leaf[m] = T.in_child[1][r];
            ++m;
        }
        for (int i = 0; i < m; ++i)
            T.w_leaf[w][i] = leaf[i];
        for (int i = 0; i < m - 1; ++i)
            T.w_int[w][i] = inner[i];
        T.w_m[w] = m;
    }
    lds_sync_wave();
    const int m = T.w_m[w];
    const int full = (1 << m) - 1;
    if (m < 3)
        return;  // two leaves: one topology only
    // areas of every subset, and the costs of single leaves
    for (int S = lane; S <= full; S += 64) {
        if (S == 0)
            continue;
        float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        for (int i = 0; i < m; ++i)
            if ((S >> i) & 1) {
                const int r = T.w_leaf[w][i];
                for (int a = 0; a < 3; ++a) {
                    b[a] = fminf(b[a], ref_box(T, r, a));
                    b[3 + a] = fmaxf(b[3 + a], ref_box(T, r, 3 + a));
                }
            }
        area[S] = half_area(b[0], b[1], b[2], b[3], b[4], b[5]);
        if ((S & (S - 1)) == 0)
            cost[S] = ref_cost(T, T.w_leaf[w][__builtin_ctz(S)]);
    }
    lds_sync_wave();
    // least cost of every subset of 2 .. m leaves, by size; a split P always
    // holds the subset's lowest leaf, so each unordered pair is seen once
    for (int size = 2; size <= m; ++size) {
        for (int S = lane; S <= full; S += 64) {
            if (__builtin_popcount(S) != size)
                continue;
            const int low = S & -S, rest = S ^ low;
            float best = INFINITY;
            int best_p = low;
            for (int sub = (rest - 1) & rest;; sub = (sub - 1) & rest) {
                const int P = low | sub;
                const float c = cost[P] + cost[S ^ P];
                if (c < best) {
                    best = c;
                    best_p = P;
                }
                if (sub == 0)
                    break;
            }
            cost[S] = kCostNode * area[S] + best;
            split[S] = (unsigned char)best_p;
        }
        lds_sync_wave();
    }
    // rewire only when the treelet gets cheaper than it is now (its subtrees
    // below may have changed this round: take the children's current costs)
    if (lane == 0 && cost[full] < node_cost(T, p) * (1.0f - 1e-6f)) {
        int free_slot = 1;  // T.w_int[w][0] is the root p
        int stack_set[kTreelet], stack_node[kTreelet], sp = 0;
        stack_set[sp] = full;
        stack_node[sp] = p;
        ++sp;
        while (sp > 0) {
            --sp;
            const int S = stack_set[sp], j = stack_node[sp];
            const int P = split[S], Q = S ^ P;
            const int parts[2] = {P, Q};
            for (int side = 0; side < 2; ++side) {
                const int part = parts[side];
                int child;
                if ((part & (part - 1)) == 0) {
                    child = T.w_leaf[w][__builtin_ctz(part)];
                } else {
                    child = T.w_int[w][free_slot++];
                    stack_set[sp] = part;
                    stack_node[sp] = child;
                    ++sp;
                }
                T.in_child[side][j] = child;
            }
            float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
            int count = 0, lo = INT32_MAX, hi = INT32_MIN;
            for (int i = 0; i < m; ++i)
                if ((S >> i) & 1) {
                    const int r = T.w_leaf[w][i];
                    for (int a = 0; a < 3; ++a) {
                        b[a] = fminf(b[a], ref_box(T, r, a));
                        b[3 + a] = fmaxf(b[3 + a], ref_box(T, r, 3 + a));
                    }
                    count += ref_count(T, r);
                    lo = min(lo, ref_lo(T, r));
                    hi = max(hi, ref_hi(T, r));
                }
            for (int a = 0; a < 6; ++a)
                T.in_box[a][j] = b[a];
            T.in_cost[j] = cost[S];
            T.in_count[j] = count;
            T.in_lo[j] = lo;
            T.in_hi[j] = hi;
        }
    }
    lds_sync_wave();
}

// Restructure the local tree in T (loaded, costs and levels not yet known).
__device__ void restructure_local(TileLds &T, int rounds) {
    const int w = threadIdx.x >> 6;
    compute_levels(T);
    refresh_bottom_up(T);
    for (int round = 0; round < rounds; ++round) {
        for (int lv = T.n_levels - 1; lv >= 0; --lv) {
            const int b0 = T.lvl_start[lv], b1 = T.lvl_start[lv + 1];
            for (int i = b0 + w; i < b1; i += kWaves) {  // wave-uniform
                const int j = T.order[i];
                if (T.in_count[j] >= kTreelet)
                    optimize_treelet(T, j, w);
            }
            __syncthreads();
            refresh_level(T, lv);  // costs above depend on this level's new subtrees
            __syncthreads();
        }
        compute_levels(T);
        refresh_bottom_up(T);
    }
}

// Load the subtree below global node `root` (an internal node) into T; a
// child becomes a local leaf when it is a leaf or when stop(child) says so
// (the nodes above the tiles stop at the tile roots).  Block-wide.
template <typename Stop, typename LeafCost>
__device__ void load_tree(TileLds &T, const Node *__restrict__ nodes, int root, Stop stop, LeafCost leaf_cost) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        T.n_in = 1;
        T.n_lf = 0;
        T.overflow = 0;
        T.in_slot[0] = root;
        T.lvl_start[0] = 0;
        T.lvl_start[1] = 1;
    }
    __syncthreads();
    // the root's own box: the union of its children's boxes
    for (int lv = 0; lv < kMaxLevels; ++lv) {
        const int b0 = T.lvl_start[lv], b1 = T.lvl_start[lv + 1];
        if (b0 == b1 || T.overflow)
            break;
        for (int j = b0 + tid; j < b1; j += blockDim.x) {
            const Node *nd = nodes + T.in_slot[j];
            const float4 L = nd->xy_left, R = nd->xy_right, Z = nd->z_both;
            const int4 refs = nd->refs;
            const float cb[2][6] = {{L.x, L.z, Z.x, L.y, L.w, Z.y}, {R.x, R.z, Z.z, R.y, R.w, Z.w}};
            if (j == 0)
                for (int a = 0; a < 3; ++a) {
                    T.in_box[a][0] = fminf(cb[0][a], cb[1][a]);
                    T.in_box[3 + a][0] = fmaxf(cb[0][3 + a], cb[1][3 + a]);
                }
            const int child[2] = {refs.x, refs.y};
            for (int side = 0; side < 2; ++side) {
                const int c = child[side];
                if (c >= 0 && !stop(c)) {
                    const int id = atomicAdd(&T.n_in, 1);
                    if (id >= kTile) {
                        T.overflow = 1;
                        continue;
                    }
                    T.in_slot[id] = c;
                    for (int a = 0; a < 6; ++a)
                        T.in_box[a][id] = cb[side][a];
                    T.in_child[side][j] = id;
                } else {
                    const int id = atomicAdd(&T.n_lf, 1);
                    if (id >= kTile) {
                        T.overflow = 1;
                        continue;
                    }
                    T.lf_ref[id] = c;
                    for (int a = 0; a < 6; ++a)
                        T.lf_box[a][id] = cb[side][a];
                    int count, lo, hi;
                    const float cost = leaf_cost(c, cb[side], count, lo, hi);
                    T.lf_cost[id] = cost;
                    T.lf_count[id] = count;
                    T.lf_lo[id] = lo;
                    T.lf_hi[id] = hi;
                    T.in_child[side][j] = ~id;
                }
            }
        }
        __syncthreads();
        if (tid == 0)
            T.lvl_start[lv + 2] = T.n_in < kTile ? T.n_in : kTile;
        __syncthreads();
    }
}

// Write the local tree back: node words, parents; returns nothing.  Block-wide.
__device__ void store_tree(const TileLds &T, Node *nodes, int32_t *parent, int n) {
    for (int j = threadIdx.x; j < T.n_in; j += blockDim.x) {
        const int g = T.in_slot[j];
        int gref[2];
        float b[2][6];
        for (int side = 0; side < 2; ++side) {
            const int c = T.in_child[side][j];
            if (c >= 0) {
                gref[side] = T.in_slot[c];
                for (int a = 0; a < 6; ++a)
                    b[side][a] = T.in_box[a][c];
            } else {
                gref[side] = T.lf_ref[~c];
                for (int a = 0; a < 6; ++a)
                    b[side][a] = T.lf_box[a][~c];
            }
            const int pslot = gref[side] >= 0 ? gref[side] : (n - 1) + ~gref[side];
            parent[pslot] = g;
        }
        Node *nd = nodes + g;
        nd->xy_left = make_float4(b[0][0], b[0][3], b[0][1], b[0][4]);
        nd->xy_right = make_float4(b[1][0], b[1][3], b[1][1], b[1][4]);
        nd->z_both = make_float4(b[0][2], b[0][5], b[1][2], b[1][5]);
        nd->refs = make_int4(gref[0], gref[1], T.in_lo[j], T.in_hi[j]);
    }
}

__device__ __forceinline__ float tri_cost(const float *b) {
    return kCostTri * half_area(b[0], b[1], b[2], b[3], b[4], b[5]);
}

// One workgroup per tile of the radix-tree kernel's list.
__global__ __launch_bounds__(kTile) void k_restructure_tiles(Node *nodes, int32_t *parent, int n,
                                                             const int32_t *__restrict__ tiles,
                                                             const int32_t *__restrict__ n_tiles,
                                                             float *__restrict__ tile_cost, int rounds) {
    extern __shared__ char lds[];
    TileLds &T = *reinterpret_cast<TileLds *>(lds);
    const int total = *n_tiles;
    for (int e = blockIdx.x; e < total; e += gridDim.x) {
        const int c = tiles[e];
        if (c < 0)
            continue;  // a one-leaf tile
        auto stop = [](int) { return false; };
        auto leaf_cost = [](int ref, const float *b, int &count, int &lo, int &hi) {
            count = 1;
            lo = hi = ~ref;
            return tri_cost(b);
        };
        load_tree(T, nodes, c, stop, leaf_cost);
        if (!T.overflow) {
            restructure_local(T, rounds);
            store_tree(T, nodes, parent, n);
            if (threadIdx.x == 0)
                tile_cost[c] = T.in_cost[0];
        }
        __syncthreads();  // LDS is reused by the next tile
    }
}

// One workgroup: the nodes above the tiles (more than kTile leaves each),
// with the tiles as fixed leaves.  Skipped when they do not fit in LDS.
__global__ __launch_bounds__(kTile) void k_restructure_top(Node *nodes, int32_t *parent, int n,
                                                           const float *__restrict__ tile_cost, int rounds) {
    extern __shared__ char lds[];
    TileLds &T = *reinterpret_cast<TileLds *>(lds);
    const Node *cn = nodes;
    auto count_of = [cn](int c) { return c < 0 ? 1 : cn[c].refs.w - cn[c].refs.z + 1; };
    if (count_of(0) <= kTile)
        return;  // the whole tree is one tile
    auto stop = [count_of](int c) { return count_of(c) <= kTile; };
    auto leaf_cost = [cn, tile_cost](int ref, const float *b, int &count, int &lo, int &hi) {
        if (ref < 0) {
            count = 1;
            lo = hi = ~ref;
            return tri_cost(b);
        }
        lo = cn[ref].refs.z;
        hi = cn[ref].refs.w;
        count = hi - lo + 1;
        return tile_cost[ref];
    };
    load_tree(T, nodes, 0, stop, leaf_cost);
    if (T.overflow)
        return;
    restructure_local(T, rounds);
    store_tree(T, nodes, parent, n);
}

}  // namespace

size_t restructure_lds_bytes() { return sizeof(TileLds); }

hipError_t launch_restructure(MeshDev &m, int rounds, hipStream_t s) {
    if (m.nt < kTreelet)
        return hipSuccess;
    int32_t *n_tiles = static_cast<int32_t *>(m.sort_tmp);  // the radix-tree kernel's tile list
    int32_t *tiles = n_tiles + 64;
    float *tile_cost = reinterpret_cast<float *>(tiles + ((m.nt + 63) & ~int64_t(63)));
    const size_t lds = sizeof(TileLds);
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_restructure_tiles),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_restructure_top),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr_set = true;
    }
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t want = (m.nt + kTile - 1) / kTile * 2;  // tiles hold up to kTile leaves, usually fewer
    const int grid = (int)(want < cus ? want : cus);
    k_restructure_tiles<<<grid, kTile, lds, s>>>(m.nodes, m.parent, (int)m.nt, tiles, n_tiles, tile_cost, rounds);
    k_restructure_top<<<1, kTile, lds, s>>>(m.nodes, m.parent, (int)m.nt, tile_cost, rounds);
    return hipGetLastError();
}

}  // namespace rsi
