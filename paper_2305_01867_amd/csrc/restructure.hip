// restructure.hip -- treelet restructuring of the BVH on gfx950.
//
// The radix tree over Morton codes splits space at fixed midpoints; for
// segments that cross a surface, the total surface area of its boxes (which
// is what a random segment's node visits follow) is well above what a
// surface-area-heuristic tree reaches.  Treelet restructuring (Karras & Aila
// 2013, "Fast parallel construction of high-quality bounding volume
// hierarchies") improves it in place: bottom-up, each node with enough leaves
// becomes the root of a treelet (grown by opening the largest-area internal
// leaf), and the treelet's internal nodes are rebuilt in the topology of
// least SAH cost, found by dynamic programming over the subsets of its
// leaves.  Treelets of 4 leaves (15 subsets) keep that search in one lane's
// registers, so all treelets of a level run at once; a few passes reach most
// of what 7-leaf treelets give.  The leaves (sorted triangles) do not move;
// only internal nodes are rewired, so every query result stays the same.
//
// On gfx950 the work is kept inside workgroups: one workgroup loads a whole
// tile (a subtree of at most 1024 leaves, listed by the radix-tree kernel)
// into LDS in one step, restructures it height by height (the nodes of one
// height compacted onto consecutive lanes, a treelet optimised per node), and
// writes it back.  No cross-workgroup synchronisation at all.  The few nodes
// above the tiles are left as the radix tree made them: restructuring them too
// (one more workgroup, the tiles as fixed leaves) cost more build time than it
// saved traversal time at every measured mesh size, 32 K to 526 K triangles.
//
// After restructuring, an internal node's leaves are no longer a contiguous
// range of sorted positions: words 14 / 15 of a node then hold the smallest
// and largest sorted leaf below it (the root still spans every leaf).
#include "rsi_internal.h"

namespace rsi {
namespace {

constexpr int kTile = 1024;            // leaves per tile
constexpr int kThreads = 512;          // lanes per workgroup (256 VGPRs per lane, no spills)
constexpr int kTreelet = 4;            // leaves per treelet (the optimisation runs in one lane's registers)
constexpr float kCostNode = 1.2f;      // SAH weight of a node visit (one 64-B node, two box tests)
constexpr float kCostTri = 1.0f;       // SAH weight of a triangle test

// LDS image of one (sub)tree, nodes and leaves in one index space: a local
// reference c below kTile is internal node c (local ids are offsets from the
// tile's first internal node), c >= kTile is leaf c - kTile.  Every per-node
// quantity is then one LDS read, whichever kind the reference is.
struct TileLds {
    int child[2][kTile];         // local references of internal node j's children
    int slot[kTile];             // global internal node index of internal node j
    int lf_ref[kTile];           // global reference of leaf k (a leaf ~g)
    float box[6][2 * kTile];     // own box of reference c: lo xyz, hi xyz
    float cost[2 * kTile];       // SAH cost of the subtree
    int count[2 * kTile];        // leaves below
    int lo[2 * kTile], hi[2 * kTile];  // smallest / largest sorted leaf below
    int parent[2 * kTile];       // local parent (internal), -1 at the root
    int arrive[kTile + 2];       // arrivals of the height climb, then per-height counters
    int height[kTile];           // 1 + the larger child height (a leaf is 0)
    int order[kTile];            // internal nodes by rising height
    int h_start[kTile + 2];      // order[h_start[h] .. h_start[h + 1]) have height h
    int n_in, n_lf, max_height;
};

__device__ __forceinline__ float half_area(float x0, float y0, float z0, float x1, float y1, float z1) {
    const float dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
    return dx * dy + dy * dz + dz * dx;  // half the surface area; the common factor 2 cancels in comparisons
}

__device__ __forceinline__ float box_area(const TileLds &T, int c) {
    return half_area(T.box[0][c], T.box[1][c], T.box[2][c], T.box[3][c], T.box[4][c], T.box[5][c]);
}

// Cost, count and leaf span of internal node j from its children.
__device__ __forceinline__ void refresh_node(TileLds &T, int j) {
    const int c0 = T.child[0][j], c1 = T.child[1][j];
    T.cost[j] = kCostNode * box_area(T, j) + T.cost[c0] + T.cost[c1];
    T.count[j] = T.count[c0] + T.count[c1];
    T.lo[j] = min(T.lo[c0], T.lo[c1]);
    T.hi[j] = max(T.hi[c0], T.hi[c1]);
}

// Splits of the subsets of four treelet leaves: {subset, part holding the
// subset's lowest leaf, last split of this subset}.
constexpr int kSplitCount = 25;
__device__ constexpr unsigned char kSplits[kSplitCount][3] = {
    {3, 1, 1},   {5, 1, 1},   {6, 2, 1},   {9, 1, 1},   {10, 2, 1},  {12, 4, 1},  {7, 1, 0},
    {7, 3, 0},   {7, 5, 1},   {11, 1, 0},  {11, 3, 0},  {11, 9, 1},  {13, 1, 0},  {13, 5, 0},
    {13, 9, 1},  {14, 2, 0},  {14, 6, 0},  {14, 10, 1}, {15, 1, 0},  {15, 3, 0},  {15, 5, 0},
    {15, 7, 0},  {15, 9, 0},  {15, 11, 0}, {15, 13, 1}};

// One lane restructures the treelet of up to kTreelet (4) leaves rooted at
// local node p: it opens the largest-area internal leaf twice, finds the
// least-cost topology over the 15 leaf subsets with every subset and split
// known at compile time (all in registers), and rewires the (at most three)
// internal nodes when that is cheaper than the current shape.
// The treelet at p (children c0, c1): opens the largest-area internal leaf
// twice; returns the number of treelet leaves (2 to 4) in leaf[], with the
// opened nodes in inner[1..] (inner[0] = p).
__device__ __forceinline__ int open_treelet(const TileLds &T, int p, int c0, int c1, int leaf[4], int inner[3]) {
    leaf[0] = c0;
    leaf[1] = c1;
    leaf[2] = leaf[3] = 0;
    inner[0] = p;
    inner[1] = inner[2] = -1;
    int m = 2;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        int best = -1;
        float best_a = -1.0f;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int r = leaf[i];
            if (i < m && r < kTile) {
                const float a = box_area(T, r);
                if (a > best_a) {
                    best_a = a;
                    best = i;
                }
            }
        }
        if (best < 0)
            break;
        int r = leaf[0];
#pragma unroll
        for (int i = 1; i < 3; ++i)
            r = best == i ? leaf[i] : r;
        const int d0 = T.child[0][r], d1 = T.child[1][r];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            leaf[i] = i == best ? d0 : leaf[i];
            leaf[i] = i == m ? d1 : leaf[i];
        }
#pragma unroll
        for (int i = 1; i < 3; ++i)
            inner[i] = i == m - 1 ? r : inner[i];
        ++m;
    }
    return m;
}

__device__ __forceinline__ void optimize_treelet(TileLds &T, int p) {
    int leaf[4], inner[3];
    const float now = T.cost[p];
    const int m = open_treelet(T, p, T.child[0][p], T.child[1][p], leaf, inner);
    if (m < 3)
        return;  // both children are leaves: one shape only
    // every subset's box, leaf count and leaf span, each from the subset
    // without its lowest leaf (with three leaves the fourth repeats the first
    // and only subsets of the first three are used)
    float sb[16][6], area[16];
    int sn[16], slo[16], shi[16];
    float cost[16], best_sum[16];
    int split[16];
#pragma unroll
    for (int S = 1; S < 16; ++S) {
        const int i = __builtin_ctz(S), R = S & (S - 1);
        const int r = i < m ? leaf[i] : leaf[0];
        if (R == 0) {
#pragma unroll
            for (int a = 0; a < 6; ++a)
                sb[S][a] = T.box[a][r];
            sn[S] = T.count[r];
            slo[S] = T.lo[r];
            shi[S] = T.hi[r];
            cost[S] = T.cost[r];
        } else {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                sb[S][a] = fminf(sb[R][a], sb[1 << i][a]);
                sb[S][3 + a] = fmaxf(sb[R][3 + a], sb[1 << i][3 + a]);
            }
            sn[S] = sn[R] + sn[1 << i];
            slo[S] = min(slo[R], slo[1 << i]);
            shi[S] = max(shi[R], shi[1 << i]);
            cost[S] = INFINITY;
        }
        area[S] = half_area(sb[S][0], sb[S][1], sb[S][2], sb[S][3], sb[S][4], sb[S][5]);
        best_sum[S] = INFINITY;
        split[S] = 0;
    }
    cost[0] = 0.0f;
    // every split (S, P | S^P) of a subset S of two or more leaves, with P
    // holding S's lowest leaf so each unordered pair appears once, listed by
    // subset size so a subset's parts are done before it; the flag marks a
    // subset's last split
#pragma unroll
    for (int e = 0; e < kSplitCount; ++e) {
        const int S = kSplits[e][0], P = kSplits[e][1];
        const float c = cost[P] + cost[S ^ P];
        if (c < best_sum[S]) {
            best_sum[S] = c;
            split[S] = P;
        }
        if (kSplits[e][2])
            cost[S] = kCostNode * area[S] + best_sum[S];
    }
    const int full = (1 << m) - 1;
    const float best_cost = m == 4 ? cost[15] : cost[7];
    if (!(best_cost < now * (1.0f - 1e-6f)))
        return;
    // mark the subsets the chosen topology uses, from the whole set down (the
    // table read backwards is by falling subset size); every index below is
    // known at compile time, so all of this stays in registers
    bool used[16];
#pragma unroll
    for (int S = 0; S < 16; ++S)
        used[S] = S == full;
#pragma unroll
    for (int e = kSplitCount - 1; e >= 0; --e) {
        const int S = kSplits[e][0], P = kSplits[e][1];
        if (used[S] && split[S] == P)
            used[P] = used[S ^ P] = true;
    }
    // node ids: the root keeps p, further internal subsets take the opened
    // nodes in turn
    int node[16];
    int taken = 1;
#pragma unroll
    for (int S = 15; S >= 3; --S) {
        node[S] = p;
        if (__builtin_popcount(S) >= 2 && S != full && used[S]) {
            node[S] = taken == 1 ? inner[1] : inner[2];
            ++taken;
        }
    }
    // write each used internal subset
#pragma unroll
    for (int S = 3; S < 16; ++S) {
        if (__builtin_popcount(S) < 2 || !used[S])
            continue;
        int child0 = 0, child1 = 0;
#pragma unroll
        for (int e = 0; e < kSplitCount; ++e) {
            if (kSplits[e][0] != S)
                continue;
            const int P = kSplits[e][1], Q = S ^ P;
            if (split[S] == P) {
                child0 = __builtin_popcount(P) == 1 ? leaf[__builtin_ctz(P)] : node[P];
                child1 = __builtin_popcount(Q) == 1 ? leaf[__builtin_ctz(Q)] : node[Q];
            }
        }
        const int j = node[S];
        T.child[0][j] = child0;
        T.child[1][j] = child1;
        T.parent[child0] = j;
        T.parent[child1] = j;
#pragma unroll
        for (int a = 0; a < 6; ++a)
            T.box[a][j] = sb[S][a];
        T.cost[j] = cost[S];
        T.count[j] = sn[S];
        T.lo[j] = slo[S];
        T.hi[j] = shi[S];
    }
}

// The same step for a level with few nodes: kGroup lanes of one wave share
// the node p, and lane g takes the leaf subset S = g.  Each lane unions its
// subset's boxes; a pair's cost follows from its leaves, a triple's from the
// pairs of the lanes that own them (shuffles), and every lane evaluates the
// whole set's splits, so the choice is the same in each.  The splits are
// tried in the order of kSplits with the same strict comparison, so the
// choice is the single-lane search's up to rounding order (the compiler may
// fuse the cost sums differently; a near tie can then go the other way).
// base is the group's first lane in the wave; control flow is uniform over
// the group.
constexpr int kGroup = 16;

__device__ __forceinline__ void treelet_group(TileLds &T, int p, int g, int base) {
    const int c0 = T.child[0][p], c1 = T.child[1][p];
    const float now = kCostNode * box_area(T, p) + T.cost[c0] + T.cost[c1];
    const int cnt = T.count[c0] + T.count[c1];
    if (g == 0) {  // refresh p
        T.cost[p] = now;
        T.count[p] = cnt;
        T.lo[p] = min(T.lo[c0], T.lo[c1]);
        T.hi[p] = max(T.hi[c0], T.hi[c1]);
    }
    if (cnt < kTreelet)
        return;
    int leaf[4], inner[3];
    const int m = open_treelet(T, p, c0, c1, leaf, inner);
    if (m < 3)
        return;
    // this lane's subset (with three leaves the fourth repeats the first; only
    // subsets of the first three are used then)
    const int S = g;
    float b[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    float lc[4];
    int n = 0, lo = INT32_MAX, hi = INT32_MIN;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = i < m ? leaf[i] : leaf[0];
        lc[i] = T.cost[r];
        if ((S >> i) & 1) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                b[a] = fminf(b[a], T.box[a][r]);
                b[3 + a] = fmaxf(b[3 + a], T.box[3 + a][r]);
            }
            n += T.count[r];
            lo = min(lo, T.lo[r]);
            hi = max(hi, T.hi[r]);
        }
    }
    const float area = half_area(b[0], b[1], b[2], b[3], b[4], b[5]);
    const int pc = __builtin_popcount(S);
    // the subset's leaves in rising order (a < e1 < e2 where present)
    const int a = __builtin_ctz(S | 16), R = S & (S - 1);
    const int e1 = __builtin_ctz(R | 16), e2 = __builtin_ctz((R & (R - 1)) | 16);
    float c = INFINITY;
    int split = 0;
    if (pc == 1) {
        c = lc[a];
    } else if (pc == 2) {
        const float sum = lc[a] + lc[e1 & 3];
        c = kCostNode * area + sum;
        split = 1 << a;
    }
    // triples: {a} | {e1, e2}, {a, e1} | {e2}, {a, e2} | {e1}
    {
        const int pa = 1 << (a & 3), p1 = 1 << (e1 & 3), p2 = 1 << (e2 & 3);
        const float v1 = __shfl(c, base + (p1 | p2), 64);
        const float v2 = __shfl(c, base + (pa | p1), 64);
        const float v3 = __shfl(c, base + (pa | p2), 64);
        if (pc == 3) {
            float best = lc[a & 3] + v1;
            int P = pa;
            const float s2 = v2 + lc[e2 & 3];
            if (s2 < best) {
                best = s2;
                P = pa | p1;
            }
            const float s3 = v3 + lc[e1 & 3];
            if (s3 < best) {
                best = s3;
                P = pa | p2;
            }
            c = kCostNode * area + best;
            split = P;
        }
    }
    // the whole set, evaluated in every lane: the cost of each part from its lane
    float ck[16];
#pragma unroll
    for (int k = 3; k < 16; ++k)
        if (__builtin_popcount(k) >= 2)
            ck[k] = __shfl(c, base + k, 64);
    int full, Pf;
    float best_cost;
    if (m == 4) {
        const float s[7] = {lc[0] + ck[14], ck[3] + ck[12], ck[5] + ck[10], ck[7] + lc[3],
                            ck[9] + ck[6], ck[11] + lc[2], ck[13] + lc[1]};
        const int P7[7] = {1, 3, 5, 7, 9, 11, 13};
        float best = s[0];
        int P = 1;
#pragma unroll
        for (int k = 1; k < 7; ++k)
            if (s[k] < best) {
                best = s[k];
                P = P7[k];
            }
        best_cost = kCostNode * __shfl(area, base + 15, 64) + best;
        full = 15;
        Pf = P;
        if (S == 15) {
            c = best_cost;
            split = P;
        }
    } else {
        best_cost = ck[7];
        full = 7;
        Pf = __shfl(split, base + 7, 64);
    }
    const int Xs = __shfl(split, base + (__builtin_popcount(Pf) == 3 ? Pf : (full ^ Pf)), 64);
    if (!(best_cost < now * (1.0f - 1e-6f)))
        return;
    // the internal subsets of the chosen topology: the whole set, its parts
    // of two or more leaves, and the parts of a triple among them
    const int Qf = full ^ Pf;
    int used = 1 << full;
    used |= __builtin_popcount(Pf) >= 2 ? 1 << Pf : 0;
    used |= __builtin_popcount(Qf) >= 2 ? 1 << Qf : 0;
    const int X = __builtin_popcount(Pf) == 3 ? Pf : (__builtin_popcount(Qf) == 3 ? Qf : 0);
    if (X) {
        const int Px = Xs, Qx = X ^ Xs;
        used |= __builtin_popcount(Px) >= 2 ? 1 << Px : 0;
        used |= __builtin_popcount(Qx) >= 2 ? 1 << Qx : 0;
    }
    // node ids: the whole set keeps p, the others take the opened nodes by
    // falling subset index
    const int others = used & ~(1 << full);
    auto ref_of = [&](int U) {
        if (__builtin_popcount(U) == 1) {
            const int i = __builtin_ctz(U);
            return i == 0 ? leaf[0] : (i == 1 ? leaf[1] : (i == 2 ? leaf[2] : leaf[3]));
        }
        if (U == full)
            return p;
        return __builtin_popcount(others >> (U + 1)) == 0 ? inner[1] : inner[2];
    };
    if ((used >> S) & 1) {
        const int j = ref_of(S);
        const int child0 = ref_of(split), child1 = ref_of(S ^ split);
        T.child[0][j] = child0;
        T.child[1][j] = child1;
        T.parent[child0] = j;
        T.parent[child1] = j;
#pragma unroll
        for (int k = 0; k < 6; ++k)
            T.box[k][j] = b[k];
        T.cost[j] = c;
        T.count[j] = n;
        T.lo[j] = lo;
        T.hi[j] = hi;
    }
}

// Heights of the local internal nodes by a bottom-up climb, one lane per
// leaf: the second lane to reach a node finds both child heights final.
// Integer work only, so the divergence of the climb costs little.
__device__ __forceinline__ void local_heights(TileLds &T) {
    for (int j = threadIdx.x; j < T.n_in; j += blockDim.x) {
        T.arrive[j] = 0;
        T.height[j] = 0;
    }
    if (threadIdx.x == 0)
        T.max_height = 0;
    __syncthreads();
    for (int k = threadIdx.x; k < T.n_lf; k += blockDim.x) {
        int j = T.parent[kTile + k];
        for (int step = 0; j >= 0 && step < T.n_in; ++step) {  // a climb is at most n_in nodes long
            if (__hip_atomic_fetch_add(&T.arrive[j], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == 0)
                break;  // the other subtree is still on its way
            const int c0 = T.child[0][j], c1 = T.child[1][j];
            const int h = 1 + max(c0 < kTile ? T.height[c0] : 0, c1 < kTile ? T.height[c1] : 0);
            T.height[j] = h;
            if (T.parent[j] < 0)
                T.max_height = h;  // the local root is the highest node
            j = T.parent[j];
        }
    }
    __syncthreads();
}

// Internal nodes grouped by height into T.order, with T.h_start[h] the first
// position of height h (a counting sort in LDS; the order inside a height
// does not matter, its nodes are independent).
__device__ __forceinline__ void order_by_height(TileLds &T) {
    const int H = T.max_height;
    for (int h = threadIdx.x; h <= H; h += blockDim.x)
        T.arrive[h] = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < T.n_in; j += blockDim.x) {
        const int h = T.height[j];
        if (h >= 1 && h <= H)  // always, in a tree the climb reached whole
            atomicAdd(&T.arrive[h], 1);
    }
    __syncthreads();
    if (threadIdx.x < 64) {  // exclusive scan of the counts by the first wave
        const int lane = threadIdx.x;
        int carry = 0;
        for (int base = 0; base <= H + 1; base += 64) {
            const int h = base + lane;
            const int v = h <= H ? T.arrive[h] : 0;
            int incl = v;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int u = __shfl_up(incl, d, 64);
                incl += lane >= d ? u : 0;
            }
            if (h <= H + 1)
                T.h_start[h] = carry + incl - v;
            carry += __shfl(incl, 63, 64);
        }
    }
    __syncthreads();
    for (int h = threadIdx.x; h <= H; h += blockDim.x)
        T.arrive[h] = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < T.n_in; j += blockDim.x) {
        const int h = T.height[j];
        if (h >= 1 && h <= H)
            T.order[T.h_start[h] + atomicAdd(&T.arrive[h], 1)] = j;
    }
    __syncthreads();
}

// Restructure the local tree in T (loaded, with parents; costs not yet
// known).  Each pass visits the internal nodes by rising height (the heights
// of the tree the pass starts from), so both subtrees of a node are final
// when it is visited, and the nodes of one height, whose subtrees are
// disjoint, run side by side on consecutive lanes: each refreshes its box
// cost and optimises the treelet rooted there, which lies inside its own
// subtree.  Compacting a height onto consecutive lanes keeps the long
// treelet optimisation from running once per wave for a few active lanes,
// as a climb from the leaves would.
__device__ __forceinline__ void restructure_local(TileLds &T, int rounds) {
    for (int round = 0; round < rounds; ++round) {
        local_heights(T);
        order_by_height(T);
        const int H = T.max_height;
        for (int h = 1; h <= H; ++h) {
            const int b = T.h_start[h], e = T.h_start[h + 1];
            if ((e - b) * kGroup <= (int)blockDim.x) {
                // few nodes (the upper levels, where the search's latency
                // adds up level by level): a lane group per node
                const int g = threadIdx.x / kGroup;
                if (b + g < e)
                    treelet_group(T, T.order[b + g], threadIdx.x & (kGroup - 1), threadIdx.x & 63 & ~(kGroup - 1));
            } else {
                for (int i = b + threadIdx.x; i < e; i += blockDim.x) {
                    const int j = T.order[i];
                    refresh_node(T, j);
                    if (T.count[j] >= kTreelet)
                        optimize_treelet(T, j);
                }
            }
            __syncthreads();
        }
    }
}

// Write the local tree back: node words, parents; returns nothing.  Block-wide.
// Load the radix-tree subtree rooted at internal node c in one parallel
// step.  In the radix-tree numbering a subtree over sorted leaves [a, b] is
// rooted at a or b and holds exactly the internal nodes [a, b - 1] (root a)
// or [a + 1, b] (root b), so local ids are offsets from that base and no
// traversal is needed.
__device__ void load_tile(TileLds &T, const Node *__restrict__ nodes, int c) {
    const int a = nodes[c].refs.z, b = nodes[c].refs.w;
    const int base = c == a ? a : a + 1;
    const int n_in = b - a < kTile ? b - a : 0;  // tiles hold at most kTile leaves
    for (int j = threadIdx.x; j < n_in; j += blockDim.x) {
        const Node *nd = nodes + base + j;
        const float4 L = nd->xy_left, R = nd->xy_right, Z = nd->z_both;
        const int4 refs = nd->refs;
        const float cb[2][6] = {{L.x, L.z, Z.x, L.y, L.w, Z.y}, {R.x, R.z, Z.z, R.y, R.w, Z.w}};
        T.slot[j] = base + j;
        const int child[2] = {refs.x, refs.y};
        for (int side = 0; side < 2; ++side) {
            const int g = child[side];
            const int id = g >= 0 ? g - base : kTile + (~g - a);
            T.parent[id] = j;
            for (int e = 0; e < 6; ++e)
                T.box[e][id] = cb[side][e];
            if (g < 0) {
                T.lf_ref[id - kTile] = g;
                T.cost[id] = kCostTri * half_area(cb[side][0], cb[side][1], cb[side][2], cb[side][3], cb[side][4],
                                                  cb[side][5]);
                T.count[id] = 1;
                T.lo[id] = T.hi[id] = ~g;
            }
            T.child[side][j] = id;
        }
        if (base + j == c) {
            T.parent[j] = -1;
            for (int e = 0; e < 3; ++e) {
                T.box[e][j] = fminf(cb[0][e], cb[1][e]);
                T.box[3 + e][j] = fmaxf(cb[0][3 + e], cb[1][3 + e]);
            }
        }
    }
    if (threadIdx.x == 0) {
        T.n_in = n_in;
        T.n_lf = n_in ? n_in + 1 : 0;
    }
    __syncthreads();
}

__device__ void store_tree(const TileLds &T, Node *nodes, int32_t *parent, int n) {
    for (int j = threadIdx.x; j < T.n_in; j += blockDim.x) {
        const int g = T.slot[j];
        int gref[2];
        float b[2][6];
        for (int side = 0; side < 2; ++side) {
            const int c = T.child[side][j];
            gref[side] = c < kTile ? T.slot[c] : T.lf_ref[c - kTile];
            for (int a = 0; a < 6; ++a)
                b[side][a] = T.box[a][c];
            const int pslot = gref[side] >= 0 ? gref[side] : (n - 1) + ~gref[side];
            parent[pslot] = g;
        }
        Node *nd = nodes + g;
        nd->xy_left = make_float4(b[0][0], b[0][3], b[0][1], b[0][4]);
        nd->xy_right = make_float4(b[1][0], b[1][3], b[1][1], b[1][4]);
        nd->z_both = make_float4(b[0][2], b[0][5], b[1][2], b[1][5]);
        nd->refs = make_int4(gref[0], gref[1], T.lo[j], T.hi[j]);
    }
}

// One workgroup per tile of the radix-tree kernel's list.
__global__ __launch_bounds__(kThreads) void k_restructure_tiles(Node *nodes, int32_t *parent, int n,
                                                             const int32_t *__restrict__ tiles,
                                                             const int32_t *__restrict__ n_tiles, int rounds) {
    extern __shared__ char lds[];
    TileLds &T = *reinterpret_cast<TileLds *>(lds);
    const int total = *n_tiles;
    for (int e = blockIdx.x; e < total; e += gridDim.x) {
        const int c = tiles[e];
        if (c < 0)
            continue;  // a one-leaf tile
        load_tile(T, nodes, c);
        restructure_local(T, rounds);
        store_tree(T, nodes, parent, n);
        __syncthreads();  // LDS is reused by the next tile
    }
}

}  // namespace

size_t restructure_lds_bytes() { return sizeof(TileLds); }

hipError_t launch_restructure(MeshDev &m, int rounds, hipStream_t s) {
    if (m.nt < kTreelet)
        return hipSuccess;
    const BuildLists L = build_lists(m.sort_tmp, m.nt);  // the radix-tree kernel's tile list
    int32_t *n_tiles = L.n_tiles;
    int32_t *tiles = L.tiles;
    const size_t lds = sizeof(TileLds);
    // above the default 64 KB of dynamic LDS: set per call (cheap on the host,
    // and right for whichever device is current; no shared flag between threads)
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_restructure_tiles),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t want = (m.nt + kTile - 1) / kTile * 2;  // tiles hold up to kTile leaves, usually fewer
    const int grid = (int)(want < cus ? want : cus);
    k_restructure_tiles<<<grid, kThreads, lds, s>>>(m.nodes, m.parent, (int)m.nt, tiles, n_tiles, rounds);
    return hipGetLastError();
}

}  // namespace rsi
