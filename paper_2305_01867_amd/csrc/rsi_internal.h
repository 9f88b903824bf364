// rsi_internal.h -- types and launchers shared by the library's own sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsi {

// Internal node: the boxes of both children plus the two child references
// (>= 0 internal node, < 0 leaf at sorted position ~ref).  One node is 64 B,
// fetched as four 16-byte loads; keeping the children's boxes in the parent
// lets one fetch decide both children.
struct alignas(16) Node {
    float4 xy_left;   // left  x lo, x hi, y lo, y hi
    float4 xy_right;  // right x lo, x hi, y lo, y hi
    float4 z_both;    // left z lo, z hi, right z lo, z hi
    int4 refs;        // left ref, right ref, first and last sorted leaf of the node
};
static_assert(sizeof(Node) == 64, "node must be 64 bytes");

// 4-wide node: the boxes of up to four children, stored axis by axis so a
// lane fetches 112 B (seven 16-byte loads) and tests all four with the same
// instructions.  A child reference is >= 0 for another 4-wide node (stored at
// the index of the binary internal node it was collapsed from), < 0 for the
// leaf at sorted position ~ref, kEmptyChild for an unused slot, whose box is
// +inf on every face so the slab test always misses it.  128 B: one L2 line.
struct alignas(16) Node4 {
    float4 lox, hix;  // x lo, x hi of children 0..3
    float4 loy, hiy;
    float4 loz, hiz;
    int4 child;
    int4 spare;
};
static_assert(sizeof(Node4) == 128, "4-wide node must be 128 bytes");
constexpr int32_t kEmptyChild = INT32_MIN;
// The first kTopSlots 4-wide nodes in breadth-first order from the root are
// also kept in a compact array (top4), which the traversal copies into LDS as
// far as its LDS budget allows.  A 4-wide child reference r >= 0 names top4[r]
// when r < kTopSlots and the node collapsed from binary node r - kTopSlots
// otherwise; the root is top4[0].  nodes4 directly follows top4 in memory
// (nodes4 = top4 + kTopSlots), so top4[r] addresses either kind.
constexpr int kTopSlots = 512;

// Leaf triangle in sorted order: first corner, the two edge vectors from it
// (rounded once, exactly as computing them on the fly would) and the input
// triangle index.  48 B, three 16-byte loads.
struct alignas(16) Tri {
    float4 a;   // A.xyz, triangle index (bit pattern of an int32)
    float4 e1;  // (B - A).xyz, 0
    float4 e2;  // (C - A).xyz, 0
};
static_assert(sizeof(Tri) == 48, "leaf triangle must be 48 bytes");

// Entries of the second pass's private stack per lane: above the radix tree's largest
// possible depth (97).  A restructured tree may be deeper; the second pass then
// tests the leaves of a subtree that finds no room, so no push is ever dropped.
constexpr int kDeepStack = 128;

// Learned proposal (mlp.hip): sizes of the network and its parameter vector
// [W1 (256 x 224), W2, W3, W4 (256 x 256), b1..b4 (256 each)], weights stored
// [out][in].
constexpr int kMlpBands = 16;
constexpr int kMlpFeat = 6 + 6 * 2 * kMlpBands;  // 198
constexpr int kMlpIn = 224;
constexpr int kMlpHidden = 256;
constexpr int kMlpOut = 256;
constexpr int kFrontierDepth = 8;
constexpr int64_t kMlpWeights = (int64_t)kMlpOut * kMlpIn + 3LL * kMlpHidden * kMlpHidden;
constexpr int64_t kMlpParams = kMlpWeights + 4LL * kMlpHidden;

struct Proposal {
    bool ready = false;      // parameters initialised or loaded
    int n_buckets = 0;       // host copy
    int64_t step = 0;        // Adam steps taken
    float *P = nullptr;      // fp32 master parameters [kMlpParams]
    float *G = nullptr;      // gradient [kMlpParams]
    float *m1 = nullptr, *m2 = nullptr;  // Adam moments
    __bf16 *Wb = nullptr;    // bf16 weights [kMlpWeights]
    __bf16 *WbT = nullptr;   // bf16 hidden weights transposed (layers 2..4, [in][out]) for the backward pass
    int32_t *bucket_ref = nullptr;    // [256] frontier node reference per bucket
    int32_t *bucket_first = nullptr;  // [256] first sorted leaf of each bucket
    int32_t *dev_n_buckets = nullptr; // [1]
    int32_t *rank = nullptr;          // [nt] sorted position of each triangle
    uint8_t *leaf_bucket = nullptr;   // [nt] bucket of each sorted leaf
    // 4-wide tree of the proposal order (meshes with a 4-wide tree): the
    // plain collapse with every frontier node starting a 4-wide node of its
    // own, laid out as the mesh's (kTopSlots top slots, then nt - 1 slots)
    Node4 *top4 = nullptr;
    int32_t *bucket_ref4 = nullptr;   // [256] frontier node reference per bucket in that tree
    int32_t *slot_bin = nullptr;      // [kTopSlots] binary index of each top slot
    int32_t *wide_flag = nullptr;     // [nt] collapse flags
    int32_t *wide_queue = nullptr;    // [nt] collapse queue
    void *block = nullptr;
};

// Device state of one built mesh.
struct MeshDev {
    int64_t nv = 0, nt = 0;
    int morton_bits = 30;
    int algorithm = 0;         // 0 radix tree + tiled bottom-up, 1 agglomerative single pass,
                               // 2 radix tree + treelet restructuring
    int root = 0;
    float *V = nullptr;        // [nv][3] copy of the vertices
    int32_t *F = nullptr;      // [nt][3] copy of the triangles
    void *keys = nullptr;      // [nt] sorted keys (uint32 or uint64)
    int32_t *ids = nullptr;    // [nt] triangle index at each sorted position
    Node *nodes = nullptr;     // [nt-1]
    Node4 *nodes4 = nullptr;   // [nt-1] slots; those of binary nodes that start a 4-wide node
    Node4 *top4 = nullptr;     // [kTopSlots] the top of the 4-wide tree, breadth-first
    int node_width = 2;        // 4 once the 4-wide tree is built (algorithms 0 and 2)
    int32_t *parent = nullptr; // [2nt-1]
    int32_t *counters = nullptr; // [nt-1]
    Tri *tris = nullptr;       // [nt]
    float *bounds = nullptr;   // [8]
    int32_t *flags = nullptr;  // [4]: [0] bad-index flag, [1] root of the agglomerative build
    void *sort_tmp = nullptr;  // key/id ping-pong + histograms
    int64_t bytes = 0;
    Proposal prop;
};

// Batched form (batch.hip): many meshes in one BVH.  Its work items are
// grouped, one group per XCD of the MI355X: the meshes are spread over the
// groups by estimated cost, so each XCD's L2 holds the trees of a few meshes.
constexpr int kItemGroups = 8;
// Batched keys: the mesh id (6 bits, at most 64 meshes) above a 30-bit Morton
// code over the mesh's own box, kept in 64-bit words.
constexpr int kBatchMortonBits = 30;
// Index in the traversal's queue words (after the queue length and the next
// segment) of the first per-group item counter; the batch's queue area holds
// them before its queue.
constexpr int kGroupNext = 8;
struct BatchDev {
    int M = 0;
    int64_t *v_off = nullptr, *t_off = nullptr;  // device [M + 1]
    int32_t *r_off = nullptr;                    // device [M + 1] first segment of each mesh
    int32_t *mesh_toff = nullptr;                // device [M] first triangle of each mesh
    int32_t *roots = nullptr;                    // device [M] subtree root (INT32_MIN: empty)
    int32_t *roots4 = nullptr;                   // device [M] the same as 4-wide references
    int32_t *slot_bin = nullptr;                 // device [kTopSlots] binary node of each top slot
    int32_t *mesh_group = nullptr;               // device [M] item group (XCD) of each mesh
    Node4 *top4g = nullptr;                      // device [kItemGroups][kTopSlots] each group's meshes' top
    int32_t *roots4g = nullptr;                  // device [kItemGroups][64] mesh roots as references in it
    int32_t *tri_mesh = nullptr;                 // device [nt]
    float *mesh_bounds = nullptr;                // device [M][8]
    int4 *items = nullptr;                       // device [n_items] (mesh, first, end, 0), grouped
    int n_items = 0;
    int32_t *group_start = nullptr;              // device [kItemGroups + 1] first item of each group
    int32_t *queue = nullptr;                    // device [n_rays]
    void *sort_ws = nullptr;                     // device ray_sort_ws_bytes(n_rays): segment order
    uint32_t *queue_len = nullptr;               // device [2]
    uint64_t *counters = nullptr;                // device [4]
    int64_t n_rays = 0;
};
hipError_t launch_batch_build(MeshDev &m, BatchDev &b, const float *V, const int32_t *F, hipStream_t s);
hipError_t launch_collapse_batch(MeshDev &m, BatchDev &b, hipStream_t s);  // wide.hip

// Build steps (build.hip).  All asynchronous on `s`.
hipError_t launch_build(MeshDev &m, const float *V, const int32_t *F, hipStream_t s, size_t sort_tmp_bytes);
size_t sort_tmp_bytes(int64_t nt, int morton_bits);
hipError_t build_from_keys64(MeshDev &m, int key_bits, hipStream_t s);
// Treelet restructuring of a built radix tree (restructure.hip); needs the
// tile list the radix-tree kernel left in m.sort_tmp.
hipError_t launch_restructure(MeshDev &m, int rounds, hipStream_t s);
hipError_t launch_collapse(MeshDev &m, hipStream_t s);  // wide.hip: the 4-wide tree
hipError_t launch_collapse_proposal(const MeshDev &m, Proposal &pr, hipStream_t s);  // ... of the proposal order

// Lists kept in a mesh's sort scratch once the sort is done: the tile count
// and tile list of the radix-tree kernel (subtrees of at most 1024 leaves), a
// node queue and a flag per internal node (4-wide collapse).
struct BuildLists {
    int32_t *n_tiles, *tiles;
    int32_t *queue, *tile_flag;
};
// tile_flag bit of the internal nodes with at most 1024 leaves (set by the
// radix-tree kernel; the tiles are the topmost of them)
constexpr int32_t kTileRootFlag = 1;
inline int64_t round64(int64_t n) { return (n + 63) & ~int64_t(63); }
inline BuildLists build_lists(void *sort_tmp, int64_t nt) {
    BuildLists L;
    L.n_tiles = static_cast<int32_t *>(sort_tmp);
    L.tiles = L.n_tiles + 64;
    L.queue = L.tiles + round64(nt);
    L.tile_flag = L.queue + round64(nt);
    return L;
}
inline size_t build_lists_bytes(int64_t nt) { return 4 * (64 + 3 * (size_t)round64(nt)); }
size_t restructure_lds_bytes();
// Stable sort of (32-bit key, id) pairs in place; tmp holds sort_u32_tmp_bytes(n).
size_t sort_u32_tmp_bytes(int64_t n);
hipError_t sort_u32_pairs(uint32_t *keys, int32_t *ids, void *tmp, int64_t n, hipStream_t s);
// Exclusive prefix sum of a[0..len) in place; partial holds 1024 entries.
hipError_t scan_u32_exclusive(uint32_t *a, int64_t len, uint32_t *partial, hipStream_t s);

// Derived outputs of the barycentric mode (derive.hip).
hipError_t launch_derive(const float *from, const float *to, int64_t n, const int32_t *tri_id, const float *uvt,
                         float *dist, float *point, hipStream_t s);
size_t compact_ws_bytes(int64_t n);
hipError_t launch_compact(const float *from, const float *to, int64_t n, const int32_t *tri_id, const float *uvt,
                          int64_t *hit_index, float *dist, int32_t *hit_tri, float *point, int64_t *n_hits,
                          void *ws, hipStream_t s);
hipError_t launch_morton_batch(MeshDev &m, const int32_t *tri_mesh, const float *mesh_bounds, hipStream_t s);

// Intersection (traverse.hip).
struct TraverseArgs {
    const float *from = nullptr, *to = nullptr;
    int64_t n = 0;
    int mode = 0;
    int certified = 0;
    int block = 256;
    int stack = 24;
    int waves_per_cu = 0;          // 0: library default
    int node_width = 0;            // 0: the mesh's widest tree, 2: binary nodes
    uint8_t *hit = nullptr;
    int32_t *tri_id = nullptr;
    float *uvt = nullptr;
    int32_t *count = nullptr;      // intercept-count mode
    uint64_t *counters = nullptr;  // [4] device
    int32_t *queue = nullptr;      // [n] device
    uint32_t *queue_len = nullptr; // [2] device (inside counters workspace): queue length, next segment
    uint32_t *visits = nullptr;    // stats only
    uint32_t *tests = nullptr;     // stats only
    const uint8_t *bucket = nullptr;      // proposal per segment (NULL: none)
    const int32_t *bucket_ref = nullptr;  // frontier node per bucket
    // batched form (NULL items: one mesh)
    const int4 *items = nullptr;          // (mesh, first segment, end segment, 0)
    int n_items = 0;
    const int32_t *group_start = nullptr; // [n_groups + 1] items grouped per XCD (NULL: one queue)
    int n_groups = 0;
    int n_meshes = 0;
    const int32_t *mesh_root = nullptr;   // subtree root per mesh (INT32_MIN: empty)
    const int32_t *mesh_root4 = nullptr;  // the same in the 4-wide tree (NULL: binary nodes only)
    const Node4 *top4g = nullptr;         // per XCD group: the top of its meshes (NULL: the combined top)
    const int32_t *roots4g = nullptr;     // per XCD group: the mesh roots as references in it
    const int32_t *mesh_toff = nullptr;   // first triangle of each mesh
    const int32_t *ray_off = nullptr;     // [n_meshes + 1] first segment of each mesh
    // segment order: 0 input order, 1 Morton code of the midpoint, 2 direction
    // octant above the Morton code of the start point (codes over the mesh box)
    int ray_sort = 0;
    const float *key_bounds = nullptr;    // [n_meshes or 1][8] lo.xyz, hi.xyz, scale, 0
    void *sort_ws = nullptr;              // ray_sort != 0: ray_sort_ws_bytes(n) bytes
};
size_t ray_sort_ws_bytes(int64_t n);
hipError_t launch_debug_certify(const float *from, const float *to, const float *corners, int64_t n, float *vals,
                                int32_t *cls, hipStream_t s);
hipError_t launch_intersect(const MeshDev &m, const TraverseArgs &a, hipStream_t s);
hipError_t launch_stats(const MeshDev &m, const TraverseArgs &a, hipStream_t s);

// Streaming copy of n16 16-byte words (membw.hip).
hipError_t launch_stream_copy(void *dst, const void *src, int64_t n16, hipStream_t s);

// Learned proposal (mlp.hip).
hipError_t proposal_frontier(const MeshDev &m, Proposal &pr, hipStream_t s);
hipError_t proposal_init(Proposal &pr, uint64_t seed, hipStream_t s);
// Training list of the segments with a first hit, in segment order; blk holds
// proposal_label_scratch(n) bytes.
size_t proposal_label_scratch(int64_t n);
hipError_t proposal_labels(const MeshDev &m, Proposal &pr, const int32_t *tri_id, int64_t n, int32_t *seg,
                           int32_t *label, uint32_t *count, int32_t *blk, hipStream_t s);
hipError_t proposal_predict(const MeshDev &m, const Proposal &pr, const float *from, const float *to, int64_t n,
                            int nb, uint8_t *bucket, hipStream_t s);
// One Adam step after a batch's gradient (step counts from 1).
struct AdamStep {
    float lr;
    int step;
};
// The gradient of one batch into pr.G (the mean loss times rows x loss_scale
// added to *loss), and with `adam` the parameter update.
hipError_t proposal_batch_grad(const MeshDev &m, Proposal &pr, const float *from, const float *to,
                               const int32_t *seg, const int32_t *lab, int64_t r0, int rows, int nb, float *loss,
                               float loss_scale, char *ws, hipStream_t s, float *logits_out, const AdamStep *adam);
size_t proposal_batch_scratch(int rows);
hipError_t proposal_features(const MeshDev &m, const float *from, const float *to, int64_t n, __bf16 *X,
                             hipStream_t s);
hipError_t proposal_set_params(Proposal &pr, hipStream_t s);

}  // namespace rsi
