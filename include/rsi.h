/*
 * rsi.h -- line-segment / triangle-mesh intersection on AMD gfx950 (MI355X).
 *
 * The operation (paper: Background section, problem statement): N_r line
 * segments l_i = (r_i_start, r_i_end) are tested against a surface of N_t
 * triangles, each a triplet of indices into N_v vertices.  The mesh is indexed
 * by a bounding volume hierarchy: Morton codes of the triangles, sorted, then a
 * binary radix tree (Karras 2012) whose node boxes are filled bottom-up; a tree
 * search per segment finds candidate triangles and a Moller-Trumbore test
 * decides (Background; Case Studies 1 and 2 show the tree's contents).  The
 * three results are those of the paper's operating modes (Background): a
 * boolean per segment, and the nearest hit's triangle with its barycentric
 * coordinates and segment parameter (from which distance and point follow).
 *
 * What counts as a hit (the reading this library implements exactly):
 *   the closed segment {O + t (E - O) : 0 <= t <= 1} meets the closed triangle
 *   {(1-u-v) A + u B + v C : u, v >= 0, u + v <= 1}, A, B, C = the triangle's
 *   vertices in index order, and the segment is not parallel to the plane.
 *   "Nearest" is the smallest t; equal t goes to the smaller triangle index.
 *   In RSI_PRECISION_CERTIFIED every decision equals the one a binary64
 *   evaluation of the Moller-Trumbore predicates makes (the paper's Epilogue
 *   offers binary64 for near-parallel rays whose binary32 result can be wrong).
 *
 * Conventions for every call:
 *   - Array arguments are DEVICE pointers (hipMalloc / hipMallocAsync / a
 *     torch CUDA tensor on a ROCm build), owned by the caller, 4-byte aligned
 *     and densely packed; host pointers are rejected with RSI_E_ARG.
 *   - Floating-point inputs are IEEE binary32; indices are int32 (the paper's
 *     Case Study 1: a 64-bit index array read through an int32 pointer
 *     silently drops triangles -- this interface only takes int32).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work
 *     is queued on it and the call returns without waiting unless stated.
 *   - A call returns a status and never throws or aborts.  Argument errors are
 *     found before any GPU work is queued.  A HIP error (including one left by
 *     earlier asynchronous work) is returned as RSI_E_HIP.  rsi_last_error()
 *     gives a message for the calling thread's last failure.
 *   - Calls that share one mesh handle may run concurrently only if they are
 *     ordered on the GPU (same stream or events); the handle itself is not
 *     changed by rsi_intersect.
 */
#ifndef RSI_H
#define RSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSI_ABI_VERSION 7  /* 2: intercept-count mode, rsi_outputs.count; 3: waves_per_cu; 4: build algorithm;
                              5: 4-wide nodes (node_width, rsi_mesh_info.node_width, RSI_EXPORT_WIDE_NODES,
                              RSI_EXPORT_WIDE_TOP); 6: RSI_EXPORT_MESH_ROOTS = 9 (was 7, the value of
                              RSI_EXPORT_WIDE_NODES), rsi_stream_copy; 7: rsi_intersect_noalloc */

typedef struct rsi_mesh_s *rsi_mesh; /* opaque; owned by the library until rsi_destroy */

typedef enum rsi_status {
    RSI_OK = 0,
    RSI_E_ARG = 1,      /* NULL / host / misaligned pointer, negative count, unknown option */
    RSI_E_RANGE = 2,    /* a triangle index outside [0, N_v) (only with check_indices) */
    RSI_E_NOMEM = 3,    /* device memory allocation failed */
    RSI_E_HIP = 4,      /* HIP runtime error, possibly from earlier asynchronous work */
    RSI_E_STATE = 5,    /* no usable gfx950 device, or a destroyed / invalid handle */
    RSI_E_CAPACITY = 6  /* a size beyond a documented limit */
} rsi_status;

typedef enum rsi_mode {
    RSI_MODE_BOOLEAN = 0,     /* paper's mode=boolean: one flag per segment */
    RSI_MODE_FIRST_HIT = 1,   /* index of the nearest hit triangle */
    RSI_MODE_BARYCENTRIC = 2, /* paper's mode=barycentric: nearest hit + (u, v, t) */
    RSI_MODE_INTERCEPT_COUNT = 3 /* paper's mode=intercept_count (Background section:
                                    the number of unique intersections per ray): the
                                    number of distinct t among the segment's hits, so
                                    triangles met at one point (a shared edge or
                                    vertex) count once.  CERTIFIED: distinct binary64 t
                                    of the binary64 decisions, as the oracle; PLAIN:
                                    distinct binary32 t of the binary32 decisions.
                                    No proposal order. */
} rsi_mode;

typedef enum rsi_precision {
    RSI_PRECISION_PLAIN = 0,     /* binary32 test; rare near-degenerate pairs may differ
                                    from the binary64 decision (paper's Epilogue) */
    RSI_PRECISION_CERTIFIED = 1  /* binary32 test with a proven error bound; pairs and
                                    orderings inside the bound are re-decided in binary64
                                    on the GPU, so results equal the binary64 decisions */
} rsi_precision;

/* Processing order of segments (rsi_intersect_opts.ray_sort).  Neighbouring
 * lanes of a wave follow similar tree paths when their segments are close in
 * space, which the Morton order of segments provides (the spatial sort of the
 * paper's Background section, applied to segments instead of triangles).
 * Codes are 30-bit, over the mesh box; the batched form keeps the mesh id
 * above them, so each mesh's segments stay within their own range. */
typedef enum rsi_ray_order {
    RSI_RAY_ORDER_INPUT = 0,         /* input order */
    RSI_RAY_ORDER_MIDPOINT = 1,      /* Morton code of the segment midpoint */
    RSI_RAY_ORDER_ORIGIN_OCTANT = 2  /* direction octant, then Morton code of the start point */
} rsi_ray_order;

/* Build options; pass NULL for defaults. */
typedef struct rsi_build_opts {
    int32_t morton_bits;   /* 30 (10 bits per axis, 32-bit keys) or 63 (21 bits per
                              axis, 64-bit keys, as the paper's uint64 codes); 0 = 30 */
    int32_t check_indices; /* nonzero: wait for the build and return RSI_E_RANGE if any
                              index is outside [0, N_v).  Without it such triangles are
                              never hit and the build does not wait. */
    int32_t algorithm;     /* 0 (default): radix tree of Karras 2012 (internal node i at
                              one end of its leaf range, root 0), then bottom-up boxes
                              in LDS tiles.  1: agglomerative single pass (Apetrei 2014,
                              as in the paper's Case Study 1 dump): the same tree with
                              internal nodes numbered by their split position; the
                              build waits once to learn the root's index.  2: the radix
                              tree, then two passes of treelet restructuring (Karras
                              & Aila 2013): internal nodes rewired to lower the tree's
                              surface-area cost, so queries visit fewer nodes; a node's
                              leaves are then no longer a contiguous range (words 14 /
                              15 of RSI_EXPORT_NODES hold their smallest and largest
                              sorted position).  Algorithms 0 and 2 also collapse the
                              binary tree into a 4-wide one (RSI_EXPORT_WIDE_NODES)
                              for the single-mesh traversal; 128 B more per triangle
                              and 64 KB per mesh.
                              Results of rsi_intersect do not depend on the algorithm. */
} rsi_build_opts;

/* Intersection options; pass NULL for defaults. */
typedef struct rsi_intersect_opts {
    int32_t precision;    /* rsi_precision; default RSI_PRECISION_PLAIN */
    int32_t block;        /* threads per workgroup of the first pass: 64, 128, 256,
                             512 or 1024 (binary nodes: at most 256, larger values
                             run as 256; a workgroup whose LDS stacks would not fit
                             runs with half as many threads until they do); 0 = the
                             library default (1024 for 4-wide nodes, 256 for binary
                             ones).  With 4-wide nodes a
                             larger workgroup keeps more of the tree's top in its
                             LDS. */
    int32_t stack_depth;  /* traversal stack entries per lane in LDS, 1..64; 0 = 20.
                             Deeper paths are finished exactly by a second pass. */
    int32_t ray_sort;     /* rsi_ray_order: order in which segments are processed.
                             Results are written at input indices in every order;
                             a value other than 0 adds a key pass and a sort of the
                             segment indices (16 B of scratch per segment). */
    int32_t proposal;     /* 1 = visit the learned proposal's bucket first (needs a
                             trained or loaded proposal); 0 = plain order */
    int32_t waves_per_cu; /* resident waves per compute unit of the persistent
                             traversal, 1..32 (capped by what registers and LDS
                             allow); 0 = the library default.  Fewer waves share a
                             CU's L1 cache among fewer tree paths. */
    int32_t node_width;   /* tree the first pass walks: 0 = the widest the mesh has
                             (4-wide for build algorithms 0 and 2 and for batches;
                             binary for algorithm 1), 2 = binary nodes, 4 = 4-wide
                             nodes (RSI_E_ARG where not built).  The proposal
                             order walks a 4-wide tree of its own in which every
                             bucket's subtree starts a node.  Results do not
                             depend on it. */
} rsi_intersect_opts;

/* Output buffers (device pointers, caller-owned).  Required per mode:
 *   BOOLEAN:     hit
 *   FIRST_HIT:   tri_id            (hit filled too when not NULL)
 *   BARYCENTRIC: tri_id and uvt    (hit filled too when not NULL)
 *   INTERCEPT_COUNT: count         (hit filled too when not NULL)
 * Results are written at the segment's input index. */
typedef struct rsi_outputs {
    uint8_t *hit;       /* [N_r] 1 if the segment meets the surface, else 0 */
    int32_t *tri_id;    /* [N_r] input index of the nearest hit triangle, -1 on a miss */
    float *uvt;         /* [N_r][3] u, v (weights of the triangle's 2nd and 3rd vertex)
                           and t of that hit, rounded from binary64 in CERTIFIED
                           precision; NaN on a miss */
    uint64_t *counters; /* optional [4]: [0] segments re-decided in binary64, [1] segments
                           that outgrew the LDS stack, [2] hitting segments whose answer
                           was not in the proposed bucket (proposal misses), [3] count-mode
                           segments with more distinct hits than a lane keeps in registers
                           (11 in CERTIFIED precision, 12 in PLAIN), finished by the second
                           pass.  Zeroed by the call before it counts.  [0] and [1] depend
                           on the order in which a wave's lanes reach their leaves, and the
                           last segments of a launch go to whichever waves are free first,
                           so these two may vary slightly from call to call; the results
                           never do. */
    int32_t *count;     /* [N_r] intercept-count mode: distinct intersections, 0 on a miss */
} rsi_outputs;

/*
 * rsi_build -- build the bounding volume hierarchy of a triangle mesh.
 *   vertices   [n_vertices][3] float, x y z of each vertex
 *   triangles  [n_triangles][3] int32, vertex indices of each triangle
 *   opts       NULL or build options
 *   stream     queue for the build
 *   out        receives the handle (set to NULL on failure)
 * Steps (paper: Background; Specific changes; Case Studies 1-2): mesh extent,
 * Morton key of every triangle centroid normalised to the extent, a stable
 * LDS radix sort of (key, index), the Karras binary radix tree over the sorted
 * keys, and a bottom-up pass (one thread per leaf, an atomic counter per
 * internal node: the second child to arrive merges both boxes and climbs).
 * The library keeps copies of what it needs (the inputs may be freed once the
 * stream passes the call) and allocates about 64 N_t + 48 N_t + 12 N_v + 12 N_t
 * + 24 N_t bytes of device memory, stream-ordered on `stream`.
 * Limits: n_triangles < 2^30, n_vertices < 2^31.  n_triangles == 0 gives a
 * mesh no segment hits.
 */
rsi_status rsi_build(const float *vertices, int64_t n_vertices,
                     const int32_t *triangles, int64_t n_triangles,
                     const rsi_build_opts *opts, void *stream, rsi_mesh *out);

/*
 * rsi_intersect -- test n_rays segments against a built mesh.
 *   rays_from, rays_to  [n_rays][3] float: start and end point of each segment
 *   mode                rsi_mode
 *   opts                NULL or intersection options
 *   out                 output buffers (see rsi_outputs)
 * Per segment (paper: Background -- tree search for candidates, then the
 * Moller-Trumbore test): traverse the tree from the root, nearer child first,
 * skipping children whose box (conservatively widened, so no binary64 hit is
 * ever culled) the segment misses; test each reached triangle.  Boolean mode
 * stops at the first hit; the other modes keep the nearest and skip boxes that
 * begin beyond it.  n_rays == 0 does nothing.  Limit: n_rays < 2^31.
 * Temporary device memory (4 n_rays + 64 bytes, plus what a proposal or a
 * segment order needs) is allocated and freed stream-ordered on `stream`.
 */
rsi_status rsi_intersect(rsi_mesh mesh, const float *rays_from, const float *rays_to,
                         int64_t n_rays, int32_t mode, const rsi_intersect_opts *opts,
                         const rsi_outputs *out, void *stream);

/*
 * rsi_intersect_noalloc -- rsi_intersect for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and results as
 * rsi_intersect; the caller still provides the inputs and outputs.  The
 * temporary memory comes from one 64 MiB device array of the library instead
 * of an allocation, so the call allocates nothing (no hipMalloc / hipFree of
 * any kind).  It needs 4 n_rays + 64 bytes rounded up to 256, plus n_rays
 * rounded up to 256 with opts->proposal = 1, plus 16 n_rays with a segment
 * order (ray_sort != 0): at most 16,777,200 segments in input order without
 * the proposal, in either precision.  A call needing more returns
 * RSI_E_CAPACITY before any GPU work.  Every GPU the library runs on holds its own copy of the array until
 * the process ends; the array's address on the current device is looked up
 * the first time this is called there.  All calls on one GPU share that
 * array: calls that may overlap on one GPU (different streams without
 * ordering between them, or different threads) race and give wrong results;
 * order them on one stream.  What must start at zero is cleared by the call's
 * own first kernel.
 */
rsi_status rsi_intersect_noalloc(rsi_mesh mesh, const float *rays_from, const float *rays_to,
                                 int64_t n_rays, int32_t mode, const rsi_intersect_opts *opts,
                                 const rsi_outputs *out, void *stream);

/* rsi_destroy -- free a mesh (stream-ordered on the stream it was built on).
 * NULL is accepted and ignored. */
rsi_status rsi_destroy(rsi_mesh mesh);

/* Host-side description of a built mesh. */
typedef struct rsi_mesh_info {
    int64_t n_vertices;
    int64_t n_triangles;
    int32_t morton_bits;
    int32_t root;            /* root reference: 0 (internal node 0), ~0 (single leaf), or
                                INT32_MIN for an empty mesh */
    int64_t device_bytes;    /* device memory held by the mesh */
    int32_t node_width;      /* 4 when the 4-wide tree is built, else 2 */
    int32_t reserved;        /* 0 */
} rsi_mesh_info;

rsi_status rsi_mesh_info_get(rsi_mesh mesh, rsi_mesh_info *info);

/* What rsi_mesh_export copies (for inspection and tests, in the spirit of the
 * paper's device-memory debugging of the BVH, Case Study 1). */
typedef enum rsi_export_what {
    RSI_EXPORT_SORTED_KEYS = 0, /* uint64 [N_t]  Morton keys in sorted order (widened)   */
    RSI_EXPORT_SORTED_IDS = 1,  /* int32  [N_t]  triangle index at each sorted position   */
    RSI_EXPORT_NODES = 2,       /* 16 x 32-bit words per internal node, [N_t - 1]:
                                   words 0-3  left  box x lo, x hi, y lo, y hi
                                   words 4-7  right box x lo, x hi, y lo, y hi
                                   words 8-11 left z lo, z hi, right z lo, z hi
                                   word 12, 13 left / right child: >= 0 internal node,
                                   < 0 leaf at sorted position ~ref; words 14, 15 the
                                   first and last sorted leaf the node covers (smallest
                                   and largest, after treelet restructuring)              */
    RSI_EXPORT_PARENTS = 3,     /* int32 [2 N_t - 1]: parent of internal node i at [i]
                                   (-1 for the root), of leaf k at [N_t - 1 + k]        */
    RSI_EXPORT_COUNTERS = 4,    /* int32 [N_t - 1]: arrivals counted at each internal
                                   node by the bottom-up pass (2 when complete)          */
    RSI_EXPORT_LEAVES = 5,      /* 12 x 32-bit words per sorted leaf, [N_t]: A.xyz,
                                   triangle index (int32), B-A xyz, 0, C-A xyz, 0        */
    RSI_EXPORT_BOUNDS = 6,      /* float [8]: mesh lo xyz, hi xyz, coordinate scale
                                   (largest |coordinate|), 0                              */
    RSI_EXPORT_WIDE_NODES = 7,  /* 32 x 32-bit words per slot, [N_t - 1] (nothing when
                                   node_width is 2): words 0-3 x lo of children 0..3,
                                   4-7 x hi, 8-11 y lo, 12-15 y hi, 16-19 z lo, 20-23
                                   z hi, 24-27 child references, word 28 the number of
                                   children, 29-31 zero.  A child reference r is a leaf
                                   at sorted position ~r when r < 0, INT32_MIN for an
                                   unused slot (its box is +inf on every face), the
                                   top node in slot r of RSI_EXPORT_WIDE_TOP when
                                   0 <= r < 512, and otherwise the 4-wide node in slot
                                   r - 512 of this array (the node collapsed from binary
                                   internal node r - 512).  Only reachable slots are
                                   defined.                                              */
    RSI_EXPORT_WIDE_TOP = 8     /* 32 x 32-bit words per slot, [512] (nothing when
                                   node_width is 2): the first 4-wide nodes in
                                   breadth-first order from the root (the root in slot
                                   0), as above, with references to other top nodes
                                   rewritten to their slots; kept in LDS by the
                                   traversal.  Slots past the tree's size are undefined. */
} rsi_export_what;

/* Copy one internal array into dst (device or host memory of dst_bytes bytes,
 * at least the size stated above).  Queued on `stream`; with a host dst the
 * call waits for the copy. */
rsi_status rsi_mesh_export(rsi_mesh mesh, int32_t what, void *dst, int64_t dst_bytes, void *stream);

/*
 * rsi_traversal_stats -- per-segment work of the same traversal rsi_intersect
 * runs with these arguments (an instrumented copy of the kernel; results are
 * not written).  node_visits[i] counts internal nodes fetched (4-wide nodes
 * when the first pass walks them, see node_width), leaf_tests[i]
 * triangles tested; both uint32 [n_rays] device arrays.  Segments finished by
 * the second (deep-stack) pass report the first pass's counts.
 */
rsi_status rsi_traversal_stats(rsi_mesh mesh, const float *rays_from, const float *rays_to,
                               int64_t n_rays, int32_t mode, const rsi_intersect_opts *opts,
                               uint32_t *node_visits, uint32_t *leaf_tests, void *stream);

/* ------------------------------------------------------------------------
 * Derived outputs of the barycentric mode (paper: Background -- the
 * intersecting rays with the intersecting triangle, the distance to and the
 * location of the nearest intersecting point; Performance section, steps
 * 3a-3d, which the paper moved from host numpy to GPU kernels).  Inputs are
 * the segments and the tri_id / uvt arrays an rsi_intersect call in
 * BARYCENTRIC mode wrote (device memory, N_r entries); a segment hits iff
 * tri_id >= 0.  Distances are t |to - from| and points from + t (to - from),
 * evaluated in binary64 from the float32 end points and t, rounded once.
 * ---------------------------------------------------------------------- */

/* Per segment: distance float [N_r] and point float [N_r][3] (either may be
 * NULL), NaN for a segment that misses.  Queued on `stream`. */
rsi_status rsi_derive(const float *rays_from, const float *rays_to, int64_t n_rays, const int32_t *tri_id,
                      const float *uvt, float *distance, float *point, void *stream);

/* The paper's result tuple, compacted: for each hitting segment in ascending
 * index, hit_index int64 (its index), distance float, hit_tri int32 (its
 * triangle) and point float [3], written to slots 0 .. *n_hits - 1 (arrays of
 * N_r entries; any may be NULL).  n_hits: device int64, required.  Queued on
 * `stream` (the call allocates 4 B per 4096 segments of scratch, stream-ordered). */
rsi_status rsi_compact_hits(const float *rays_from, const float *rays_to, int64_t n_rays, const int32_t *tri_id,
                            const float *uvt, int64_t *hit_index, float *distance, int32_t *hit_tri, float *point,
                            int64_t *n_hits, void *stream);

/*
 * rsi_debug_certify -- the CERTIFIED precision's binary32 test on n given
 * (segment, triangle) pairs, for checking its error bounds (the paper's
 * Epilogue: binary32 Moller-Trumbore can misjudge near-parallel segments, and
 * binary64 intermediates fix that; the bound decides which pairs binary32 may
 * settle).  Pair i is segment rays_from[i] -> rays_to[i] and the triangle with
 * corners corners[i][0..2] (xyz each), set up as the traversal does (direction
 * and edges rounded to binary32).  Device arrays:
 *   values  float [n][10]: det, U, W, T (binary32), their bounds B(det), B(U),
 *           B(W), B(T), and for a sure hit the interval [tlo, thi] around t
 *           (NaN otherwise).  The bounds claim |X32 - X| <= B(X) and
 *           |X32 - X64| <= B(X) for the exact value X and the binary64 value X64
 *           computed in the oracle's operation order.
 *   classes int32 [n]: 0 sure miss, 1 sure hit, 2 unsure (decided in binary64).
 * Queued on `stream`; RSI_E_ARG for NULL or misaligned pointers or n < 0.
 */
rsi_status rsi_debug_certify(const float *rays_from, const float *rays_to, const float *corners, int64_t n,
                             float *values, int32_t *classes, void *stream);

/* ------------------------------------------------------------------------
 * Learned subtree proposal.  A small MLP predicts, per segment, the depth-8
 * subtree ("bucket") of the tree that holds its first hit; rsi_intersect with
 * opts->proposal = 1 traverses that subtree first (and, in boolean mode, stops
 * at a sure hit there), then the rest of the tree without it (on 4-wide nodes
 * a second collapse, made when the proposal is created or loaded, keeps every
 * bucket's subtree as a node of its own: 128 (N_t + 511) bytes more).  The exact
 * traversal and test decide every result, so results are identical to
 * proposal = 0; only the amount of work changes.
 * Network: inputs = the 6 end-point coordinates normalised to [-1, 1] over the
 * mesh box and sin/cos(pi f_k x) of each for f_k = 2^(k/2), k = 0..15 (198,
 * padded to 224); three hidden layers of 256 with ReLU; 256 logits, one per
 * frontier bucket (buckets past the frontier's size are masked).  bf16 weights
 * and activations, fp32 accumulation on the matrix cores, fp32 master weights
 * and Adam for training.  Parameters are one fp32 vector of RSI_MLP_PARAMS:
 * W1 [256][224], W2, W3, W4 [256][256] (row = output unit), then b1..b4 [256].
 * All proposal calls need a mesh with at least one triangle.
 * ---------------------------------------------------------------------- */
#define RSI_MLP_PARAMS 254976
#define RSI_MLP_INPUTS 224
#define RSI_MLP_BUCKETS 256

typedef struct rsi_train_opts {
    int32_t epochs;   /* passes over the labelled segments; 0 = 2 */
    int32_t batch;    /* segments per Adam step, 64..65536; 0 = 4096 */
    float lr;         /* Adam learning rate; 0 = 1e-3 */
    int32_t reinit;   /* nonzero: draw fresh initial weights even if trained */
    uint64_t seed;    /* initial-weight seed */
} rsi_train_opts;

/* Train on segments the method labels itself: a CERTIFIED first-hit pass over
 * (from, to) gives each hitting segment's triangle, hence its bucket; then
 * `epochs` passes of minibatch Adam on cross-entropy.  epoch_loss (device
 * float [epochs], may be NULL) receives the mean loss of each epoch;
 * *n_labelled (host, may be NULL) the number of hitting segments used.
 * Waits for the stream (the label count sets the batch schedule). */
rsi_status rsi_proposal_train(rsi_mesh mesh, const float *rays_from, const float *rays_to, int64_t n_rays,
                              const rsi_train_opts *opts, float *epoch_loss, int64_t *n_labelled, void *stream);

/* Bucket per segment (device uint8 [n_rays]) from the fused inference kernel. */
rsi_status rsi_proposal_predict(rsi_mesh mesh, const float *rays_from, const float *rays_to, int64_t n_rays,
                                uint8_t *bucket, void *stream);

/* what = 0: copy the fp32 parameters to buf; what = 1: replace them with buf
 * (bf16 copies refreshed, Adam state reset).  buf: device float [RSI_MLP_PARAMS]. */
rsi_status rsi_proposal_params(rsi_mesh mesh, int32_t what, float *buf, void *stream);

/* One minibatch without an update, for checking the kernels: segments
 * (from, to) [n_rays <= 65536] with labels (device int32 [n_rays], bucket
 * index).  Writes the gradient of the mean cross-entropy (device float
 * [RSI_MLP_PARAMS]), the logits (device float [n_rays][256]) and the mean loss
 * (device float [1]). */
rsi_status rsi_proposal_gradient(rsi_mesh mesh, const float *rays_from, const float *rays_to,
                                 const int32_t *labels, int64_t n_rays, float *grad, float *logits, float *loss,
                                 void *stream);

/* The network inputs of each segment: device bf16 bit patterns [n_rays][224]. */
rsi_status rsi_proposal_features(rsi_mesh mesh, const float *rays_from, const float *rays_to, int64_t n_rays,
                                 uint16_t *features, void *stream);

/* The frontier: node reference of each bucket (>= 0 internal node, < 0 leaf
 * ~k), first sorted leaf of each bucket (device int32 [256] each, unused
 * entries untouched), and the bucket count (host). */
rsi_status rsi_proposal_frontier(rsi_mesh mesh, int32_t *bucket_ref, int32_t *bucket_first, int32_t *n_buckets,
                                 void *stream);

/* Save / load the parameters and Adam state (raw little-endian binary with a
 * header: magic, layer sizes, parameter count, step, triangle count, bucket
 * count).  Loading checks the header against this mesh.  Both wait. */
rsi_status rsi_proposal_save(rsi_mesh mesh, const char *path);
rsi_status rsi_proposal_load(rsi_mesh mesh, const char *path);

/* ------------------------------------------------------------------------
 * Batched form: up to 64 meshes of uneven size and their segment batches in
 * one BVH build and one persistent traversal launch.  Mesh m owns vertices
 * [vertex_offsets[m], vertex_offsets[m+1]) of the concatenated vertex array,
 * triangles [triangle_offsets[m], ...+1) whose indices are relative to its
 * own first vertex, and segments [ray_offsets[m], ...+1).  Keys are the mesh
 * id (6 bits, bits 30..35 of the exported 64-bit keys) above a 30-bit Morton
 * code (10 bits per axis of the mesh's own box), so one sort (five 8-bit
 * passes), one radix tree and one bottom-up pass cover all meshes
 * and each mesh is one subtree.  The traversal takes (mesh, segment range)
 * items of up to 512 segments from a queue.  Reported triangle indices are
 * relative to the segment's mesh.  rsi_batch_create allocates everything
 * (including ~16 B per segment for the optional segment ordering);
 * rsi_batch_build and rsi_batch_intersect allocate nothing and never wait, so
 * both may be captured in a HIP graph and replayed (inputs at the same
 * addresses).  Triangles with an index outside their mesh are never hit.
 * ---------------------------------------------------------------------- */
typedef struct rsi_batch_s *rsi_batch;

#define RSI_BATCH_MAX_MESHES 64

/* Offsets: host int64 arrays of n_meshes + 1 entries, starting at 0 and
 * non-decreasing.  Totals: triangles < 2^30, vertices and segments < 2^31. */
rsi_status rsi_batch_create(int32_t n_meshes, const int64_t *vertex_offsets, const int64_t *triangle_offsets,
                            const int64_t *ray_offsets, void *stream, rsi_batch *out);
/* vertices: device float [total][3]; triangles: device int32 [total][3]. */
rsi_status rsi_batch_build(rsi_batch batch, const float *vertices, const int32_t *triangles, void *stream);
/* Segments: device float [total][3] each; outputs as rsi_intersect, over all
 * segments.  opts->proposal must be 0. */
rsi_status rsi_batch_intersect(rsi_batch batch, const float *rays_from, const float *rays_to, int32_t mode,
                               const rsi_intersect_opts *opts, const rsi_outputs *out, void *stream);
/* The combined BVH's arrays as rsi_mesh_export, plus RSI_EXPORT_MESH_ROOTS:
 * int32 [n_meshes], each mesh's subtree root (INT32_MIN for an empty mesh). */
#define RSI_EXPORT_MESH_ROOTS 9
rsi_status rsi_batch_export(rsi_batch batch, int32_t what, void *dst, int64_t dst_bytes, void *stream);
rsi_status rsi_batch_destroy(rsi_batch batch);

/* ------------------------------------------------------------------------
 * Measurement helper: the achievable HBM bandwidth that the traversal's
 * measured memory traffic is compared with.  Copies `bytes` (a multiple of
 * 16) from src to dst, both 16-byte aligned device buffers that do not
 * overlap, with a streaming kernel: each lane moves 16-byte words in a
 * grid-stride loop, four in flight, non-temporal loads and stores, eight
 * 256-thread workgroups per compute unit.  Queued on `stream`; RSI_E_ARG for a
 * size, alignment or pointer that breaks these rules.
 * ---------------------------------------------------------------------- */
rsi_status rsi_stream_copy(void *dst, const void *src, int64_t bytes, void *stream);

const char *rsi_status_string(rsi_status status);
const char *rsi_last_error(void);   /* message of this thread's last failure, "" if none */
int32_t rsi_abi_version(void);      /* RSI_ABI_VERSION of the built library */

#ifdef __cplusplus
}
#endif

#endif /* RSI_H */
