// traverse.hip -- tree search and Moller-Trumbore leaf tests on gfx950.
//
// Paper: Background -- a tree search gathers the candidate triangles of each
// segment and the Moller-Trumbore test (Moller & Trumbore 1997) decides; the
// operating modes boolean / barycentric; Epilogue -- binary32 can misjudge
// near-parallel rays, binary64 intermediates fix it.
//
// Pass 1 (k_traverse): one lane per segment, stack of pending subtrees in LDS
// (stack_depth entries per lane), nearer child first, binary32 arithmetic.
//   PLAIN      the binary32 predicates decide.
//   CERTIFIED  each predicate X comes with a proven bound B(X) on its distance
//              from the exact value and from the binary64 value; |X| > B(X)
//              fixes the sign of the binary64 result, so the pair is a sure
//              hit or a sure miss.  Otherwise the pair is "unsure" and the
//              lane decides it at once with the binary64 test in the
//              oracle's operation order (no contraction, correctly rounded
//              division).  Nearest-hit choice uses proven intervals around
//              the binary64 t, and the binary64 t themselves where two
//              intervals overlap.
// A segment whose path outgrows the LDS stack (or, in count mode, whose list
// of distinct t overflows or holds nearly equal ones) is appended to a queue
// and finished by pass 2 (k_finish): a deep private stack and, in CERTIFIED
// precision, the binary64 test on every candidate.
//
// Box test: the slab test on each child box widened by eta = 2^-20 max(|coord|)
// of the segment and mesh.  That margin exceeds every rounding of the slab
// arithmetic, so a point within eta/4 of a box is never culled -- in
// particular any binary64 hit of a non-grazing segment.
#include "rsi_internal.h"

#include <cstdlib>
#include <type_traits>

namespace rsi {
namespace {

constexpr float kEtaRel = 0x1p-20f;
constexpr float kBoundK = 12.0f * 0x1p-24f;  // >= 8 u32 (binary32) + 8 u64 (binary64) with slack
constexpr float kBoundTiny = 0x1p-140f;      // absorbs underflow in the products
constexpr int kMiss = 0, kHit = 1, kUnsure = 2;
enum { MODE_BOOL = 0, MODE_FIRST = 1, MODE_BARY = 2, MODE_COUNT = 3 };
// distinct t a lane keeps in registers in count mode: binary32 values (plain),
// or intervals of two floats each (certified: 11, which keeps the kernel
// within its 128 VGPRs with few spills; the segments with more go to the
// second pass -- 27k of 1e7 at the paper's scale, 6.38 -> 6.28 ms against 12)
template <bool CERT>
constexpr int kCountSlots = CERT ? 11 : 12;

struct Ray {
    float3 o, d;   // start point, direction E - O (rounded)
    float3 inv;    // 1 / direction (components below eta/4 raised to eta/4)
    float3 nra;    // -(O + eta) * inv   (lower box faces)
    float3 nrb;    // -(O - eta) * inv   (upper box faces)
};

__device__ __forceinline__ bool finite3(float3 v) {
    return __builtin_isfinite(v.x) && __builtin_isfinite(v.y) && __builtin_isfinite(v.z);
}

__device__ __forceinline__ float widen_dir(float d, float dmin) {
    return fabsf(d) < dmin ? copysignf(dmin, d) : d;
}

// Returns false for segments whose setup is not finite.
__device__ __forceinline__ bool setup_ray(const float *__restrict__ from, const float *__restrict__ to,
                                          int64_t i, float scale, Ray &r) {
    // streamed once: non-temporal, so the segments do not push the tree out of L2
    r.o = make_float3(__builtin_nontemporal_load(from + 3 * i), __builtin_nontemporal_load(from + 3 * i + 1),
                      __builtin_nontemporal_load(from + 3 * i + 2));
    const float3 e = make_float3(__builtin_nontemporal_load(to + 3 * i), __builtin_nontemporal_load(to + 3 * i + 1),
                                 __builtin_nontemporal_load(to + 3 * i + 2));
    r.d = make_float3(e.x - r.o.x, e.y - r.o.y, e.z - r.o.z);
    float m = fmaxf(scale, fmaxf(fmaxf(fabsf(r.o.x), fabsf(r.o.y)), fabsf(r.o.z)));
    m = fmaxf(m, fmaxf(fmaxf(fabsf(e.x), fabsf(e.y)), fabsf(e.z)));
    const float eta = m * kEtaRel;
    const float dmin = 0.25f * eta;
    r.inv = make_float3(1.0f / widen_dir(r.d.x, dmin), 1.0f / widen_dir(r.d.y, dmin), 1.0f / widen_dir(r.d.z, dmin));
    r.nra = make_float3(-((r.o.x + eta) * r.inv.x), -((r.o.y + eta) * r.inv.y), -((r.o.z + eta) * r.inv.z));
    r.nrb = make_float3(-((r.o.x - eta) * r.inv.x), -((r.o.y - eta) * r.inv.y), -((r.o.z - eta) * r.inv.z));
    return finite3(r.o) && finite3(e) && finite3(r.d) && finite3(r.inv) && finite3(r.nra) && finite3(r.nrb) &&
           __builtin_isfinite(eta);
}

// Widened slab test of one box against t in [0, tlimit]; returns the entry t.
__device__ __forceinline__ bool slab(float xlo, float xhi, float ylo, float yhi, float zlo, float zhi,
                                     const Ray &r, float tlimit, float &tenter) {
    const float tx0 = fmaf(xlo, r.inv.x, r.nra.x), tx1 = fmaf(xhi, r.inv.x, r.nrb.x);
    const float ty0 = fmaf(ylo, r.inv.y, r.nra.y), ty1 = fmaf(yhi, r.inv.y, r.nrb.y);
    const float tz0 = fmaf(zlo, r.inv.z, r.nra.z), tz1 = fmaf(zhi, r.inv.z, r.nrb.z);
    const float tmin = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
    const float tmax = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), tlimit));
    tenter = tmin;
    return tmin <= tmax;
}

// The same test with the near and far face of each axis given (the lower
// face is the near one for a direction component >= 0, the upper one
// otherwise, with the matching offsets nn / nf of nra / nrb).  For a box with
// lo <= hi the sign picks exactly the operands min / max pick in slab(), so
// the decisions are the same bit for bit; a box that is +inf on every face
// still misses.
__device__ __forceinline__ bool slab_nf(float nx, float fx, float ny, float fy, float nz, float fz,
                                        const float3 &inv, const float3 &nn, const float3 &nf, float tlimit,
                                        float &tenter) {
    const float tnx = fmaf(nx, inv.x, nn.x), tfx = fmaf(fx, inv.x, nf.x);
    const float tny = fmaf(ny, inv.y, nn.y), tfy = fmaf(fy, inv.y, nf.y);
    const float tnz = fmaf(nz, inv.z, nn.z), tfz = fmaf(fz, inv.z, nf.z);
    const float tmin = fmaxf(fmaxf(tnx, tny), fmaxf(tnz, 0.0f));
    const float tmax = fminf(fminf(tfx, tfy), fminf(tfz, tlimit));
    tenter = tmin;
    return tmin <= tmax;
}

struct MT32 {
    float det, U, W, T;
    float3 s;
};

// Binary32 Moller-Trumbore quantities (contraction allowed: the bound below
// holds for any grouping into fused operations).
__device__ __forceinline__ MT32 mt32(const Tri &tri, const Ray &r) {
    MT32 m;
    const float3 e1 = make_float3(tri.e1.x, tri.e1.y, tri.e1.z);
    const float3 e2 = make_float3(tri.e2.x, tri.e2.y, tri.e2.z);
    m.s = make_float3(r.o.x - tri.a.x, r.o.y - tri.a.y, r.o.z - tri.a.z);
    const float px = r.d.y * e2.z - r.d.z * e2.y;
    const float py = r.d.z * e2.x - r.d.x * e2.z;
    const float pz = r.d.x * e2.y - r.d.y * e2.x;
    const float qx = m.s.y * e1.z - m.s.z * e1.y;
    const float qy = m.s.z * e1.x - m.s.x * e1.z;
    const float qz = m.s.x * e1.y - m.s.y * e1.x;
    m.det = e1.x * px + e1.y * py + e1.z * pz;
    m.U = m.s.x * px + m.s.y * py + m.s.z * pz;
    m.W = r.d.x * qx + r.d.y * qy + r.d.z * qz;
    m.T = e2.x * qx + e2.y * qy + e2.z * qz;
    return m;
}

// The binary32 decision, same predicates as the definition.
__device__ __forceinline__ bool decide32(const MT32 &m) {
    if (!(m.det != 0.0f))
        return false;
    const float g = m.det > 0.0f ? 1.0f : -1.0f;
    const float a = g * m.U, b = g * m.W, tt = g * m.T, D = g * m.det;
    return a >= 0.0f && b >= 0.0f && a + b <= D && tt >= 0.0f && tt <= D;
}

// Certified classification.  Every binary32 quantity X (det, U, W, T) is a sum
// of six signed products of three rounded differences, formed with at most 8
// roundings per product; so |X32 - X| <= gamma_8 M(X) with M(X) the same sum
// over absolute values, and the binary64 evaluation obeys the same form with
// unit roundoff 2^-53.  B(X) = 12 * 2^-24 * M(X) covers both with room for the
// roundings of M itself.  For a hit the interval [tlo, thi] holds the exact t
// and the binary64 t.
struct Bounds {
    float d, U, W, T;
};

__device__ __forceinline__ Bounds mt_bounds(const MT32 &m, const Tri &tri, const Ray &r) {
    const float adx = fabsf(r.d.x), ady = fabsf(r.d.y), adz = fabsf(r.d.z);
    const float asx = fabsf(m.s.x), asy = fabsf(m.s.y), asz = fabsf(m.s.z);
    const float a1x = fabsf(tri.e1.x), a1y = fabsf(tri.e1.y), a1z = fabsf(tri.e1.z);
    const float a2x = fabsf(tri.e2.x), a2y = fabsf(tri.e2.y), a2z = fabsf(tri.e2.z);
    const float Pmx = ady * a2z + adz * a2y, Pmy = adz * a2x + adx * a2z, Pmz = adx * a2y + ady * a2x;
    const float Qmx = asy * a1z + asz * a1y, Qmy = asz * a1x + asx * a1z, Qmz = asx * a1y + asy * a1x;
    Bounds b;
    b.d = fmaf(kBoundK, a1x * Pmx + a1y * Pmy + a1z * Pmz, kBoundTiny);
    b.U = fmaf(kBoundK, asx * Pmx + asy * Pmy + asz * Pmz, kBoundTiny);
    b.W = fmaf(kBoundK, adx * Qmx + ady * Qmy + adz * Qmz, kBoundTiny);
    b.T = fmaf(kBoundK, a2x * Qmx + a2y * Qmy + a2z * Qmz, kBoundTiny);
    return b;
}

__device__ __forceinline__ int classify(const MT32 &m, const Tri &tri, const Ray &r, float &tlo, float &thi) {
    const Bounds bb = mt_bounds(m, tri, r);
    const float Bd = bb.d, BU = bb.U, BW = bb.W, BT = bb.T;
    const float aD = fabsf(m.det);
    // a hit needs |U|, |W|, |T| <= |det| in binary64; a sure excess is a sure miss
    const float cap = aD + Bd;
    if (fabsf(m.U) - BU > cap || fabsf(m.W) - BW > cap || fabsf(m.T) - BT > cap)
        return kMiss;
    if (!(aD > Bd))
        return kUnsure;  // sign of det (or det == 0) not certain; also NaN
    const float g = m.det > 0.0f ? 1.0f : -1.0f;
    const float a = g * m.U, b = g * m.W, tt = g * m.T;
    const float w = g * ((m.det - m.U) - m.W);  // D - a - b
    const float z = g * (m.det - m.T);          // D - tt
    const float Bw = Bd + BU + BW + 0x1p-22f * (aD + fabsf(m.U) + fabsf(m.W));
    const float Bz = Bd + BT + 0x1p-22f * (aD + fabsf(m.T));
    if (a < -BU || b < -BW || w < -Bw || tt < -BT || z < -Bz)
        return kMiss;
    if (a > BU && b > BW && w > Bw && tt > BT && z > Bz) {
        tlo = (tt - BT) / (aD + Bd) * (1.0f - 0x1p-21f);
        thi = (tt + BT) / (aD - Bd) * (1.0f + 0x1p-21f);
        return kHit;
    }
    return kUnsure;
}

// Binary64 test in the definition's operation order: differences, cross
// products, dot products summed left to right, no fused operations, correctly
// rounded division.
struct MT64 {
    bool hit;
    double u, v, t;
};

__device__ __forceinline__ MT64 mt64(double ox, double oy, double oz, double ex, double ey, double ez,
                                     const float *__restrict__ V, const int32_t *__restrict__ F, int t) {
#pragma clang fp contract(off)
    const int32_t i0 = F[3 * (int64_t)t], i1 = F[3 * (int64_t)t + 1], i2 = F[3 * (int64_t)t + 2];
    const double Ax = V[3 * (int64_t)i0], Ay = V[3 * (int64_t)i0 + 1], Az = V[3 * (int64_t)i0 + 2];
    const double Bx = V[3 * (int64_t)i1], By = V[3 * (int64_t)i1 + 1], Bz = V[3 * (int64_t)i1 + 2];
    const double Cx = V[3 * (int64_t)i2], Cy = V[3 * (int64_t)i2 + 1], Cz = V[3 * (int64_t)i2 + 2];
    const double dx = ex - ox, dy = ey - oy, dz = ez - oz;
    const double e1x = Bx - Ax, e1y = By - Ay, e1z = Bz - Az;
    const double e2x = Cx - Ax, e2y = Cy - Ay, e2z = Cz - Az;
    const double sx = ox - Ax, sy = oy - Ay, sz = oz - Az;
    const double px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    const double qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    const double det = (e1x * px + e1y * py) + e1z * pz;
    const double U = (sx * px + sy * py) + sz * pz;
    const double W = (dx * qx + dy * qy) + dz * qz;
    const double T = (e2x * qx + e2y * qy) + e2z * qz;
    MT64 r{false, 0.0, 0.0, 0.0};
    if (det == 0.0)
        return r;
    const double g = det > 0.0 ? 1.0 : -1.0;
    const double a = g * U, b = g * W, tt = g * T, D = g * det;
    if (a >= 0.0 && b >= 0.0 && a + b <= D && tt >= 0.0 && tt <= D) {
        r.hit = true;
        r.u = U / det;
        r.v = W / det;
        r.t = T / det;
    }
    return r;
}

__device__ __forceinline__ bool valid_tri(const int32_t *__restrict__ F, int64_t nv, int t) {
    const int32_t i0 = F[3 * (int64_t)t], i1 = F[3 * (int64_t)t + 1], i2 = F[3 * (int64_t)t + 2];
    return i0 >= 0 && i1 >= 0 && i2 >= 0 && i0 < nv && i1 < nv && i2 < nv;
}

struct Outs {
    uint8_t *hit;
    int32_t *id;
    float *uvt;
    int32_t *count;
};

__device__ __forceinline__ void write_count(const Outs &o, int64_t i, int32_t c) {
    if (o.hit)
        o.hit[i] = c > 0 ? 1 : 0;
    o.count[i] = c;
}

__device__ __forceinline__ void write_out(const Outs &o, int64_t i, int mode, int id, float u, float v, float t) {
    if (mode == MODE_COUNT) {
        write_count(o, i, id >= 0 ? 1 : 0);
        return;
    }
    if (o.hit)
        o.hit[i] = id >= 0 ? 1 : 0;
    if (mode != MODE_BOOL)
        o.id[i] = id;
    if (mode == MODE_BARY) {
        o.uvt[3 * i] = id >= 0 ? u : NAN;
        o.uvt[3 * i + 1] = id >= 0 ? v : NAN;
        o.uvt[3 * i + 2] = id >= 0 ? t : NAN;
    }
}

struct TravParams {
    const Node *__restrict__ nodes;
    const Node4 *__restrict__ nodes4;  // the 4-wide tree the first pass walks, or NULL
    const Node4 *__restrict__ top4;    // its first kTopSlots nodes, breadth-first
    int top_lds;                       // how many of them each workgroup keeps in LDS
    int bary_after;                    // certified barycentric, one mesh: (u, v, t) by k_bary64
    const Tri *__restrict__ tris;
    const float *__restrict__ V;
    const int32_t *__restrict__ F;
    const float *__restrict__ bounds;
    int64_t nv;
    int64_t nt;
    int root;
    const float *__restrict__ from;
    const float *__restrict__ to;
    int64_t n;
    Outs out;
    int stack_depth;
    int waves_per_cu;
    int32_t *queue;
    uint32_t *queue_len;
    uint32_t *next_ray;
    unsigned long long *counters;
    uint32_t *visits;
    uint32_t *tests;
    const uint8_t *bucket;
    const int32_t *bucket_ref;
    const int4 *items;
    int n_items;
    const int32_t *group_start;  // [n_groups + 1] first item of each group, or NULL: one queue
    int n_groups;
    int n_meshes;
    const int32_t *mesh_root;
    const int32_t *mesh_root4;  // the mesh roots as 4-wide references (first pass over 4-wide nodes)
    // batched form, 4-wide, every top slot in LDS: each workgroup keeps the
    // top of its XCD group's meshes (group blockIdx.x mod n_groups) instead
    // of the combined tree's, with the mesh roots as references in it
    const Node4 *top4g;
    const int32_t *roots4g;
    int top_group;
    const int32_t *mesh_toff;
    const int32_t *ray_off;
    const int32_t *order;  // segment at each processing position (NULL: input order)
    int stage_ok;          // boolean results may be staged per wave (4-byte aligned output)
    int deep_cap;          // second pass: entries of a lane's private stack (<= kDeepStack)
    int wave_cap;          // second pass: entries of a wave's shared stack (<= its LDS array)
};

__device__ __forceinline__ void enqueue(const TravParams &p, int64_t i, int why) {
    const uint32_t slot = atomicAdd(p.queue_len, 1u);
    p.queue[slot] = (int32_t)i;
    atomicAdd(p.counters + why, 1ull);
}


// Pointers into LDS by address space, so reads of the LDS copy of the tree's
// top compile to ds_read and are not merged with the global path.
typedef const __attribute__((address_space(3))) char *LdsBytes;
typedef float F4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 lds_f4(LdsBytes p) {
    const F4v v = *reinterpret_cast<const __attribute__((address_space(3))) F4v *>(p);
    return make_float4(v.x, v.y, v.z, v.w);
}

// Compare-exchange of (entry t, child) pairs: the nearer first.
__device__ __forceinline__ void order2(float &ka, int &ca, float &kb, int &cb) {
    const bool sw = kb < ka;
    const float lo = fminf(ka, kb), hi = fmaxf(ka, kb);
    const int cl = sw ? cb : ca, ch = sw ? ca : cb;
    ka = lo;
    kb = hi;
    ca = cl;
    cb = ch;
}

// ------------------------------------------------------------------ pass 1
// Persistent waves.  Each wave owns a contiguous range of segments; a lane
// whose segment is finished is refilled from that range while the others go
// on, so a wave's time follows the mean cost of a segment instead of the
// slowest of its 64 (no atomics: a shared counter across eight XCDs costs more
// than the imbalance of ~1e3 segments per wave).  Leaf tests are postponed: a lane holds up to
// kPend leaves aside and continues with internal nodes; the leaf phase runs
// once a set share of the wave is waiting (on a further leaf, or done), so the
// leaf code runs for many lanes at once.
constexpr int kRefillMin = 8;     // refill when at least this many lanes idle
// The node phase hands over to the leaf phase once more than 1/kLeafShare of
// the active lanes wait on a leaf: early for the modes that test few leaves
// per segment (node steps keep more lanes busy), at half for the count mode,
// which tests every leaf it reaches (measured on the paper-scale workload).
template <int MODE>
constexpr int kLeafShare = MODE == MODE_COUNT ? 2 : 3;
// Leaves a lane may hold aside while it goes on with internal nodes: two
// keep more lanes in the node phase (boolean -2%, intercept count -5% at the
// paper's scale against one; three gain nothing more).
template <int MODE>
constexpr int kPend = 2;
// Resident waves per CU of the persistent traversal unless asked otherwise:
// fewer waves than registers allow share the CU's L1 among fewer tree paths.
constexpr int kDefaultWavesPerCU = 16;
constexpr int kDone = INT32_MIN;  // nothing left for the lane's segment
// One mesh: the share of the segments handed out in chunks at the end of the
// launch (1/kTailDiv of them), and the chunk size.  At the paper's scale a
// sixth measured best (a quarter, an eighth, a tenth, a twelfth and a
// sixteenth all ended later).
constexpr int64_t kTailDiv = 6;
constexpr int kTailChunk = 64;

// Boolean results of one mesh in input order are staged per wave in LDS and
// written out a window of kStageWin segments at a time (whole lines instead
// of single bytes as segments finish): two windows per wave, each a value
// and a done bitmap and a count of finished segments.  A wave's range starts
// at a multiple of 4, so a window's groups of four are 4-byte aligned (a
// coarser alignment would unbalance the waves' ranges).
constexpr int kStageWin = 256;
constexpr int kStageWords = 2 * kStageWin / 32 + 1;  // value bits, done bits, count
constexpr int kStageWaveWords = 2 * kStageWords + 2;  // two windows, padded to 16 bytes

// PROP: proposal-first order.  Phase 0 traverses the predicted frontier
// subtree; phase 1 the whole tree with that subtree left out.  Together they
// visit exactly what the plain order visits, so results do not change.
template <int MODE, bool CERT, bool STATS, bool PROP, bool WIDE>
__device__ __forceinline__ void traverse_pass1(TravParams p, int *lds_stack) {
    int *stk = lds_stack + threadIdx.x;
    const int stride = blockDim.x;
    const int lane = threadIdx.x & 63;
    const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    const float scale = p.bounds[6];
    const int n_internal = (int)p.nt - 1;
    const int max_steps = 2 * (int)p.nt + 8;  // N_t < 2^30
    const int depth_lim = p.stack_depth * stride;  // stack offsets are kept in units of lanes
    // 4-wide: the top of the tree in LDS, after the stacks (read-only once filled)
    const int ref_lim = WIDE ? n_internal + kTopSlots : n_internal;
    float4 *top_cache = reinterpret_cast<float4 *>(lds_stack + (p.stack_depth + 3) * stride);
    const int group = p.n_groups > 0 ? (int)(blockIdx.x % p.n_groups) : 0;
    if (WIDE) {
        const Node4 *top = p.top_group ? p.top4g + (int64_t)group * kTopSlots : p.top4;
        const float4 *src = reinterpret_cast<const float4 *>(top);
        for (int i = threadIdx.x; i < 8 * p.top_lds; i += stride)
            top_cache[i] = src[i];
        __syncthreads();
    }
    const int32_t *roots4 = p.top_group ? p.roots4g + (int64_t)group * 64 : p.mesh_root4;

    // One mesh: each wave owns a contiguous range of segments and its lanes
    // draw from it.  Batched form: waves take (mesh, segment range) items from
    // a shared queue, one atomic per item.  Wave-uniform state.
    const bool batch = p.items != nullptr;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t wave_id = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    // boolean results staged in LDS (one mesh, input order, 4-byte aligned output)
    const bool stage = MODE == MODE_BOOL && !STATS && !batch && p.order == nullptr && p.stage_ok;
    // One mesh: the first segments are split evenly over the waves; the rest
    // (1/kTailDiv, from a multiple of 4) is a pool of kTailChunk-segment chunks
    // that waves take in turn once their own share is handed out, so the waves
    // whose shares cost more do not hold up the end of the launch.
    const int64_t n_static = batch ? 0 : (p.n - p.n / kTailDiv) & ~int64_t(3);
    int64_t cursor = batch ? 0 : n_static * wave_id / waves;
    int64_t range_end = batch ? 0 : n_static * (wave_id + 1) / waves;
    if (stage) {  // ranges start at multiples of 4
        cursor &= ~int64_t(3);
        range_end = wave_id + 1 == waves ? n_static : (range_end & ~int64_t(3));
    }
    uint32_t *stage_w = nullptr;  // this wave's two windows
    int64_t win_base = cursor;    // first segment of the older window
    int win_old = 0;              // which of the two holds the older window
    if (stage) {
        // after the stacks (stack_depth + 3 entries per lane with 4-wide nodes,
        // + 1 with binary ones) and the top nodes
        stage_w = reinterpret_cast<uint32_t *>(lds_stack + (p.stack_depth + (WIDE ? 3 : 1)) * stride +
                                               32 * p.top_lds) +
                  (threadIdx.x >> 6) * kStageWaveWords;
        if (lane < kStageWaveWords)
            stage_w[lane] = 0u;
    }
    // write the finished entries of the older window (all of them once its
    // count is complete) and make the newer one the older
    auto stage_flush = [&]() {
        const uint32_t *W = stage_w + win_old * kStageWords;
        const int j = 4 * lane;
        const uint32_t v = (W[j >> 5] >> (j & 31)) & 0xfu, d = (W[8 + (j >> 5)] >> (j & 31)) & 0xfu;
        const int64_t i = win_base + j;
        if (d == 0xfu && i + 3 < range_end) {
            const uint32_t word = (v & 1u) | ((v >> 1) & 1u) << 8 | ((v >> 2) & 1u) << 16 | ((v >> 3) & 1u) << 24;
            *reinterpret_cast<uint32_t *>(p.out.hit + i) = word;
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (((d >> k) & 1u) && i + k < range_end)
                    p.out.hit[i + k] = (uint8_t)((v >> k) & 1u);
        }
        if (lane < kStageWords)
            stage_w[win_old * kStageWords + lane] = 0u;  // read above by every lane first (in wave order)
        win_base += kStageWin;
        win_old ^= 1;
    };
    // a finished boolean segment: into its window, or straight out if its
    // window has been written already (a segment that outlasted it)
    auto put_hit = [&](int64_t i, uint32_t v) {
        const int64_t off = i - win_base;
        if (stage && off >= 0 && off < 2 * kStageWin) {
            uint32_t *W = stage_w + ((win_old + (int)(off >> 8)) & 1) * kStageWords;
            const int j = (int)(off & (kStageWin - 1));
            if (v)
                atomicOr(W + (j >> 5), 1u << (j & 31));
            atomicOr(W + 8 + (j >> 5), 1u << (j & 31));
            atomicAdd(W + 16, 1u);
        } else {
            p.out.hit[i] = (uint8_t)v;
        }
    };
    bool items_left = batch || n_static < p.n;  // batch items, or the pool's chunks
    uint32_t groups_done = 0;  // item groups found empty (wave-uniform)
    int cur_root = p.root, cur_toff = 0;
    int lane_root = p.root, lane_toff = 0;  // of the lane's current segment

    int64_t ray = -1;
    Ray r;
    // 4-wide: byte offsets in a node of the near-face rows (x lo or hi at 0 /
    // 16, y at 32 / 48, z at 64 / 80; the far row is the other of each pair)
    // and the matching slab offsets, fixed per segment by the direction signs
    int offx = 0, offy = 32, offz = 64;
    float3 nn = make_float3(0.0f, 0.0f, 0.0f), nf = nn;
    int ref = kDone, sp = 0;  // sp: offset of the next free slot (a multiple of stride)
    int held[kPend<MODE>];    // leaves held aside (-1: free), tested in this order
#pragma unroll
    for (int k = 0; k < kPend<MODE>; ++k)
        held[k] = -1;
    auto none_held = [&]() {
        bool none = true;
#pragma unroll
        for (int k = 0; k < kPend<MODE>; ++k)
            none = none && held[k] < 0;
        return none;
    };
    auto drop_held = [&]() {
#pragma unroll
        for (int k = 0; k < kPend<MODE>; ++k)
            held[k] = -1;
    };
    float tlimit = 1.0f;
    int best_id = -1;
    float best_t = INFINITY, best_lo = INFINITY, best_hi = INFINITY, best_u = 0.0f, best_v = 0.0f;
    // certified nearest hit: its binary64 t when computed (it decided a tie)
    bool best_exact = false;
    double best_t64 = 0.0;
    bool found = false, flagged = false, overflow = false;
    uint32_t n_nodes = 0, n_tests = 0;
    int steps = 0;
    int phase = 1, skip = kDone;  // kDone never equals a child reference
    bool best_late = false;       // best hit found in phase 1 (a proposal miss)
    uint32_t n_late = 0;          // this lane's proposal misses, summed per wave at exit
    uint32_t n_redecided = 0;     // boolean, certified: pairs of this segment decided in binary64
    uint32_t seg_redecided = 0;   // this lane's segments with such a pair, summed per wave at exit
    // count mode: the distinct t found so far -- binary32 values (plain), or
    // intervals that each hold one hit's binary64 t (certified): disjoint
    // intervals hold distinct values, so only overlapping ones need the exact
    // second pass
    float tk[kCountSlots<CERT>], tk_hi[kCountSlots<CERT>];
    int nk = 0;
    bool list_full = false;

    auto pop = [&]() -> int { return sp > 0 ? stk[sp -= stride] : kDone; };

    for (;;) {
        // ---- refill idle lanes
        const uint64_t idle = __ballot(ray < 0);
        if (!batch && items_left && cursor >= range_end && idle) {
            uint32_t k = 0;
            if (lane == 0)
                k = atomicAdd(p.next_ray, 1u);
            k = __shfl(k, 0);
            const int64_t start = n_static + (int64_t)k * kTailChunk;
            if (start < p.n) {
                if (stage) {
                    // what the old range left in its windows goes out (against
                    // the old range end); then the windows start at the chunk.
                    // Segments of the old range still in flight come before
                    // it, so they are written straight out when they finish.
                    if (win_base < range_end)
                        stage_flush();
                    if (win_base < range_end)
                        stage_flush();
                    win_base = start;
                    win_old = 0;
                }
                cursor = start;
                range_end = start + kTailChunk < p.n ? start + kTailChunk : p.n;
            } else {
                items_left = false;
            }
        }
        if (batch && items_left && cursor >= range_end && idle) {
            int item = -1;
            if (p.group_start) {
                // items are grouped by XCD (workgroups are spread over the
                // eight XCDs in turn): this workgroup's group first, so each
                // XCD's L2 serves a few meshes; then the others, so no XCD
                // idles while work is left
#pragma unroll 1
                for (int t = 0; t < p.n_groups && item < 0; ++t) {
                    const int g = (group + t) % p.n_groups;
                    if (groups_done & (1u << g))
                        continue;
                    uint32_t k = 0;
                    if (lane == 0)
                        k = atomicAdd(p.queue_len + kGroupNext + g, 1u);
                    k = __shfl(k, 0);
                    const int first = p.group_start[g], count = p.group_start[g + 1] - first;
                    if (k < (uint32_t)count)
                        item = first + (int)k;
                    else
                        groups_done |= 1u << g;
                }
            } else {
                uint32_t k = 0;
                if (lane == 0)
                    k = atomicAdd(p.next_ray, 1u);
                k = __shfl(k, 0);
                item = k < (uint32_t)p.n_items ? (int)k : -1;
            }
            if (item >= 0) {
                const int4 it = p.items[item];
                cursor = it.y;
                range_end = it.z;
                cur_root = WIDE ? roots4[it.x] : p.mesh_root[it.x];
                cur_toff = p.mesh_toff[it.x];
            } else {
                items_left = false;
            }
        }
        if (cursor < range_end && idle && (__popcll(idle) >= kRefillMin || idle == ~0ull)) {
            const int cnt = __popcll(idle);
            if (stage && cursor + cnt > win_base + 2 * kStageWin)
                stage_flush();  // the older window waits on a slow segment: write what is done
            const int64_t base = cursor;
            cursor = base + cnt < range_end ? base + cnt : range_end;
            if (ray < 0) {
                const int64_t idx = base + __popcll(idle & lt_mask);
                if (idx < range_end) {
                    ray = p.order ? p.order[idx] : idx;
                    lane_root = cur_root;
                    lane_toff = cur_toff;
                    ref = lane_root;
                    drop_held();
                    sp = 0;
                    tlimit = 1.0f;
                    best_id = -1;
                    best_t = best_lo = best_hi = INFINITY;
                    best_exact = false;
                    best_u = best_v = 0.0f;
                    found = flagged = overflow = false;
                    n_redecided = 0;
                    n_nodes = n_tests = 0;
                    nk = 0;
                    list_full = false;
                    steps = 0;
                    best_late = false;
                    if (PROP) {
                        skip = p.bucket_ref[p.bucket[ray]];
                        ref = skip;
                        phase = 0;
                    }
                    if (!setup_ray(p.from, p.to, ray, scale, r)) {
                        if (STATS) {
                            p.visits[ray] = 0;
                            p.tests[ray] = 0;
                        } else if (CERT) {
                            enqueue(p, ray, 0);
                            if (MODE == MODE_BOOL)
                                put_hit(ray, 0u);  // written again by the second pass
                        } else if (MODE == MODE_BOOL) {
                            put_hit(ray, 0u);
                        } else {
                            write_out(p.out, ray, MODE, -1, 0.0f, 0.0f, 0.0f);
                        }
                        ray = -1;
                    } else if (WIDE) {
                        const bool sx = r.inv.x < 0.0f, sy = r.inv.y < 0.0f, sz = r.inv.z < 0.0f;
                        offx = sx ? 16 : 0;
                        offy = sy ? 48 : 32;
                        offz = sz ? 80 : 64;
                        nn = make_float3(sx ? r.nrb.x : r.nra.x, sy ? r.nrb.y : r.nra.y, sz ? r.nrb.z : r.nra.z);
                        nf = make_float3(sx ? r.nra.x : r.nrb.x, sy ? r.nra.y : r.nrb.y, sz ? r.nra.z : r.nrb.z);
                    }
                }
            }
        }
        const uint64_t active = __ballot(ray >= 0);
        if (!active) {
            if (cursor >= range_end && !items_left)
                break;
            continue;
        }

        // ---- node phase
        // Push and pop are branch-free: every lane has one spare LDS slot past
        // its stack_depth entries, so the push slot is written unconditionally
        // (a slot at or above sp holds nothing live), and the top of stack is
        // read ahead of the node fetch and used only if the node yields nothing.
        for (;;) {
            if (ray >= 0 && ref < 0 && ref != kDone) {  // a leaf: hold it aside if a slot is free
                bool put = false;
#pragma unroll
                for (int k = 0; k < kPend<MODE>; ++k)
                    if (!put && held[k] < 0) {
                        held[k] = ~ref;
                        put = true;
                    }
                if (put)
                    ref = pop();
            }
            const bool want = ray >= 0 && ref >= 0;
            const uint64_t w = __ballot(want);
            if (!w)
                break;
            const uint64_t waiting = active & ~w;
            if (kLeafShare<MODE> * __popcll(waiting) > __popcll(active))
                break;
            if (want) {
                if (++steps > max_steps || ref >= ref_lim) {
                    overflow = true;  // cannot happen for a well-formed tree
                    ref = kDone;
                    drop_held();
                } else {
                    const int top = stk[sp > 0 ? sp - stride : 0];
                    if (STATS)
                        ++n_nodes;
                    if (WIDE) {
                        // four children per fetch; the hits after the next one
                        // go on the stack, at most three slots past sp (the
                        // lane has three spare slots past stack_depth)
                        // each load fetches a face row of all four children:
                        // near and far faces chosen by the segment's signs
                        float4 nx, fx, ny, fy, nz, fz;
                        int4 ch;
                        if (ref < p.top_lds) {  // the top of the tree, from LDS (ds_read)
                            const LdsBytes c = (LdsBytes)(top_cache + 8 * ref);  // generic -> LDS
                            nx = lds_f4(c + offx);
                            fx = lds_f4(c + (offx ^ 16));
                            ny = lds_f4(c + offy);
                            fy = lds_f4(c + (offy ^ 16));
                            nz = lds_f4(c + offz);
                            fz = lds_f4(c + (offz ^ 16));
                            const float4 cf = lds_f4(c + 96);
                            ch = make_int4(__float_as_int(cf.x), __float_as_int(cf.y), __float_as_int(cf.z),
                                           __float_as_int(cf.w));
                        } else {
                            // nodes4 follows top4: one address for both kinds of reference
                            const char *c = reinterpret_cast<const char *>(p.top4 + ref);
                            nx = *reinterpret_cast<const float4 *>(c + offx);
                            fx = *reinterpret_cast<const float4 *>(c + (offx ^ 16));
                            ny = *reinterpret_cast<const float4 *>(c + offy);
                            fy = *reinterpret_cast<const float4 *>(c + (offy ^ 16));
                            nz = *reinterpret_cast<const float4 *>(c + offz);
                            fz = *reinterpret_cast<const float4 *>(c + (offz ^ 16));
                            ch = *reinterpret_cast<const int4 *>(c + 96);
                        }
                        float k0, k1, k2, k3;
                        bool h0 = slab_nf(nx.x, fx.x, ny.x, fy.x, nz.x, fz.x, r.inv, nn, nf, tlimit, k0);
                        bool h1 = slab_nf(nx.y, fx.y, ny.y, fy.y, nz.y, fz.y, r.inv, nn, nf, tlimit, k1);
                        bool h2 = slab_nf(nx.z, fx.z, ny.z, fy.z, nz.z, fz.z, r.inv, nn, nf, tlimit, k2);
                        bool h3 = slab_nf(nx.w, fx.w, ny.w, fy.w, nz.w, fz.w, r.inv, nn, nf, tlimit, k3);
                        int c0 = ch.x, c1 = ch.y, c2 = ch.z, c3 = ch.w;
                        if (PROP) {  // in phase 1 the proposed subtree is done already
                            h0 = h0 && c0 != skip;
                            h1 = h1 && c1 != skip;
                            h2 = h2 && c2 != skip;
                            h3 = h3 && c3 != skip;
                        }
                        const int nh = (int)h0 + (int)h1 + (int)h2 + (int)h3;
                        if (MODE != MODE_COUNT) {
                            // nearest first: a boolean segment meets a hit
                            // sooner, the nearest-hit modes' shrinking t limit
                            // prunes the rest
                            k0 = h0 ? k0 : INFINITY;
                            k1 = h1 ? k1 : INFINITY;
                            k2 = h2 ? k2 : INFINITY;
                            k3 = h3 ? k3 : INFINITY;
                            order2(k0, c0, k1, c1);
                            order2(k2, c2, k3, c3);
                            order2(k0, c0, k2, c2);
                            order2(k1, c1, k3, c3);
                            order2(k1, c1, k2, c2);
                            stk[sp] = nh == 4 ? c3 : (nh == 3 ? c2 : c1);
                            stk[sp + stride] = nh == 4 ? c2 : c1;
                            stk[sp + 2 * stride] = c1;
                        } else {
                            // count mode visits every candidate whatever the
                            // order: the first hit child is next, the others go
                            // on the stack in child order
                            const int p1 = h0, p2 = p1 + h1, p3 = p2 + h2;
                            if (h1 && p1)
                                stk[sp] = c1;
                            if (h2 && p2)
                                stk[sp + (p2 - 1) * stride] = c2;
                            if (h3 && p3)
                                stk[sp + (p3 - 1) * stride] = c3;
                            c0 = h0 ? c0 : (h1 ? c1 : (h2 ? c2 : c3));
                        }
                        ref = nh ? c0 : (sp > 0 ? top : kDone);
                        sp += nh > 1 ? (nh - 1) * stride : (nh == 0 && sp > 0 ? -stride : 0);
                        if (sp > depth_lim) {
                            overflow = true;  // the segment goes to the deep-stack pass
                            ref = kDone;
                            drop_held();
                        }
                    } else {
                        const Node *nd = p.nodes + ref;
                        const float4 L = nd->xy_left, R = nd->xy_right, Z = nd->z_both;
                        const int4 refs = nd->refs;
                        float tl, tr;
                        bool hl = slab(L.x, L.y, L.z, L.w, Z.x, Z.y, r, tlimit, tl);
                        bool hr = slab(R.x, R.y, R.z, R.w, Z.z, Z.w, r, tlimit, tr);
                        if (PROP) {  // in phase 1 the proposed subtree is done already
                            hl = hl && refs.x != skip;
                            hr = hr && refs.y != skip;
                        }
                        const bool both = hl && hr, any = hl || hr;
                        const bool left_first = both ? tl <= tr : hl;
                        stk[sp] = left_first ? refs.y : refs.x;
                        const int next = left_first ? refs.x : refs.y;
                        overflow = overflow || (both && sp >= depth_lim);
                        ref = any ? next : (sp > 0 ? top : kDone);
                        sp += both ? stride : (!any && sp > 0 ? -stride : 0);
                        if (both && sp > depth_lim) {
                            ref = kDone;  // overflow: the segment goes to the deep-stack pass
                            drop_held();
                        }
                    }
                }
            }
        }

        // ---- leaf phase: the leaves held aside, in the order they were met;
        // a decided segment drops the rest
        auto test_leaf = [&](const int leaf) {
            if (leaf >= p.nt) {
                overflow = true;  // cannot happen for a well-formed tree
                ref = kDone;
            } else {
                const Tri tri = p.tris[leaf];
                if (STATS)
                    ++n_tests;
                const MT32 m = mt32(tri, r);
                const int id = __float_as_int(tri.a.w);
                if (MODE == MODE_COUNT) {
                    // every hit counts once per distinct t; no early exit, no pruning
                    if (!CERT) {
                        if (decide32(m)) {
                            const float t = m.T / m.det;
                            bool dup = false;
#pragma unroll
                            for (int k = 0; k < kCountSlots<CERT>; ++k)
                                dup = dup || (k < nk && tk[k] == t);
                            if (!dup) {
                                if (nk == kCountSlots<CERT>) {
                                    list_full = true;  // finished by the second pass
                                    ref = kDone;
                                } else {
#pragma unroll
                                    for (int k = 0; k < kCountSlots<CERT>; ++k)
                                        if (k == nk)
                                            tk[k] = t;
                                    ++nk;
                                }
                            }
                        }
                    } else {
                        // a sure hit brings an interval holding its binary64 t;
                        // an unsure pair is decided in binary64 here
                        float lo = 0.0f, hi = 0.0f;
                        const int c = classify(m, tri, r, lo, hi);
                        bool take = c == kHit;
                        if (c == kUnsure && valid_tri(p.F, p.nv, id)) {
                            const float *o = p.from + 3 * ray, *e = p.to + 3 * ray;
                            const MT64 h = mt64(o[0], o[1], o[2], e[0], e[1], e[2], p.V, p.F, id);
                            take = h.hit;
                            lo = __double2float_rd(h.t);
                            hi = __double2float_ru(h.t);
                        }
                        if (take) {
                            bool meet = false;
#pragma unroll
                            for (int k = 0; k < kCountSlots<CERT>; ++k)
                                meet = meet || (k < nk && !(hi < tk[k] || lo > tk_hi[k]));
                            if (meet) {
                                flagged = true;  // equal or nearly equal t: counted exactly by the second pass
                                ref = kDone;
                            } else if (nk == kCountSlots<CERT>) {
                                list_full = true;
                                ref = kDone;
                            } else {
#pragma unroll
                                for (int k = 0; k < kCountSlots<CERT>; ++k)
                                    if (k == nk) {
                                        tk[k] = lo;
                                        tk_hi[k] = hi;
                                    }
                                ++nk;
                            }
                        }
                    }
                } else if (!CERT) {
                    if (decide32(m)) {
                        if (MODE == MODE_BOOL) {
                            found = true;
                            best_late = phase == 1;
                            ref = kDone;
                        } else {
                            const float t = m.T / m.det;
                            if (t < best_t || (t == best_t && id < best_id)) {
                                best_t = t;
                                best_id = id;
                                best_late = phase == 1;
                                if (MODE == MODE_BARY) {
                                    best_u = m.U / m.det;
                                    best_v = m.W / m.det;
                                }
                                tlimit = best_t;
                            }
                        }
                    }
                } else {
                    float lo = 0.0f, hi = 0.0f;
                    const int c = classify(m, tri, r, lo, hi);
                    if (MODE == MODE_BOOL) {
                        bool hit = c == kHit;
                        if (c == kUnsure) {
                            // decided here in binary64, in the oracle's
                            // operation order: a segment aimed at an edge or a
                            // vertex would otherwise search on for a sure hit
                            // through everything its box overlaps
                            ++n_redecided;
                            if (valid_tri(p.F, p.nv, id)) {
                                const float *o = p.from + 3 * ray, *e = p.to + 3 * ray;
                                hit = mt64(o[0], o[1], o[2], e[0], e[1], e[2], p.V, p.F, id).hit;
                            }
                        }
                        if (hit) {
                            found = true;
                            best_late = phase == 1;
                            ref = kDone;
                        }
                    } else {
                        // an unsure pair is decided here in binary64, in the
                        // oracle's operation order; a hit then takes part
                        // like a sure one, its interval holding the exact t
                        bool hit = c == kHit, exact = false;
                        double t64 = 0.0;
                        const float *o = p.from + 3 * ray, *e = p.to + 3 * ray;
                        if (c == kUnsure) {
                            ++n_redecided;
                            hit = false;
                            if (valid_tri(p.F, p.nv, id)) {
                                const MT64 h = mt64(o[0], o[1], o[2], e[0], e[1], e[2], p.V, p.F, id);
                                hit = h.hit;
                                exact = true;
                                t64 = h.t;
                                lo = __double2float_rd(h.t);
                                hi = __double2float_ru(h.t);
                            }
                        }
                        if (hit && !(best_id < 0 || hi < best_lo) && !(lo > best_hi)) {
                            // the intervals overlap: compare the binary64 t
                            // themselves (both pairs are binary64 hits), ties
                            // to the smaller triangle id, as the oracle
                            if (!exact) {
                                t64 = mt64(o[0], o[1], o[2], e[0], e[1], e[2], p.V, p.F, id).t;
                                exact = true;
                            }
                            if (!best_exact) {
                                best_t64 = mt64(o[0], o[1], o[2], e[0], e[1], e[2], p.V, p.F, best_id).t;
                                best_exact = true;
                            }
                            ++n_redecided;
                            hit = t64 < best_t64 || (t64 == best_t64 && id < best_id);
                            lo = __double2float_rd(t64);
                            hi = __double2float_ru(t64);
                        } else if (hit && best_id >= 0 && !(hi < best_lo)) {
                            hit = false;  // beyond the best hit
                        }
                        if (hit) {
                            best_lo = lo;
                            best_hi = hi;
                            best_id = id;
                            best_exact = exact;
                            best_t64 = t64;
                            best_late = phase == 1;
                            tlimit = fminf(tlimit, hi * (1.0f + 0x1p-20f));
                        }
                    }
                }
            }
        };
#pragma unroll
        for (int k = 0; k < kPend<MODE>; ++k)
            if (ray >= 0 && held[k] >= 0) {
                const int leaf = held[k];
                held[k] = -1;
                if (!(found || flagged || list_full || overflow))
                    test_leaf(leaf);
            }

        // ---- proposal: the predicted subtree is exhausted, go on with the rest
        if (PROP && ray >= 0 && ref == kDone && none_held() && phase == 0 && !found && !flagged && !overflow) {
            phase = 1;
            ref = lane_root == skip ? kDone : lane_root;
        }

        // ---- finish lanes whose segment is decided
        if (ray >= 0 && ref == kDone && none_held()) {
            if (PROP && !STATS && best_late && (found || (MODE != MODE_BOOL && best_id >= 0 && !flagged && !overflow)))
                ++n_late;  // the proposal did not hold the answer
            if (STATS) {
                p.visits[ray] = n_nodes;
                p.tests[ray] = n_tests;
            } else if (MODE == MODE_COUNT) {
                if (overflow)
                    enqueue(p, ray, 1);
                else if (list_full)
                    enqueue(p, ray, 3);
                else if (CERT && flagged)
                    enqueue(p, ray, 0);
                else
                    write_count(p.out, ray, nk);
            } else if (MODE == MODE_BOOL) {
                // a queued segment counts as finished here (0); the second
                // pass writes its result after this kernel
                if (!found && overflow)
                    enqueue(p, ray, 1);
                seg_redecided += n_redecided > 0 ? 1u : 0u;
                put_hit(ray, found ? 1u : 0u);
            } else {
                if (CERT && n_redecided > 0 && !flagged)
                    ++seg_redecided;  // (a flagged segment is counted when queued)
                if (overflow) {
                    enqueue(p, ray, 1);
                } else if (CERT && flagged) {
                    enqueue(p, ray, 0);
                } else if (CERT && MODE == MODE_BARY && best_id >= 0) {
                    if (p.bary_after) {  // (u, v, t) after both passes, a lane per segment
                        if (p.out.hit)
                            p.out.hit[ray] = 1;
                        p.out.id[ray] = best_id - lane_toff;
                    } else {
                        const float *o = p.from + 3 * ray, *e = p.to + 3 * ray;
                        const MT64 h = mt64(o[0], o[1], o[2], e[0], e[1], e[2], p.V, p.F, best_id);
                        write_out(p.out, ray, MODE, best_id - lane_toff, (float)h.u, (float)h.v, (float)h.t);
                    }
                } else {
                    write_out(p.out, ray, MODE, best_id >= 0 ? best_id - lane_toff : -1, best_u, best_v, best_t);
                }
            }
            ray = -1;
        }
        if (stage) {  // a complete older window goes out whole (then perhaps the next one)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int64_t need = range_end - win_base < kStageWin ? range_end - win_base : kStageWin;
                if (need > 0 && stage_w[win_old * kStageWords + 16] == (uint32_t)need)
                    stage_flush();
            }
        }
    }
    if (stage) {  // every segment is finished: whatever is left in the windows
        if (win_base < range_end)
            stage_flush();
        if (win_base < range_end)
            stage_flush();
    }
    if (MODE != MODE_COUNT && CERT && !STATS) {
        // segments with a pair decided in binary64 in this pass, one atomic per wave
        uint32_t w = seg_redecided;
        for (int off = 32; off > 0; off >>= 1)
            w += __shfl_xor(w, off);
        if (lane == 0 && w)
            atomicAdd(p.counters, (unsigned long long)w);
    }
    if (PROP && !STATS) {
        // one atomic per wave: a shared counter across eight XCDs is costly
        uint32_t w = n_late;
        for (int off = 32; off > 0; off >>= 1)
            w += __shfl_xor(w, off);
        if (lane == 0 && w)
            atomicAdd(p.counters + 2, (unsigned long long)w);
    }
}

// Workgroup bound per node width: the binary kernels keep 256 (a larger
// bound changed their code and cost the batched form 18%); the 4-wide ones
// take up to 1024 threads, whose workgroups keep more of the tree's top.
template <bool WIDE>
constexpr int kMaxBlock = WIDE ? 1024 : 256;

template <int MODE, bool CERT, bool STATS, bool PROP, bool WIDE>
__global__ __attribute__((amdgpu_flat_work_group_size(1, kMaxBlock<WIDE>))) void k_traverse(TravParams p) {
    extern __shared__ float4 lds_dyn[];  // 16-byte aligned: the 4-wide top nodes follow the stacks
    traverse_pass1<MODE, CERT, STATS, PROP, WIDE>(p, reinterpret_cast<int *>(lds_dyn));
}

// Count mode holds its list of distinct t in registers; the register budget
// is fixed at four waves per SIMD (the default resident count) so the list
// cannot lower occupancy.
template <bool CERT, bool STATS, bool WIDE>
__global__ __attribute__((amdgpu_flat_work_group_size(1, kMaxBlock<WIDE>), amdgpu_waves_per_eu(4))) void k_traverse_count(
    TravParams p) {
    extern __shared__ float4 lds_dyn[];
    traverse_pass1<MODE_COUNT, CERT, STATS, false, WIDE>(p, reinterpret_cast<int *>(lds_dyn));
}

// ------------------------------------------------------------------ pass 2
// Queued segments are finished exactly: a stack deep enough for any radix
// tree, and in CERTIFIED precision every candidate not already a proven
// binary32 miss decided in binary64 with the oracle's operation order.  A
// segment whose binary32 setup is not finite is tested against every
// triangle under its root.
//
// Two shapes, chosen per launch from the queue length (uniform per block):
//   short queue: one wave per segment.  The wave shares an LDS stack and pops
//     up to 64 subtrees per step, one per lane, so a segment takes about
//     (tree depth + candidates / 64) steps instead of one dependent load per
//     visited node.
//   long queue: one lane per segment with a private deep stack (throughput).
constexpr int kFinishThreads = 64;
constexpr int kCountList = 256;  // hits a wave collects per segment in count mode (more: rounds)
constexpr int kWaveFinishMax = 8192;                      // queue length up to which a wave takes a segment
constexpr int kWaveStack = kDeepStack * kFinishThreads;  // shared entries (same LDS as the private stacks)
// Steps that pop k entries push at most 2k; popping at most (soft - size),
// soft = capacity - kDeepStack, keeps the stack at or below soft, and above it
// single pops (a plain depth-first walk) add at most one entry per tree level.
// Count mode always takes the wave shape, so its blocks need only the shared
// stack (a soft limit of 1024 entries plus the depth-first headroom) and a
// short hit list: about 7 KB of LDS instead of 48, so eight times as many
// segments are in flight (its queue holds every segment with more distinct
// hits than the first pass keeps, ~14k of 1e7 at the paper's scale).
template <int MODE>
constexpr int kWaveCap = MODE == MODE_COUNT ? 1024 + kDeepStack : kWaveStack;

template <int MODE, bool CERT>
struct Finish {
    Ray r;
    double ox, oy, oz, ex, ey, ez;
    int best_id;
    double bu, bv, bt;
    float t32, u32, v32;
    float tlimit;
    bool done;
    // count mode: only hits beyond the last counted t take part; with
    // `list` set, every such hit's t is appended there instead
    double floor64;
    float floor32;
    double *list;
    int *list_len;

    __device__ void reset_best() {
        best_id = -1;
        bu = bv = bt = 0.0;
        t32 = INFINITY;
        u32 = v32 = 0.0f;
        tlimit = 1.0f;
        done = false;
    }

    __device__ bool init(const TravParams &p, int64_t i) {
        reset_best();
        floor64 = -INFINITY;
        floor32 = -INFINITY;
        list = nullptr;
        list_len = nullptr;
        const float *o = p.from + 3 * i, *e = p.to + 3 * i;
        ox = o[0]; oy = o[1]; oz = o[2];
        ex = e[0]; ey = e[1]; ez = e[2];
        return setup_ray(p.from, p.to, i, p.bounds[6], r);
    }

    __device__ void test_leaf(const TravParams &p, int leaf) {
        const Tri tri = p.tris[leaf];
        const int id = __float_as_int(tri.a.w);
        const MT32 m = mt32(tri, r);
        if (CERT) {
            float lo, hi;
            if (classify(m, tri, r, lo, hi) == kMiss)
                return;  // the bound proves the binary64 test misses too
            MT64 h{false, 0.0, 0.0, 0.0};
            if (valid_tri(p.F, p.nv, id))
                h = mt64(ox, oy, oz, ex, ey, ez, p.V, p.F, id);
            if (!h.hit || !(h.t > floor64))
                return;
            if (MODE == MODE_COUNT && list) {
                append(h.t);
                return;
            }
            if (MODE == MODE_BOOL) {
                best_id = id;
                done = true;
                return;
            }
            if (best_id < 0 || h.t < bt || (h.t == bt && id < best_id)) {
                best_id = id;
                bu = h.u;
                bv = h.v;
                bt = h.t;
                // round up, then widen: no box holding a hit at t <= bt is culled
                tlimit = fminf(tlimit, __double2float_ru(h.t) * (1.0f + 0x1p-20f));
            }
        } else if (decide32(m)) {
            if (MODE == MODE_BOOL) {
                best_id = id;
                done = true;
                return;
            }
            const float t = m.T / m.det;
            if (!(t > floor32))
                return;
            if (MODE == MODE_COUNT && list) {
                append((double)t);
                return;
            }
            if (t < t32 || (t == t32 && id < best_id)) {
                t32 = t;
                best_id = id;
                u32 = m.U / m.det;
                v32 = m.W / m.det;
                tlimit = t;
            }
        }
    }

    // Every leaf of subtree c, exactly: the second pass's answer when a
    // subtree finds no room on the stack (a tree deeper than the stack), so a
    // push is never dropped.  The span [smallest, largest sorted leaf] holds
    // the subtree's leaves (after treelet restructuring it may hold others of
    // the same mesh too; testing a triangle twice or one outside the subtree
    // never changes a result: each is decided exactly, and equal t count once).
    __device__ void test_span(const TravParams &p, int c) {
        int first = ~c, last = ~c;
        if (c >= 0) {
            const int4 r = p.nodes[c].refs;
            first = r.z;
            last = r.w;
        }
        for (int leaf = first; leaf <= last && leaf >= 0 && leaf < p.nt && !done; ++leaf)
            test_leaf(p, leaf);
    }

    __device__ void append(double t) {
        const int k = atomicAdd(list_len, 1);
        if (k < kCountList)
            list[k] = t;
    }

    __device__ void write(const TravParams &p, int64_t i, int toff) const {
        const int local = best_id >= 0 ? best_id - toff : -1;
        if (CERT)
            write_out(p.out, i, MODE, local, (float)bu, (float)bv, (float)bt);
        else
            write_out(p.out, i, MODE, local, u32, v32, t32);
    }

    // Wave-wide result: the smallest (t, triangle id) of all lanes' hits.
    __device__ void reduce_wave() {
        for (int off = 32; off > 0; off >>= 1) {
            const int oid = __shfl_xor(best_id, off);
            if (CERT) {
                const double ot = __shfl_xor(bt, off), ou = __shfl_xor(bu, off), ov = __shfl_xor(bv, off);
                if (oid >= 0 && (best_id < 0 || ot < bt || (ot == bt && oid < best_id))) {
                    best_id = oid;
                    bt = ot;
                    bu = ou;
                    bv = ov;
                }
            } else {
                const float ot = __shfl_xor(t32, off), ou = __shfl_xor(u32, off), ov = __shfl_xor(v32, off);
                if (oid >= 0 && (best_id < 0 || ot < t32 || (ot == t32 && oid < best_id))) {
                    best_id = oid;
                    t32 = ot;
                    u32 = ou;
                    v32 = ov;
                }
            }
        }
    }
};

__device__ __forceinline__ void segment_root(const TravParams &p, int64_t i, int &root, int &toff) {
    root = p.root;
    toff = 0;
    if (p.items) {  // batched form: the mesh of segment i
        int lo = 0, hi = p.n_meshes - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (p.ray_off[mid] <= i)
                lo = mid;
            else
                hi = mid - 1;
        }
        root = p.mesh_root[lo];
        toff = p.mesh_toff[lo];
    }
}

// The wave's search for one segment from `root`: every lane's share of the
// candidates goes through f.test_leaf; the caller reduces across the wave.
template <int MODE, bool CERT>
__device__ void wave_search(const TravParams &p, Finish<MODE, CERT> &f, bool ok, int root, int *stk) {
    const int lane = threadIdx.x;
    const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    const int n_internal = (int)p.nt - 1;
    if (root == kDone) {
        // empty mesh: nothing to test
    } else if (!ok) {
        if (CERT) {
            const int64_t first = root < 0 ? ~root : p.nodes[root].refs.z;
            const int64_t last = root < 0 ? ~root : p.nodes[root].refs.w;
            for (int64_t base = first; base <= last; base += 64) {
                if (base + lane <= last)
                    f.test_leaf(p, (int)(base + lane));
                if (MODE == MODE_BOOL && __ballot(f.done))
                    break;
            }
        }
    } else {
        int size = 1;
        if (lane == 0)
            stk[0] = root;
        __syncthreads();
        const int64_t max_steps = 2 * p.nt + 8;  // every step pops at least one of < 2 nt subtrees
        // soft limit: a step that pops k entries pushes at most 2k, and past
        // the soft limit single pops add at most one entry per tree level
        const int cap = p.wave_cap;
        const int soft = cap - (kDeepStack < cap / 2 ? kDeepStack : cap / 2);
        for (int64_t step = 0; step < max_steps && size > 0; ++step) {
            const int room = soft - size;
            int k = room < 1 ? 1 : (room < 64 ? room : 64);
            k = k < size ? k : size;
            const int ref = lane < k ? stk[size - 1 - lane] : kDone;
            __syncthreads();
            size -= k;
            int c0 = kDone, c1 = kDone;  // subtrees to push, nearer one on top
            if (ref >= 0 && ref < n_internal) {
                const Node *nd = p.nodes + ref;
                const float4 L = nd->xy_left, R = nd->xy_right, Z = nd->z_both;
                const int4 refs = nd->refs;
                float tl, tr;
                const bool hl = slab(L.x, L.y, L.z, L.w, Z.x, Z.y, f.r, f.tlimit, tl);
                const bool hr = slab(R.x, R.y, R.z, R.w, Z.z, Z.w, f.r, f.tlimit, tr);
                if (hl && hr) {
                    const bool left_first = tl <= tr;
                    c0 = left_first ? refs.y : refs.x;
                    c1 = left_first ? refs.x : refs.y;
                } else if (hl || hr) {
                    c0 = hl ? refs.x : refs.y;
                }
            } else if (ref != kDone && ref < 0 && ~ref < p.nt) {
                f.test_leaf(p, ~ref);
            }
            const uint64_t m0 = __ballot(c0 != kDone), m1 = __ballot(c1 != kDone);
            const int o = size + __popcll(m0 & lt_mask) + __popcll(m1 & lt_mask);
            // a subtree past the stack's capacity is searched leaf by leaf here
            if (c0 != kDone) {
                if (o < cap)
                    stk[o] = c0;
                else
                    f.test_span(p, c0);
            }
            if (c1 != kDone) {
                if (o + 1 < cap)
                    stk[o + 1] = c1;
                else
                    f.test_span(p, c1);
            }
            size += __popcll(m0) + __popcll(m1);
            size = size < cap ? size : cap;
            __syncthreads();
            if (MODE == MODE_BOOL) {
                if (__ballot(f.done))
                    break;
            } else {
                float tl = f.tlimit;  // any lane's hit bounds the nearest one
                for (int off = 32; off > 0; off >>= 1)
                    tl = fminf(tl, __shfl_xor(tl, off));
                f.tlimit = tl;
            }
        }
    }
    __syncthreads();  // the stack is reused by the next search
}

// One wave (the whole 64-thread block) finishes segment i.  Count mode
// collects the t of every hit in LDS and counts the distinct values; a
// segment with more hits than the list holds asks instead, round by round,
// for the nearest hit beyond the last counted t until there is none.
template <int MODE, bool CERT>
__device__ void finish_wave(const TravParams &p, int64_t i, int *stk) {
    int root, toff;
    segment_root(p, i, root, toff);
    Finish<MODE, CERT> f;
    const bool ok = f.init(p, i);
    if constexpr (MODE == MODE_COUNT) {
        // one search collecting every hit's t; the distinct values are then
        // counted in LDS.  Only a list that overflows falls back to rounds.
        __shared__ double list[kCountList];
        __shared__ int list_len;
        if (threadIdx.x == 0)
            list_len = 0;
        __syncthreads();
        f.list = list;
        f.list_len = &list_len;
        wave_search<MODE, CERT>(p, f, ok, root, stk);
        const int m = list_len;
        f.list = nullptr;
        if (m <= kCountList) {
            int distinct = 0;
            for (int j = threadIdx.x; j < m; j += blockDim.x) {
                const double v = list[j];
                bool first = true;
                for (int k = 0; k < j && first; ++k)
                    first = list[k] != v;
                distinct += first ? 1 : 0;
            }
            for (int off = 32; off > 0; off >>= 1)
                distinct += __shfl_xor(distinct, off);
            if (threadIdx.x == 0)
                write_count(p.out, i, distinct);
            __syncthreads();  // the list is reused by the block's next segment
            return;
        }
        int32_t cnt = 0;
        for (int64_t q = 0; q <= p.nt; ++q) {  // at most one round per triangle
            f.reset_best();
            wave_search<MODE, CERT>(p, f, ok, root, stk);
            f.reduce_wave();
            if (f.best_id < 0)
                break;
            ++cnt;
            if (CERT)
                f.floor64 = f.bt;
            else
                f.floor32 = f.t32;
        }
        if (threadIdx.x == 0)
            write_count(p.out, i, cnt);
        __syncthreads();
        return;
    } else {
        wave_search<MODE, CERT>(p, f, ok, root, stk);
        if (MODE == MODE_BOOL) {
            f.best_id = __ballot(f.best_id >= 0) ? 0 : -1;
            toff = 0;
        } else {
            f.reduce_wave();
        }
        if (threadIdx.x == 0)
            f.write(p, i, toff);
    }
}

// One lane finishes segment i with its private stack (stride kFinishThreads).
template <int MODE, bool CERT>
__device__ void finish_lane(const TravParams &p, int64_t i, int *stk) {
    int root, toff;
    segment_root(p, i, root, toff);
    Finish<MODE, CERT> f;
    const bool ok = f.init(p, i);
    if (root == kDone) {
        // empty mesh: nothing to test
    } else if (!ok) {
        if (CERT) {
            // brute force over every leaf under the root: the box test is not reliable here
            const int first = root < 0 ? ~root : p.nodes[root].refs.z;
            const int last = root < 0 ? ~root : p.nodes[root].refs.w;
            for (int leaf = first; leaf <= last && !f.done; ++leaf)
                f.test_leaf(p, leaf);
        }
    } else {
        int sp = 0;
        int ref = root;
        const int64_t max_steps = 2 * p.nt + 8;
        const int n_internal = (int)p.nt - 1;
        for (int64_t steps = 0; steps <= max_steps && ref < n_internal && ~ref < p.nt; ++steps) {
            if (ref >= 0) {
                const Node *nd = p.nodes + ref;
                const float4 L = nd->xy_left, R = nd->xy_right, Z = nd->z_both;
                const int4 refs = nd->refs;
                float tl, tr;
                const bool hl = slab(L.x, L.y, L.z, L.w, Z.x, Z.y, f.r, f.tlimit, tl);
                const bool hr = slab(R.x, R.y, R.z, R.w, Z.z, Z.w, f.r, f.tlimit, tr);
                if (hl && hr) {
                    const bool left_first = tl <= tr;
                    const int far = left_first ? refs.y : refs.x;
                    if (sp < p.deep_cap)
                        stk[(sp++) * kFinishThreads] = far;
                    else
                        f.test_span(p, far);  // deeper than the stack: that subtree leaf by leaf
                    if (f.done)
                        break;
                    ref = left_first ? refs.x : refs.y;
                    continue;
                }
                if (hl || hr) {
                    ref = hl ? refs.x : refs.y;
                    continue;
                }
            } else {
                f.test_leaf(p, ~ref);
                if (f.done)
                    break;
            }
            if (sp == 0)
                break;
            ref = stk[(--sp) * kFinishThreads];
        }
    }
    f.write(p, i, toff);
}

template <int MODE, bool CERT>
__global__ __launch_bounds__(kFinishThreads) void k_finish(TravParams p) {
    __shared__ int deep[kWaveCap<MODE>];
    const uint32_t count = *p.queue_len;
    if (MODE == MODE_COUNT || count <= (uint32_t)kWaveFinishMax) {
        for (uint32_t qi = blockIdx.x; qi < count; qi += gridDim.x)
            finish_wave<MODE, CERT>(p, p.queue[qi], deep);
    } else {
        if constexpr (MODE != MODE_COUNT)
            for (uint32_t qi = blockIdx.x * blockDim.x + threadIdx.x; qi < count; qi += gridDim.x * blockDim.x)
                finish_lane<MODE, CERT>(p, p.queue[qi], deep + threadIdx.x);
    }
}

// ------------------------------------------------------------ segment order
// Spatially coherent processing order: neighbouring lanes then take segments
// that start (or lie) close together and head the same way, so they share
// tree paths and cached nodes.  30-bit keys; in the batched form the top six
// bits are the mesh, so each mesh's segments stay in its own position range
// and the work items stay valid.
__device__ __forceinline__ uint32_t spread_bits(uint32_t v) {  // bit k -> bit 3k, 10 bits
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t cell(float x, float lo, float hi, int bits) {
    const float f = hi > lo ? (x - lo) / (hi - lo) : 0.0f;
    const float c = fminf(fmaxf(f, 0.0f), 1.0f) * (float)(1u << bits);  // NaN -> 0
    const uint32_t q = (uint32_t)c;
    return q < (1u << bits) ? q : (1u << bits) - 1u;
}

__global__ void k_ray_keys(const float *__restrict__ from, const float *__restrict__ to, int64_t n, int kind,
                           const float *__restrict__ bounds, const int32_t *__restrict__ ray_off, int n_meshes,
                           uint32_t *__restrict__ keys, int32_t *__restrict__ ids) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    int m = 0;
    if (ray_off) {
        int lo = 0, hi = n_meshes - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ray_off[mid] <= i)
                lo = mid;
            else
                hi = mid - 1;
        }
        m = lo;
    }
    const float *b = bounds + 8 * m;
    const float ox = from[3 * i], oy = from[3 * i + 1], oz = from[3 * i + 2];
    const float ex = to[3 * i], ey = to[3 * i + 1], ez = to[3 * i + 2];
    const int mesh_bits = ray_off ? 6 : 0;
    const int oct_bits = kind == 2 ? 3 : 0;
    const int bits = (30 - mesh_bits - oct_bits) / 3;
    float px = ox, py = oy, pz = oz;
    if (kind == 1) {
        px = 0.5f * (ox + ex);
        py = 0.5f * (oy + ey);
        pz = 0.5f * (oz + ez);
    }
    const uint32_t code = (spread_bits(cell(pz, b[2], b[5], bits)) << 2) |
                          (spread_bits(cell(py, b[1], b[4], bits)) << 1) | spread_bits(cell(px, b[0], b[3], bits));
    uint32_t key = code;
    if (kind == 2) {
        const uint32_t oct = (ex < ox ? 1u : 0u) | (ey < oy ? 2u : 0u) | (ez < oz ? 4u : 0u);
        key |= oct << (3 * bits);
    }
    key |= (uint32_t)m << (30 - mesh_bits);
    keys[i] = key;
    ids[i] = (int32_t)i;
}

__global__ void k_reset(uint32_t *queue_len, unsigned long long *counters, int n_groups) {
    if (threadIdx.x < 2)
        queue_len[threadIdx.x] = 0;  // queue length, next segment of pass 1
    if (threadIdx.x < n_groups)
        queue_len[kGroupNext + threadIdx.x] = 0;  // next item of each group
    if (threadIdx.x < 4)
        counters[threadIdx.x] = 0;
}

// Certified barycentric output of one mesh: the binary64 (u, v, t) of each
// segment's nearest triangle, from the original corners in the oracle's
// operation order.  Run after both passes with a lane per segment, so the
// binary64 work is not spread over the traversal's divergent lanes.
__global__ void k_bary64(const float *__restrict__ from, const float *__restrict__ to, const float *__restrict__ V,
                         const int32_t *__restrict__ F, const int32_t *__restrict__ tri_id, float *__restrict__ uvt,
                         int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    const int id = tri_id[i];
    if (id < 0)
        return;  // a miss: written by the passes
    const MT64 h = mt64(from[3 * i], from[3 * i + 1], from[3 * i + 2], to[3 * i], to[3 * i + 1], to[3 * i + 2], V, F,
                        id);
    uvt[3 * i] = (float)h.u;
    uvt[3 * i + 1] = (float)h.v;
    uvt[3 * i + 2] = (float)h.t;
}

__global__ void k_fill_miss(Outs out, int64_t n, int mode) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        write_out(out, i, mode, -1, 0.0f, 0.0f, 0.0f);
}

// Default workgroup size: 256 for binary nodes; 1024 for 4-wide ones, whose
// workgroups keep the top of the tree in LDS (a larger workgroup holds more
// of it for the same resident waves: all 512 top nodes at 1024 threads and
// depth-20 stacks; 0.2-1% faster than 512 threads in every mode at the
// paper's scale).
constexpr int kDefaultBlock = 256, kDefaultBlockWide = 1024;

template <int MODE, bool CERT, bool STATS, bool PROP, bool WIDE>
void launch_pass1(const TravParams &p, int block, hipStream_t s) {
    if (block == 0)
        block = WIDE ? kDefaultBlockWide : kDefaultBlock;
    if (block > kMaxBlock<WIDE>)
        block = kMaxBlock<WIDE>;
    // spare slots per lane past stack_depth: one for the binary push, three
    // for the 4-wide one; the 4-wide traversal also keeps the top of the tree
    // in what is left of the CU's LDS for the resident workgroups asked for
    int dev = 0, cus = 256, per_cu = 0, lds_cu = 160 * 1024, lds_block = 64 * 1024;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    (void)hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
    if (hipDeviceGetAttribute(&lds_block, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess ||
        lds_block <= 0)
        (void)hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    // a workgroup whose stacks do not fit in LDS runs with fewer threads
    const size_t lane_bytes = (size_t)(p.stack_depth + (WIDE ? 3 : 1)) * sizeof(int);
    // the boolean staging windows (per wave), after the stacks and the top nodes
    const bool staged = MODE == MODE_BOOL && !STATS && p.stage_ok && p.items == nullptr && p.order == nullptr;
    const size_t wave_stage = staged ? kStageWaveWords * sizeof(uint32_t) : 0;
    while (block > 64 && lane_bytes * block + wave_stage * (block / 64) > (size_t)lds_block)
        block /= 2;
    const size_t stack_bytes = lane_bytes * block;
    const size_t stage_bytes = wave_stage * (size_t)(block / 64);
    TravParams q = p;
    q.top_lds = 0;
    q.stage_ok = stage_bytes > 0 ? 1 : 0;
    if (WIDE) {
        int blocks_cu = p.waves_per_cu / (block / 64);
        blocks_cu = blocks_cu < 1 ? 1 : blocks_cu;
        int64_t room = lds_cu / blocks_cu;
        room = room < lds_block ? room : lds_block;
        room -= (int64_t)(stack_bytes + stage_bytes);
        const int64_t slots = room > 0 ? room / (int64_t)sizeof(Node4) : 0;
        q.top_lds = (int)(slots < kTopSlots ? slots : kTopSlots);
    }
    // a group's top replaces the combined one only when all of it is in LDS
    // (a slot fetched from memory is read at the combined top's address)
    q.top_group = (WIDE && p.items && p.top4g && q.top_lds == kTopSlots) ? 1 : 0;
    const size_t lds = stack_bytes + (size_t)q.top_lds * sizeof(Node4) + stage_bytes;
    void (*kern)(TravParams) = nullptr;
    if constexpr (MODE == MODE_COUNT)
        kern = &k_traverse_count<CERT, STATS, WIDE>;
    else
        kern = &k_traverse<MODE, CERT, STATS, PROP, WIDE>;
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern), block, lds);
    const int cap = p.waves_per_cu / (block / 64);  // resident blocks per CU asked for
    per_cu = per_cu < cap ? per_cu : cap;
    if (per_cu < 1)
        per_cu = 1;
    const int64_t want = (p.n + block - 1) / block;
    const int64_t resident = (int64_t)cus * per_cu;
    const int grid = (int)(want < resident ? want : resident);
    kern<<<grid, block, lds, s>>>(q);
}

// make_params leaves nodes4 NULL where the binary tree is walked; with the
// proposal order it names the proposal's own 4-wide tree.
template <int MODE, bool STATS, bool CERT>
void dispatch_order(const TravParams &p, bool prop, int block, hipStream_t s) {
    const bool wide = p.nodes4 != nullptr;
    if (prop)
        wide ? launch_pass1<MODE, CERT, STATS, true, true>(p, block, s)
             : launch_pass1<MODE, CERT, STATS, true, false>(p, block, s);
    else
        wide ? launch_pass1<MODE, CERT, STATS, false, true>(p, block, s)
             : launch_pass1<MODE, CERT, STATS, false, false>(p, block, s);
}

template <int MODE, bool STATS>
void dispatch_mode(const TravParams &p, bool cert, bool prop, int block, hipStream_t s) {
    cert ? dispatch_order<MODE, STATS, true>(p, prop, block, s) : dispatch_order<MODE, STATS, false>(p, prop, block, s);
}

template <bool STATS>
void dispatch_pass1(const TravParams &p, int mode, bool cert, int block, hipStream_t s) {
    const bool prop = p.bucket != nullptr;
    if (mode == MODE_BOOL)
        dispatch_mode<MODE_BOOL, STATS>(p, cert, prop, block, s);
    else if (mode == MODE_FIRST)
        dispatch_mode<MODE_FIRST, STATS>(p, cert, prop, block, s);
    else if (mode == MODE_BARY)
        dispatch_mode<MODE_BARY, STATS>(p, cert, prop, block, s);
    else if (cert)  // count mode has no proposal order
        p.nodes4 ? launch_pass1<MODE_COUNT, true, STATS, false, true>(p, block, s)
                 : launch_pass1<MODE_COUNT, true, STATS, false, false>(p, block, s);
    else
        p.nodes4 ? launch_pass1<MODE_COUNT, false, STATS, false, true>(p, block, s)
                 : launch_pass1<MODE_COUNT, false, STATS, false, false>(p, block, s);
}

TravParams make_params(const MeshDev &m, const TraverseArgs &a) {
    TravParams p;
    p.nodes = m.nodes;
    // the 4-wide tree for one mesh unless binary nodes are asked for: the
    // mesh's own in the plain order, the proposal's (frontier nodes start
    // 4-wide nodes) in the proposal order
    const bool wide = m.node_width == 4 && a.node_width != 2 && (a.items == nullptr || a.mesh_root4 != nullptr);
    if (wide && a.bucket == nullptr) {
        p.nodes4 = m.nodes4;
        p.top4 = m.top4;
    } else if (wide && m.prop.top4 != nullptr) {
        p.nodes4 = m.prop.top4 + kTopSlots;
        p.top4 = m.prop.top4;
    } else {
        p.nodes4 = nullptr;
        p.top4 = nullptr;
    }
    p.top_lds = 0;
    p.bary_after = (a.mode == MODE_BARY && a.certified && a.items == nullptr && a.uvt != nullptr) ? 1 : 0;
    p.tris = m.tris;
    p.V = m.V;
    p.F = m.F;
    p.bounds = m.bounds;
    p.nv = m.nv;
    p.nt = m.nt;
    p.root = m.root;
    p.from = a.from;
    p.to = a.to;
    p.n = a.n;
    p.out = Outs{a.hit, a.tri_id, a.uvt, a.count};
    p.stack_depth = a.stack;
    p.waves_per_cu = a.waves_per_cu > 0 ? a.waves_per_cu : kDefaultWavesPerCU;
    p.queue = a.queue;
    p.queue_len = a.queue_len;
    p.next_ray = a.queue_len + 1;
    p.counters = reinterpret_cast<unsigned long long *>(a.counters);
    p.visits = a.visits;
    p.tests = a.tests;
    p.bucket = a.bucket;
    p.bucket_ref = p.nodes4 && a.bucket ? m.prop.bucket_ref4 : a.bucket_ref;
    p.items = a.items;
    p.n_items = a.n_items;
    p.group_start = a.items ? a.group_start : nullptr;
    p.n_groups = p.group_start ? a.n_groups : 0;
    p.n_meshes = a.n_meshes;
    p.mesh_root = a.mesh_root;
    p.mesh_root4 = p.nodes4 ? a.mesh_root4 : nullptr;
    p.top4g = p.nodes4 && a.items ? a.top4g : nullptr;
    p.roots4g = p.top4g ? a.roots4g : nullptr;
    p.top_group = 0;
    p.mesh_toff = a.mesh_toff;
    p.ray_off = a.ray_off;
    p.order = nullptr;
    p.stage_ok = (reinterpret_cast<uintptr_t>(a.hit) & 3u) == 0 ? 1 : 0;
    p.deep_cap = kDeepStack;
    p.wave_cap = a.mode == MODE_COUNT ? kWaveCap<MODE_COUNT> : kWaveCap<MODE_BOOL>;
    // RSI_DEBUG_PASS2_STACK=k (2..kDeepStack) shrinks both second-pass stacks
    // to k entries, so tests reach the leaf-span path that a tree deeper than
    // the stacks takes; results do not change
    if (const char *env = getenv("RSI_DEBUG_PASS2_STACK")) {
        const int k = atoi(env);
        if (k >= 2 && k <= kDeepStack) {
            p.deep_cap = k;
            p.wave_cap = k;
        }
    }
    return p;
}

// Keys and a stable sort of the segment indices; p.order then lists them.
hipError_t order_segments(const TraverseArgs &a, TravParams &p, hipStream_t s) {
    if (a.ray_sort == 0 || a.n < 2)
        return hipSuccess;
    uint32_t *keys = static_cast<uint32_t *>(a.sort_ws);
    int32_t *ids = reinterpret_cast<int32_t *>(keys + ((a.n + 63) & ~int64_t(63)));
    void *tmp = ids + ((a.n + 63) & ~int64_t(63));
    k_ray_keys<<<(int)((a.n + 255) / 256), 256, 0, s>>>(a.from, a.to, a.n, a.ray_sort, a.key_bounds, a.ray_off,
                                                       a.n_meshes, keys, ids);
    const hipError_t e = sort_u32_pairs(keys, ids, tmp, a.n, s);
    p.order = ids;
    return e;
}

}  // namespace

size_t ray_sort_ws_bytes(int64_t n) {
    const int64_t padded = (n + 63) & ~int64_t(63);
    return 8 * (size_t)padded + sort_u32_tmp_bytes(n) + 256;
}

hipError_t launch_intersect(const MeshDev &m, const TraverseArgs &a, hipStream_t s) {
    TravParams p = make_params(m, a);
    k_reset<<<1, 64, 0, s>>>(a.queue_len, p.counters, p.group_start ? p.n_groups : 0);
    if (a.n == 0)
        return hipGetLastError();
    if (m.nt == 0) {
        k_fill_miss<<<(int)((a.n + 255) / 256), 256, 0, s>>>(p.out, a.n, a.mode);
        return hipGetLastError();
    }
    const hipError_t e = order_segments(a, p, s);
    if (e != hipSuccess)
        return e;
    dispatch_pass1<false>(p, a.mode, a.certified != 0, a.block, s);
    // enough blocks for one per segment of a short queue; a long queue is
    // taken 64 segments per block (count mode: a wave per segment, with
    // small blocks that fit many per CU)
    const int64_t cap2 = a.mode == MODE_COUNT ? 8192 : 2048;
    const int grid2 = (int)(a.n < cap2 ? a.n : cap2);
    if (a.mode == MODE_BOOL)
        a.certified ? k_finish<MODE_BOOL, true><<<grid2, kFinishThreads, 0, s>>>(p) : k_finish<MODE_BOOL, false><<<grid2, kFinishThreads, 0, s>>>(p);
    else if (a.mode == MODE_FIRST)
        a.certified ? k_finish<MODE_FIRST, true><<<grid2, kFinishThreads, 0, s>>>(p) : k_finish<MODE_FIRST, false><<<grid2, kFinishThreads, 0, s>>>(p);
    else if (a.mode == MODE_BARY)
        a.certified ? k_finish<MODE_BARY, true><<<grid2, kFinishThreads, 0, s>>>(p) : k_finish<MODE_BARY, false><<<grid2, kFinishThreads, 0, s>>>(p);
    else
        a.certified ? k_finish<MODE_COUNT, true><<<grid2, kFinishThreads, 0, s>>>(p) : k_finish<MODE_COUNT, false><<<grid2, kFinishThreads, 0, s>>>(p);
    if (p.bary_after)
        k_bary64<<<(int)((a.n + 255) / 256), 256, 0, s>>>(a.from, a.to, m.V, m.F, a.tri_id, a.uvt, a.n);
    return hipGetLastError();
}

namespace {
// Diagnostics of the certified test on given pairs: the same ray and triangle
// set-up as the traversal, then the binary32 quantities, their bounds and the
// classification.  vals[i] = det, U, W, T, B(det), B(U), B(W), B(T), tlo, thi.
__global__ void k_debug_certify(const float *__restrict__ from, const float *__restrict__ to,
                                const float *__restrict__ corners, int64_t n, float *__restrict__ vals,
                                int32_t *__restrict__ cls) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    Ray r;
    r.o = make_float3(from[3 * i], from[3 * i + 1], from[3 * i + 2]);
    r.d = make_float3(to[3 * i] - r.o.x, to[3 * i + 1] - r.o.y, to[3 * i + 2] - r.o.z);
    const float *c = corners + 9 * i;
    Tri tri;
    tri.a = make_float4(c[0], c[1], c[2], 0.0f);
    tri.e1 = make_float4(c[3] - c[0], c[4] - c[1], c[5] - c[2], 0.0f);
    tri.e2 = make_float4(c[6] - c[0], c[7] - c[1], c[8] - c[2], 0.0f);
    const MT32 m = mt32(tri, r);
    const Bounds b = mt_bounds(m, tri, r);
    float tlo = NAN, thi = NAN;
    cls[i] = classify(m, tri, r, tlo, thi);
    float *v = vals + 10 * i;
    v[0] = m.det; v[1] = m.U; v[2] = m.W; v[3] = m.T;
    v[4] = b.d; v[5] = b.U; v[6] = b.W; v[7] = b.T;
    v[8] = tlo; v[9] = thi;
}
}  // namespace

hipError_t launch_debug_certify(const float *from, const float *to, const float *corners, int64_t n, float *vals,
                                int32_t *cls, hipStream_t s) {
    if (n > 0)
        k_debug_certify<<<(int)((n + 255) / 256), 256, 0, s>>>(from, to, corners, n, vals, cls);
    return hipGetLastError();
}

hipError_t launch_stats(const MeshDev &m, const TraverseArgs &a, hipStream_t s) {
    TravParams p = make_params(m, a);
    k_reset<<<1, 64, 0, s>>>(a.queue_len, p.counters, p.group_start ? p.n_groups : 0);
    if (m.nt == 0 || a.n == 0)
        return hipGetLastError();
    const hipError_t e = order_segments(a, p, s);
    if (e != hipSuccess)
        return e;
    dispatch_pass1<true>(p, a.mode, a.certified != 0, a.block, s);
    return hipGetLastError();
}

}  // namespace rsi
