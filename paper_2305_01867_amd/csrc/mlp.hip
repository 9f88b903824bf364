// mlp.hip -- the learned subtree proposal: a small MLP that predicts, per
// segment, which depth-8 subtree of the BVH holds its first hit, so the
// traversal can visit that subtree first and stop early on a sure hit.  The
// exact traversal still decides every result; the proposal only changes the
// order of work.
//
// Network: 6 endpoint coordinates normalised to [-1, 1] over the mesh box,
// plus sin / cos (pi f_k x) for 16 bands f_k = 2^(k/2) per coordinate
// (198 features, padded to 224), three hidden layers of 256 with ReLU, 256
// logits (one per frontier bucket; unused buckets masked).  bf16 weights and
// activations, fp32 accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16);
// fp32 master weights and Adam for training.
//
// MFMA 16x16x32 bf16 operand layout on a wave of 64 lanes (lane l):
//   A (16 x 32): row l % 16, k = 8 (l / 16) + j, j = 0..7
//   B (32 x 16): col l % 16, k = 8 (l / 16) + j
//   D (16 x 16): row 4 (l / 16) + i, col l % 16, i = 0..3
#include "rsi_internal.h"

namespace rsi {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// -------------------------------------------------------------- features
// Feature j of one segment (j < kMlpIn; zero past kMlpFeat).  Coordinates are
// normalised as n = (p - lo) / (hi - lo) (0 on a flat axis), x = 2 n - 1; the
// band frequencies are the float32 values 2^(k/2).
__device__ __forceinline__ float band_freq(int k) {
    return ldexpf((k & 1) ? 1.41421354f : 1.0f, k >> 1);
}

__device__ __forceinline__ float norm_coord(float p, float lo, float hi) {
#pragma clang fp contract(off)
    const float ext = hi - lo;
    const float n = ext > 0.0f ? (p - lo) / ext : 0.0f;
    return n * 2.0f - 1.0f;
}

// sin(pi a) and cos(pi a): the hardware sine / cosine take their argument in
// turns, so a / 2 is reduced exactly to [-1/2, 1/2] first.  The features are
// rounded to bf16 (8 bits), far coarser than the instruction's error.
__device__ __forceinline__ void sincospi_fast(float a, float &sn, float &cs) {
    float t = 0.5f * a;
    t = t - rintf(t);
    sn = __builtin_amdgcn_sinf(t);
    cs = __builtin_amdgcn_cosf(t);
}

// Writes the 33 features that depend on coordinate c (its value, then
// sin / cos of the 16 bands) into row[].
__device__ __forceinline__ void coord_features(float x, int c, __bf16 *row) {
#pragma clang fp contract(off)
    row[c] = (__bf16)x;
    for (int k = 0; k < kMlpBands; ++k) {
        const float a = band_freq(k) * x;
        float sn, cs;
        sincospi_fast(a, sn, cs);
        row[6 + c * 2 * kMlpBands + 2 * k] = (__bf16)sn;
        row[6 + c * 2 * kMlpBands + 2 * k + 1] = (__bf16)cs;
    }
}

__device__ __forceinline__ float seg_coord(const float *__restrict__ from, const float *__restrict__ to, int64_t i,
                                           int c) {
    return c < 3 ? from[3 * i + c] : to[3 * i + c - 3];
}

// X[r][0..kMlpIn) for rows [0, rows): segment index = ids ? ids[r0 + r] : r0 + r.
__global__ __launch_bounds__(256) void k_features(const float *__restrict__ from, const float *__restrict__ to,
                                                  const int32_t *__restrict__ ids, int64_t r0, int64_t rows,
                                                  const float *__restrict__ bounds, __bf16 *__restrict__ X) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = t / 7;
    const int part = (int)(t % 7);
    if (r >= rows)
        return;
    __bf16 *row = X + r * kMlpIn;
    if (part == 6) {
        for (int j = kMlpFeat; j < kMlpIn; ++j)
            row[j] = (__bf16)0.0f;
        return;
    }
    const int64_t seg = ids ? ids[r0 + r] : r0 + r;
    const int c = part;
    const float x = norm_coord(seg_coord(from, to, seg, c), bounds[c % 3], bounds[3 + c % 3]);
    coord_features(x, c, row);
}

// ------------------------------------------------- weight gradients
// dW_l[n][k] = sum_r dZ_l[r][n] H_l[r][k] for the four layers in one launch:
// workgroup z covers layer z / chunks over rows [c k_chunk, (c + 1) k_chunk)
// of chunk c = z % chunks and a 128 x 128 tile of (n, k); four waves of
// 64 x 64.  Both operands are the training pass's column-major arrays,
// contiguous along r, staged through LDS kDStage rows at a time (the next
// stage loads into registers while the current one multiplies); the sum over
// r runs in r order.  A split writes raw partial sums [chunk][256][K_l],
// added in chunk order by k_grad_finish; one chunk writes the gradient.
constexpr int kSplitMax = 16;    // row chunks of the weight gradients at most
constexpr int kSplitRows = 256;  // rows per chunk (a multiple of kDStage)
constexpr int kDT = 128, kDStage = 128, kDPitch = kDStage + 8;
constexpr size_t kDwLds = 2 * (size_t)kDT * kDPitch * sizeof(__bf16);

struct DwArgs {
    const __bf16 *A[4];  // dZ_l, [256][ld]
    const __bf16 *B[4];  // the layer's input, [K_l][ld]
    float *out[4];       // [chunks][256][K_l] partial sums, or the gradient (one chunk)
    int64_t ld;
    int k_chunk, chunks;
};

// rows [m0, m0 + 128) x r [r0, r0 + kDStage) of a [rows][ld] operand, 8 16-byte loads per lane
__device__ __forceinline__ void dw_load(const __bf16 *__restrict__ P, int rows, int64_t ld, int m0, int r0, int rend,
                                        int tid, bf16x8 (&v)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int idx = tid + 256 * q, m = idx >> 4, c = 8 * (idx & 15);
        if (m0 + m < rows && r0 + c < rend)
            v[q] = *reinterpret_cast<const bf16x8 *>(P + (int64_t)(m0 + m) * ld + r0 + c);
        else
            v[q] = bf16x8{};
    }
}

__device__ __forceinline__ void dw_store(__bf16 *S, int tid, const bf16x8 (&v)[8]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int idx = tid + 256 * q;
        *reinterpret_cast<bf16x8 *>(S + (idx >> 4) * kDPitch + 8 * (idx & 15)) = v[q];
    }
}

__global__ __launch_bounds__(256) void k_dw(DwArgs d) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __bf16 *As = reinterpret_cast<__bf16 *>(lds_raw);  // [kDT][kDPitch]: n x r
    __bf16 *Bs = As + kDT * kDPitch;                    // [kDT][kDPitch]: k x r
    const int layer = blockIdx.z / d.chunks, chunk = blockIdx.z % d.chunks;
    const int N = kMlpOut, K = layer == 0 ? kMlpIn : kMlpHidden;
    const int n0 = blockIdx.y * kDT, k0 = blockIdx.x * kDT;
    if (k0 >= K)
        return;  // layer 1 has fewer inputs; uniform per workgroup
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wn = (wave >> 1) * 64, wk = (wave & 1) * 64;
    const int rb = chunk * d.k_chunk;
    const int re = min((int)d.ld, rb + d.k_chunk);
    const __bf16 *A = d.A[layer], *B = d.B[layer];
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
            acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    bf16x8 va[8], vb[8];
    dw_load(A, N, d.ld, n0, rb, re, tid, va);
    dw_load(B, K, d.ld, k0, rb, re, tid, vb);
    const int kq = 8 * (lane >> 4);
    for (int r0 = rb; r0 < re; r0 += kDStage) {
        __syncthreads();  // the previous stage's reads are done
        dw_store(As, tid, va);
        dw_store(Bs, tid, vb);
        __syncthreads();
        if (r0 + kDStage < re) {
            dw_load(A, N, d.ld, n0, r0 + kDStage, re, tid, va);
            dw_load(B, K, d.ld, k0, r0 + kDStage, re, tid, vb);
        }
        const int steps = min(kDStage, re - r0) / 32;
        for (int j = 0; j < steps; ++j) {
            bf16x8 fa[4], fb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
                fa[a] = *reinterpret_cast<const bf16x8 *>(As + (wn + 16 * a + (lane & 15)) * kDPitch + 32 * j + kq);
#pragma unroll
            for (int b = 0; b < 4; ++b)
                fb[b] = *reinterpret_cast<const bf16x8 *>(Bs + (wk + 16 * b + (lane & 15)) * kDPitch + 32 * j + kq);
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = mfma16(fa[a], fb[b], acc[a][b]);
        }
    }
    float *out = d.out[layer] + (int64_t)chunk * N * K;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int n = n0 + wn + 16 * a + 4 * (lane >> 4) + i;
                const int k = k0 + wk + 16 * b + (lane & 15);
                if (n < N && k < K)
                    out[(int64_t)n * K + k] = acc[a][b][i];
            }
}

// Uniform(-a, a) initial weights from a counter-based hash (seed, index).
__device__ __forceinline__ uint32_t mix32(uint64_t x) {
    x ^= x >> 33;
    x *= 0xff51afd7ed558ccdull;
    x ^= x >> 33;
    x *= 0xc4ceb9fe1a85ec53ull;
    x ^= x >> 33;
    return (uint32_t)x;
}

// The bf16 weights are kept in MFMA fragment order: a layer with K inputs is
// a sequence of 16-column x 32-k blocks (column tile major, then k step),
// each 1 KB block laid out as the B operand's lanes take it (lane l: column
// l % 16, k = 8 (l / 16) .. + 7), so one wave-wide 16-byte load reads one
// whole block, eight full cache lines.
__host__ __device__ constexpr int64_t frag_index(int col, int k, int K) {
    return ((((int64_t)(col >> 4) * (K >> 5) + (k >> 5)) * 64 + (col & 15) + 16 * ((k & 31) >> 3)) << 3) + (k & 7);
}

// bf16 copies of weight i (layer l's W[out][in]): Wb in fragment order with
// columns = outputs (the forward product), and for layers 2..4 WbT in
// fragment order with columns = inputs (the backward product)
__device__ __forceinline__ void store_weight(__bf16 *__restrict__ Wb, __bf16 *__restrict__ WbT, int64_t i, float w) {
    const __bf16 h = (__bf16)w;
    const int64_t first = (int64_t)kMlpOut * kMlpIn, hh = (int64_t)kMlpHidden * kMlpHidden;
    if (i < first) {
        Wb[frag_index((int)(i / kMlpIn), (int)(i % kMlpIn), kMlpIn)] = h;
    } else {
        const int64_t l = (i - first) / hh, j = (i - first) % hh;
        const int o = (int)(j / kMlpHidden), in = (int)(j % kMlpHidden);
        Wb[first + l * hh + frag_index(o, in, kMlpHidden)] = h;
        WbT[l * hh + frag_index(in, o, kMlpHidden)] = h;
    }
}

__global__ __launch_bounds__(256) void k_init_params(float *__restrict__ P, __bf16 *__restrict__ Wb,
                                                     __bf16 *__restrict__ WbT, float *__restrict__ m1,
                                                     float *__restrict__ m2, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpParams)
        return;
    float w = 0.0f;
    if (i < kMlpWeights) {
        const int fan_in = i < (int64_t)kMlpOut * kMlpIn ? kMlpFeat : kMlpHidden;
        const float a = sqrtf(6.0f / (float)fan_in);
        const float u = (mix32(seed * 0x9e3779b97f4a7c15ull + (uint64_t)i) >> 8) * 0x1p-24f;
        w = (2.0f * u - 1.0f) * a;
        if (i < (int64_t)kMlpOut * kMlpIn && (i % kMlpIn) >= kMlpFeat)
            w = 0.0f;  // padding features carry no weight
        store_weight(Wb, WbT, i, w);
    }
    P[i] = w;
    m1[i] = 0.0f;
    m2[i] = 0.0f;
}

// ------------------------------------------------ fused inference kernel
// 96 segments per tile; four waves, wave w producing output columns
// [64 w, 64 w + 64) of every layer for all 96 rows (24 MFMA per k step, so
// each weight fragment fetched from L2 feeds 6 row tiles).  Activations stay
// in LDS in one bf16 buffer that each layer overwrites once every wave has
// read it (54 KB with the argmax scratch: two workgroups per CU, 246 VGPRs
// and two waves per SIMD; 112 or 128 rows spill).  Weight fragments load two
// k steps ahead of the multiplies that use them (measured at the paper's
// scale: 64 rows with two buffers and a one-step register copy 11.0 ms per
// 1e7 segments, this layout 7.6 ms; eight waves of 32 columns each, at four
// waves per SIMD, are no faster).  The accumulation order over k is
// the one k_gemm uses, so the logits are bit-identical to the training
// forward pass.
constexpr int kPRows = 96;
constexpr int kPPitch = kMlpHidden + 8;
constexpr int kPRowTiles = kPRows / 16;
constexpr int kPWaves = 4;                          // waves per workgroup, each owning a column slice
constexpr int kPThreads = 64 * kPWaves;
constexpr int kPColTiles = kMlpHidden / 16 / kPWaves;  // 16-column tiles per wave
constexpr int kPAhead = 2;                          // k steps the weight loads run ahead (1: 8.0 ms, 2: 7.6, 3: 7.6, 4: 7.7)

template <int RT>
__device__ __forceinline__ void tile_step(const __bf16 *__restrict__ xrow, int k0, const bf16x8 (&fb)[kPColTiles],
                                          f32x4 (&acc)[RT][kPColTiles]) {
#pragma unroll
    for (int a = 0; a < RT; ++a) {
        const bf16x8 fa = *reinterpret_cast<const bf16x8 *>(xrow + 16 * a * kPPitch + k0);
#pragma unroll
        for (int b = 0; b < kPColTiles; ++b)
            acc[a][b] = mfma16(fa, fb[b], acc[a][b]);
    }
}

// K (224 or 256) is known at compile time and the k loop fully unrolled, so
// every step's weight fragments are registers of their own: step st + kPAhead's
// loads are issued before step st multiplies and stay in flight across it,
// with no register copy that would wait for them.
// RT row tiles of 16 (activations in LDS at pitch kPPitch), the wave's
// kPColTiles column tiles, weight loads AHEAD k steps early.
template <int K, int RT = kPRowTiles, int AHEAD = kPAhead>
__device__ __forceinline__ void layer_tile(const __bf16 *__restrict__ Xin, const __bf16 *__restrict__ Wt, int wave,
                                           int lane, f32x4 (&acc)[RT][kPColTiles]) {
    static_assert(K % 32 == 0, "K must be a multiple of 32");
    constexpr int kSteps = K / 32;
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int b = 0; b < kPColTiles; ++b)
            acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int kq = 8 * (lane >> 4);
    // the wave's first column tile, this lane's 16 bytes of each block
    const __bf16 *wfrag = Wt + (int64_t)kPColTiles * wave * kSteps * 512 + 8 * lane;
    const __bf16 *xrow = Xin + (lane & 15) * kPPitch + kq;
    bf16x8 f[kSteps][kPColTiles];
#pragma unroll
    for (int st = 0; st < AHEAD && st < kSteps; ++st)
#pragma unroll
        for (int b = 0; b < kPColTiles; ++b)
            f[st][b] = *reinterpret_cast<const bf16x8 *>(wfrag + (int64_t)(b * kSteps + st) * 512);
#pragma unroll
    for (int st = 0; st < kSteps; ++st) {
        if (st + AHEAD < kSteps)
#pragma unroll
            for (int b = 0; b < kPColTiles; ++b)
                f[st + AHEAD][b] = *reinterpret_cast<const bf16x8 *>(wfrag + (int64_t)(b * kSteps + st + AHEAD) * 512);
        tile_step<RT>(xrow, 32 * st, f[st], acc);
        __builtin_amdgcn_sched_barrier(0);  // keep each step's loads in its step: no hoisting past the register budget
    }
}

// layer_tile for a chain of layers: the first AHEAD k steps' fragments come
// in pf, and the last AHEAD steps load the next layer's first AHEAD steps
// (from Wn, with KN inputs; none when Wn is NULL) into pf, so a layer starts
// without waiting on memory and the epilogue between two layers hides the
// loads' latency.
template <int KN, int AHEAD>
__device__ __forceinline__ void prefetch_layer(const __bf16 *__restrict__ Wn, int wave, int lane,
                                               bf16x8 (&pf)[AHEAD][kPColTiles]) {
    constexpr int kStepsN = KN / 32;
    const __bf16 *nfrag = Wn + (int64_t)kPColTiles * wave * kStepsN * 512 + 8 * lane;
#pragma unroll
    for (int st = 0; st < AHEAD; ++st)
#pragma unroll
        for (int b = 0; b < kPColTiles; ++b)
            pf[st][b] = *reinterpret_cast<const bf16x8 *>(nfrag + (int64_t)(b * kStepsN + st) * 512);
}

template <int K, int KN, int RT, int AHEAD>
__device__ __forceinline__ void layer_chain(const __bf16 *__restrict__ Xin, const __bf16 *__restrict__ Wt,
                                            const __bf16 *__restrict__ Wn, int wave, int lane,
                                            f32x4 (&acc)[RT][kPColTiles], bf16x8 (&pf)[AHEAD][kPColTiles]) {
    constexpr int kSteps = K / 32, kStepsN = KN / 32;
    static_assert(K % 32 == 0 && KN % 32 == 0 && AHEAD <= kSteps && AHEAD <= kStepsN, "whole k steps");
#pragma unroll
    for (int a = 0; a < RT; ++a)
#pragma unroll
        for (int b = 0; b < kPColTiles; ++b)
            acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    const int kq = 8 * (lane >> 4);
    const __bf16 *wfrag = Wt + (int64_t)kPColTiles * wave * kSteps * 512 + 8 * lane;
    const __bf16 *nfrag = Wn ? Wn + (int64_t)kPColTiles * wave * kStepsN * 512 + 8 * lane : nullptr;
    const __bf16 *xrow = Xin + (lane & 15) * kPPitch + kq;
    bf16x8 f[kSteps][kPColTiles];
#pragma unroll
    for (int st = 0; st < AHEAD; ++st)
#pragma unroll
        for (int b = 0; b < kPColTiles; ++b)
            f[st][b] = pf[st][b];
#pragma unroll
    for (int st = 0; st < kSteps; ++st) {
        if (st + AHEAD < kSteps) {
#pragma unroll
            for (int b = 0; b < kPColTiles; ++b)
                f[st + AHEAD][b] = *reinterpret_cast<const bf16x8 *>(wfrag + (int64_t)(b * kSteps + st + AHEAD) * 512);
        } else if (nfrag) {
#pragma unroll
            for (int b = 0; b < kPColTiles; ++b)
                pf[st + AHEAD - kSteps][b] =
                    *reinterpret_cast<const bf16x8 *>(nfrag + (int64_t)(b * kStepsN + st + AHEAD - kSteps) * 512);
        }
        tile_step<RT>(xrow, 32 * st, f[st], acc);
        __builtin_amdgcn_sched_barrier(0);
    }
}

__global__ __launch_bounds__(kPThreads) __attribute__((amdgpu_waves_per_eu(kPWaves / 2))) void k_mlp_propose(const float *__restrict__ from, const float *__restrict__ to,
                                                     int64_t n, const float *__restrict__ bounds,
                                                     const __bf16 *__restrict__ Wb, const float *__restrict__ P,
                                                     int nb, uint8_t *__restrict__ bucket) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __bf16 *X = reinterpret_cast<__bf16 *>(lds_raw);  // activations, overwritten layer by layer
    float *best_v = reinterpret_cast<float *>(X + kPRows * kPPitch);  // [kPWaves][kPRows]
    int *best_i = reinterpret_cast<int *>(best_v + kPWaves * kPRows);  // [kPWaves][kPRows]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float *bias = P + kMlpWeights;
    const int64_t tiles = (n + kPRows - 1) / kPRows;
#pragma unroll 1
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t r0 = tile * kPRows;
        // features -> X (pitch kPPitch)
#pragma unroll 1
        for (int q = tid; q < kPRows * 7; q += kPThreads) {
            const int r = q / 7, part = q % 7;
            __bf16 *row = X + r * kPPitch;
            if (part == 6) {
                for (int j = kMlpFeat; j < kMlpIn; ++j)
                    row[j] = (__bf16)0.0f;
                continue;
            }
            const int64_t seg = r0 + r < n ? r0 + r : n - 1;
            const float x = norm_coord(seg_coord(from, to, seg, part), bounds[part % 3], bounds[3 + part % 3]);
            coord_features(x, part, row);
        }
        __syncthreads();
        // the four layers through one call site, so the accumulators keep one
        // register set; a layer's outputs go over its inputs in X once every
        // wave has read them
        f32x4 acc[kPRowTiles][kPColTiles];
#pragma unroll 1
        for (int l = 0; l < 4; ++l) {
            const __bf16 *in = X;
            __bf16 *out = X;
            const int64_t woff = l == 0 ? 0 : (int64_t)kMlpOut * kMlpIn + (int64_t)(l - 1) * kMlpHidden * kMlpHidden;
            if (l == 0)
                layer_tile<kMlpIn>(in, Wb + woff, wave, lane, acc);
            else
                layer_tile<kMlpHidden>(in, Wb + woff, wave, lane, acc);
            if (l == 3)
                break;
            const float *bl = bias + l * kMlpHidden;
            __syncthreads();  // every wave has read `in` before it is overwritten
#pragma unroll
            for (int b = 0; b < kPColTiles; ++b) {
                const int col = 16 * kPColTiles * wave + 16 * b + (lane & 15);
                const float bv = bl[col];
#pragma unroll
                for (int a = 0; a < kPRowTiles; ++a)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int row = 16 * a + 4 * (lane >> 4) + i;
                        out[row * kPPitch + col] = (__bf16)fmaxf(acc[a][b][i] + bv, 0.0f);
                    }
            }
            __syncthreads();
        }
        const float *b4 = bias + 3 * kMlpHidden;
        float b4v[kPColTiles];
#pragma unroll
        for (int b = 0; b < kPColTiles; ++b)
            b4v[b] = b4[16 * kPColTiles * wave + 16 * b + (lane & 15)];
        // argmax over valid buckets (smallest index on ties)
#pragma unroll
        for (int a = 0; a < kPRowTiles; ++a)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float bv = -INFINITY;
                int bi = INT32_MAX;
#pragma unroll
                for (int b = 0; b < kPColTiles; ++b) {
                    const int col = 16 * kPColTiles * wave + 16 * b + (lane & 15);
                    const float v = acc[a][b][i] + b4v[b];
                    if (col < nb && (v > bv || (v == bv && col < bi))) {
                        bv = v;
                        bi = col;
                    }
                }
#pragma unroll
                for (int off = 1; off < 16; off <<= 1) {
                    const float ov = __shfl_xor(bv, off);
                    const int oi = __shfl_xor(bi, off);
                    if (ov > bv || (ov == bv && oi < bi)) {
                        bv = ov;
                        bi = oi;
                    }
                }
                if ((lane & 15) == 0) {
                    const int row = 16 * a + 4 * (lane >> 4) + i;
                    best_v[wave * kPRows + row] = bv;
                    best_i[wave * kPRows + row] = bi;
                }
            }
        __syncthreads();
        if (tid < kPRows && r0 + tid < n) {
            float bv = best_v[tid];
            int bi = best_i[tid];
            for (int w = 1; w < kPWaves; ++w) {
                const float v = best_v[w * kPRows + tid];
                const int i2 = best_i[w * kPRows + tid];
                if (v > bv || (v == bv && i2 < bi)) {
                    bv = v;
                    bi = i2;
                }
            }
            bucket[r0 + tid] = (uint8_t)(bi >= 0 && bi < nb ? bi : 0);
        }
        __syncthreads();
    }
}

constexpr size_t kProposeLds = (size_t)kPRows * kPPitch * sizeof(__bf16) + 2 * kPWaves * (size_t)kPRows * 4;

// ------------------------------------------------ fused training pass
// One workgroup per kTRows rows of a batch: the features, the four layers
// forward, softmax cross-entropy and the chain of input gradients back to
// the first layer, with the activations and gradients of the tile in LDS and
// written out (bf16, column-major) for the weight gradients.  The layer
// products run through layer_tile, the inference kernel's, so the logits
// equal those of k_mlp_propose bit for bit.  A workgroup
// also writes the column sums of each layer's gradient over its rows (the
// bias gradients, added over the tiles in order by k_grad_finish) and the sum
// of its rows' losses.  The backward products read the transposed copy of
// the hidden weights, so both directions load 16 contiguous bytes per lane.
constexpr int kTRows = 32;
constexpr int kTRowTiles = kTRows / 16;
constexpr int kTAhead = 4;
static_assert(kTRows % 16 == 0 && kTRows <= 64, "whole row tiles; the loss sum reads one row per lane");

struct TrainArgs {
    const float *from, *to;
    const int32_t *seg;  // segment of batch row r0 + r (NULL: the segment is r0 + r)
    const int32_t *lab;  // label of batch row r0 + r
    int64_t r0;
    int rows, nb;
    const float *bounds;
    const __bf16 *Wb;    // [out][in] per layer
    const __bf16 *WbT;   // layers 2..4 transposed, [in][out]
    const float *bias;   // [4][256]
    int64_t ld;          // rows rounded up to whole tiles: the row stride of the arrays below
    __bf16 *X0;          // [224][ld]: the features, column-major
    __bf16 *H;           // [3][256][ld]: the hidden activations, column-major
    __bf16 *dZ;          // [4][256][ld]: gradients of the pre-activations, column-major
    float *logits;       // [rows][256], or NULL
    float *bias_part;    // [tiles][4][256]
    float *loss_part;    // [tiles]
    float inv_rows, loss_scale;
};

// LDS: the activations (the logits later take their place and more), the
// gradients, the ReLU masks as wave ballots in the MFMA output layout, and
// the per-wave column sums and row losses of the softmax.
constexpr int kTMaskWords = kTRowTiles * kPColTiles * 4 * 4;  // (row tile, col tile, i, wave) per layer
constexpr size_t kTActBytes = (size_t)kTRows * kPPitch * sizeof(__bf16);
constexpr int kLPitch = kMlpOut + 16;  // logits row pitch (floats): four rows on disjoint LDS banks
constexpr size_t kTLogitBytes = (size_t)kTRows * kLPitch * sizeof(float);
static_assert(kTLogitBytes >= kTActBytes, "the logits take the activations' place");
constexpr size_t kTrainLds = kTLogitBytes + kTActBytes + 3 * (size_t)kTMaskWords * sizeof(uint64_t) +
                             4 * (size_t)kMlpOut * sizeof(float) + (size_t)kTRows * sizeof(float);

// The tile's rows of an LDS array (pitch kPPitch, `cols` columns) into a
// column-major global array T[col][ld] at rows t0 .. t0 + kTRows (padding
// rows go out too: zero features, zero gradients), 16 bytes per lane, four
// lanes per column: the weight-gradient product then reads both operands
// contiguous along the rows.
__device__ __forceinline__ void copy_cols(const __bf16 *S, __bf16 *T, int64_t ld, int t0, int cols, int tid) {
    constexpr int kG = kTRows / 8;
    for (int i = tid; i < cols * kG; i += 256) {
        const int col = i / kG, g = i % kG;
        bf16x8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j)
            v[j] = S[(8 * g + j) * kPPitch + col];
        *reinterpret_cast<bf16x8 *>(T + (int64_t)col * ld + t0 + 8 * g) = v;
    }
}

// Max / sum over the 16 lanes of a DPP row, every lane ending with the same
// value: rotations by 8, 4, 2 and 1 within the row, each step adding two
// operands that are equal up to order (so every lane rounds the same sums).
__device__ __forceinline__ float dpp_ror(float v, int n) {
    switch (n) {
    case 8: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x128, 0xf, 0xf, false));
    case 4: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x124, 0xf, 0xf, false));
    case 2: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x122, 0xf, 0xf, false));
    default: return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x121, 0xf, 0xf, false));
    }
}
__device__ __forceinline__ float row16_max(float v) {
    v = fmaxf(v, dpp_ror(v, 8));
    v = fmaxf(v, dpp_ror(v, 4));
    v = fmaxf(v, dpp_ror(v, 2));
    return fmaxf(v, dpp_ror(v, 1));
}
__device__ __forceinline__ float row16_sum(float v) {
    v += dpp_ror(v, 8);
    v += dpp_ror(v, 4);
    v += dpp_ror(v, 2);
    return v + dpp_ror(v, 1);
}

__global__ __launch_bounds__(256) void k_train_tile(TrainArgs a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __bf16 *X = reinterpret_cast<__bf16 *>(lds_raw);                  // activations [kTRows][kPPitch]
    float *L = reinterpret_cast<float *>(lds_raw);                     // logits [kTRows][256], over X
    __bf16 *D = reinterpret_cast<__bf16 *>(lds_raw + kTLogitBytes);    // gradients [kTRows][kPPitch]
    uint64_t *Msk = reinterpret_cast<uint64_t *>(lds_raw + kTLogitBytes + kTActBytes);  // [3][kTMaskWords]
    float *csum = reinterpret_cast<float *>(Msk + 3 * kTMaskWords);   // [4 waves][256]
    float *rl = csum + 4 * kMlpOut;                                    // [kTRows] row losses
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tile = blockIdx.x, t0 = tile * kTRows;
    const int nrows = min(kTRows, a.rows - t0);
    // features; rows past the batch are zero
    for (int q = tid; q < kTRows * 7; q += 256) {
        const int r = q / 7, part = q % 7;
        __bf16 *row = X + r * kPPitch;
        if (part == 6) {
            for (int j = kMlpFeat; j < kMlpIn; ++j)
                row[j] = (__bf16)0.0f;
        } else if (r < nrows) {
            const int64_t br = a.r0 + t0 + r;
            const int64_t seg = a.seg ? a.seg[br] : br;
            const float x = norm_coord(seg_coord(a.from, a.to, seg, part), a.bounds[part % 3], a.bounds[3 + part % 3]);
            coord_features(x, part, row);
        } else {
            row[part] = (__bf16)0.0f;
            for (int k = 0; k < 2 * kMlpBands; ++k)
                row[6 + part * 2 * kMlpBands + k] = (__bf16)0.0f;
        }
    }
    __syncthreads();
    copy_cols(X, a.X0, a.ld, t0, kMlpIn, tid);
    // forward: each layer's output over its input in X once every wave has read it
    f32x4 acc[kTRowTiles][kPColTiles];
    bf16x8 pf[kTAhead][kPColTiles];  // the next layer's first k steps, loaded ahead
    auto wlayer = [&](int l) -> const __bf16 * {  // forward l = 0..3, then backward l = 3..1 as 4..6
        if (l == 0)
            return a.Wb;
        if (l < 4)
            return a.Wb + (int64_t)kMlpOut * kMlpIn + (int64_t)(l - 1) * kMlpHidden * kMlpHidden;
        return a.WbT + (int64_t)(6 - l) * kMlpHidden * kMlpHidden;
    };
    prefetch_layer<kMlpIn, kTAhead>(a.Wb, wave, lane, pf);
#pragma unroll 1
    for (int l = 0; l < 4; ++l) {
        const float *bl = a.bias + l * kMlpHidden;
        float bvs[kPColTiles];  // this layer's biases, loaded while it multiplies
#pragma unroll
        for (int b = 0; b < kPColTiles; ++b)
            bvs[b] = bl[16 * kPColTiles * wave + 16 * b + (lane & 15)];
        if (l == 0)
            layer_chain<kMlpIn, kMlpHidden, kTRowTiles, kTAhead>(X, wlayer(0), wlayer(1), wave, lane, acc, pf);
        else
            layer_chain<kMlpHidden, kMlpHidden, kTRowTiles, kTAhead>(X, wlayer(l), wlayer(l + 1), wave, lane, acc, pf);
        __syncthreads();
#pragma unroll
        for (int b = 0; b < kPColTiles; ++b) {
            const int col = 16 * kPColTiles * wave + 16 * b + (lane & 15);
            const float bv = bvs[b];
#pragma unroll
            for (int t = 0; t < kTRowTiles; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * t + 4 * (lane >> 4) + i;
                    const float v = acc[t][b][i] + bv;
                    if (l < 3) {
                        const __bf16 h = (__bf16)fmaxf(v, 0.0f);
                        X[row * kPPitch + col] = h;
                        // ReLU mask of the backward pass, kept in the layout its epilogue reads
                        const uint64_t m = __ballot((float)h > 0.0f);
                        if (lane == 0)
                            Msk[l * kTMaskWords + ((t * kPColTiles + b) * 4 + i) * 4 + wave] = m;
                    } else {
                        L[row * kLPitch + col] = v;
                    }
                }
        }
        __syncthreads();
        if (l < 3)
            copy_cols(X, a.H + (int64_t)l * kMlpHidden * a.ld, a.ld, t0, kMlpHidden, tid);
        else if (a.logits)
            for (int i = tid; i < nrows * kMlpOut; i += 256)
                a.logits[(int64_t)t0 * kMlpOut + i] = L[(i / kMlpOut) * kLPitch + i % kMlpOut];
    }
    // softmax cross-entropy: four rows of a wave at a time, 16 lanes (one DPP
    // row) per row, lane l16 holding columns l16 + 16 j
    const int g4 = lane >> 4, l16 = lane & 15;
    float cs[16];  // this lane's column sums of the bf16 gradient over its rows
#pragma unroll
    for (int j = 0; j < 16; ++j)
        cs[j] = 0.0f;
#pragma unroll
    for (int p = 0; p < kTRows / 16; ++p) {
        const int row = (kTRows / 4) * wave + 4 * p + g4;
        const float *z = L + row * kLPitch;
        float v[16];
        float mx = -INFINITY;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int c = l16 + 16 * j;
            v[j] = c < a.nb ? z[c] : -INFINITY;
            mx = fmaxf(mx, v[j]);
        }
        mx = row16_max(mx);
        float sum = 0.0f;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            v[j] = (l16 + 16 * j) < a.nb ? expf(v[j] - mx) : 0.0f;
            sum += v[j];
        }
        sum = row16_sum(sum);
        const bool valid = row < nrows;
        const int label = valid ? a.lab[a.r0 + t0 + row] : -1;
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int c = l16 + 16 * j;
            const float g = valid && c < a.nb ? (v[j] / sum - (c == label ? 1.0f : 0.0f)) * a.inv_rows : 0.0f;
            const __bf16 gb = (__bf16)g;
            D[row * kPPitch + c] = gb;
            cs[j] += (float)gb;
        }
        if (l16 == 0)
            rl[row] = valid && label >= 0 && label < a.nb ? (logf(sum) + mx - z[label]) * a.loss_scale : 0.0f;
    }
    // the wave's column sums: add the four lane groups
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        float x = cs[j];
        x += __shfl_xor(x, 16);
        x += __shfl_xor(x, 32);
        cs[j] = x;
    }
    if (lane < 16)
#pragma unroll
        for (int j = 0; j < 16; ++j)
            csum[wave * kMlpOut + l16 + 16 * j] = cs[j];
    __syncthreads();
    copy_cols(D, a.dZ + (int64_t)3 * kMlpOut * a.ld, a.ld, t0, kMlpOut, tid);
    a.bias_part[((int64_t)tile * 4 + 3) * kMlpOut + tid] =
        ((csum[tid] + csum[kMlpOut + tid]) + csum[2 * kMlpOut + tid]) + csum[3 * kMlpOut + tid];
    if (wave == 0) {
        float v = lane < kTRows ? rl[lane] : 0.0f;
        for (int off = 32; off > 0; off >>= 1)
            v += __shfl_xor(v, off);
        if (lane == 0)
            a.loss_part[tile] = v;
    }
    // backward: dZ(l - 1) = (dZ(l) W_l) where H_l > 0, in place in D; the
    // column sums (bias gradients) from the registers, over the lanes that
    // share a column
#pragma unroll 1
    for (int l = 3; l > 0; --l) {
        layer_chain<kMlpHidden, kMlpHidden, kTRowTiles, kTAhead>(D, wlayer(7 - l), l > 1 ? wlayer(8 - l) : nullptr,
                                                                 wave, lane, acc, pf);
        __syncthreads();
        const uint64_t *mk = Msk + (l - 1) * kTMaskWords;
#pragma unroll
        for (int b = 0; b < kPColTiles; ++b) {
            const int col = 16 * kPColTiles * wave + 16 * b + (lane & 15);
            float colsum = 0.0f;
#pragma unroll
            for (int t = 0; t < kTRowTiles; ++t)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int row = 16 * t + 4 * (lane >> 4) + i;
                    const bool on = (mk[((t * kPColTiles + b) * 4 + i) * 4 + wave] >> lane) & 1ull;
                    const __bf16 gb = (__bf16)(on ? acc[t][b][i] : 0.0f);
                    D[row * kPPitch + col] = gb;
                    colsum += (float)gb;
                }
            colsum += __shfl_xor(colsum, 16);
            colsum += __shfl_xor(colsum, 32);
            if (lane < 16)
                a.bias_part[((int64_t)tile * 4 + (l - 1)) * kMlpOut + col] = colsum;
        }
        __syncthreads();
        copy_cols(D, a.dZ + (int64_t)(l - 1) * kMlpOut * a.ld, a.ld, t0, kMlpOut, tid);
    }
}

// The gradient of every parameter: a weight's split-K partial sums added in
// chunk order (or the value already in G), a bias's tile sums added in tile
// order; the loss parts added in tile order.  With adam set, the Adam step on
// the fp32 master parameters and the bf16 copies follow.
struct FinishArgs {
    const float *split;  // [4][kSplitMax][256][256] partials, or NULL: the weight gradients are in G
    int chunks;
    const float *bias_part;
    int tiles;
    const float *loss_part;
    float *loss;
    float *G;
    int adam;
    float *P, *m1, *m2;
    __bf16 *Wb, *WbT;
    float lr, b1, b2, eps, c1, c2;
};

__global__ __launch_bounds__(256) void k_grad_finish(FinishArgs f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && f.loss) {
        float sum = 0.0f;
#pragma unroll 32
        for (int t = 0; t < f.tiles; ++t)
            sum += f.loss_part[t];
        *f.loss += sum;
    }
    if (i >= kMlpParams)
        return;
    float g;
    if (i < kMlpWeights) {
        if (f.split) {
            const int64_t first = (int64_t)kMlpOut * kMlpIn, hh = (int64_t)kMlpHidden * kMlpHidden;
            const int l = i < first ? 0 : 1 + (int)((i - first) / hh);
            const int64_t j = i < first ? i : (i - first) % hh;
            const int64_t mn = l == 0 ? first : hh;
            const float *pp = f.split + (int64_t)l * kSplitMax * kMlpOut * kMlpHidden + j;
            g = 0.0f;
#pragma unroll 4
            for (int z = 0; z < f.chunks; ++z)
                g += pp[z * mn];
        } else {
            g = f.G[i];
        }
    } else {
        const int b = (int)(i - kMlpWeights), l = b / kMlpHidden, n = b % kMlpHidden;
        g = 0.0f;
#pragma unroll 32
        for (int t = 0; t < f.tiles; ++t)
            g += f.bias_part[((int64_t)t * 4 + l) * kMlpOut + n];
    }
    f.G[i] = g;
    if (!f.adam)
        return;
    const float m = f.b1 * f.m1[i] + (1.0f - f.b1) * g;
    const float v = f.b2 * f.m2[i] + (1.0f - f.b2) * g * g;
    f.m1[i] = m;
    f.m2[i] = v;
    const float w = f.P[i] - f.lr * (m * f.c1) / (sqrtf(v * f.c2) + f.eps);
    f.P[i] = w;
    if (i < kMlpWeights)
        store_weight(f.Wb, f.WbT, i, w);
}

// ------------------------------------------------ frontier and labels
// Left-to-right frontier of the tree at depth 8: internal nodes at depth 8
// and leaves shallower than that.  One lane walks it level by level (at most
// 511 nodes); then each bucket's first sorted leaf is found by descending left.
__global__ void k_frontier(const Node *__restrict__ nodes, const int32_t *__restrict__ parent, int root, int nt,
                           int32_t *__restrict__ bucket_ref, int32_t *__restrict__ bucket_first,
                           int32_t *__restrict__ n_buckets, uint8_t *__restrict__ leaf_bucket) {
    __shared__ int cur[kMlpOut], nxt[kMlpOut];
    __shared__ int count;
    if (threadIdx.x == 0) {
        int nc = 1;
        cur[0] = root;
        for (int d = 0; d < kFrontierDepth; ++d) {
            int nn = 0;
            for (int j = 0; j < nc; ++j) {
                const int r = cur[j];
                if (r >= 0) {
                    nxt[nn++] = nodes[r].refs.x;
                    nxt[nn++] = nodes[r].refs.y;
                } else {
                    nxt[nn++] = r;
                }
            }
            for (int j = 0; j < nn; ++j)
                cur[j] = nxt[j];
            nc = nn;
        }
        count = nc;
        *n_buckets = nc;
    }
    __syncthreads();
    const int b = threadIdx.x;
    if (b < count) {
        int r = cur[b];
        bucket_ref[b] = r;
        int x = r;
        for (int guard = 0; x >= 0 && guard < nt; ++guard)  // a path has fewer than nt internal nodes
            x = nodes[x].refs.x;
        bucket_first[b] = ~x;
        // mark every leaf of the bucket's subtree: a walk without a stack (down
        // the left children, then up until a left child with an unvisited right
        // sibling), bounded by the subtree's 2 N_t node steps
        auto up = [&](int c) { return c >= 0 ? parent[c] : parent[(nt - 1) + ~c]; };
        x = r;
        for (int64_t step = 0; step < 4 * (int64_t)nt + 8; ++step) {
            while (x >= 0 && step++ < 4 * (int64_t)nt + 8)
                x = nodes[x].refs.x;
            if (x < 0 && ~x < nt)
                leaf_bucket[~x] = (uint8_t)b;
            // climb until x is a left child whose parent's right child is unvisited
            int c = x;
            bool next = false;
            while (c != r && step++ < 4 * (int64_t)nt + 8) {
                const int q = up(c);
                if (q < 0 || q >= nt - 1)
                    break;
                if (nodes[q].refs.x == c) {
                    x = nodes[q].refs.y;
                    next = true;
                    break;
                }
                c = q;
            }
            if (!next)
                break;
        }
    }
}

// rank[ids[k]] = k: sorted position of each input triangle.
__global__ void k_rank(const int32_t *__restrict__ ids, int nt, int32_t *__restrict__ rank) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nt)
        rank[ids[k]] = k;
}

// The training list: for every segment with a first hit, in segment order,
// the segment and its bucket (the frontier subtree that holds the hit leaf).
// A stable compaction -- per-workgroup counts, one scan of them, then each
// workgroup writes at its offset in order -- so the list, and the training
// that walks it batch by batch, do not depend on scheduling.
constexpr int kLabSeg = 16;                   // segments per lane
constexpr int kLabPerBlock = 256 * kLabSeg;   // per workgroup of 256

// Exclusive prefix sum of v over a 256-lane workgroup; total = the sum.
__device__ __forceinline__ int block_excl_scan(int v, int &total) {
    __shared__ int wsum[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(incl, d, 64);
        incl += lane >= d ? u : 0;
    }
    if (lane == 63)
        wsum[w] = incl;
    __syncthreads();
    int off = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        off += k < w ? wsum[k] : 0;
        total += wsum[k];
    }
    __syncthreads();  // wsum is reused by the next call
    return off + incl - v;
}

__device__ __forceinline__ int lane_hits(const int32_t *__restrict__ tri_id, int64_t n, int64_t base) {
    int c = 0;
    for (int j = 0; j < kLabSeg; ++j)
        c += base + j < n && tri_id[base + j] >= 0;
    return c;
}

__global__ __launch_bounds__(256) void k_label_count(const int32_t *__restrict__ tri_id, int64_t n,
                                                     int32_t *__restrict__ blk) {
    const int64_t base = (int64_t)blockIdx.x * kLabPerBlock + (int64_t)threadIdx.x * kLabSeg;
    int total;
    block_excl_scan(lane_hits(tri_id, n, base), total);
    if (threadIdx.x == 0)
        blk[blockIdx.x] = total;
}

// blk[b] = the list position of workgroup b's first entry; *count = the total.
__global__ __launch_bounds__(256) void k_label_scan(int32_t *__restrict__ blk, int nblk, uint32_t *__restrict__ count) {
    uint32_t carry = 0;
    for (int b0 = 0; b0 < nblk; b0 += 256) {
        const int b = b0 + threadIdx.x;
        const int v = b < nblk ? blk[b] : 0;
        int total;
        const int ex = block_excl_scan(v, total);
        if (b < nblk)
            blk[b] = (int32_t)(carry + ex);
        carry += (uint32_t)total;
    }
    if (threadIdx.x == 0)
        *count = carry;
}

__global__ __launch_bounds__(256) void k_labels(const int32_t *__restrict__ tri_id, int64_t n,
                                                const int32_t *__restrict__ rank,
                                                const uint8_t *__restrict__ leaf_bucket,
                                                const int32_t *__restrict__ blk, int32_t *__restrict__ seg_out,
                                                int32_t *__restrict__ label_out) {
    const int64_t base = (int64_t)blockIdx.x * kLabPerBlock + (int64_t)threadIdx.x * kLabSeg;
    int total;
    int pos = blk[blockIdx.x] + block_excl_scan(lane_hits(tri_id, n, base), total);
    for (int j = 0; j < kLabSeg; ++j) {
        const int64_t i = base + j;
        const int t = i < n ? tri_id[i] : -1;
        if (t >= 0) {
            seg_out[pos] = (int32_t)i;
            label_out[pos] = leaf_bucket[rank[t]];
            ++pos;
        }
    }
}

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

}  // namespace

// ===================================================================== host
hipError_t proposal_frontier(const MeshDev &m, Proposal &pr, hipStream_t s) {
    if (m.nt < 1)
        return hipErrorInvalidValue;
    k_rank<<<cdiv(m.nt, 256), 256, 0, s>>>(m.ids, (int)m.nt, pr.rank);
    k_frontier<<<1, kMlpOut, 0, s>>>(m.nodes, m.parent, m.root, (int)m.nt, pr.bucket_ref, pr.bucket_first,
                                     pr.dev_n_buckets, pr.leaf_bucket);
    return hipGetLastError();
}

hipError_t proposal_init(Proposal &pr, uint64_t seed, hipStream_t s) {
    k_init_params<<<cdiv(kMlpParams, 256), 256, 0, s>>>(pr.P, pr.Wb, pr.WbT, pr.m1, pr.m2, seed);
    return hipGetLastError();
}

size_t proposal_label_scratch(int64_t n) { return 4 * (size_t)(n / kLabPerBlock + 1); }

hipError_t proposal_labels(const MeshDev &m, Proposal &pr, const int32_t *tri_id, int64_t n, int32_t *seg,
                           int32_t *label, uint32_t *count, int32_t *blk, hipStream_t s) {
    const int nblk = (int)((n + kLabPerBlock - 1) / kLabPerBlock);
    if (nblk == 0)
        return hipSuccess;
    k_label_count<<<nblk, 256, 0, s>>>(tri_id, n, blk);
    k_label_scan<<<1, 256, 0, s>>>(blk, nblk, count);
    k_labels<<<nblk, 256, 0, s>>>(tri_id, n, pr.rank, pr.leaf_bucket, blk, seg, label);
    return hipGetLastError();
}

hipError_t proposal_predict(const MeshDev &m, const Proposal &pr, const float *from, const float *to, int64_t n,
                            int nb, uint8_t *bucket, hipStream_t s) {
    if (n == 0)
        return hipSuccess;
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t tiles = (n + kPRows - 1) / kPRows;
    const int grid = (int)(tiles < 2 * cus ? tiles : 2 * cus);
    static_assert(kProposeLds <= 64 * 1024, "the fused inference kernel fits the default dynamic LDS");
    k_mlp_propose<<<grid, kPThreads, kProposeLds, s>>>(from, to, n, m.bounds, pr.Wb, pr.P, nb, bucket);
    return hipGetLastError();
}

// Forward + backward of one batch (rows segments listed in seg[r0..r0+rows),
// labels lab[r0..]) in three launches: k_train_tile (features, forward,
// softmax cross-entropy, input gradients and bias / loss parts per tile of
// kTRows rows), k_gemm4 (every layer's weight gradient, split over the rows)
// and k_grad_finish (the sums in fixed order into pr.G, the loss, and with
// `adam` the Adam step).  ws must hold proposal_batch_scratch(rows) bytes.
hipError_t proposal_batch_grad(const MeshDev &m, Proposal &pr, const float *from, const float *to,
                               const int32_t *seg, const int32_t *lab, int64_t r0, int rows, int nb, float *loss,
                               float loss_scale, char *ws, hipStream_t s, float *logits_out, const AdamStep *adam) {
    const int tiles = cdiv(rows, kTRows);
    const int64_t ld = (int64_t)tiles * kTRows;
    __bf16 *X0 = reinterpret_cast<__bf16 *>(ws);           // [224][ld]
    __bf16 *H = X0 + ld * kMlpIn;                          // [3][256][ld]
    __bf16 *dZ0 = H + 3 * ld * kMlpHidden;                 // [4][256][ld]
    float *split = reinterpret_cast<float *>(dZ0 + 4 * ld * kMlpOut);  // [4][kSplitMax][256][256]
    float *bias_part = split + 4 * (int64_t)kSplitMax * kMlpOut * kMlpHidden;       // [tiles][4][256]
    float *loss_part = bias_part + (int64_t)tiles * 4 * kMlpOut;                   // [tiles]
    TrainArgs a{};
    a.from = from;
    a.to = to;
    a.seg = seg;
    a.lab = lab;
    a.r0 = r0;
    a.rows = rows;
    a.nb = nb;
    a.bounds = m.bounds;
    a.Wb = pr.Wb;
    a.WbT = pr.WbT;
    a.bias = pr.P + kMlpWeights;
    a.ld = ld;
    a.X0 = X0;
    a.H = H;
    a.dZ = dZ0;
    a.logits = logits_out;
    a.bias_part = bias_part;
    a.loss_part = loss_part;
    a.inv_rows = 1.0f / rows;
    a.loss_scale = loss_scale > 0.0f ? loss_scale : 1.0f / rows;
    // above the default 64 KB of dynamic LDS: set per call (cheap on the
    // host, right for whichever device is current)
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_train_tile),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTrainLds);
    if (e != hipSuccess)
        return e;
    k_train_tile<<<tiles, 256, kTrainLds, s>>>(a);
    // every layer's weight gradient in one launch, split over the rows (a
    // batch of at most kSplitRows rows is not split: its sums go straight to
    // the gradient); padding rows add exact zeros, their gradients being zero
    float *G = pr.G;
    DwArgs dw{};
    dw.ld = ld;
    dw.chunks = ld > kSplitRows ? cdiv(ld, kSplitRows) : 1;
    if (dw.chunks > kSplitMax)
        dw.chunks = kSplitMax;
    dw.k_chunk = cdiv(cdiv(ld, dw.chunks), kDStage) * kDStage;
    dw.chunks = cdiv(ld, dw.k_chunk);
    const bool split_k = dw.chunks > 1;
    for (int l = 0; l < 4; ++l) {
        const int64_t woff = l == 0 ? 0 : (int64_t)kMlpOut * kMlpIn + (int64_t)(l - 1) * kMlpHidden * kMlpHidden;
        dw.A[l] = dZ0 + (int64_t)l * kMlpOut * ld;
        dw.B[l] = l == 0 ? X0 : H + (int64_t)(l - 1) * kMlpHidden * ld;
        dw.out[l] = split_k ? split + (int64_t)l * kSplitMax * kMlpOut * kMlpHidden : G + woff;
    }
    e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_dw), hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)kDwLds);
    if (e != hipSuccess)
        return e;
    k_dw<<<dim3(cdiv(kMlpHidden, kDT), cdiv(kMlpOut, kDT), 4 * dw.chunks), 256, kDwLds, s>>>(dw);
    FinishArgs f{};
    f.split = split_k ? split : nullptr;
    f.chunks = dw.chunks;
    f.bias_part = bias_part;
    f.tiles = tiles;
    f.loss_part = loss_part;
    f.loss = loss;
    f.G = G;
    if (adam) {
        f.adam = 1;
        f.P = pr.P;
        f.m1 = pr.m1;
        f.m2 = pr.m2;
        f.Wb = pr.Wb;
        f.WbT = pr.WbT;
        f.lr = adam->lr;
        f.b1 = 0.9f;
        f.b2 = 0.999f;
        f.eps = 1e-8f;
        f.c1 = 1.0f / (1.0f - powf(f.b1, (float)adam->step));
        f.c2 = 1.0f / (1.0f - powf(f.b2, (float)adam->step));
    }
    k_grad_finish<<<cdiv(kMlpParams, 256), 256, 0, s>>>(f);
    return hipGetLastError();
}

namespace {
__global__ void k_params_to_bf16(const float *__restrict__ P, __bf16 *__restrict__ Wb, __bf16 *__restrict__ WbT) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMlpWeights)
        store_weight(Wb, WbT, i, P[i]);
}
}  // namespace

hipError_t proposal_set_params(Proposal &pr, hipStream_t s) {
    k_params_to_bf16<<<cdiv(kMlpWeights, 256), 256, 0, s>>>(pr.P, pr.Wb, pr.WbT);
    return hipGetLastError();
}

size_t proposal_batch_scratch(int rows) {
    const size_t tiles = (size_t)cdiv(rows, kTRows);
    return tiles * kTRows * (kMlpIn + 3 * kMlpHidden + 4 * kMlpOut) * 2 +
           4 * (size_t)kSplitMax * kMlpOut * kMlpHidden * 4 + tiles * 4 * kMlpOut * 4 + tiles * 4 + 256;
}

hipError_t proposal_features(const MeshDev &m, const float *from, const float *to, int64_t n, __bf16 *X,
                             hipStream_t s) {
    if (n == 0)
        return hipSuccess;
    k_features<<<cdiv(n * 7, 256), 256, 0, s>>>(from, to, nullptr, 0, n, m.bounds, X);
    return hipGetLastError();
}

}  // namespace rsi
