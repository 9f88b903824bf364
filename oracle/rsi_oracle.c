/*
 * rsi_oracle.c -- plain CPU oracle for segment/triangle-mesh intersection.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the GPU path.
 *
 * What it computes (paper: Background section, problem statement; the test is
 * the Moller-Trumbore ray/triangle test of the cited Moller & Trumbore 1997):
 *   ray i is the closed segment O_i + t (E_i - O_i), t in [0, 1];
 *   triangle j is the closed triangle (1-u-v) A + u B + v C, u, v >= 0,
 *   u + v <= 1, with A, B, C = V[F[j][0]], V[F[j][1]], V[F[j][2]].
 * Every pair is evaluated (exhaustive search, Background section), in IEEE
 * binary64 with round-to-nearest, no fused multiply-add (build flag
 * -ffp-contract=off), dot products summed left to right, and the decision made
 * without division:
 *   d = E-O, e1 = B-A, e2 = C-A, s = O-A, p = d x e2, q = s x e1,
 *   det = e1.p, U = s.p, W = d.q, T = e2.q;
 *   det == 0 -> miss (segment parallel to the plane, no epsilon);
 *   with g = sign(det): hit iff gU >= 0, gW >= 0, gU + gW <= g det,
 *   gT >= 0 and gT <= g det; then u = U/det, v = W/det, t = T/det.
 * Per ray: boolean = any hit; first hit = the smallest t, ties to the smallest
 * triangle index; (u, v, t) of that triangle (Background section: the three
 * operating modes).
 *
 * The BVH-structure functions (binary radix tree of Karras 2012, section 3, and
 * per-node bounding boxes) follow the paper's description of the BVH built over
 * Morton-sorted triangles (Background section; Case Study 1 listings).
 */
#include <stdint.h>
#include <stddef.h>
#include <math.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* One segment against one triangle, binary64, in the order stated above.  */
/* Returns 1 on a hit and writes the three quotients.                       */
/* ---------------------------------------------------------------------- */
static int oracle_pair(const double O[3], const double E[3],
                       const double A[3], const double B[3], const double C[3],
                       double *u_out, double *v_out, double *t_out)
{
    double d[3], e1[3], e2[3], s[3], p[3], q[3];
    int k;
    for (k = 0; k < 3; ++k) {
        d[k] = E[k] - O[k];
        e1[k] = B[k] - A[k];
        e2[k] = C[k] - A[k];
        s[k] = O[k] - A[k];
    }
    /* p = d x e2, q = s x e1 */
    p[0] = d[1] * e2[2] - d[2] * e2[1];
    p[1] = d[2] * e2[0] - d[0] * e2[2];
    p[2] = d[0] * e2[1] - d[1] * e2[0];
    q[0] = s[1] * e1[2] - s[2] * e1[1];
    q[1] = s[2] * e1[0] - s[0] * e1[2];
    q[2] = s[0] * e1[1] - s[1] * e1[0];

    double det = (e1[0] * p[0] + e1[1] * p[1]) + e1[2] * p[2];
    double U = (s[0] * p[0] + s[1] * p[1]) + s[2] * p[2];
    double W = (d[0] * q[0] + d[1] * q[1]) + d[2] * q[2];
    double T = (e2[0] * q[0] + e2[1] * q[1]) + e2[2] * q[2];

    if (det == 0.0)
        return 0;
    double g = det > 0.0 ? 1.0 : -1.0;
    double a = g * U, b = g * W, tt = g * T, D = g * det;
    if (a >= 0.0 && b >= 0.0 && a + b <= D && tt >= 0.0 && tt <= D) {
        *u_out = U / det;
        *v_out = W / det;
        *t_out = T / det;
        return 1;
    }
    return 0;
}

/*
 * Exhaustive search: n_rays segments against n_tri triangles.
 *   V        float [n_vert][3]      vertex coordinates
 *   F        int32 [n_tri][3]       vertex indices (must lie in [0, n_vert))
 *   from,to  float [n_rays][3]      segment end points
 * Outputs (host memory, caller-owned):
 *   hit      uint8 [n_rays]         1 if any triangle is hit
 *   id       int32 [n_rays]         first-hit triangle index, -1 on a miss
 *   uvt      double[n_rays][3]      (u, v, t) of the first hit, NaN on a miss
 *   n_hits   int32 [n_rays]         number of triangles hit (may be NULL)
 * Returns 0, or -1 if an index is out of range (nothing written then).
 */
int rsi_oracle_intersect(const float *V, int64_t n_vert,
                         const int32_t *F, int64_t n_tri,
                         const float *from, const float *to, int64_t n_rays,
                         uint8_t *hit, int32_t *id, double *uvt, int32_t *n_hits,
                         int n_threads)
{
    int64_t j, i;
    for (j = 0; j < 3 * n_tri; ++j)
        if (F[j] < 0 || (int64_t)F[j] >= n_vert)
            return -1;

    /* Promote every triangle's corners to binary64 once (exact). */
    double *tri = (double *)malloc(sizeof(double) * 9 * (size_t)(n_tri > 0 ? n_tri : 1));
    if (!tri)
        return -2;
    for (j = 0; j < n_tri; ++j)
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k)
                tri[9 * j + 3 * c + k] = (double)V[3 * (int64_t)F[3 * j + c] + k];

#ifdef _OPENMP
    if (n_threads > 0)
        omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
    for (i = 0; i < n_rays; ++i) {
        double O[3], E[3];
        for (int k = 0; k < 3; ++k) {
            O[k] = (double)from[3 * i + k];
            E[k] = (double)to[3 * i + k];
        }
        int32_t best = -1, count = 0;
        double bu = NAN, bv = NAN, bt = NAN;
        for (int64_t jj = 0; jj < n_tri; ++jj) {
            double u, v, t;
            const double *T = tri + 9 * jj;
            if (oracle_pair(O, E, T, T + 3, T + 6, &u, &v, &t)) {
                ++count;
                /* ascending j with a strict test keeps the smallest index on ties */
                if (best < 0 || t < bt) {
                    best = (int32_t)jj;
                    bu = u;
                    bv = v;
                    bt = t;
                }
            }
        }
        hit[i] = (uint8_t)(best >= 0);
        id[i] = best;
        uvt[3 * i + 0] = bu;
        uvt[3 * i + 1] = bv;
        uvt[3 * i + 2] = bt;
        if (n_hits)
            n_hits[i] = count;
    }
    free(tri);
    return 0;
}

/* Threads the OpenMP runtime would use for the call above. */
int rsi_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Every (u, v, t, j) hit of one segment, in ascending j.  Used by tests that
 * look at more than the first hit.  Returns the number of hits written
 * (at most cap), or -1 on a bad index.
 */
int rsi_oracle_all_hits(const float *V, int64_t n_vert, const int32_t *F, int64_t n_tri,
                        const float from[3], const float to[3],
                        int32_t *ids, double *uvt, int cap)
{
    double O[3], E[3], A[3], B[3], C[3];
    int n = 0;
    for (int k = 0; k < 3; ++k) {
        O[k] = (double)from[k];
        E[k] = (double)to[k];
    }
    for (int64_t j = 0; j < n_tri; ++j) {
        for (int c = 0; c < 3; ++c)
            if (F[3 * j + c] < 0 || (int64_t)F[3 * j + c] >= n_vert)
                return -1;
        for (int k = 0; k < 3; ++k) {
            A[k] = (double)V[3 * (int64_t)F[3 * j + 0] + k];
            B[k] = (double)V[3 * (int64_t)F[3 * j + 1] + k];
            C[k] = (double)V[3 * (int64_t)F[3 * j + 2] + k];
        }
        double u, v, t;
        if (oracle_pair(O, E, A, B, C, &u, &v, &t)) {
            if (n < cap) {
                ids[n] = (int32_t)j;
                uvt[3 * n + 0] = u;
                uvt[3 * n + 1] = v;
                uvt[3 * n + 2] = t;
            }
            ++n;
        }
    }
    return n;
}

/*
 * Number of distinct intersections of each segment with the surface (paper:
 * Background -- the experimental intercept-count mode, the number of unique
 * intersections per ray).  Reading: the number of distinct binary64 t values
 * among the segment's hits, each decided exactly as above, so several
 * triangles hit at the same t (a shared edge or vertex) count once.
 *   count   int32 [n_rays]   output
 * Returns 0, -1 on a bad index, -2 if memory runs out.
 */
static int cmp_double(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

int rsi_oracle_intercept_count(const float *V, int64_t n_vert,
                               const int32_t *F, int64_t n_tri,
                               const float *from, const float *to, int64_t n_rays,
                               int32_t *count, int n_threads)
{
    int64_t j, i;
    for (j = 0; j < 3 * n_tri; ++j)
        if (F[j] < 0 || (int64_t)F[j] >= n_vert)
            return -1;
    double *tri = (double *)malloc(sizeof(double) * 9 * (size_t)(n_tri > 0 ? n_tri : 1));
    if (!tri)
        return -2;
    for (j = 0; j < n_tri; ++j)
        for (int c = 0; c < 3; ++c)
            for (int k = 0; k < 3; ++k)
                tri[9 * j + 3 * c + k] = (double)V[3 * (int64_t)F[3 * j + c] + k];
    int failed = 0;
#ifdef _OPENMP
    if (n_threads > 0)
        omp_set_num_threads(n_threads);
#pragma omp parallel reduction(| : failed)
#endif
    {
        size_t cap = 64;
        double *ts = (double *)malloc(sizeof(double) * cap);
        if (!ts)
            failed = 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
        for (i = 0; i < n_rays; ++i) {
            if (!ts) {
                count[i] = -1;
                continue;
            }
            double O[3], E[3];
            for (int k = 0; k < 3; ++k) {
                O[k] = (double)from[3 * i + k];
                E[k] = (double)to[3 * i + k];
            }
            size_t n = 0;
            for (int64_t jj = 0; jj < n_tri; ++jj) {
                double u, v, t;
                const double *T = tri + 9 * jj;
                if (!oracle_pair(O, E, T, T + 3, T + 6, &u, &v, &t))
                    continue;
                if (n == cap) {
                    double *grown = (double *)realloc(ts, sizeof(double) * 2 * cap);
                    if (!grown) {
                        failed = 1;
                        break;
                    }
                    ts = grown;
                    cap *= 2;
                }
                ts[n++] = t;
            }
            qsort(ts, n, sizeof(double), cmp_double);
            int32_t distinct = 0;
            for (size_t k = 0; k < n; ++k)
                if (k == 0 || ts[k] != ts[k - 1])
                    ++distinct;
            count[i] = distinct;
        }
        free(ts);
    }
    free(tri);
    return failed ? -2 : 0;
}

/* ---------------------------------------------------------------------- */
/* Binary radix tree over sorted keys (Karras 2012, section 3).            */
/* ---------------------------------------------------------------------- */

/* Number of significant bits of x (0 for x == 0). */
static int bit_length(uint64_t x)
{
    int n = 0;
    while (x) {
        ++n;
        x >>= 1;
    }
    return n;
}

/*
 * Length of the longest common prefix of the bit strings key_i || i and
 * key_j || j, where keys are key_bits wide and indices 32 bits wide (equal keys
 * are told apart by their positions); -1 when j lies outside [0, n).
 */
static int common_prefix(const uint64_t *keys, int64_t n, int key_bits, int64_t i, int64_t j)
{
    if (j < 0 || j >= n)
        return -1;
    if (keys[i] != keys[j])
        return key_bits - bit_length(keys[i] ^ keys[j]);
    return key_bits + 32 - bit_length((uint64_t)((uint32_t)i ^ (uint32_t)j));
}

/*
 * For each internal node i in [0, n-2] find the key range it covers and the
 * split inside it, as in Karras 2012 section 3: the range grows from i in the
 * direction whose neighbour shares the longer prefix; its far end is the last
 * position whose prefix with i is longer than the prefix i shares with the
 * neighbour on the other side; the split is the last position whose prefix
 * with i is longer than the prefix common to the whole range.
 * Children: left covers [min end, split], right [split+1, max end]; a child
 * covering a single key is leaf `split` (left) or `split+1` (right), otherwise
 * internal node `split` (left) or `split+1` (right).
 * Outputs int32 [n-1]: left, right child index, left_leaf, right_leaf flags,
 * first/last (range ends).
 */
void rsi_oracle_radix_tree(const uint64_t *keys, int64_t n, int key_bits,
                           int32_t *left, int32_t *right,
                           uint8_t *left_leaf, uint8_t *right_leaf,
                           int32_t *first, int32_t *last)
{
    for (int64_t i = 0; i + 1 < n; ++i) {
        int dir = common_prefix(keys, n, key_bits, i, i + 1) >
                          common_prefix(keys, n, key_bits, i, i - 1) ? 1 : -1;
        int lower = common_prefix(keys, n, key_bits, i, i - dir);

        /* grow an upper bound for the range length by doubling */
        int64_t len_max = 2;
        while (common_prefix(keys, n, key_bits, i, i + len_max * dir) > lower)
            len_max *= 2;
        /* then find the exact length bit by bit */
        int64_t len = 0;
        for (int64_t step = len_max / 2; step >= 1; step /= 2)
            if (common_prefix(keys, n, key_bits, i, i + (len + step) * dir) > lower)
                len += step;
        int64_t j = i + len * dir;
        int node_prefix = common_prefix(keys, n, key_bits, i, j);

        /* split: largest offset s in [0, len) whose prefix with i exceeds node_prefix */
        int64_t s = 0;
        int64_t div = 2;
        for (;;) {
            int64_t step = (len + div - 1) / div;
            if (common_prefix(keys, n, key_bits, i, i + (s + step) * dir) > node_prefix)
                s += step;
            if (step == 1)
                break;
            div *= 2;
        }
        int64_t split = i + s * dir + (dir < 0 ? -1 : 0);
        int64_t lo = i < j ? i : j, hi = i < j ? j : i;
        left[i] = (int32_t)split;
        right[i] = (int32_t)(split + 1);
        left_leaf[i] = (uint8_t)(lo == split);
        right_leaf[i] = (uint8_t)(hi == split + 1);
        first[i] = (int32_t)lo;
        last[i] = (int32_t)hi;
    }
}

/*
 * Bounding box of every internal node: the component-wise min / max over the
 * corners of all triangles in its key range [first, last] (by definition of a
 * bounding volume over the node's leaves).  order[k] is the triangle at sorted
 * position k.  Output float [n-1][6] = lo.xyz, hi.xyz.
 */
void rsi_oracle_node_boxes(const float *V, const int32_t *F, const int32_t *order, int64_t n,
                           const int32_t *first, const int32_t *last, float *boxes)
{
    for (int64_t i = 0; i + 1 < n; ++i) {
        float lo[3] = {INFINITY, INFINITY, INFINITY};
        float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int64_t k = first[i]; k <= last[i]; ++k) {
            int64_t t = order[k];
            for (int c = 0; c < 3; ++c) {
                const float *P = V + 3 * (int64_t)F[3 * t + c];
                for (int a = 0; a < 3; ++a) {
                    if (P[a] < lo[a]) lo[a] = P[a];
                    if (P[a] > hi[a]) hi[a] = P[a];
                }
            }
        }
        for (int a = 0; a < 3; ++a) {
            boxes[6 * i + a] = lo[a];
            boxes[6 * i + 3 + a] = hi[a];
        }
    }
}
