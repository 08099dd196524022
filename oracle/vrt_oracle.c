/*
 * vrt_oracle.c -- plain, slow CPU oracle for voxel ray tracing of dynamic
 * line sets (arXiv 2510.09081, Sections 3.1-3.5).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant table with
 * the HIP implementation.
 *
 * Arithmetic:
 *   - voxel membership, counts, mips, erosion and culling: exact integers
 *     (int64), on endpoints quantized to 1/256 voxel;
 *   - the per-fragment occupancy quantum: a fixed IEEE binary32 operation
 *     sequence (it decides an integer, so both sides use the same precision);
 *   - primary-ray directions: a fixed binary32 sequence (both sides trace the
 *     same ray);
 *   - everything else in the trace (hits, order, compositing): binary64.
 * Build with -ffp-contract=off so that no multiply-add is fused.
 *
 * Voxel arrays here are dense, x fastest: v = (z*Gy + y)*Gx + x.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define QS 256             /* fixed-point steps per voxel */
#define RMIN_Q 128         /* PWAA minimum radius: half a voxel (Alg. 3) */
#define ST_OK 0
#define ST_RANGE 2
#define ST_COUNT_OVERFLOW 5

/* ------------------------------------------------------------------ */
/* small integer helpers                                               */

static int64_t floordiv(int64_t a, int64_t b) /* b > 0 */
{
    int64_t q = a / b;
    if ((a % b) != 0 && a < 0) q -= 1;
    return q;
}

static int64_t ceil_sqrt_i64(int64_t n) /* smallest w >= 0 with w*w >= n */
{
    if (n <= 0) return 0;
    int64_t w = (int64_t)sqrt((double)n);
    while (w * w < n) w++;
    while (w > 0 && (w - 1) * (w - 1) >= n) w--;
    return w;
}

static int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
static int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }

/* ------------------------------------------------------------------ */
/* Quantization of endpoints, radius and eye.                          */

/* Each coordinate becomes q = rint((x - origin) * s), s = 256/voxel_size
 * rounded once to binary32; the subtraction and the product are two separate
 * binary32 operations.  |q| must stay below 2^20. */
int orc_quantize(const float *xyz, int64_t nv, const float *origin, float voxel_size, int32_t *q)
{
    float s = (float)(256.0 / (double)voxel_size);
    int status = ST_OK;
    for (int64_t i = 0; i < nv; i++) {
        for (int c = 0; c < 3; c++) {
            float t = xyz[3 * i + c] - origin[c];
            float u = t * s;
            if (!(fabsf(u) < 1048576.0f)) { status = ST_RANGE; q[3 * i + c] = 0; continue; }
            q[3 * i + c] = (int32_t)rintf(u);
            if (q[3 * i + c] >= (1 << 20) || q[3 * i + c] <= -(1 << 20)) status = ST_RANGE;
        }
    }
    return status;
}

/* Radius in 1/256 voxel, rounded to nearest even in binary64. */
int64_t orc_radius_q(float radius, float voxel_size)
{
    return (int64_t)rint((double)radius * 256.0 / (double)voxel_size);
}

/* Eye position in 1/256 voxel relative to the grid corner. */
void orc_eye_q(const float *eye, const float *origin, float voxel_size, int64_t *eq)
{
    double s = 256.0 / (double)voxel_size;
    for (int c = 0; c < 3; c++) eq[c] = (int64_t)rint(((double)eye[c] - (double)origin[c]) * s);
}

/* Clip-plane normals (Section 3.1, after Gross & Gumhold): the tangent at an
 * interior vertex by central differences, T = V[i+1] - V[i-1] (exact
 * integers), normalized in binary32 as f32(T_c) / sqrt(f32(T.T)).  End
 * vertices of a polyline, and zero tangents, get no clip plane (n = 0,
 * interior = 0).  seg_valid[i] = 1 iff vertex i starts a segment, i.e. it is
 * not the last vertex of its polyline (primitive index i, Section 3.3). */
void orc_vertex_attrs(const int32_t *q, const int32_t *offsets, int64_t np, float *nrm,
                      uint8_t *interior, uint8_t *seg_valid)
{
    for (int64_t p = 0; p < np; p++) {
        int64_t a = offsets[p], b = offsets[p + 1];
        for (int64_t i = a; i < b; i++) {
            seg_valid[i] = (uint8_t)(i + 1 < b);
            interior[i] = 0;
            nrm[3 * i] = nrm[3 * i + 1] = nrm[3 * i + 2] = 0.0f;
            if (i > a && i + 1 < b) {
                int64_t T[3], TT = 0;
                for (int c = 0; c < 3; c++) {
                    T[c] = (int64_t)q[3 * (i + 1) + c] - (int64_t)q[3 * (i - 1) + c];
                    TT += T[c] * T[c];
                }
                if (TT > 0) {
                    float len = sqrtf((float)TT);
                    for (int c = 0; c < 3; c++) nrm[3 * i + c] = (float)T[c] / len;
                    interior[i] = 1;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Conservative capsule voxelization (Section 3.1, Alg. 1 and Eq. 1).   */

typedef void (*visit_fn)(void *ctx, int64_t x, int64_t y, int64_t z);

/* Corrected form, in integers (Q = 256 steps per voxel):
 *  1. d = B - A; the major axis a0 has the largest |d| (lowest index on a
 *     tie); if d[a0] < 0 the endpoints are swapped (the set does not change).
 *  2. The capsule's closed AABB [min - r, max + r] gives the voxel range
 *     [floor((lo-1)/Q), floor(hi/Q)] per axis, clipped to the grid; this is
 *     the major-axis walk from the extended vertices, both ends included.
 *  3. For each major-axis slab x, with [ta, tb] its part of the AABB, the
 *     capsule's minor coordinate i lies within the segment's line at ta and
 *     tb widened by R_i = r*sqrt(1 + (d_i/d_a0)^2) -- the projected radius
 *     that is conservative in 3D (Eq. 1 under-estimates it when both minor
 *     components are non-zero).  Scaled by D = d_a0: centre numerator
 *     A_i*D + d_i*(t - A_a0), half-width W_i = ceil(sqrt(r^2 (D^2 + d_i^2))).
 *  4. Every voxel of the slab's 2D box (clipped to the AABB range) is visited.
 * A zero-length segment is a ball: its AABB range. */
static int64_t segment_voxels_exact(const int32_t *Ai, const int32_t *Bi, int64_t rq, const int32_t *G,
                                    visit_fn fn, void *ctx)
{
    int64_t A[3], B[3], d[3];
    for (int c = 0; c < 3; c++) { A[c] = Ai[c]; B[c] = Bi[c]; d[c] = B[c] - A[c]; }
    int a0 = 0;
    for (int c = 1; c < 3; c++)
        if (llabs(d[c]) > llabs(d[a0])) a0 = c;
    if (d[a0] < 0) {
        for (int c = 0; c < 3; c++) { int64_t t = A[c]; A[c] = B[c]; B[c] = t; d[c] = -d[c]; }
    }
    int a1 = (a0 + 1) % 3, a2 = (a0 + 2) % 3;
    int64_t D = d[a0];
    int64_t lo[3], hi[3], vlo[3], vhi[3];
    for (int c = 0; c < 3; c++) {
        lo[c] = imin(A[c], B[c]) - rq;
        hi[c] = imax(A[c], B[c]) + rq;
        vlo[c] = imax(floordiv(lo[c] - 1, QS), 0);
        vhi[c] = imin(floordiv(hi[c], QS), (int64_t)G[c] - 1);
        if (vlo[c] > vhi[c]) return 0;
    }
    int64_t W[3] = {0, 0, 0};
    if (D > 0) {
        W[a1] = ceil_sqrt_i64(rq * rq * (D * D + d[a1] * d[a1]));
        W[a2] = ceil_sqrt_i64(rq * rq * (D * D + d[a2] * d[a2]));
    }
    int64_t n = 0;
    for (int64_t x = vlo[a0]; x <= vhi[a0]; x++) {
        int64_t ta = imax(lo[a0], x * QS), tb = imin(hi[a0], (x + 1) * QS);
        int64_t rlo[3], rhi[3];
        int ax[2] = {a1, a2};
        for (int k = 0; k < 2; k++) {
            int i = ax[k];
            if (D == 0) { rlo[i] = vlo[i]; rhi[i] = vhi[i]; continue; }
            int64_t ca = A[i] * D + d[i] * (ta - A[a0]);
            int64_t cb = A[i] * D + d[i] * (tb - A[a0]);
            int64_t nlo = imin(ca, cb) - W[i], nhi = imax(ca, cb) + W[i];
            rlo[i] = imax(floordiv(nlo - 1, D * QS), vlo[i]);
            rhi[i] = imin(floordiv(nhi, D * QS), vhi[i]);
        }
        for (int64_t j = rlo[a1]; j <= rhi[a1]; j++)
            for (int64_t k = rlo[a2]; k <= rhi[a2]; k++) {
                int64_t C[3];
                C[a0] = x; C[a1] = j; C[a2] = k;
                if (fn) fn(ctx, C[0], C[1], C[2]);
                n++;
            }
    }
    return n;
}

/* Alg. 1 as printed, in binary64 voxel units, for comparison only: Eq. (1)
 * radius, walk while t0 < t_max, int() read as floor, no AABB clamp. */
static int64_t segment_voxels_literal(const int32_t *Ai, const int32_t *Bi, int64_t rq, const int32_t *G,
                                      visit_fn fn, void *ctx)
{
    double A[3], B[3], d[3], r = (double)rq / QS;
    for (int c = 0; c < 3; c++) { A[c] = Ai[c] / (double)QS; B[c] = Bi[c] / (double)QS; d[c] = B[c] - A[c]; }
    int a0 = 0;
    for (int c = 1; c < 3; c++)
        if (fabs(d[c]) > fabs(d[a0])) a0 = c;
    if (d[a0] < 0) {
        for (int c = 0; c < 3; c++) { double t = A[c]; A[c] = B[c]; B[c] = t; d[c] = -d[c]; }
    }
    if (d[a0] == 0.0) return 0;
    int a1 = (a0 + 1) % 3, a2 = (a0 + 2) % 3;
    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double s[3], v0[3], rh[3];
    for (int c = 0; c < 3; c++) { s[c] = d[c] / d[a0]; v0[c] = A[c] - s[c] * r; }
    rh[a1] = r / sqrt(1.0 - (d[a1] / len) * (d[a1] / len));
    rh[a2] = r / sqrt(1.0 - (d[a2] / len) * (d[a2] / len));
    double tmin = v0[a0], tmax = B[a0] + s[a0] * r, t0 = tmin;
    double p0[3] = {v0[0], v0[1], v0[2]};
    int64_t n = 0;
    while (t0 < tmax) {
        double t1 = fmin(tmax, floor(t0 + 1.0));
        double p1[3];
        for (int c = 0; c < 3; c++) p1[c] = v0[c] + s[c] * (t1 - tmin);
        int64_t jmin = (int64_t)floor(fmin(p0[a1], p1[a1]) - rh[a1]);
        int64_t jmax = (int64_t)floor(fmax(p0[a1], p1[a1]) + rh[a1]);
        int64_t kmin = (int64_t)floor(fmin(p0[a2], p1[a2]) - rh[a2]);
        int64_t kmax = (int64_t)floor(fmax(p0[a2], p1[a2]) + rh[a2]);
        int64_t x = (int64_t)floor(t0);
        for (int64_t j = jmin; j <= jmax; j++)
            for (int64_t k = kmin; k <= kmax; k++) {
                int64_t C[3];
                C[a0] = x; C[a1] = j; C[a2] = k;
                if (C[0] < 0 || C[1] < 0 || C[2] < 0 || C[0] >= G[0] || C[1] >= G[1] || C[2] >= G[2]) continue;
                if (fn) fn(ctx, C[0], C[1], C[2]);
                n++;
            }
        t0 = t1;
        for (int c = 0; c < 3; c++) p0[c] = p1[c];
    }
    return n;
}

/* The two comparison voxelizers of Section 4.1 (Table 2), from their
 * definitions.  Neither is conservative for capsules; they are measured
 * against the capsule voxelizer, not used for rendering.
 *
 * Thin line ("DDA"): the voxels whose open interior the open segment (A, B)
 * meets, plus the voxels holding A and B (half-open cells); the radius plays
 * no part.  Each voxel of the segment's voxel box is tested on its own: the
 * parameters t in (0, 1) at which the segment is strictly inside the cube on
 * one axis form an open interval (lo_c/den_c, hi_c/den_c), and the cube's
 * interior is met iff every lower end is below every upper end (exact
 * integer cross-multiplication). */
static int open_segment_meets_voxel(const int64_t *A, const int64_t *d, const int64_t *v)
{
    int64_t ln[4] = {0, 0, 0, 0}, ld[4] = {1, 1, 1, 1};  /* lower ends n/d, d > 0 (the first is t = 0) */
    int64_t un[4] = {1, 1, 1, 1}, ud[4] = {1, 1, 1, 1};  /* upper ends (the first is t = 1) */
    for (int c = 0; c < 3; c++) {
        int64_t lo = v[c] * QS, hi = (v[c] + 1) * QS;
        if (d[c] == 0) {
            if (!(lo < A[c] && A[c] < hi)) return 0;
            continue;
        }
        int64_t n1 = lo - A[c], n2 = hi - A[c], den = d[c];
        if (den < 0) { int64_t t = -n1; n1 = -n2; n2 = t; den = -den; }
        ln[c + 1] = n1; ld[c + 1] = den;
        un[c + 1] = n2; ud[c + 1] = den;
    }
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++)
            if (!(ln[i] * ud[j] < un[j] * ld[i])) return 0;
    return 1;
}

static int64_t segment_voxels_thin(const int32_t *Ai, const int32_t *Bi, const int32_t *G, visit_fn fn, void *ctx)
{
    int64_t A[3], B[3], d[3], lo[3], hi[3], ca[3], cb[3];
    for (int c = 0; c < 3; c++) {
        A[c] = Ai[c]; B[c] = Bi[c]; d[c] = B[c] - A[c];
        ca[c] = floordiv(A[c], QS); cb[c] = floordiv(B[c], QS);
        lo[c] = imax(imin(ca[c], cb[c]) - 1, 0);
        hi[c] = imin(imax(ca[c], cb[c]) + 1, (int64_t)G[c] - 1);
    }
    int64_t n = 0;
    for (int64_t z = lo[2]; z <= hi[2]; z++)
        for (int64_t y = lo[1]; y <= hi[1]; y++)
            for (int64_t x = lo[0]; x <= hi[0]; x++) {
                int64_t v[3] = {x, y, z};
                int endp = (x == ca[0] && y == ca[1] && z == ca[2]) || (x == cb[0] && y == cb[1] && z == cb[2]);
                if (endp || open_segment_meets_voxel(A, d, v)) {
                    if (fn) fn(ctx, x, y, z);
                    n++;
                }
            }
    return n;
}

/* Capsule AABB: every voxel that touches the capsule's closed bounding box
 * (the range of step 2 of the capsule voxelizer). */
static int64_t segment_voxels_aabb(const int32_t *Ai, const int32_t *Bi, int64_t rq, const int32_t *G, visit_fn fn,
                                   void *ctx)
{
    int64_t vlo[3], vhi[3];
    for (int c = 0; c < 3; c++) {
        vlo[c] = imax(floordiv(imin(Ai[c], Bi[c]) - rq - 1, QS), 0);
        vhi[c] = imin(floordiv(imax(Ai[c], Bi[c]) + rq, QS), (int64_t)G[c] - 1);
        if (vlo[c] > vhi[c]) return 0;
    }
    int64_t n = 0;
    for (int64_t z = vlo[2]; z <= vhi[2]; z++)
        for (int64_t y = vlo[1]; y <= vhi[1]; y++)
            for (int64_t x = vlo[0]; x <= vhi[0]; x++) {
                if (fn) fn(ctx, x, y, z);
                n++;
            }
    return n;
}

/* Membership by mode: 0 the capsule voxelizer (Alg. 1, corrected Eq. (1)),
 * 1 the printed Alg. 1 + Eq. (1), 2 the thin line, 3 the capsule AABB. */
static int64_t segment_voxels_mode(int mode, const int32_t *A, const int32_t *B, int64_t rq, const int32_t *G,
                                   visit_fn fn, void *ctx)
{
    switch (mode) {
    case 1: return segment_voxels_literal(A, B, rq, G, fn, ctx);
    case 2: return segment_voxels_thin(A, B, G, fn, ctx);
    case 3: return segment_voxels_aabb(A, B, rq, G, fn, ctx);
    default: return segment_voxels_exact(A, B, rq, G, fn, ctx);
    }
}

typedef struct { int32_t *out; int64_t cap, n; } list_ctx;
static void visit_list(void *ctx, int64_t x, int64_t y, int64_t z)
{
    list_ctx *L = (list_ctx *)ctx;
    if (L->n < L->cap) {
        L->out[3 * L->n] = (int32_t)x; L->out[3 * L->n + 1] = (int32_t)y; L->out[3 * L->n + 2] = (int32_t)z;
    }
    L->n++;
}

/* Voxel set S(s) of one segment; writes up to cap (x,y,z) triples and returns
 * the full count.  mode: see segment_voxels_mode. */
int64_t orc_segment_voxels(const int32_t *A, const int32_t *B, int64_t rq, const int32_t *G, int32_t *out,
                           int64_t cap, int mode)
{
    list_ctx L = {out, cap, 0};
    return segment_voxels_mode(mode, A, B, rq, G, visit_list, &L);
}

/* ------------------------------------------------------------------ */
/* Occupancy quantum of one (segment, voxel) pair (Alg. 2 and Alg. 3).  */

/* Clipped-capsule SDF sampled at the voxel centre, with the radius clamped to
 * r_min = 0.5 voxel and the occupancy scaled by (r / r_clamp)^2 (PWAA), as a
 * fixed binary32 sequence (no fused multiply-add, sums left to right,
 * correctly rounded division and square root).  Lengths are in 1/256 voxel.
 * Returns q = rint(256 * occupancy) in [0, 256]. */
int orc_occupancy_q(const int32_t *A, const int32_t *B, const float *n0, const float *n1, int a_interior,
                    int b_interior, float rc, float corr, int64_t vx, int64_t vy, int64_t vz)
{
    int64_t P[3] = {vx * QS + QS / 2, vy * QS + QS / 2, vz * QS + QS / 2};
    float pa[3], pb[3], d[3];
    for (int c = 0; c < 3; c++) {
        pa[c] = (float)(P[c] - (int64_t)A[c]);
        pb[c] = (float)(P[c] - (int64_t)B[c]);
        d[c] = (float)((int64_t)B[c] - (int64_t)A[c]);
    }
    float hn = pa[0] * d[0];
    hn = hn + pa[1] * d[1];
    hn = hn + pa[2] * d[2];
    float dd = d[0] * d[0];
    dd = dd + d[1] * d[1];
    dd = dd + d[2] * d[2];
    float h = 0.0f;
    if (dd > 0.0f) {
        h = hn / dd;
        h = fminf(fmaxf(h, 0.0f), 1.0f);
    }
    float e0 = pa[0] - d[0] * h, e1 = pa[1] - d[1] * h, e2 = pa[2] - d[2] * h;
    float ss = e0 * e0;
    ss = ss + e1 * e1;
    ss = ss + e2 * e2;
    float sdf = sqrtf(ss) - rc;
    if (a_interior) {
        float s0 = pa[0] * n0[0];
        s0 = s0 + pa[1] * n0[1];
        s0 = s0 + pa[2] * n0[2];
        sdf = fmaxf(sdf, -s0);
    }
    if (b_interior) {
        float s1 = pb[0] * n1[0];
        s1 = s1 + pb[1] * n1[1];
        s1 = s1 + pb[2] * n1[2];
        sdf = fmaxf(sdf, s1);
    }
    float occ = 0.5f - sdf / 256.0f;
    occ = fminf(fmaxf(occ, 0.0f), 1.0f);
    occ = occ * corr;
    return (int)rintf(occ * 256.0f);
}

/* PWAA constants from the quantized radius: r_clamp and (r / r_clamp)^2,
 * evaluated in binary64 and rounded once to binary32. */
void orc_pwaa_consts(int64_t rq, float *rc, float *corr)
{
    int64_t rcl = rq > RMIN_Q ? rq : RMIN_Q;
    double ratio = (double)rq / (double)rcl;
    *rc = (float)rcl;
    *corr = (float)(ratio * ratio);
}

/* ------------------------------------------------------------------ */
/* Pass 1: per-voxel count and occupancy, packed in one 32-bit word      */
/* (Section 3.1: count in the low 16 bits, occupancy sum in the high).    */

typedef struct {
    const int32_t *q;
    const float *nrm;
    const uint8_t *interior;
    int64_t seg;
    float rc, corr;
    const int32_t *G;
    int64_t *count;
    int64_t *occ;
} vox_ctx;

static void visit_accumulate(void *ctx, int64_t x, int64_t y, int64_t z)
{
    vox_ctx *V = (vox_ctx *)ctx;
    int64_t i = V->seg;
    int64_t v = (z * V->G[1] + y) * V->G[0] + x;
    int qv = orc_occupancy_q(V->q + 3 * i, V->q + 3 * (i + 1), V->nrm + 3 * i, V->nrm + 3 * (i + 1),
                             V->interior[i], V->interior[i + 1], V->rc, V->corr, x, y, z);
    V->count[v] += 1;
    V->occ[v] += qv;
}

/* Fills words[v] = (count + occupancy_sum * 2^16) mod 2^32.  A segment
 * longer than 2^16 steps along an axis is a range error; a voxel with more
 * than 65535 fragments is a count overflow.  mode selects the membership
 * (segment_voxels_mode; only 0 is conservative, the others are comparisons). */
int orc_voxelize(const int32_t *q, const float *nrm, const uint8_t *interior, const uint8_t *seg_valid,
                 int64_t nv, int64_t rq, const int32_t *G, uint32_t *words, int64_t *n_fragments, int mode)
{
    int64_t nvox = (int64_t)G[0] * G[1] * G[2];
    int64_t *count = (int64_t *)calloc((size_t)nvox, sizeof(int64_t));
    int64_t *occ = (int64_t *)calloc((size_t)nvox, sizeof(int64_t));
    float rc, corr;
    orc_pwaa_consts(rq, &rc, &corr);
    int status = ST_OK;
    vox_ctx V = {q, nrm, interior, 0, rc, corr, G, count, occ};
    int64_t nf = 0;
    for (int64_t i = 0; i + 1 < nv; i++) {
        if (!seg_valid[i]) continue;
        int bad = 0;
        for (int c = 0; c < 3; c++)
            if (llabs((int64_t)q[3 * (i + 1) + c] - (int64_t)q[3 * i + c]) >= 65536) bad = 1;
        if (bad) { status = ST_RANGE; continue; }
        V.seg = i;
        nf += segment_voxels_mode(mode, q + 3 * i, q + 3 * (i + 1), rq, G, visit_accumulate, &V);
    }
    for (int64_t v = 0; v < nvox; v++) {
        if (count[v] > 65535 && status == ST_OK) status = ST_COUNT_OVERFLOW;
        words[v] = (uint32_t)(((uint64_t)count[v] + ((uint64_t)occ[v] << 16)) & 0xFFFFFFFFu);
    }
    free(count);
    free(occ);
    if (n_fragments) *n_fragments = nf;
    return status;
}

/* ------------------------------------------------------------------ */
/* Occupancy pyramid (Section 3.1, averaging mipmap).                    */

/* Level 0 in 1/256 units: saturated at 256 (a fraction of the voxel); a
 * voxel with 256 or more fragments is full (its 16-bit sum may wrap). */
void orc_occupancy_level0(const uint32_t *words, int64_t nvox, uint16_t *o0)
{
    for (int64_t v = 0; v < nvox; v++) {
        uint32_t cnt = words[v] & 0xFFFFu, sum = words[v] >> 16;
        o0[v] = (uint16_t)(cnt >= 256 ? 256 : (sum > 256 ? 256 : sum));
    }
}

/* One averaging step: parent = floor((sum of children inside the grid + 4) / 8);
 * parent dims are ceil(child dims / 2). */
void orc_mip_average(const uint16_t *src, const int32_t *ds, uint16_t *dst)
{
    int64_t dx = (ds[0] + 1) / 2, dy = (ds[1] + 1) / 2, dz = (ds[2] + 1) / 2;
    for (int64_t z = 0; z < dz; z++)
        for (int64_t y = 0; y < dy; y++)
            for (int64_t x = 0; x < dx; x++) {
                int64_t s = 0;
                for (int k = 0; k < 8; k++) {
                    int64_t cx = 2 * x + (k & 1), cy = 2 * y + ((k >> 1) & 1), cz = 2 * z + (k >> 2);
                    if (cx < ds[0] && cy < ds[1] && cz < ds[2]) s += src[(cz * ds[1] + cy) * ds[0] + cx];
                }
                dst[(z * dy + y) * dx + x] = (uint16_t)((s + 4) / 8);
            }
}

/* Culling pyramid step: parent visible iff any child is visible (Section 3.2). */
void orc_mip_or(const uint8_t *src, const int32_t *ds, uint8_t *dst)
{
    int64_t dx = (ds[0] + 1) / 2, dy = (ds[1] + 1) / 2, dz = (ds[2] + 1) / 2;
    for (int64_t z = 0; z < dz; z++)
        for (int64_t y = 0; y < dy; y++)
            for (int64_t x = 0; x < dx; x++) {
                uint8_t any = 0;
                for (int k = 0; k < 8; k++) {
                    int64_t cx = 2 * x + (k & 1), cy = 2 * y + ((k >> 1) & 1), cz = 2 * z + (k >> 2);
                    if (cx < ds[0] && cy < ds[1] && cz < ds[2] && src[(cz * ds[1] + cy) * ds[0] + cx]) any = 1;
                }
                dst[(z * dy + y) * dx + x] = any;
            }
}

/* ------------------------------------------------------------------ */
/* Culling (Section 3.2).                                                */

/* Erosion: the minimum level-0 occupancy over the voxel and its six face
 * neighbours (outside the grid counts as empty); a voxel blocks culling rays
 * when its eroded occupancy is full (>= 256, i.e. 1.0). */
void orc_erode_blocking(const uint16_t *o0, const int32_t *G, uint8_t *blocking)
{
    int64_t gx = G[0], gy = G[1], gz = G[2];
    for (int64_t z = 0; z < gz; z++)
        for (int64_t y = 0; y < gy; y++)
            for (int64_t x = 0; x < gx; x++) {
                int64_t v = (z * gy + y) * gx + x;
                int e = o0[v];
                const int64_t nb[6][3] = {{x - 1, y, z}, {x + 1, y, z}, {x, y - 1, z},
                                          {x, y + 1, z}, {x, y, z - 1}, {x, y, z + 1}};
                for (int k = 0; k < 6; k++) {
                    int64_t a = nb[k][0], b = nb[k][1], c = nb[k][2];
                    int on = 0;
                    if (a >= 0 && b >= 0 && c >= 0 && a < gx && b < gy && c < gz) on = o0[(c * gy + b) * gx + a];
                    if (on < e) e = on;
                }
                blocking[v] = (uint8_t)(e >= 256);
            }
}

/* Number of blocking voxels met by the open segment from the centre of voxel
 * (x,y,z) to the eye, stopping at `limit`.  Exact integer Amanatides-Woo:
 * the next boundary crossing on each axis is compared by cross-multiplying
 * distances; axes that tie are stepped together, so voxels the segment only
 * touches along an edge or at a corner are not visited.  The walk ends when
 * the segment leaves the grid or reaches the eye. */
int64_t orc_culling_ray(int64_t x, int64_t y, int64_t z, const int64_t *E, const int32_t *G,
                        const uint8_t *blocking, int64_t limit, int64_t *n_visited)
{
    int64_t cur[3] = {x, y, z}, c[3], delta[3], adel[3], step[3], g[3];
    for (int a = 0; a < 3; a++) {
        c[a] = cur[a] * QS + QS / 2;
        delta[a] = E[a] - c[a];
        adel[a] = llabs(delta[a]);
        step[a] = delta[a] > 0 ? 1 : (delta[a] < 0 ? -1 : 0);
        g[a] = QS / 2; /* distance from the centre to the next boundary */
    }
    int64_t n = 0, visited = 0;
    for (;;) {
        int best = -1;
        for (int a = 0; a < 3; a++) {
            if (step[a] == 0) continue;
            if (best < 0 || g[a] * adel[best] < g[best] * adel[a]) best = a;
        }
        if (best < 0) break;                 /* eye at the centre */
        if (!(g[best] < adel[best])) break;  /* next crossing at or beyond the eye */
        int tie[3] = {0, 0, 0};
        for (int a = 0; a < 3; a++)
            if (step[a] != 0 && g[a] * adel[best] == g[best] * adel[a]) tie[a] = 1;
        int out = 0;
        for (int a = 0; a < 3; a++)
            if (tie[a]) {
                cur[a] += step[a];
                g[a] += QS;
                if (cur[a] < 0 || cur[a] >= G[a]) out = 1;
            }
        if (out) break;
        visited++;
        if (blocking[(cur[2] * G[1] + cur[1]) * G[0] + cur[0]]) {
            n++;
            if (n >= limit) break;
        }
    }
    if (n_visited) *n_visited = visited;
    return n;
}

/* Level-0 culling: a voxel is visible iff it is occupied (count > 0) and its
 * ray to the eye meets fewer than `limit` blocking voxels; limit < 0 disables
 * culling (every occupied voxel is visible). */
void orc_visibility(const uint32_t *words, const uint8_t *blocking, const int32_t *G, const int64_t *E,
                    int64_t limit, uint8_t *vis)
{
    int64_t gx = G[0], gy = G[1], gz = G[2];
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t z = 0; z < gz; z++)
        for (int64_t y = 0; y < gy; y++)
            for (int64_t x = 0; x < gx; x++) {
                int64_t v = (z * gy + y) * gx + x;
                if ((words[v] & 0xFFFFu) == 0) { vis[v] = 0; continue; }
                if (limit < 0) { vis[v] = 1; continue; }
                vis[v] = (uint8_t)(orc_culling_ray(x, y, z, E, G, blocking, limit, NULL) < limit);
            }
}

/* ------------------------------------------------------------------ */
/* Per-voxel fragment lists (Section 3.3).                               */

/* Position of voxel (x,y,z) in brick-major order: 8^3 bricks in x-fastest
 * order, voxels x-fastest inside a brick. */
static int64_t brick_major(int64_t x, int64_t y, int64_t z, const int32_t *G)
{
    int64_t nbx = G[0] / 8, nby = G[1] / 8;
    int64_t b = ((z / 8) * nby + (y / 8)) * nbx + (x / 8);
    return b * 512 + ((z % 8) * 64 + (y % 8) * 8 + (x % 8));
}

/* offsets[v] = exclusive prefix sum of count*visible over brick-major order
 * (stored at the dense index v); returns the total.  Dims must be multiples of 8. */
int64_t orc_offsets(const uint32_t *words, const uint8_t *vis, const int32_t *G, uint32_t *offsets)
{
    int64_t gx = G[0], gy = G[1], gz = G[2], nvox = gx * gy * gz;
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)nvox);
    for (int64_t z = 0; z < gz; z++)
        for (int64_t y = 0; y < gy; y++)
            for (int64_t x = 0; x < gx; x++) order[brick_major(x, y, z, G)] = (z * gy + y) * gx + x;
    int64_t run = 0;
    for (int64_t k = 0; k < nvox; k++) {
        int64_t v = order[k];
        offsets[v] = (uint32_t)run;
        if (vis[v]) run += (int64_t)(words[v] & 0xFFFFu);
    }
    free(order);
    return run;
}

typedef struct { const int32_t *G; const uint8_t *vis; uint32_t *cursor; uint32_t *ids; int64_t seg; } fill_ctx;
static void visit_fill(void *ctx, int64_t x, int64_t y, int64_t z)
{
    fill_ctx *F = (fill_ctx *)ctx;
    int64_t v = (z * F->G[1] + y) * F->G[0] + x;
    if (F->vis[v]) F->ids[F->cursor[v]++] = (uint32_t)F->seg;
}

/* ids: for every visible voxel, the ascending list of segments whose voxel
 * set contains it, stored at [offsets[v], offsets[v] + count[v]). */
void orc_fill_lists(const int32_t *q, const uint8_t *seg_valid, int64_t nv, int64_t rq, const int32_t *G,
                    const uint8_t *vis, const uint32_t *offsets, uint32_t *ids, int mode)
{
    int64_t nvox = (int64_t)G[0] * G[1] * G[2];
    uint32_t *cursor = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nvox);
    memcpy(cursor, offsets, sizeof(uint32_t) * (size_t)nvox);
    fill_ctx F = {G, vis, cursor, ids, 0};
    for (int64_t i = 0; i + 1 < nv; i++) {
        if (!seg_valid[i]) continue;
        int bad = 0;
        for (int c = 0; c < 3; c++)
            if (llabs((int64_t)q[3 * (i + 1) + c] - (int64_t)q[3 * i + c]) >= 65536) bad = 1;
        if (bad) continue;
        F.seg = i;
        segment_voxels_mode(mode, q + 3 * i, q + 3 * (i + 1), rq, G, visit_fill, &F);
    }
    free(cursor);
}

/* ------------------------------------------------------------------ */
/* Voxel-space shading (Section 3.4): ambient occlusion from cones traced  */
/* through the occupancy pyramid and a directional shadow ray, evaluated   */
/* for the visible voxels only; the tracer takes one value per hit.         */

/* Cone directions: the K points of a Fibonacci sphere (z evenly spaced,
 * longitude advancing by the golden angle), in 1/256 units, rounded to the
 * nearest integer in binary64. */
void orc_shade_dirs(int32_t K, int32_t *U)
{
    const double golden = M_PI * (3.0 - sqrt(5.0));
    for (int32_t k = 0; k < K; k++) {
        double z = 1.0 - (2.0 * k + 1.0) / (double)K;
        double r = sqrt(1.0 - z * z), phi = golden * (double)k;
        U[3 * k] = (int32_t)rint(256.0 * r * cos(phi));
        U[3 * k + 1] = (int32_t)rint(256.0 * r * sin(phi));
        U[3 * k + 2] = (int32_t)rint(256.0 * z);
    }
}

/* Light direction in 1/256 units (normalized, then rounded in binary64). */
void orc_shade_light(const float *l, int32_t *L)
{
    double n = sqrt((double)l[0] * l[0] + (double)l[1] * l[1] + (double)l[2] * l[2]);
    for (int c = 0; c < 3; c++) L[c] = (int32_t)rint(256.0 * (double)l[c] / n);
}

/* Occupancy (fraction) of cell c at pyramid level lv (dims d); 0 outside. */
static double occ_cell(const uint16_t *lv, const int64_t *d, const int64_t *c)
{
    for (int a = 0; a < 3; a++)
        if (c[a] < 0 || c[a] >= d[a]) return 0.0;
    return lv[(c[2] * d[1] + c[1]) * d[0] + c[0]] / 256.0;
}

/* For every voxel v with vis[v] != 0 (dense x-fastest arrays, grid G):
 *   ambient occlusion: for each cone k, samples j = 1..J at 2^j voxels from
 *     the voxel centre along U_k, each read from the level-j cell holding it
 *     (floor division in 1/256 units); the cone's opacity accumulates front
 *     to back, a += (1 - a) o_j, and AO(v) is the mean of 1 - a over the K
 *     cones;
 *   shadow: the ray from the voxel centre along L through the level-0 grid
 *     (integer walk, tied axes step together, v itself excluded) until it
 *     leaves the grid; S(v) is the product of 1 - o0(u) over the voxels u
 *     it enters;
 *   lit(v) = AO(v) (ambient + (1 - ambient) S(v)).
 * levels[j] points at occupancy level j (dims ceil(G / 2^j)), j = 0..J.
 * Invisible voxels get ao = sh = lit = 0. */
void orc_shade(const int32_t *G, const uint16_t *const *levels, int32_t J, const uint8_t *vis, int32_t K,
               const int32_t *U, const int32_t *L, double ambient, double *ao, double *sh, double *lit)
{
    int64_t nvox = (int64_t)G[0] * G[1] * G[2];
    int64_t dims[8][3];
    for (int32_t j = 0; j <= J; j++)
        for (int a = 0; a < 3; a++) {
            int64_t d = G[a];
            for (int32_t t = 0; t < j; t++) d = (d + 1) / 2;
            dims[j][a] = d;
        }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t v = 0; v < nvox; v++) {
        ao[v] = sh[v] = lit[v] = 0.0;
        if (!vis[v]) continue;
        int64_t p[3] = {v % G[0], (v / G[0]) % G[1], v / ((int64_t)G[0] * G[1])};
        int64_t C[3];
        for (int a = 0; a < 3; a++) C[a] = p[a] * QS + QS / 2;
        double sum = 0.0;
        for (int32_t k = 0; k < K; k++) {
            double acc = 0.0;
            for (int32_t j = 1; j <= J; j++) {
                int64_t cell[3];
                for (int a = 0; a < 3; a++)
                    cell[a] = floordiv(C[a] + (int64_t)U[3 * k + a] * ((int64_t)1 << j), (int64_t)QS << j);
                acc += (1.0 - acc) * occ_cell(levels[j], dims[j], cell);
            }
            sum += 1.0 - acc;
        }
        ao[v] = sum / (double)K;
        /* shadow walk: next crossing on axis a at parameter (X_a - C_a) / L_a */
        double T = 1.0;
        int64_t u[3] = {p[0], p[1], p[2]};
        int any = L[0] != 0 || L[1] != 0 || L[2] != 0;
        while (any) {
            int64_t num[3], den[3];
            int best = -1;
            for (int a = 0; a < 3; a++) {
                den[a] = llabs((int64_t)L[a]);
                if (den[a] == 0) continue;
                int64_t X = (u[a] + (L[a] > 0)) * QS;
                num[a] = llabs(X - C[a]);
                if (best < 0 || num[a] * den[best] < num[best] * den[a]) best = a;
            }
            int out = 0;
            for (int a = 0; a < 3; a++) {
                if (den[a] == 0 || num[a] * den[best] != num[best] * den[a]) continue;
                u[a] += L[a] > 0 ? 1 : -1;
                if (u[a] < 0 || u[a] >= G[a]) out = 1;
            }
            if (out) break;
            T *= 1.0 - occ_cell(levels[0], dims[0], u);
        }
        sh[v] = T;
        lit[v] = ao[v] * (ambient + (1.0 - ambient) * T);
    }
}

/* ------------------------------------------------------------------ */
/* Primary rays (Section 3.5: one ray per pixel through its centre).     */

/* Camera basis in binary64, then rounded to binary32:
 *   f = normalize(target - eye), right = normalize(f x up), up' = right x f,
 *   R = right * tan(fovy/2) * W/H, U = up' * tan(fovy/2).
 * Per pixel in binary32 (row 0 at the top):
 *   u = 2(x + 0.5)/W - 1, v = 1 - 2(y + 0.5)/H, d = (f + u R) + v U, D = d/|d|. */
void orc_camera_consts(const float *eye, const float *target, const float *up, float fovy_deg, int32_t W,
                       int32_t H, float *F, float *R, float *U)
{
    double f[3], r[3], u[3], n;
    for (int c = 0; c < 3; c++) f[c] = (double)target[c] - (double)eye[c];
    n = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    for (int c = 0; c < 3; c++) f[c] = f[c] / n;
    double up0 = up[0], up1 = up[1], up2 = up[2];
    r[0] = f[1] * up2 - f[2] * up1;
    r[1] = f[2] * up0 - f[0] * up2;
    r[2] = f[0] * up1 - f[1] * up0;
    n = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (int c = 0; c < 3; c++) r[c] = r[c] / n;
    u[0] = r[1] * f[2] - r[2] * f[1];
    u[1] = r[2] * f[0] - r[0] * f[2];
    u[2] = r[0] * f[1] - r[1] * f[0];
    double th = tan((double)fovy_deg * M_PI / 360.0);
    double aspect = (double)W / (double)H;
    for (int c = 0; c < 3; c++) {
        F[c] = (float)f[c];
        R[c] = (float)(r[c] * (th * aspect));
        U[c] = (float)(u[c] * th);
    }
}

void orc_ray_dirs(const float *F, const float *R, const float *U, int32_t W, int32_t H, const int64_t *pix,
                  int64_t npix, float *dirs)
{
    for (int64_t k = 0; k < npix; k++) {
        int64_t px = pix[k] % W, py = pix[k] / W;
        float u = (2.0f * ((float)px + 0.5f)) / (float)W - 1.0f;
        float v = 1.0f - (2.0f * ((float)py + 0.5f)) / (float)H;
        float d[3];
        for (int c = 0; c < 3; c++) {
            float a = u * R[c];
            float b = v * U[c];
            d[c] = (F[c] + a) + b;
        }
        float ss = d[0] * d[0];
        ss = ss + d[1] * d[1];
        ss = ss + d[2] * d[2];
        float len = sqrtf(ss);
        for (int c = 0; c < 3; c++) dirs[3 * k + c] = d[c] / len;
    }
}

/* ------------------------------------------------------------------ */
/* Ray tracing (Section 3.5) in binary64.                                */

typedef struct {
    int hit;          /* 1 if the ray enters the capsule at t > 0 from outside */
    double t;         /* entry parameter (voxel units) */
    double P[3];      /* entry point */
    int accepted;     /* entry point on the kept side of both clip planes */
    double clip_margin;
    double miss_margin; /* | min distance(ray, segment) - r | */
    double t_near;      /* ray parameter of the closest approach */
} seg_hit;

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Closest approach between the ray O + tD (t >= 0, |D| = 1) and segment
 * A + h(B - A), h in [0, 1]: the squared distance is a convex quadratic in
 * (t, h), so its minimum over the half-strip is the stationary point when
 * feasible, else the clamped minimum along one of the three edges. */
static void ray_segment_closest(const double *O, const double *D, const double *A, const double *B,
                                double *dist, double *t_ray)
{
    double ba[3], oa[3];
    for (int c = 0; c < 3; c++) { ba[c] = B[c] - A[c]; oa[c] = O[c] - A[c]; }
    double a = dot3(ba, ba), b = dot3(ba, D), e = dot3(oa, D), f = dot3(oa, ba);
    double ct[4], ch[4];
    int nc = 0;
    double den = a - b * b;
    if (a > 0 && den > 0) { ct[nc] = (b * f - e * a) / den; ch[nc] = (f - b * e) / den; nc++; }
    ct[nc] = 0.0; ch[nc] = a > 0 ? f / a : 0.0; nc++;  /* edge t = 0 */
    ct[nc] = -e; ch[nc] = 0.0; nc++;                  /* edge h = 0 */
    ct[nc] = b - e; ch[nc] = 1.0; nc++;               /* edge h = 1 */
    double best = INFINITY, bt = 0.0;
    for (int k = 0; k < nc; k++) {
        double t = ct[k] < 0 ? 0.0 : ct[k];
        double h = ch[k] < 0 ? 0.0 : (ch[k] > 1 ? 1.0 : ch[k]);
        double w[3];
        for (int c = 0; c < 3; c++) w[c] = oa[c] + t * D[c] - h * ba[c];
        double dd = dot3(w, w);
        if (dd < best) { best = dd; bt = t; }
    }
    *dist = sqrt(best);
    *t_ray = bt;
}

/* Entry of the ray into the capsule {p : dist(p, AB) <= r}: the capsule is
 * the union of a finite cylinder and two balls, so its first point along the
 * ray is the earliest entry into any of the three.  The ray origin is moved
 * next to the segment first (binary64 stays accurate for far eyes). */
static void capsule_hit(const double *O, const double *D, const double *A, const double *B, const double *n0,
                        const double *n1, int a_int, int b_int, double r, seg_hit *H)
{
    H->hit = 0; H->accepted = 0; H->clip_margin = INFINITY;
    double dist, tn;
    ray_segment_closest(O, D, A, B, &dist, &tn);
    H->miss_margin = fabs(dist - r);
    H->t_near = tn;
    double oa0[3];
    for (int c = 0; c < 3; c++) oa0[c] = O[c] - A[c];
    double odist2;
    {   /* origin inside the capsule: no entry */
        double ba[3];
        for (int c = 0; c < 3; c++) ba[c] = B[c] - A[c];
        double baba = dot3(ba, ba), h = baba > 0 ? dot3(oa0, ba) / baba : 0.0;
        h = h < 0 ? 0 : (h > 1 ? 1 : h);
        double w[3];
        for (int c = 0; c < 3; c++) w[c] = oa0[c] - h * ba[c];
        odist2 = dot3(w, w);
        if (odist2 <= r * r) return;
    }
    double t0 = -dot3(oa0, D); /* rebase: parameter of the point nearest A */
    if (t0 < 0) t0 = 0;
    double Ob[3];
    for (int c = 0; c < 3; c++) Ob[c] = O[c] + t0 * D[c];
    double best = INFINITY;
    const double *ctr[2] = {A, B};
    for (int k = 0; k < 2; k++) {
        double oc[3];
        for (int c = 0; c < 3; c++) oc[c] = Ob[c] - ctr[k][c];
        double b = dot3(oc, D), cc = dot3(oc, oc) - r * r, disc = b * b - cc;
        if (disc >= 0) {
            double t = t0 + (-b - sqrt(disc));
            if (t > 0 && t < best) best = t;
        }
    }
    double ba[3], oa[3];
    for (int c = 0; c < 3; c++) { ba[c] = B[c] - A[c]; oa[c] = Ob[c] - A[c]; }
    double baba = dot3(ba, ba);
    if (baba > 0) {
        double dba = dot3(D, ba) / baba, oba = dot3(oa, ba) / baba, Dp[3], Op[3];
        for (int c = 0; c < 3; c++) { Dp[c] = D[c] - ba[c] * dba; Op[c] = oa[c] - ba[c] * oba; }
        double a = dot3(Dp, Dp), b = dot3(Dp, Op), cc = dot3(Op, Op) - r * r;
        if (a > 0) {
            double disc = b * b - a * cc;
            if (disc >= 0) {
                double s = (-b - sqrt(disc)) / a;
                double h = oba + s * dba;
                double t = t0 + s;
                if (t > 0 && h >= 0 && h <= 1 && t < best) best = t;
            }
        }
    }
    if (!(best < INFINITY)) return;
    H->hit = 1;
    H->t = best;
    for (int c = 0; c < 3; c++) H->P[c] = O[c] + best * D[c];
    int acc = 1;
    if (a_int) {
        double w[3];
        for (int c = 0; c < 3; c++) w[c] = H->P[c] - A[c];
        double s = dot3(w, n0);
        if (!(s >= 0)) acc = 0;
        if (fabs(s) < H->clip_margin) H->clip_margin = fabs(s);
    }
    if (b_int) {
        double w[3];
        for (int c = 0; c < 3; c++) w[c] = H->P[c] - B[c];
        double s = dot3(w, n1);
        if (!(s < 0)) acc = 0;
        if (fabs(s) < H->clip_margin) H->clip_margin = fabs(s);
    }
    H->accepted = acc;
}

/* Voxel containing a point, half-open in the direction of travel. */
static void voxel_of(const double *P, const double *D, int64_t *v)
{
    for (int c = 0; c < 3; c++) v[c] = D[c] < 0 ? (int64_t)ceil(P[c]) - 1 : (int64_t)floor(P[c]);
}

typedef struct {
    int32_t Gx, Gy, Gz;
    const int32_t *q;        /* quantized vertices */
    const float *nrm;        /* binary32 clip normals */
    const uint8_t *interior;
    const uint8_t *seg_valid;
    int64_t nv;
    double r;                /* radius, voxel units */
    const uint8_t *vis;      /* level-0 visibility (dense) */
    const uint32_t *words;
    const uint32_t *offsets; /* dense; list of v at [offsets[v], offsets[v] + count) */
    const uint32_t *ids;
    double O[3];             /* eye, voxel units */
    int mode;                /* 0 opaque, 1 transparent */
    double alpha, tau;       /* alpha: opacity of a hit on a segment without its own colour */
    const float *rgba;       /* NULL, or per segment s: colour and opacity at rgba[4 s .. 4 s + 3] */
    const double *lit;       /* NULL, or the voxel-space shading (dense): a hit's colour is scaled by the
                                value of the voxel holding its point (Section 3.4, one sample per hit) */
} trace_in;

typedef struct {
    int64_t id;
    double t;
    int64_t vox[3];
    int counted;
    double col[3];
    double alpha;   /* opacity of this hit when composited */
    double face_margin;
} acc_hit;

static int in_grid(const trace_in *T, const int64_t *v)
{
    return v[0] >= 0 && v[1] >= 0 && v[2] >= 0 && v[0] < T->Gx && v[1] < T->Gy && v[2] < T->Gz;
}

static int64_t dense(const trace_in *T, const int64_t *v) { return (v[2] * T->Gy + v[1]) * T->Gx + v[0]; }

static int list_has(const trace_in *T, int64_t v, int64_t id)
{
    int64_t lo = T->offsets[v], n = T->words[v] & 0xFFFFu, hi = lo + n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if ((int64_t)T->ids[mid] == id) return 1;
        if ((int64_t)T->ids[mid] < id) lo = mid + 1; else hi = mid - 1;
    }
    return 0;
}

/* counted: the hit lies in a visible voxel inside the grid */
static int counted_at(const trace_in *T, const int64_t *v) { return in_grid(T, v) && T->vis[dense(T, v)]; }

/* Smallest distance from P to a face of its voxel across which the
 * "counted and listed" status of segment id changes. */
static double face_margin(const trace_in *T, const double *P, const int64_t *v, int64_t id, int counted_here)
{
    double m = INFINITY;
    for (int a = 0; a < 3; a++)
        for (int s = -1; s <= 1; s += 2) {
            int64_t n[3] = {v[0], v[1], v[2]};
            n[a] += s;
            int cn = counted_at(T, n) && list_has(T, dense(T, n), id);
            if (cn == counted_here) continue;
            double dist = s < 0 ? P[a] - (double)v[a] : (double)(v[a] + 1) - P[a];
            if (dist < m) m = dist;
        }
    return m;
}

static int cmp_hit(const void *a, const void *b)
{
    const acc_hit *x = (const acc_hit *)a, *y = (const acc_hit *)b;
    if (x->t < y->t) return -1;
    if (x->t > y->t) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

typedef struct {
    acc_hit *h;
    int64_t n, cap;
} hitbuf;

static void hb_push(hitbuf *B, const acc_hit *x)
{
    if (B->n == B->cap) {
        B->cap = B->cap ? 2 * B->cap : 64;
        B->h = (acc_hit *)realloc(B->h, sizeof(acc_hit) * (size_t)B->cap);
    }
    B->h[B->n++] = *x;
}

/* open-addressing set of segment ids already evaluated for this ray */
typedef struct { int64_t *k; int64_t cap, n; } idset;

static int idset_add(idset *S, int64_t id)
{
    if (2 * (S->n + 1) > S->cap) {
        int64_t oc = S->cap, *ok = S->k;
        S->cap = oc ? 2 * oc : 256;
        S->k = (int64_t *)malloc(sizeof(int64_t) * (size_t)S->cap);
        for (int64_t i = 0; i < S->cap; i++) S->k[i] = -1;
        S->n = 0;
        for (int64_t i = 0; i < oc; i++)
            if (ok[i] >= 0) idset_add(S, ok[i]);
        free(ok);
    }
    uint64_t h = ((uint64_t)id * 0x9E3779B97F4A7C15ull) & (uint64_t)(S->cap - 1);
    while (S->k[h] >= 0) {
        if (S->k[h] == id) return 0;
        h = (h + 1) & (uint64_t)(S->cap - 1);
    }
    S->k[h] = id;
    S->n++;
    return 1;
}

/* Composites hits sorted by (t, id) front to back, each with its own
 * opacity a_k: C += T*a_k*c_k, T *= (1 - a_k), stopping before a hit once
 * T < tau.  Returns the number of hits composited. */
static int64_t composite(const acc_hit *h, int64_t n, double tau, double *rgba)
{
    double T = 1.0, C[3] = {0, 0, 0};
    int64_t k = 0;
    for (; k < n; k++) {
        if (T < tau) break;
        for (int c = 0; c < 3; c++) C[c] += T * h[k].alpha * h[k].col[c];
        T *= (1.0 - h[k].alpha);
    }
    rgba[0] = C[0]; rgba[1] = C[1]; rgba[2] = C[2]; rgba[3] = 1.0 - T;
    return k;
}

/* Number of the sorted hits composited before transmittance drops below tau. */
static int64_t layers_before_tau(const acc_hit *h, int64_t n, double tau)
{
    double T = 1.0;
    int64_t k = 0;
    while (k < n && !(T < tau)) { T *= (1.0 - h[k].alpha); k++; }
    return k;
}

static void segment_geom(const trace_in *T, int64_t s, double *A, double *B, double *n0, double *n1)
{
    for (int c = 0; c < 3; c++) {
        A[c] = T->q[3 * s + c] / (double)QS;
        B[c] = T->q[3 * (s + 1) + c] / (double)QS;
        n0[c] = T->nrm[3 * s + c];
        n1[c] = T->nrm[3 * (s + 1) + c];
    }
}

/* Colour and opacity of a hit on segment s: the caller's per-segment RGBA
 * (opacity clamped to [0, 1]), else the absolute unit tangent with the
 * default opacity. */
static void segment_colour(const trace_in *T, int64_t s, const double *A, const double *B, double *col,
                           double *alpha)
{
    if (T->rgba) {
        for (int c = 0; c < 3; c++) col[c] = (double)T->rgba[4 * s + c];
        double a = (double)T->rgba[4 * s + 3];
        *alpha = a < 0.0 ? 0.0 : (a > 1.0 ? 1.0 : a);
        return;
    }
    double d[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]}, n = sqrt(dot3(d, d));
    for (int c = 0; c < 3; c++) col[c] = n > 0 ? fabs(d[c]) / n : 0.0;
    *alpha = T->alpha;
}

typedef struct { double m, t; } near_rec; /* hit/miss or clip margin, at ray parameter t */

/* Two segments with the same quantized endpoints and the same clip planes are
 * the same capsule: every implementation computes the same hit parameter for
 * both, so their order is decided by the id rule alone, never by rounding.
 * Gaps between such hits are not ordering decisions. */
static int same_capsule(const trace_in *T, int64_t a, int64_t b)
{
    for (int c = 0; c < 6; c++)
        if (T->q[3 * a + c] != T->q[3 * b + c]) return 0;
    for (int e = 0; e < 2; e++) {
        if (T->interior[a + e] != T->interior[b + e]) return 0;
        for (int c = 0; c < 3; c++)
            if (T->nrm[3 * (a + e) + c] != T->nrm[3 * (b + e) + c]) return 0;
    }
    return 1;
}

/* Evaluates one candidate segment: records its entry hit (counted or not)
 * and the hit/miss and clip margins with the ray parameter they apply at. */
static void eval_candidate(const trace_in *T, const double *D, int64_t s, hitbuf *B, near_rec *nr)
{
    double A[3], Bv[3], n0[3], n1[3];
    segment_geom(T, s, A, Bv, n0, n1);
    seg_hit H;
    capsule_hit(T->O, D, A, Bv, n0, n1, T->interior[s], T->interior[s + 1], T->r, &H);
    nr->m = H.miss_margin;
    nr->t = H.t_near;
    if (!H.hit) return;
    if (H.clip_margin < nr->m) nr->m = H.clip_margin;
    acc_hit x;
    x.id = s;
    x.t = H.t;
    voxel_of(H.P, D, x.vox);
    segment_colour(T, s, A, Bv, x.col, &x.alpha);
    if (!H.accepted) return; /* a rejected entry never counts; its clip margin is in nr */
    x.counted = counted_at(T, x.vox);
    if (T->lit && x.counted)
        for (int c = 0; c < 3; c++) x.col[c] *= T->lit[dense(T, x.vox)];
    x.face_margin = face_margin(T, H.P, x.vox, s, x.counted);
    hb_push(B, &x);
}

/* Parameter up to which the result is decided by the counted hits so far:
 * opaque, the first counted hit; transparent, the first hit that is no
 * longer composited. */
static double result_extent(const trace_in *T, const hitbuf *B)
{
    acc_hit *c = (acc_hit *)malloc(sizeof(acc_hit) * (size_t)(B->n + 1));
    int64_t n = 0;
    for (int64_t k = 0; k < B->n; k++)
        if (B->h[k].counted) c[n++] = B->h[k];
    double ext = INFINITY;
    if (n > 0) {
        qsort(c, (size_t)n, sizeof(acc_hit), cmp_hit);
        if (T->mode == 0) ext = c[0].t;
        else {
            int64_t k = layers_before_tau(c, n, T->tau);
            if (k < n) ext = c[k].t;
        }
    }
    free(c);
    return ext;
}

/* Traces one ray.  Candidates are the lists of the visible voxels the ray
 * walks through (binary64 Amanatides-Woo); by conservative voxelization
 * every counted hit -- an accepted entry whose point lies in a visible
 * voxel -- is among them.  The walk ends two voxels past the parameter at
 * which the result is decided.  brute != 0 takes every segment instead.
 * Margins (voxel units):
 *   m_geom: the smallest hit/miss, clip-plane or ordering margin of any
 *           decision that can change the result;
 *   m_face: the smallest distance of a relevant hit point to a face of its
 *           voxel across which its counted/listed status changes. */
static void trace_one(const trace_in *T, const double *D, int brute, int64_t *out_id, double *out_t,
                      double *rgba, double *m_geom, double *m_face, int64_t *n_comp)
{
    hitbuf B = {0};
    idset S = {0};
    near_rec *nr = NULL;
    int64_t nnr = 0, capnr = 0;
#define EVAL(sid)                                                                   \
    do {                                                                            \
        if (nnr == capnr) {                                                         \
            capnr = capnr ? 2 * capnr : 256;                                        \
            nr = (near_rec *)realloc(nr, sizeof(near_rec) * (size_t)capnr);         \
        }                                                                           \
        eval_candidate(T, D, (sid), &B, &nr[nnr]);                                  \
        nnr++;                                                                      \
    } while (0)

    if (brute) {
        for (int64_t s = 0; s + 1 < T->nv; s++)
            if (T->seg_valid[s]) EVAL(s);
    } else {
        double G[3] = {T->Gx, T->Gy, T->Gz}, tin = 0.0, tout = INFINITY;
        int ok = 1;
        for (int a = 0; a < 3; a++) {
            if (D[a] == 0.0) {
                if (T->O[a] < 0 || T->O[a] > G[a]) ok = 0;
                continue;
            }
            double t1 = (0.0 - T->O[a]) / D[a], t2 = (G[a] - T->O[a]) / D[a];
            if (t1 > t2) { double tmp = t1; t1 = t2; t2 = tmp; }
            if (t1 > tin) tin = t1;
            if (t2 < tout) tout = t2;
        }
        if (ok && tin < tout) {
            int64_t v[3], step[3];
            double tnext[3];
            for (int a = 0; a < 3; a++) {
                double p = T->O[a] + tin * D[a];
                v[a] = (int64_t)floor(p);
                if (D[a] < 0 && p == floor(p)) v[a] -= 1;
                if (v[a] < 0) v[a] = 0;
                if (v[a] >= (int64_t)G[a]) v[a] = (int64_t)G[a] - 1;
                step[a] = D[a] > 0 ? 1 : (D[a] < 0 ? -1 : 0);
                tnext[a] = step[a] == 0 ? INFINITY : ((double)(v[a] + (step[a] > 0)) - T->O[a]) / D[a];
            }
            double tcur = tin, tstop = INFINITY;
            for (;;) {
                int64_t dv = dense(T, v);
                uint32_t n = T->words[dv] & 0xFFFFu;
                if (T->vis[dv] && n) {
                    int64_t o = T->offsets[dv], before = B.n;
                    for (int64_t k = 0; k < (int64_t)n; k++)
                        if (idset_add(&S, T->ids[o + k])) EVAL((int64_t)T->ids[o + k]);
                    if (B.n > before) tstop = result_extent(T, &B);
                }
                int a = 0;
                for (int c = 1; c < 3; c++)
                    if (tnext[c] < tnext[a]) a = c;
                double tn = tnext[a];
                if (!(tn < tout)) break;
                v[a] += step[a];
                if (v[a] < 0 || v[a] >= (int64_t)G[a]) break;
                tnext[a] = ((double)(v[a] + (step[a] > 0)) - T->O[a]) / D[a];
                tcur = tn;
                if (tcur > tstop + 2.0) break;
            }
        }
    }
#undef EVAL
    /* counted hits in (t, id) order */
    acc_hit *cnt = (acc_hit *)malloc(sizeof(acc_hit) * (size_t)(B.n + 1));
    int64_t nc = 0;
    for (int64_t k = 0; k < B.n; k++)
        if (B.h[k].counted) cnt[nc++] = B.h[k];
    qsort(cnt, (size_t)nc, sizeof(acc_hit), cmp_hit);

    double t_rel;
    rgba[0] = rgba[1] = rgba[2] = rgba[3] = 0.0;
    *m_geom = INFINITY;
    *m_face = INFINITY;
    *out_id = nc > 0 ? cnt[0].id : -1;
    *out_t = nc > 0 ? cnt[0].t : INFINITY;
    if (T->mode == 0) {
        if (nc > 0) {
            rgba[0] = cnt[0].col[0]; rgba[1] = cnt[0].col[1]; rgba[2] = cnt[0].col[2]; rgba[3] = 1.0;
            for (int64_t k = 1; k < nc; k++)
                if (!same_capsule(T, cnt[k].id, cnt[0].id)) { *m_geom = cnt[k].t - cnt[0].t; break; }
            *n_comp = 1;
        } else {
            *n_comp = 0;
        }
        t_rel = *out_t;
    } else {
        int64_t k = composite(cnt, nc, T->tau, rgba);
        *n_comp = k;
        t_rel = (k < nc) ? cnt[k].t : INFINITY;
        for (int64_t i = 0; i + 1 < nc && i < k; i++) {
            if (same_capsule(T, cnt[i + 1].id, cnt[i].id)) continue;
            double g = cnt[i + 1].t - cnt[i].t;
            if (g < *m_geom) *m_geom = g;
        }
    }
    for (int64_t k = 0; k < nnr; k++)
        if (nr[k].t <= t_rel + T->r + 1e-3 && nr[k].m < *m_geom) *m_geom = nr[k].m;
    for (int64_t k = 0; k < B.n; k++) {
        if (B.h[k].t > t_rel + 1e-3) continue;
        if (B.h[k].face_margin < *m_face) *m_face = B.h[k].face_margin;
    }
    free(cnt);
    free(nr);
    free(S.k);
    free(B.h);
}

/* The paper's per-voxel rule (Section 3.5): walk the voxels front to back;
 * in each visible voxel test its list and keep only hits whose point lies in
 * that voxel; opaque rays stop after the first voxel with a hit.  Used to
 * check that lists are conservative enough for the rule to reach the
 * brute-force result (no margins are computed). */
static void trace_invoxel(const trace_in *T, const double *D, int64_t *out_id, double *out_t, double *rgba,
                          int64_t *n_comp)
{
    hitbuf B = {0};
    double G[3] = {T->Gx, T->Gy, T->Gz}, tin = 0.0, tout = INFINITY;
    int ok = 1;
    for (int a = 0; a < 3; a++) {
        if (D[a] == 0.0) {
            if (T->O[a] < 0 || T->O[a] > G[a]) ok = 0;
            continue;
        }
        double t1 = (0.0 - T->O[a]) / D[a], t2 = (G[a] - T->O[a]) / D[a];
        if (t1 > t2) { double tmp = t1; t1 = t2; t2 = tmp; }
        if (t1 > tin) tin = t1;
        if (t2 < tout) tout = t2;
    }
    int64_t done = 0;
    if (ok && tin < tout) {
        int64_t v[3], step[3];
        double tnext[3];
        for (int a = 0; a < 3; a++) {
            double p = T->O[a] + tin * D[a];
            v[a] = (int64_t)floor(p);
            if (D[a] < 0 && p == floor(p)) v[a] -= 1;
            if (v[a] < 0) v[a] = 0;
            if (v[a] >= (int64_t)G[a]) v[a] = (int64_t)G[a] - 1;
            step[a] = D[a] > 0 ? 1 : (D[a] < 0 ? -1 : 0);
            tnext[a] = step[a] == 0 ? INFINITY : ((double)(v[a] + (step[a] > 0)) - T->O[a]) / D[a];
        }
        for (;;) {
            int64_t dv = dense(T, v);
            uint32_t n = T->words[dv] & 0xFFFFu;
            int64_t before = B.n;
            if (T->vis[dv] && n) {
                for (int64_t k = 0; k < (int64_t)n; k++) {
                    int64_t s = T->ids[T->offsets[dv] + k];
                    double A[3], Bv[3], n0[3], n1[3];
                    segment_geom(T, s, A, Bv, n0, n1);
                    seg_hit H;
                    capsule_hit(T->O, D, A, Bv, n0, n1, T->interior[s], T->interior[s + 1], T->r, &H);
                    if (!H.hit || !H.accepted) continue;
                    int64_t pv[3];
                    voxel_of(H.P, D, pv);
                    if (pv[0] != v[0] || pv[1] != v[1] || pv[2] != v[2]) continue;
                    acc_hit x;
                    x.id = s; x.t = H.t; x.counted = 1; x.face_margin = INFINITY;
                    x.vox[0] = v[0]; x.vox[1] = v[1]; x.vox[2] = v[2];
                    segment_colour(T, s, A, Bv, x.col, &x.alpha);
                    if (T->lit)
                        for (int c = 0; c < 3; c++) x.col[c] *= T->lit[dense(T, v)];
                    hb_push(&B, &x);
                }
                if (B.n > before) qsort(B.h + before, (size_t)(B.n - before), sizeof(acc_hit), cmp_hit);
            }
            if (T->mode == 0 && B.n > 0) break;
            if (T->mode == 1 && layers_before_tau(B.h, B.n, T->tau) < B.n) break;
            int a = 0;
            for (int c = 1; c < 3; c++)
                if (tnext[c] < tnext[a]) a = c;
            if (!(tnext[a] < tout)) break;
            v[a] += step[a];
            if (v[a] < 0 || v[a] >= (int64_t)G[a]) break;
            tnext[a] = ((double)(v[a] + (step[a] > 0)) - T->O[a]) / D[a];
        }
    }
    (void)done;
    rgba[0] = rgba[1] = rgba[2] = rgba[3] = 0.0;
    *out_id = B.n > 0 ? B.h[0].id : -1;
    *out_t = B.n > 0 ? B.h[0].t : INFINITY;
    if (T->mode == 0) {
        if (B.n > 0) { rgba[0] = B.h[0].col[0]; rgba[1] = B.h[0].col[1]; rgba[2] = B.h[0].col[2]; rgba[3] = 1.0; }
        *n_comp = B.n > 0;
    } else {
        *n_comp = composite(B.h, B.n, T->tau, rgba);
    }
    free(B.h);
}

/* Traces the given pixels.  Outputs per pixel: first counted segment id (-1
 * if none), its parameter t (voxel units), RGBA (opaque: colour of the first
 * hit with alpha 1; transparent: premultiplied composite, A = 1 - T), the
 * two certification margins and the number of composited hits.
 * method 0: the definition over the candidates the lists supply (with
 *           margins); 1: every segment (tiny inputs only); 2: the per-voxel
 *           rule over the lists (no margins). */
void orc_trace(int32_t Gx, int32_t Gy, int32_t Gz, const int32_t *q, const float *nrm, const uint8_t *interior,
               const uint8_t *seg_valid, int64_t nv, int64_t rq, const uint8_t *vis, const uint32_t *words,
               const uint32_t *offsets, const uint32_t *ids, const int64_t *eye_q, const float *dirs,
               int64_t npix, int mode, double alpha, double tau, const float *seg_rgba, const double *lit, int brute,
               int64_t *out_id, double *out_t, double *out_rgba, double *m_geom, double *m_face, int64_t *n_comp)
{
    trace_in T;
    T.Gx = Gx; T.Gy = Gy; T.Gz = Gz;
    T.q = q; T.nrm = nrm; T.interior = interior; T.seg_valid = seg_valid; T.nv = nv;
    T.r = (double)rq / QS;
    T.vis = vis; T.words = words; T.offsets = offsets; T.ids = ids;
    for (int c = 0; c < 3; c++) T.O[c] = (double)eye_q[c] / QS;
    T.mode = mode; T.alpha = alpha; T.tau = tau; T.rgba = seg_rgba; T.lit = lit;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t k = 0; k < npix; k++) {
        double D[3] = {dirs[3 * k], dirs[3 * k + 1], dirs[3 * k + 2]};
        if (brute == 2) {
            trace_invoxel(&T, D, &out_id[k], &out_t[k], &out_rgba[4 * k], &n_comp[k]);
            m_geom[k] = m_face[k] = INFINITY;
        } else {
            trace_one(&T, D, brute, &out_id[k], &out_t[k], &out_rgba[4 * k], &m_geom[k], &m_face[k], &n_comp[k]);
        }
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
