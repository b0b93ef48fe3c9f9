/*
 * CubismZ wavelet stage -- CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, single-threaded, slow and
 * obviously-correct statement of what the GPU path computes.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it; the
 * product library never does, and the two share no code, header or table.
 *
 * Paper: Hadjidoukas & Wermelinger, "A Parallel Data Compression Framework for
 * Large Scale 3D Scientific Data" (CubismZ), arXiv 1903.07761.
 *   Sec. 2.2  one quantity at a time; the grid block is the unit of work.
 *   Sec. 2.3  "Wavelet-based compression": per-block forward wavelet transform
 *             with filters "on the interval" (blocks are independent),
 *             decimation of detail coefficients at a threshold eps, output =
 *             bit-set mask + stream of significant coefficients.
 *   Sec. 2.3  "Wavelet types": fourth-order interpolating (W4), its lifted
 *             form (W4_li) and third-order average-interpolating (W3_ai).
 *   Sec. 2.3  "Data decompression": block-level inverse transform.
 *   Sec. 3    Eq. (1): PSNR.
 *
 * The paper names the schemes but not their stencils, boundary rules, depth,
 * coefficient order or mask layout.  The readings taken here:
 *   - W4: an odd sample is predicted by the cubic through the four nearest
 *     existing even samples of the line (Donoho's interpolating transform; on
 *     the interval the window is one-sided at the ends, and the last odd
 *     sample is extrapolated).  Detail = odd - prediction, coarse = even.
 *   - W4_li: the W4 predict, then a lifting update s = e + U d (Sweldens'
 *     lifting): U = P~^T / 2 with P~ the centred four-point predict, i.e.
 *     the update (-1, 9, 9, -1)/32 over d_k-2 .. d_k+1, keeping the terms
 *     whose detail exists.  (Transposing the one-sided boundary rows instead
 *     would give a coarse operator I - P^T P / 2 of spectral radius ~4.9:
 *     coarse values would grow ~5x per axis and level, against the paper's
 *     aim for this scheme of smaller errors than W4.)
 *   - W3_ai: values are cell averages; coarse = mean of a pair; detail = left
 *     child - the average over the left half-cell of the quadratic whose
 *     averages over the three nearest existing coarse cells match (Donoho's
 *     average-interpolation).  The right child's residual is -detail.
 *   - 3D: separable, level by level: at size n the x-lines, then the y-lines,
 *     then the z-lines of the region [0,n)^3 are transformed, each writing
 *     coarse to [0,n/2) and details to [n/2,n) (Mallat layout); n runs
 *     N, N/2, ..., 8, leaving a 4^3 coarse corner.  The inverse runs n =
 *     8..N, z then y then x.
 *   - Decimation after the whole forward transform: keep q if q lies in the
 *     4^3 coarse corner or (double)|c_q| >= eps.
 *   - Arithmetic in the field precision T, IEEE round-to-nearest, no fused
 *     multiply-add, every weighted sum formed left to right in ascending
 *     source index starting from its first term.  All weights are dyadic
 *     rationals and are derived below from their definitions in double, which
 *     holds them exactly.
 *
 * Stream (little-endian): 64-byte header; (nblocks+1) u64 record offsets
 * relative to the payload; zero pad to a 16-byte boundary; per block in block
 * order a record = u32 nnz, u32 flags (0), N^3/8 mask bytes (bit q = bit q&7
 * of byte q>>3), nnz values of type T in ascending q, zero pad to 16 bytes.
 */
#include <math.h>
#include <stdlib.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>

#define CZO_W4 0
#define CZO_W4LI 1
#define CZO_W3AI 2

#define CZO_OK 0
#define CZO_ERR_ARG (-1)
#define CZO_ERR_SHAPE (-2)
#define CZO_ERR_CAPACITY (-3)
#define CZO_ERR_NONFINITE (-4)
#define CZO_ERR_FORMAT (-5)

#define CZO_MAXN 64
#define CZO_HDR 64

/* ---------------------------------------------------------------- weights */

/* Lagrange basis polynomial j of the nodes x[0..k) evaluated at t. */
static double lagrange(const double *x, int k, int j, double t)
{
    double num = 1.0, den = 1.0;
    for (int i = 0; i < k; i++) {
        if (i == j)
            continue;
        num *= t - x[i];
        den *= x[j] - x[i];
    }
    return num / den;
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* W4 / W4_li predict of odd sample m on a line with h even samples.  Even
 * sample k sits at coarse coordinate k, odd sample m at m + 1/2.  The cubic
 * goes through the four nearest existing evens s..s+3.  Returns s. */
static int w4_stencil(int h, int m, double w[4])
{
    int s = clampi(m - 1, 0, h - 4);
    double x[4] = {s, s + 1, s + 2, s + 3};
    for (int j = 0; j < 4; j++)
        w[j] = lagrange(x, 4, j, m + 0.5);
    return s;
}

/* Weight that the centred four-point predict of odd sample m (cubic through
 * the evens m-1, m, m+1, m+2, wherever those lie) gives to even k; 0 when k is
 * not one of them.  In the interior this is the W4 predict itself. */
static double w4_centred_weight(int m, int k)
{
    int s = m - 1;
    if (k < s || k > s + 3)
        return 0.0;
    double x[4] = {s, s + 1, s + 2, s + 3};
    return lagrange(x, 4, k - s, m + 0.5);
}

/* W3_ai predict of the left child of coarse cell k (cell k = [k, k+1] in
 * coarse units).  The quadratic q has averages C_s, C_s+1, C_s+2 over the
 * three nearest existing cells; its primitive F is the cubic through the
 * cumulative sums F(s+j) = C_s + ... + C_s+j-1 at the cell edges.  The left
 * child is the average of q over [k, k+1/2]:
 *     2 (F(k + 1/2) - F(k)) = sum_i w_i C_s+i
 * with w_i = 2 (sum_{j>i} L_j(k + 1/2) - [edge s+i+1 <= k]).  Returns s. */
static int w3_stencil(int h, int k, double w[3])
{
    int s = clampi(k - 1, 0, h - 3);
    double x[4] = {s, s + 1, s + 2, s + 3};
    double L[4];
    for (int j = 0; j < 4; j++)
        L[j] = lagrange(x, 4, j, k + 0.5);
    for (int i = 0; i < 3; i++) {
        double tail = 0.0;
        for (int j = i + 1; j < 4; j++)
            tail += L[j];
        double below = (s + i + 1 <= k) ? 1.0 : 0.0;
        w[i] = 2.0 * (tail - below);
    }
    return s;
}

static int ilog2(int n)
{
    int l = 0;
    while ((1 << l) < n)
        l++;
    return l;
}

static int valid_block(int N) { return N == 8 || N == 16 || N == 32 || N == 64; }

static size_t roundup16(size_t v) { return (v + 15u) & ~(size_t)15u; }

static void put_u32(uint8_t *p, uint32_t v) { memcpy(p, &v, 4); }
static void put_u64(uint8_t *p, uint64_t v) { memcpy(p, &v, 8); }
static uint32_t get_u32(const uint8_t *p) { uint32_t v; memcpy(&v, p, 4); return v; }
static uint64_t get_u64(const uint8_t *p) { uint64_t v; memcpy(&v, p, 8); return v; }

/* Payload start: header + (nblocks+1) offsets, rounded up to 16 bytes. */
static size_t payload_start(uint64_t nblocks) { return roundup16(CZO_HDR + 8u * (nblocks + 1u)); }

/* Largest record: every coefficient kept. */
static size_t record_bound(int N, int elem)
{
    size_t n3 = (size_t)N * N * N;
    return roundup16(8u + n3 / 8u + n3 * (size_t)elem);
}

size_t czo_compress_bound(uint32_t nx, uint32_t ny, uint32_t nz, int N, int elem)
{
    if (!valid_block(N) || (elem != 4 && elem != 8) || nx % N || ny % N || nz % N)
        return 0;
    uint64_t nb = (uint64_t)(nx / N) * (ny / N) * (nz / N);
    return payload_start(nb) + nb * record_bound(N, elem);
}

/* Eq. (1): PSNR = 20 log10((max_R - min_R) / (2 sqrt(MSE))), MSE in double.
 * Returns +inf when MSE is 0. */
double czo_psnr(const void *ref, const void *dec, size_t count, int elem)
{
    double lo = INFINITY, hi = -INFINITY, sse = 0.0;
    for (size_t i = 0; i < count; i++) {
        double r = elem == 4 ? (double)((const float *)ref)[i] : ((const double *)ref)[i];
        double d = elem == 4 ? (double)((const float *)dec)[i] : ((const double *)dec)[i];
        if (r < lo)
            lo = r;
        if (r > hi)
            hi = r;
        sse += (r - d) * (r - d);
    }
    double mse = sse / (double)count;
    if (mse == 0.0)
        return INFINITY;
    return 20.0 * log10((hi - lo) / (2.0 * sqrt(mse)));
}

/* ------------------------------------------------- precision instantiation */

#define T float
#define SFX(name) name##_f32
#include "cz_oracle_t.h"
#undef T
#undef SFX

#define T double
#define SFX(name) name##_f64
#include "cz_oracle_t.h"
#undef T
#undef SFX
