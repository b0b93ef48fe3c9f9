/*
 * CPU oracle, precision-generic part (TEST INFRASTRUCTURE ONLY).
 * Included twice by cz_oracle.c with T = float and T = double; SFX(name)
 * appends the precision suffix.  Every operation is rounded in T.
 */

/* ((w0 x0 + w1 x1) + w2 x2) + ... : left to right, each step rounded in T. */
static T SFX(dot)(const double *w, const T *x, int k)
{
    T acc = (T)w[0] * x[0];
    for (int j = 1; j < k; j++)
        acc = acc + (T)w[j] * x[j];
    return acc;
}

/* W4 prediction of odd sample m from the evens e[0..h). */
static T SFX(w4_pred)(const T *e, int h, int m)
{
    double w[4];
    int s = w4_stencil(h, m, w);
    return SFX(dot)(w, e + s, 4);
}

/* W4_li update of even k: u_k = sum over m ascending of U_km d_m with
 * U = P~^T / 2, P~ the centred four-point predict (nodes m-1..m+2), taken over
 * the existing details m and evens k only (see w4_centred_weight). */
static T SFX(w4_update)(const T *d, int h, int k)
{
    T acc = 0;
    int first = 1;
    for (int m = 0; m < h; m++) {
        double w = w4_centred_weight(m, k);
        if (w == 0.0)
            continue;
        T term = (T)(0.5 * w) * d[m];
        if (first) {
            acc = term;
            first = 0;
        } else {
            acc = acc + term;
        }
    }
    return acc;
}

/* W3_ai prediction of the left child of coarse cell k from C[0..h). */
static T SFX(w3_pred)(const T *C, int h, int k)
{
    double w[3];
    int s = w3_stencil(h, k, w);
    return SFX(dot)(w, C + s, 3);
}

/* One forward level along a line of length n (even, >= 8):
 * out[0..h) = coarse, out[h..n) = details. */
void SFX(czo_fwd1)(int scheme, int n, const T *v, T *out)
{
    int h = n / 2;
    T a[CZO_MAXN / 2], d[CZO_MAXN / 2];
    if (scheme == CZO_W3AI) {
        for (int k = 0; k < h; k++)
            a[k] = (v[2 * k] + v[2 * k + 1]) * (T)0.5;
        for (int k = 0; k < h; k++)
            d[k] = v[2 * k] - SFX(w3_pred)(a, h, k);
    } else {
        T o[CZO_MAXN / 2];
        for (int k = 0; k < h; k++) {
            a[k] = v[2 * k];
            o[k] = v[2 * k + 1];
        }
        for (int m = 0; m < h; m++)
            d[m] = o[m] - SFX(w4_pred)(a, h, m);
        if (scheme == CZO_W4LI) {
            T s[CZO_MAXN / 2];
            for (int k = 0; k < h; k++)
                s[k] = a[k] + SFX(w4_update)(d, h, k);
            memcpy(a, s, sizeof(T) * h);
        }
    }
    memcpy(out, a, sizeof(T) * h);
    memcpy(out + h, d, sizeof(T) * h);
}

/* One inverse level: w = [coarse | details] -> line v of length n. */
void SFX(czo_inv1)(int scheme, int n, const T *w, T *v)
{
    int h = n / 2;
    const T *d = w + h;
    if (scheme == CZO_W3AI) {
        const T *C = w;
        for (int k = 0; k < h; k++) {
            T a = SFX(w3_pred)(C, h, k) + d[k];
            v[2 * k] = a;
            v[2 * k + 1] = (C[k] + C[k]) - a;
        }
        return;
    }
    T e[CZO_MAXN / 2];
    for (int k = 0; k < h; k++)
        e[k] = scheme == CZO_W4LI ? w[k] - SFX(w4_update)(d, h, k) : w[k];
    for (int k = 0; k < h; k++)
        v[2 * k] = e[k];
    for (int m = 0; m < h; m++)
        v[2 * m + 1] = d[m] + SFX(w4_pred)(e, h, m);
}

/* Full-depth 1D transform of a line of length n: levels n, n/2, ..., 8. */
void SFX(czo_fwd_line)(int scheme, int n, T *v)
{
    T out[CZO_MAXN];
    for (int len = n; len >= 8; len /= 2) {
        SFX(czo_fwd1)(scheme, len, v, out);
        memcpy(v, out, sizeof(T) * len);
    }
}

void SFX(czo_inv_line)(int scheme, int n, T *v)
{
    T out[CZO_MAXN];
    for (int len = 8; len <= n; len *= 2) {
        SFX(czo_inv1)(scheme, len, v, out);
        memcpy(v, out, sizeof(T) * len);
    }
}

/* Apply one level (fwd or inv) along axis (0 = x, 1 = y, 2 = z) to every line
 * of the region [0,n)^3 of the N^3 block B (q = x + N (y + N z)). */
static void SFX(axis_pass)(int scheme, int inverse, int axis, int N, int n, T *B)
{
    const size_t stride[3] = {1, (size_t)N, (size_t)N * N};
    size_t sa = stride[axis], s1 = stride[axis == 0 ? 1 : 0], s2 = stride[axis == 2 ? 1 : 2];
    T line[CZO_MAXN], out[CZO_MAXN];
    for (int j = 0; j < n; j++) {
        for (int i = 0; i < n; i++) {
            T *base = B + i * s1 + j * s2;
            for (int t = 0; t < n; t++)
                line[t] = base[t * sa];
            if (inverse)
                SFX(czo_inv1)(scheme, n, line, out);
            else
                SFX(czo_fwd1)(scheme, n, line, out);
            for (int t = 0; t < n; t++)
                base[t * sa] = out[t];
        }
    }
}

/* Forward 3D multilevel transform of one N^3 block, in place. */
void SFX(czo_fwd_block)(int scheme, int N, T *B)
{
    for (int n = N; n >= 8; n /= 2) {
        SFX(axis_pass)(scheme, 0, 0, N, n, B);
        SFX(axis_pass)(scheme, 0, 1, N, n, B);
        SFX(axis_pass)(scheme, 0, 2, N, n, B);
    }
}

/* Inverse 3D multilevel transform of one N^3 block, in place. */
void SFX(czo_inv_block)(int scheme, int N, T *B)
{
    for (int n = 8; n <= N; n *= 2) {
        SFX(axis_pass)(scheme, 1, 2, N, n, B);
        SFX(axis_pass)(scheme, 1, 1, N, n, B);
        SFX(axis_pass)(scheme, 1, 0, N, n, B);
    }
}

/* Decimate the transformed block C and write its record at rec (which must
 * have room for the largest record).  Returns the record size in bytes. */
static size_t SFX(pack_block)(int N, double eps, const T *C, uint8_t *rec)
{
    size_t n3 = (size_t)N * N * N;
    uint8_t *mask = rec + 8;
    T *vals = (T *)(void *)(mask + n3 / 8);
    memset(mask, 0, n3 / 8);
    uint32_t nnz = 0;
    for (size_t q = 0; q < n3; q++) {
        size_t x = q % N, y = (q / N) % N, z = q / ((size_t)N * N);
        int coarse = x < 4 && y < 4 && z < 4;
        if (coarse || fabs((double)C[q]) >= eps) {
            mask[q >> 3] |= (uint8_t)(1u << (q & 7));
            memcpy(&vals[nnz], &C[q], sizeof(T));
            nnz++;
        }
    }
    put_u32(rec, nnz);
    put_u32(rec + 4, 0);
    size_t used = 8 + n3 / 8 + (size_t)nnz * sizeof(T);
    size_t total = roundup16(used);
    memset(rec + used, 0, total - used);
    return total;
}

/* Block (bx, by, bz) of the field <-> the N^3 block array B. */
static void SFX(gather_block)(const T *field, uint32_t nx, uint32_t ny, int N, uint32_t bx, uint32_t by,
                              uint32_t bz, T *B)
{
    for (int z = 0; z < N; z++)
        for (int y = 0; y < N; y++)
            for (int x = 0; x < N; x++) {
                size_t g = ((size_t)(bz * N + z) * ny + (by * N + y)) * nx + (bx * N + x);
                B[x + N * (y + N * z)] = field[g];
            }
}

static void SFX(scatter_block)(const T *B, uint32_t nx, uint32_t ny, int N, uint32_t bx, uint32_t by,
                               uint32_t bz, T *field)
{
    for (int z = 0; z < N; z++)
        for (int y = 0; y < N; y++)
            for (int x = 0; x < N; x++) {
                size_t g = ((size_t)(bz * N + z) * ny + (by * N + y)) * nx + (bx * N + x);
                field[g] = B[x + N * (y + N * z)];
            }
}

static int SFX(all_finite)(const T *B, size_t n)
{
    for (size_t i = 0; i < n; i++)
        if (!isfinite(B[i]))
            return 0;
    return 1;
}

/* Compress an nx*ny*nz field (x fastest) into the stream at out.  Blocks are
 * visited in order b = bx + nbx (by + nby bz).  On success *out_bytes holds
 * the stream size; on CZO_ERR_CAPACITY it holds the size required. */
int SFX(czo_compress)(uint32_t nx, uint32_t ny, uint32_t nz, int N, int scheme, double eps,
                      const T *field, uint8_t *out, size_t cap, size_t *out_bytes)
{
    if (!out || !out_bytes || scheme < 0 || scheme > 2 || !(eps >= 0.0) || isinf(eps))
        return CZO_ERR_ARG;
    if (!valid_block(N) || nx % N || ny % N || nz % N)
        return CZO_ERR_SHAPE;
    uint32_t nbx = nx / N, nby = ny / N, nbz = nz / N;
    uint64_t nb = (uint64_t)nbx * nby * nbz;
    if (!field && nb)
        return CZO_ERR_ARG;
    size_t bound = czo_compress_bound(nx, ny, nz, N, (int)sizeof(T));
    if (cap < bound) {
        *out_bytes = bound;
        return CZO_ERR_CAPACITY;
    }
    size_t n3 = (size_t)N * N * N, p0 = payload_start(nb);
    T *B = (T *)malloc(sizeof(T) * n3);
    if (!B)
        return CZO_ERR_ARG;
    memset(out, 0, p0);
    int rc = CZO_OK;
    uint64_t off = 0;
    for (uint64_t b = 0; b < nb && rc == CZO_OK; b++) {
        uint32_t bx = (uint32_t)(b % nbx), by = (uint32_t)((b / nbx) % nby), bz = (uint32_t)(b / ((uint64_t)nbx * nby));
        SFX(gather_block)(field, nx, ny, N, bx, by, bz, B);
        if (!SFX(all_finite)(B, n3)) {
            rc = CZO_ERR_NONFINITE;
            break;
        }
        SFX(czo_fwd_block)(scheme, N, B);
        if (!SFX(all_finite)(B, n3)) {
            rc = CZO_ERR_NONFINITE;
            break;
        }
        off += SFX(pack_block)(N, eps, B, out + p0 + off);
        put_u64(out + CZO_HDR + 8 * (b + 1), off);
    }
    free(B);
    if (rc != CZO_OK)
        return rc;
    memcpy(out, "CZB1", 4);
    put_u32(out + 4, 1);
    put_u32(out + 8, (uint32_t)scheme);
    put_u32(out + 12, (uint32_t)sizeof(T));
    put_u32(out + 16, (uint32_t)N);
    put_u32(out + 20, (uint32_t)(ilog2(N) - 2));
    put_u32(out + 24, nx);
    put_u32(out + 28, ny);
    put_u32(out + 32, nz);
    put_u32(out + 36, 0);
    memcpy(out + 40, &eps, 8);
    put_u64(out + 48, nb);
    put_u64(out + 56, off);
    *out_bytes = p0 + off;
    return CZO_OK;
}

/* Unpack record rec (size rec_bytes) into the coefficient block B: kept
 * coefficients from the value stream in ascending q, dropped ones +0. */
static int SFX(unpack_record)(const uint8_t *rec, uint64_t rec_bytes, int N, T *B)
{
    size_t n3 = (size_t)N * N * N;
    if (rec_bytes < 8 + n3 / 8)
        return CZO_ERR_FORMAT;
    uint32_t nnz = get_u32(rec);
    if (nnz > n3 || roundup16(8 + n3 / 8 + (size_t)nnz * sizeof(T)) != rec_bytes)
        return CZO_ERR_FORMAT;
    const uint8_t *mask = rec + 8, *vals = mask + n3 / 8;
    uint32_t r = 0;
    for (size_t q = 0; q < n3; q++) {
        if (mask[q >> 3] >> (q & 7) & 1u) {
            if (r >= nnz)
                return CZO_ERR_FORMAT;
            memcpy(&B[q], vals + (size_t)r * sizeof(T), sizeof(T));
            r++;
        } else {
            B[q] = (T)0;
        }
    }
    return r == nnz ? CZO_OK : CZO_ERR_FORMAT;
}

/* Rebuild the field from a stream.  field_cap is in elements. */
int SFX(czo_decompress)(const uint8_t *in, size_t in_bytes, T *field, size_t field_cap)
{
    if (!in || in_bytes < CZO_HDR)
        return CZO_ERR_FORMAT;
    if (memcmp(in, "CZB1", 4) != 0 || get_u32(in + 4) != 1)
        return CZO_ERR_FORMAT;
    int scheme = (int)get_u32(in + 8), elem = (int)get_u32(in + 12), N = (int)get_u32(in + 16);
    uint32_t levels = get_u32(in + 20), nx = get_u32(in + 24), ny = get_u32(in + 28), nz = get_u32(in + 32);
    uint64_t nb = get_u64(in + 48), payload = get_u64(in + 56);
    if (scheme < 0 || scheme > 2 || elem != (int)sizeof(T) || !valid_block(N) || levels != (uint32_t)(ilog2(N) - 2))
        return CZO_ERR_FORMAT;
    if (nx % N || ny % N || nz % N)
        return CZO_ERR_FORMAT;
    uint32_t nbx = nx / N, nby = ny / N, nbz = nz / N;
    if (nb != (uint64_t)nbx * nby * nbz)
        return CZO_ERR_FORMAT;
    size_t p0 = payload_start(nb);
    if (p0 > in_bytes || payload > in_bytes - p0)
        return CZO_ERR_FORMAT;
    if (get_u64(in + CZO_HDR) != 0 || get_u64(in + CZO_HDR + 8 * nb) != payload)
        return CZO_ERR_FORMAT;
    if (!field && nb)
        return CZO_ERR_ARG;
    if (field_cap < (size_t)nx * ny * nz)
        return CZO_ERR_CAPACITY;
    T *B = (T *)malloc(sizeof(T) * (size_t)N * N * N);
    if (!B)
        return CZO_ERR_ARG;
    int rc = CZO_OK;
    for (uint64_t b = 0; b < nb && rc == CZO_OK; b++) {
        uint64_t o0 = get_u64(in + CZO_HDR + 8 * b), o1 = get_u64(in + CZO_HDR + 8 * (b + 1));
        if (o1 < o0 || o1 > payload) {
            rc = CZO_ERR_FORMAT;
            break;
        }
        rc = SFX(unpack_record)(in + p0 + o0, o1 - o0, N, B);
        if (rc != CZO_OK)
            break;
        SFX(czo_inv_block)(scheme, N, B);
        uint32_t bx = (uint32_t)(b % nbx), by = (uint32_t)((b / nbx) % nby), bz = (uint32_t)(b / ((uint64_t)nbx * nby));
        SFX(scatter_block)(B, nx, ny, N, bx, by, bz, field);
    }
    free(B);
    return rc;
}

/* Forward transform + decimation of blocks [b0, b1) only, each record written
 * to recs + (b - b0) * record_bound (used to time or sample a subset of a
 * large field).  rec_bytes[b - b0] receives each record's size. */
int SFX(czo_compress_blocks)(uint32_t nx, uint32_t ny, uint32_t nz, int N, int scheme, double eps,
                             const T *field, uint64_t b0, uint64_t b1, uint8_t *recs, uint64_t *rec_bytes)
{
    if (!valid_block(N) || nx % N || ny % N || nz % N)
        return CZO_ERR_SHAPE;
    uint32_t nbx = nx / N, nby = ny / N;
    size_t n3 = (size_t)N * N * N, rb = record_bound(N, (int)sizeof(T));
    T *B = (T *)malloc(sizeof(T) * n3);
    if (!B)
        return CZO_ERR_ARG;
    int rc = CZO_OK;
    for (uint64_t b = b0; b < b1; b++) {
        uint32_t bx = (uint32_t)(b % nbx), by = (uint32_t)((b / nbx) % nby), bz = (uint32_t)(b / ((uint64_t)nbx * nby));
        SFX(gather_block)(field, nx, ny, N, bx, by, bz, B);
        SFX(czo_fwd_block)(scheme, N, B);
        if (!SFX(all_finite)(B, n3))
            rc = CZO_ERR_NONFINITE;
        rec_bytes[b - b0] = SFX(pack_block)(N, eps, B, recs + (b - b0) * rb);
    }
    free(B);
    return rc;
}

/* Inverse of czo_compress_blocks: decode records laid out at record_bound
 * strides and write blocks [b0, b1) of the field. */
int SFX(czo_decompress_blocks)(uint32_t nx, uint32_t ny, uint32_t nz, int N, int scheme, const uint8_t *recs,
                               const uint64_t *rec_bytes, uint64_t b0, uint64_t b1, T *field)
{
    if (!valid_block(N) || nx % N || ny % N || nz % N)
        return CZO_ERR_SHAPE;
    uint32_t nbx = nx / N, nby = ny / N;
    size_t n3 = (size_t)N * N * N, rb = record_bound(N, (int)sizeof(T));
    T *B = (T *)malloc(sizeof(T) * n3);
    if (!B)
        return CZO_ERR_ARG;
    int rc = CZO_OK;
    for (uint64_t b = b0; b < b1 && rc == CZO_OK; b++) {
        rc = SFX(unpack_record)(recs + (b - b0) * rb, rec_bytes[b - b0], N, B);
        if (rc != CZO_OK)
            break;
        SFX(czo_inv_block)(scheme, N, B);
        uint32_t bx = (uint32_t)(b % nbx), by = (uint32_t)((b / nbx) % nby), bz = (uint32_t)(b / ((uint64_t)nbx * nby));
        SFX(scatter_block)(B, nx, ny, N, bx, by, bz, field);
    }
    free(B);
    return rc;
}
