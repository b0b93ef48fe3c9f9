/*
 * CPU oracle on all host cores -- TEST INFRASTRUCTURE ONLY, timing build.
 *
 * The paper's node layer (Sec. 2.1) compresses the blocks a node owns with
 * OpenMP threads, each thread taking whole blocks.  These routines do the
 * same with the oracle's own block-range routines, unchanged: an OpenMP
 * parallel-for over chunks of consecutive blocks, each chunk handled by
 * czo_compress_blocks / czo_decompress_blocks exactly as one thread would.
 * Records land at record-bound strides as in those routines, so the output
 * equals that of a single call over the whole range (tests check this).
 * Linked with cz_oracle.c into its own library; used only to time the
 * benchmark's CPU baseline on all cores.
 */
#include <omp.h>
#include <stddef.h>
#include <stdint.h>

int czo_compress_blocks_f32(uint32_t nx, uint32_t ny, uint32_t nz, int N, int scheme, double eps, const float *field,
                            uint64_t b0, uint64_t b1, uint8_t *recs, uint64_t *rec_bytes);
int czo_compress_blocks_f64(uint32_t nx, uint32_t ny, uint32_t nz, int N, int scheme, double eps, const double *field,
                            uint64_t b0, uint64_t b1, uint8_t *recs, uint64_t *rec_bytes);
int czo_decompress_blocks_f32(uint32_t nx, uint32_t ny, uint32_t nz, int N, int scheme, const uint8_t *recs,
                              const uint64_t *rec_bytes, uint64_t b0, uint64_t b1, float *field);
int czo_decompress_blocks_f64(uint32_t nx, uint32_t ny, uint32_t nz, int N, int scheme, const uint8_t *recs,
                              const uint64_t *rec_bytes, uint64_t b0, uint64_t b1, double *field);

/* Blocks a thread takes at a time. */
#define CZO_PAR_CHUNK 4

static size_t rec_stride(int N, size_t elem)
{
    size_t n3 = (size_t)N * N * N;
    return (8 + n3 / 8 + n3 * elem + 15) & ~(size_t)15;
}

int czo_par_max_threads(void) { return omp_get_max_threads(); }

#define CZO_PAR(SFX, T)                                                                                             \
    int czo_compress_blocks_par_##SFX(uint32_t nx, uint32_t ny, uint32_t nz, int N, int scheme, double eps,      \
                                      const T *field, uint64_t b0, uint64_t b1, uint8_t *recs,                    \
                                      uint64_t *rec_bytes, int threads)                                          \
    {                                                                                                              \
        const size_t rb = rec_stride(N, sizeof(T));                                                                \
        const int64_t nchunks = (int64_t)((b1 - b0 + CZO_PAR_CHUNK - 1) / CZO_PAR_CHUNK);                         \
        int rc = 0;                                                                                                \
        _Pragma("omp parallel for schedule(dynamic, 1) num_threads(threads)")                                      \
        for (int64_t c = 0; c < nchunks; c++) {                                                                    \
            const uint64_t lo = b0 + (uint64_t)c * CZO_PAR_CHUNK;                                                  \
            const uint64_t hi = lo + CZO_PAR_CHUNK < b1 ? lo + CZO_PAR_CHUNK : b1;                                 \
            const int r = czo_compress_blocks_##SFX(nx, ny, nz, N, scheme, eps, field, lo, hi,                     \
                                                    recs + (lo - b0) * rb, rec_bytes + (lo - b0));                 \
            if (r != 0) {                                                                                          \
                _Pragma("omp atomic write") rc = r;                                                                \
            }                                                                                                      \
        }                                                                                                          \
        return rc;                                                                                                 \
    }                                                                                                              \
    int czo_decompress_blocks_par_##SFX(uint32_t nx, uint32_t ny, uint32_t nz, int N, int scheme,                \
                                        const uint8_t *recs, const uint64_t *rec_bytes, uint64_t b0, uint64_t b1, \
                                        T *field, int threads)                                                    \
    {                                                                                                              \
        const size_t rb = rec_stride(N, sizeof(T));                                                                \
        const int64_t nchunks = (int64_t)((b1 - b0 + CZO_PAR_CHUNK - 1) / CZO_PAR_CHUNK);                         \
        int rc = 0;                                                                                                \
        _Pragma("omp parallel for schedule(dynamic, 1) num_threads(threads)")                                      \
        for (int64_t c = 0; c < nchunks; c++) {                                                                    \
            const uint64_t lo = b0 + (uint64_t)c * CZO_PAR_CHUNK;                                                  \
            const uint64_t hi = lo + CZO_PAR_CHUNK < b1 ? lo + CZO_PAR_CHUNK : b1;                                 \
            const int r = czo_decompress_blocks_##SFX(nx, ny, nz, N, scheme, recs + (lo - b0) * rb,                \
                                                      rec_bytes + (lo - b0), lo, hi, field);                       \
            if (r != 0) {                                                                                          \
                _Pragma("omp atomic write") rc = r;                                                                \
            }                                                                                                      \
        }                                                                                                          \
        return rc;                                                                                                 \
    }

CZO_PAR(f32, float)
CZO_PAR(f64, double)
