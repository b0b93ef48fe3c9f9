/*
 * cz.h -- C ABI of the CubismZ wavelet stage on MI355X (gfx950).
 *
 * The operation (Hadjidoukas & Wermelinger, arXiv 1903.07761):
 *   Sec. 2.1-2.2  the field is one scalar quantity on a grid of equal cubic
 *                 blocks of power-of-two edge N; blocks are the unit of work.
 *   Sec. 2.3      "Wavelet-based compression": per block, a 3D forward wavelet
 *                 transform with filters on the interval (no data from
 *                 neighbouring blocks), then decimation of the detail
 *                 coefficients below eps, output = bit-set mask + stream of
 *                 significant coefficients.  "Wavelet types": W4 (fourth-order
 *                 interpolating), W4_li (its lifted form), W3_ai (third-order
 *                 average-interpolating).
 *   Sec. 2.3      "Data decompression": block-level inverse transform.
 *   Sec. 2.2      the exclusive prefix scan of compressed sizes that places
 *                 each piece in the output.
 *
 * Stream format (little-endian), produced by cz_compress, consumed by
 * cz_decompress:
 *   [0, 64)      header: char magic[4] = "CZB1"; u32 version = 1, scheme,
 *                elem_bytes, N, levels = log2(N) - 2, nx, ny, nz, reserved = 0;
 *                f64 epsilon; u64 nblocks; u64 payload_bytes
 *   [64, ...)    (nblocks + 1) u64 record offsets relative to the payload,
 *                off[0] = 0, off[b+1] = off[b] + record_bytes(b)
 *   pad          zeros up to payload start P = roundup16(64 + 8 (nblocks + 1))
 *   P + off[b]   record of block b = bx + nbx (by + nby bz):
 *                  u32 nnz (kept coefficients, the 64 coarse ones included),
 *                  u32 flags = 0,
 *                  N^3 / 8 mask bytes: bit q (q = x + N (y + N z), Mallat
 *                  layout) is bit (q & 7) of byte (q >> 3),
 *                  nnz values of the field type in ascending q,
 *                  zero padding to a multiple of 16 bytes.
 *   total bytes  P + off[nblocks]
 *
 * The transform (all arithmetic in the field precision, no fused
 * multiply-add, weighted sums left to right in ascending source index):
 *   one level of a line of n samples -> [n/2 coarse | n/2 details]:
 *     W4    detail m = odd m - cubic through the four nearest existing evens
 *           at m + 1/2; coarse = evens.
 *     W4_li W4, then coarse k += sum over details m = k-2..k+1 (those that
 *           exist) of (-1, 9, 9, -1)/32 d_m.
 *     W3_ai coarse k = (v[2k] + v[2k+1]) / 2; detail k = v[2k] - the average
 *           over [k, k+1/2] of the quadratic matching the three nearest
 *           existing coarse averages.
 *   3D: for n = N, N/2, ..., 8: x-lines, then y-lines, then z-lines of
 *   [0,n)^3; inverse for n = 8..N: z, y, x.  Decimation keeps q when q lies
 *   in the 4^3 coarse corner or (double)|c_q| >= eps; dropped values decode
 *   as +0.0.
 *
 * Blocks up to 32^3 stay on chip (VGPRs + LDS); 64^3 blocks (1 MiB float,
 * 2 MiB double) are staged in per-workgroup scratch slots the context owns
 * (two per workgroup: one block is transformed while the previous one waits
 * for its offset).
 *
 * Conventions.  Every pointer named d_* is device memory of the context's
 * device, owned by the caller; the library keeps none of them after a call
 * returns, and never allocates on the compress/decompress paths once the
 * context's workspace is large enough (cz_reserve).  Calls are ordered on the
 * given HIP stream (hipStream_t passed as void*; NULL = the null stream).  A
 * context's workspace is shared by its calls: calls on one context must not
 * overlap in time (issue them on one stream, or synchronise between them).
 * All functions return 0 (CZ_OK) or a negative CZ_ERR_* code; nothing throws.
 */
#ifndef CZ_H
#define CZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { CZ_W4 = 0, CZ_W4_LI = 1, CZ_W3_AI = 2 };

enum {
    CZ_OK = 0,
    CZ_ERR_ARG = -1,       /* null pointer, bad enum, eps < 0 or non-finite   */
    CZ_ERR_SHAPE = -2,     /* N not in {8,16,32,64}, an edge not a multiple,  */
                           /* or a grid too large for 32-bit block addressing */
    CZ_ERR_CAPACITY = -3,  /* output buffer too small (required size returned) */
    CZ_ERR_NONFINITE = -4, /* non-finite input or coefficient; output undefined */
    CZ_ERR_FORMAT = -5,    /* corrupt or inconsistent stream                   */
    CZ_ERR_HIP = -6,       /* HIP runtime failure                              */
    CZ_ERR_BUDGET = -7,    /* request larger than a server's memory budget     */
    CZ_ERR_TIMEOUT = -8,   /* a device-side wait exceeded its bound             */
    CZ_ERR_SCRATCH = -9    /* beyond the fixed scratch of cz_compress_noalloc   */
};

typedef struct {
    uint32_t nx, ny, nz;  /* grid edges, x fastest in memory (C order [z][y][x]) */
    uint32_t block;       /* N in {8, 16, 32, 64}; every edge a multiple of N    */
    uint32_t scheme;      /* CZ_W4 | CZ_W4_LI | CZ_W3_AI                          */
    uint32_t elem_bytes;  /* 4 (float) or 8 (double)                              */
    double epsilon;       /* absolute decimation threshold, finite and >= 0      */
} cz_params;

typedef struct cz_ctx cz_ctx;

/* Create a context on HIP device `device` (allocates a small workspace and a
 * pinned status word).  Returns CZ_ERR_HIP if the device is unusable. */
int cz_create(cz_ctx **out, int device);
void cz_destroy(cz_ctx *ctx);

/* Grow the context's workspace so that fields of up to max_blocks blocks need
 * no allocation later: the look-back flags (8 bytes a block) and the slots in
 * which single-field compression of 32^3 blocks parks records of at most
 * 8 KiB until their offsets are known (8 KiB + 4 bytes a block).  64^3 blocks
 * also need scratch slots sized by the launch, not by the field (up to about
 * 1 GiB for double data), which the first call with N = 64 allocates.
 * Optional: compress/decompress grow the workspace on demand. */
int cz_reserve(cz_ctx *ctx, uint64_t max_blocks);

/* Worst-case stream size (every coefficient kept) for params p, or 0 when p
 * is invalid.  = P + nblocks * roundup16(8 + N^3/8 + N^3 elem_bytes). */
size_t cz_compress_bound(const cz_params *p);

/* Compress the device field d_field (nx*ny*nz elements, [z][y][x]) into the
 * stream at d_out (capacity out_cap bytes, >= cz_compress_bound or
 * CZ_ERR_CAPACITY with the bound written to *h_out_bytes when non-null).
 * Synchronous when h_out_bytes != NULL: waits for the stream and returns the
 * stream size and any device-detected error (CZ_ERR_NONFINITE,
 * CZ_ERR_TIMEOUT), which is then cleared.  Otherwise fully asynchronous: the size is written to the
 * device u64 *d_out_bytes (if non-null) and device errors are read with
 * cz_get_status before the context's next call. */
int cz_compress(cz_ctx *ctx, const cz_params *p, const void *d_field, void *d_out, size_t out_cap,
                uint64_t *d_out_bytes, size_t *h_out_bytes, void *stream);

/* In-situ extraction (Sec. 2.1: the compressor takes the quantity of
 * interest out of the solver's blocks, whose cells hold all quantities):
 * compress quantity `comp` of an interleaved state d_state, a C-order
 * [nz][ny][nx][ncomp] array of the field type (cell (x, y, z) holds its
 * ncomp quantities contiguously).  The blocks are read with strided loads
 * straight from the state; the stream is byte-identical to cz_compress of the
 * extracted field.  Other arguments and returns as cz_compress; CZ_ERR_ARG for
 * comp >= ncomp, CZ_ERR_SHAPE when a block row of the state spans 2^31 bytes
 * or more. */
int cz_compress_strided(cz_ctx *ctx, const cz_params *p, const void *d_state, uint32_t ncomp, uint32_t comp,
                        void *d_out, size_t out_cap, uint64_t *d_out_bytes, size_t *h_out_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): cz_compress
 * with no allocation of any kind.  The call's scratch -- its ticket, status
 * and size words, its descriptor and one look-back flag per block -- lives in
 * a fixed array in the library's device code (one copy per device, held until
 * the process ends, located once per device by cz_create), never in the
 * context's growable workspace.  Limits: N <= 32 and at most
 * CZ_NOALLOC_MAX_BLOCKS blocks; anything larger returns CZ_ERR_SCRATCH before
 * any work is issued (use cz_compress there).  Arguments, stream contents and
 * the other returns are exactly those of cz_compress.  Synchronous when
 * h_out_bytes != NULL (size and device error returned); otherwise the size
 * goes to *d_out_bytes and the call's device error is folded into the
 * context's status word, read with cz_get_status.  Every call on one device
 * shares that device's array and starts by clearing it (with a kernel, not a
 * memset): two calls that overlap in time on one device race, whatever their
 * contexts or streams. */
#define CZ_NOALLOC_MAX_BLOCKS 1048576u /* 2^20 blocks: 8 MiB of flags */
int cz_compress_noalloc(cz_ctx *ctx, const cz_params *p, const void *d_field, void *d_out, size_t out_cap,
                        uint64_t *d_out_bytes, size_t *h_out_bytes, void *stream);

/* Rebuild the field from the stream d_in (in_bytes long) into d_field
 * (field_cap bytes).  With expected == NULL the 64-byte header is read back
 * (synchronous), and the call waits for completion and returns (and clears)
 * any device-detected error (CZ_ERR_FORMAT for an inconsistent record; such
 * blocks are left unwritten).  With
 * expected != NULL (it must match the header) the call is asynchronous and
 * device errors are read with cz_get_status. */
int cz_decompress(cz_ctx *ctx, const cz_params *expected, const void *d_in, size_t in_bytes, void *d_field,
                  size_t field_cap, void *stream);

/* Wait for `stream`, then return and clear the error latched by the
 * context's asynchronous calls (CZ_OK if none). */
int cz_get_status(cz_ctx *ctx, void *stream);

/* Parse a host copy of a stream header (n >= 64 bytes). */
int cz_read_header(const void *h_hdr, size_t n, cz_params *out, uint64_t *nblocks, uint64_t *total_bytes);

const char *cz_strerror(int code);

/* ------------------------------------------------------------ kernel tuning
 *
 * Each (N, precision) has one or more register/LDS tilings of the same
 * transform (how many z-columns a thread owns, how many planes stay in LDS);
 * every variant yields byte-identical streams and fields.  cz_variant_count
 * returns how many exist (0 for an unsupported pair); cz_set_variant selects
 * one for later calls of ctx on (block, elem_bytes, scheme) (default 0).
 * Returns CZ_ERR_ARG for an unknown variant. */
int cz_variant_count(uint32_t block, uint32_t elem_bytes);
int cz_set_variant(cz_ctx *ctx, uint32_t block, uint32_t elem_bytes, uint32_t scheme, int variant);

/* ------------------------------------------------------------------ batches
 *
 * Several independent fields (Sec. 2.2: each quantity of a time step is
 * compressed on its own) in one call.  Fields are grouped by (N, precision,
 * scheme, variant); each group runs as one launch that pulls blocks of all its
 * fields from a device work queue, and the groups run concurrently on streams
 * forked from `stream` and joined back to it.  Every output is byte-identical
 * to the single-field call with the same parameters.
 *
 * cz_compress_batch: field i (params ps[i], device d_fields[i]) -> stream at
 * d_outs[i] of capacity caps[i] (>= cz_compress_bound(&ps[i]), else
 * CZ_ERR_CAPACITY and, when h_out_bytes != NULL, the bound in h_out_bytes[i]).
 * Sizes go to the device array d_out_bytes[n] (if non-null) and, when
 * h_out_bytes != NULL, to h_out_bytes[n] after waiting (synchronous; device
 * errors are returned and cleared as for cz_compress).  Otherwise the call is
 * asynchronous and errors are read with cz_get_status.
 *
 * cz_decompress_batch: stream i (d_ins[i], in_bytes[i] = its total size, its
 * header matching ps[i]) -> field d_fields[i] of capacity caps[i] bytes.
 * Asynchronous; device errors (CZ_ERR_FORMAT, ...) via cz_get_status.
 *
 * At most 24 groups per call; the host arrays are read before the call
 * returns.  The pointer arrays are host memory, the pointers in them device
 * memory. */
int cz_compress_batch(cz_ctx *ctx, int n, const cz_params *ps, const void *const *d_fields, void *const *d_outs,
                      const size_t *caps, uint64_t *d_out_bytes, size_t *h_out_bytes, void *stream);
int cz_decompress_batch(cz_ctx *ctx, int n, const cz_params *ps, const void *const *d_ins, const size_t *in_bytes,
                        void *const *d_fields, const size_t *caps, void *stream);

/* ------------------------------------------------------------ captured plans
 *
 * A plan fixes the parameters of a batch (op 0 = compress, 1 = decompress) and
 * owns its workspace; its first run records the batch's launches into a HIP
 * graph (descriptor upload, per-group kernels on forked streams, status fold,
 * size readback) and every later run replays it with new buffers, so a
 * repeated batch costs one graph launch.  cz_plan_run takes the same buffer
 * arrays as the batch calls (src_bytes: stream sizes for op 1, ignored for
 * op 0) and is asynchronous; cz_plan_result waits for `stream` and returns the
 * run's error (cleared) and, for op 0, the stream sizes in h_out_bytes[n].
 * A plan shares the status word of its context: runs of plans of one context
 * must not overlap with each other or with the context's other calls. */
typedef struct cz_plan cz_plan;
int cz_plan_create(cz_ctx *ctx, int op, int n, const cz_params *ps, cz_plan **out);
int cz_plan_run(cz_plan *plan, const void *const *srcs, const size_t *src_bytes, void *const *dsts,
                const size_t *dst_caps, void *stream);
int cz_plan_result(cz_plan *plan, void *stream, size_t *h_out_bytes);
void cz_plan_destroy(cz_plan *plan);

/* ---------------------------------------------- lossless-stage preconditioning
 *
 * Sec. 2.3 ("Lossless compression", "Wavelet types") and Sec. 4.1 (Exp. 2):
 * before the lossless coder the aggregate stream may be byte-shuffled, and the
 * low bits of the detail coefficients zeroed (Z4 / Z8).
 *
 * cz_shuffle: byte j of element i of d_in (elem = 4 or 8 bytes, n = nbytes /
 * elem whole elements) goes to d_out[j * n + i]; the nbytes % elem tail bytes
 * are copied to the end unchanged.  cz_unshuffle is its inverse.  d_in (for
 * cz_shuffle) or d_out (for cz_unshuffle) must be elem-aligned; the buffers
 * must not overlap.  Asynchronous on `stream`; CZ_ERR_ARG on bad arguments.
 *
 * cz_zero_details: in place, clear the `bits` least significant bits of every
 * stored detail coefficient of the stream d_stream (nbytes long, made with
 * parameters p): every value outside the 4^3 coarse corner.  Keep decisions
 * are unchanged (the stream was decimated with the exact coefficients); only
 * values change, by less than 2^bits units in the last place.  bits <= 23
 * (float) or 52 (double), else CZ_ERR_ARG.  Asynchronous; a record
 * inconsistent with the offsets is left alone and CZ_ERR_FORMAT is latched
 * for cz_get_status. */
int cz_shuffle(const void *d_in, size_t nbytes, uint32_t elem, void *d_out, void *stream);
int cz_unshuffle(const void *d_in, size_t nbytes, uint32_t elem, void *d_out, void *stream);
int cz_zero_details(cz_ctx *ctx, const cz_params *p, void *d_stream, size_t nbytes, uint32_t bits, void *stream);

/* -------------------------------------------------------- GPU lossless stage
 *
 * Sec. 2.2-2.3: the second substage is a general-purpose lossless coder over
 * the (optionally shuffled) output of the first.  This one runs on the GPU: a
 * byte-oriented canonical Huffman code with lengths limited to 12 bits
 * (package-merge over the byte histogram), over chunks of 4 KiB of input
 * that decode independently.  Container "CZH1" (little-endian): 32-byte
 * header {magic, u32 version 1, u64 raw bytes, u32 chunk bytes 4096,
 * u32 chunks, u32 max length 12, u32 0}, 256 code lengths (u8), (chunks + 1)
 * u64 chunk offsets relative to the payload, zero pad to 16 bytes, then each
 * chunk's codes, bit-reversed and least significant bit first in little-endian
 * 32-bit words, padded to a whole word.
 *
 * cz_huff_bound: worst-case container size for nbytes of input.
 * cz_huff_encode: encode d_in[0, nbytes) into d_out (8-byte aligned, capacity out_cap >=
 * cz_huff_bound, else CZ_ERR_CAPACITY with the bound in *h_out_bytes);
 * synchronous (the code is built on the host from the histogram): returns
 * the container size in *h_out_bytes.
 * cz_huff_decode: decode the container d_in (16-byte aligned, in_bytes long) into d_out
 * (4-byte aligned, out_cap >= raw bytes); reads the header synchronously,
 * then asynchronous; a corrupt chunk latches CZ_ERR_FORMAT for
 * cz_get_status.  Both use the context's workspace. */
size_t cz_huff_bound(size_t nbytes);
int cz_huff_encode(cz_ctx *ctx, const void *d_in, size_t nbytes, void *d_out, size_t out_cap, size_t *h_out_bytes,
                   void *stream);
int cz_huff_decode(cz_ctx *ctx, const void *d_in, size_t in_bytes, void *d_out, size_t out_cap, void *stream);

/* ------------------------------------------------------------ random access
 *
 * Sec. 2.3 ("Data decompression"): decompression works block by block; a
 * reader fetches only the records it needs through the offsets table and
 * keeps recently decoded blocks in a cache.  Decoding uses the same inverse
 * kernels, so every decoded block is bit-identical to the same block of a
 * full cz_decompress.
 *
 * cz_decompress_blocks: decode the blocks h_blocks[0, n) (host array of block
 * indices b = bx + nbx (by + nby bz), each < nblocks) of the stream d_in
 * (in_bytes long, made with parameters p) into d_out: block k lands dense,
 * [z][y][x] with x fastest, at element offset k N^3.  out_cap >= n N^3
 * elem_bytes (else CZ_ERR_CAPACITY).  Asynchronous; a record inconsistent
 * with the offsets is left unwritten and CZ_ERR_FORMAT latched for
 * cz_get_status.  Uses the context's workspace like cz_decompress.
 *
 * cz_cache: a device pool of capacity_blocks decoded N^3 blocks of one stream
 * (parameters p), least recently used replacement.  cz_cache_fetch makes the
 * blocks h_blocks[0, n) resident (n <= capacity; repeated blocks allowed),
 * decoding only those not already in the pool, and returns in h_ptrs[i] the
 * device address of block h_blocks[i] (dense [z][y][x]); the addresses stay
 * valid until a later fetch evicts them.  Passing another stream buffer or
 * size empties the pool first.  cz_cache_region decodes (through the pool)
 * the box origin[0..2] (x, y, z) + [0, extent) of the field into d_out
 * ([ez][ey][ex], x fastest); the blocks it touches must fit the pool.
 * cz_cache_stats returns the requested blocks served from the pool (hits) and
 * decoded (misses).  A cache uses its context's work queue: its calls must
 * not overlap with the context's other calls. */
int cz_decompress_blocks(cz_ctx *ctx, const cz_params *p, const void *d_in, size_t in_bytes, const uint32_t *h_blocks,
                         size_t n, void *d_out, size_t out_cap, void *stream);
typedef struct cz_cache cz_cache;
int cz_cache_create(cz_ctx *ctx, const cz_params *p, size_t capacity_blocks, cz_cache **out);
int cz_cache_fetch(cz_cache *c, const void *d_in, size_t in_bytes, const uint32_t *h_blocks, size_t n,
                   void **h_ptrs, void *stream);
int cz_cache_region(cz_cache *c, const void *d_in, size_t in_bytes, const uint32_t origin[3], const uint32_t extent[3],
                    void *d_out, size_t out_cap, void *stream);
int cz_cache_stats(cz_cache *c, uint64_t *hits, uint64_t *misses);
void cz_cache_destroy(cz_cache *c);

/* ------------------------------------------------------------------ serving
 *
 * A scheduler for a stream of independent requests (the in-situ use of
 * Sec. 1-2: each quantity is handed over as the simulation produces it).  A
 * worker thread admits requests from an arrival FIFO, strictly in order, while
 * the admitted-but-unfinished requests number at most max_inflight and their
 * device footprint (compress: raw field + cz_compress_bound; decompress:
 * src_bytes + raw field) stays within hbm_budget_bytes, and launches whatever
 * it admitted at once as one batch (grouped by kernel class as in
 * cz_compress_batch), with up to four batches in flight.  Outputs are
 * byte-identical to the single-field calls.
 *
 * The caller owns every buffer; a request's source must be complete (its
 * producing stream synchronised) before cz_submit, and its buffers must stay
 * valid until it is done.  The server keeps its own device workspace; the
 * context's variant table must not change while the server runs.  Times are
 * seconds on the server's monotonic clock (cz_server_time), from its start. */
typedef struct cz_server cz_server;

typedef struct {
    int op;              /* 0 = compress, 1 = decompress                        */
    cz_params p;         /* decompress: the parameters the stream was made with */
    const void *d_src;   /* compress: the field; decompress: the stream         */
    size_t src_bytes;    /* decompress: stream size (ignored for compress)      */
    void *d_dst;         /* compress: stream buffer; decompress: the field      */
    size_t dst_cap;      /* capacity of d_dst in bytes                          */
    uint64_t user_tag;   /* returned untouched                                  */
} cz_request;

/* Start a server on ctx's device.  CZ_ERR_ARG for max_inflight < 1 or a zero
 * budget. */
int cz_server_start(cz_ctx *ctx, size_t hbm_budget_bytes, int max_inflight, cz_server **out);

/* Queue a request (non-blocking).  Validation errors (CZ_ERR_ARG, _SHAPE,
 * _CAPACITY, _FORMAT) and CZ_ERR_BUDGET (footprint above the budget) are
 * returned at once and nothing is queued; otherwise *ticket identifies it. */
int cz_submit(cz_server *s, const cz_request *r, uint64_t *ticket);

/* State of a request: *done = 1 once finished, with its CZ_* status, the
 * stream size (compress) and its arrival, admission and completion times
 * (-1 until they happen).  Any output pointer but done may be NULL. */
int cz_poll(cz_server *s, uint64_t ticket, int *done, int *status, size_t *out_bytes, double *t_arrive,
            double *t_admit, double *t_done);

/* Block until the request is done; returns its status. */
int cz_wait(cz_server *s, uint64_t ticket);

/* Seconds since the server started, on the clock of cz_poll's times. */
double cz_server_time(cz_server *s);

/* Finish every queued request, stop the worker and free the server.
 * Returns CZ_ERR_HIP if the device failed while serving, else CZ_OK. */
int cz_server_stop(cz_server *s);

#ifdef __cplusplus
}
#endif

#endif /* CZ_H */
