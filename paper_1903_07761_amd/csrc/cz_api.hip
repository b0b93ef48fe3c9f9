// Host side of the C ABI declared in include/cz.h: parameter validation,
// stream layout arithmetic, workspace ownership and kernel launches.
//
// The problem statement (arXiv 1903.07761, Sec. 2.1-2.3): a grid of equal
// cubic blocks of power-of-two edge, one scalar quantity at a time, a wavelet
// scheme, a precision and a decimation threshold.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "../../include/cz.h"
#include "cz_kernels.h"

struct cz_ctx {
    int device = 0;
    int num_cu = 0;
    czk::CzWork *work = nullptr;  // device: ticket, status, total
    uint64_t *flags = nullptr;    // device: look-back flags
    uint64_t cap_blocks = 0;
    czk::CzWork *pinned = nullptr;  // host-pinned mirror of *work for sync reads
    void *scratch = nullptr;        // N = 64 blocks: one slot per resident workgroup
    size_t scratch_bytes = 0;
};

namespace {

constexpr uint32_t MAGIC = 0x31425A43u;  // "CZB1" little-endian
constexpr uint64_t MAX_BLOCKS = 1ull << 31;
constexpr uint64_t HDR = 64;

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess)
            prev = -1;
        if (prev != dev)
            (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev)
            (void)hipSetDevice(prev);
    }
};

uint64_t roundup16(uint64_t v) { return (v + 15u) & ~uint64_t(15); }

int ilog2(uint32_t n)
{
    int l = 0;
    while ((1u << l) < n)
        ++l;
    return l;
}

bool supported_block(uint32_t n) { return n == 8 || n == 16 || n == 32 || n == 64; }

// Shared validation of a parameter block; fills nblocks on success.
int check_params(const cz_params *p, uint64_t *nblocks)
{
    if (!p)
        return CZ_ERR_ARG;
    if (p->scheme > 2 || (p->elem_bytes != 4 && p->elem_bytes != 8))
        return CZ_ERR_ARG;
    if (!(p->epsilon >= 0.0) || !std::isfinite(p->epsilon))
        return CZ_ERR_ARG;
    if (!supported_block(p->block))
        return CZ_ERR_SHAPE;
    const uint32_t N = p->block;
    if (p->nx % N || p->ny % N || p->nz % N)
        return CZ_ERR_SHAPE;
    // a block row span (N rows of nx elements) is addressed with 32-bit offsets
    if ((uint64_t)p->nx * N * p->elem_bytes >= (1ull << 31))
        return CZ_ERR_SHAPE;
    const uint64_t nb = (uint64_t)(p->nx / N) * (p->ny / N) * (p->nz / N);
    // blocks up to 32^3 launch one workgroup of at most N^2 threads per block:
    // the grid's thread count must stay below 2^32
    if (nb >= MAX_BLOCKS || (N <= 32 && nb * N * N >= (1ull << 32)))
        return CZ_ERR_SHAPE;
    *nblocks = nb;
    return CZ_OK;
}

uint64_t payload_start(uint64_t nblocks) { return roundup16(HDR + 8 * (nblocks + 1)); }

uint64_t record_bound(uint32_t N, uint32_t elem)
{
    const uint64_t n3 = (uint64_t)N * N * N;
    return roundup16(8 + n3 / 8 + n3 * elem);
}

void build_header(const cz_params *p, uint64_t nblocks, uint32_t out[16])
{
    std::memset(out, 0, 64);
    out[0] = MAGIC;
    out[1] = 1;
    out[2] = p->scheme;
    out[3] = p->elem_bytes;
    out[4] = p->block;
    out[5] = (uint32_t)(ilog2(p->block) - 2);
    out[6] = p->nx;
    out[7] = p->ny;
    out[8] = p->nz;
    out[9] = 0;
    std::memcpy(&out[10], &p->epsilon, 8);
    std::memcpy(&out[12], &nblocks, 8);
    // out[14..15] payload bytes: written by the last block
}

int ensure_capacity(cz_ctx *ctx, uint64_t nblocks)
{
    if (nblocks <= ctx->cap_blocks)
        return CZ_OK;
    uint64_t want = ctx->cap_blocks ? ctx->cap_blocks : 4096;
    while (want < nblocks)
        want *= 2;
    uint64_t *fresh = nullptr;
    if (hipMalloc(&fresh, want * sizeof(uint64_t)) != hipSuccess)
        return CZ_ERR_HIP;
    if (ctx->flags) {
        (void)hipDeviceSynchronize();  // previous calls may still use the old flags
        (void)hipFree(ctx->flags);
    }
    ctx->flags = fresh;
    ctx->cap_blocks = want;
    return CZ_OK;
}

int status_to_error(uint32_t st)
{
    if (st & czk::STATUS_NONFINITE)
        return CZ_ERR_NONFINITE;
    if (st & czk::STATUS_FORMAT)
        return CZ_ERR_FORMAT;
    if (st & czk::STATUS_TIMEOUT)
        return CZ_ERR_TIMEOUT;
    return CZ_OK;
}

// Copy the workspace header to pinned memory and wait for the stream.
int read_work(cz_ctx *ctx, hipStream_t st)
{
    if (hipMemcpyAsync(ctx->pinned, ctx->work, sizeof(czk::CzWork), hipMemcpyDeviceToHost, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (hipStreamSynchronize(st) != hipSuccess)
        return CZ_ERR_HIP;
    return CZ_OK;
}

// Synchronous calls report their device-side error and consume it.
int take_status(cz_ctx *ctx, hipStream_t st)
{
    const int rc = status_to_error(ctx->pinned->status);
    if (ctx->pinned->status != 0 && czk::launch_prep_inv(ctx->work, st) != hipSuccess)
        return CZ_ERR_HIP;
    return rc;
}

// Scratch for the N = 64 kernels: one N^3 slot per workgroup of the grid.
int ensure_scratch(cz_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->scratch_bytes)
        return CZ_OK;
    void *fresh = nullptr;
    if (hipMalloc(&fresh, bytes) != hipSuccess)
        return CZ_ERR_HIP;
    if (ctx->scratch) {
        (void)hipDeviceSynchronize();
        (void)hipFree(ctx->scratch);
    }
    ctx->scratch = fresh;
    ctx->scratch_bytes = bytes;
    return CZ_OK;
}

int grid_for(cz_ctx *ctx, const czk::KernelKey &key, bool inverse, uint64_t nblocks)
{
    int per_cu = czk::occupancy(key, inverse);
    if (per_cu < 1)
        per_cu = 1;
    uint64_t g = (uint64_t)per_cu * (uint64_t)ctx->num_cu;
    if (g > nblocks)
        g = nblocks;
    return (int)(g ? g : 1);
}

}  // namespace

extern "C" {

int cz_create(cz_ctx **out, int device)
{
    if (!out)
        return CZ_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count)
        return CZ_ERR_HIP;
    DeviceGuard guard(device);
    cz_ctx *ctx = new (std::nothrow) cz_ctx();
    if (!ctx)
        return CZ_ERR_ARG;
    ctx->device = device;
    if (hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        hipMalloc(&ctx->work, sizeof(czk::CzWork)) != hipSuccess ||
        hipMemset(ctx->work, 0, sizeof(czk::CzWork)) != hipSuccess ||
        hipHostMalloc(&ctx->pinned, sizeof(czk::CzWork), hipHostMallocDefault) != hipSuccess ||
        ensure_capacity(ctx, 4096) != CZ_OK) {
        cz_destroy(ctx);
        return CZ_ERR_HIP;
    }
    *out = ctx;
    return CZ_OK;
}

void cz_destroy(cz_ctx *ctx)
{
    if (!ctx)
        return;
    DeviceGuard guard(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->flags)
        (void)hipFree(ctx->flags);
    if (ctx->work)
        (void)hipFree(ctx->work);
    if (ctx->pinned)
        (void)hipHostFree(ctx->pinned);
    if (ctx->scratch)
        (void)hipFree(ctx->scratch);
    delete ctx;
}

int cz_reserve(cz_ctx *ctx, uint64_t max_blocks)
{
    if (!ctx)
        return CZ_ERR_ARG;
    if (max_blocks >= MAX_BLOCKS)
        return CZ_ERR_SHAPE;
    DeviceGuard guard(ctx->device);
    return ensure_capacity(ctx, max_blocks);
}

size_t cz_compress_bound(const cz_params *p)
{
    uint64_t nb = 0;
    if (check_params(p, &nb) != CZ_OK)
        return 0;
    return (size_t)(payload_start(nb) + nb * record_bound(p->block, p->elem_bytes));
}

int cz_compress(cz_ctx *ctx, const cz_params *p, const void *d_field, void *d_out, size_t out_cap,
                uint64_t *d_out_bytes, size_t *h_out_bytes, void *stream)
{
    if (!ctx)
        return CZ_ERR_ARG;
    uint64_t nb = 0;
    int rc = check_params(p, &nb);
    if (rc != CZ_OK)
        return rc;
    const uint64_t bound = payload_start(nb) + nb * record_bound(p->block, p->elem_bytes);
    if (out_cap < bound) {
        if (h_out_bytes)
            *h_out_bytes = (size_t)bound;
        return CZ_ERR_CAPACITY;
    }
    if (!d_out || (nb && !d_field))
        return CZ_ERR_ARG;
    DeviceGuard guard(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = ensure_capacity(ctx, nb)) != CZ_OK)
        return rc;

    czk::PrepArgs pa{};
    pa.out = static_cast<uint8_t *>(d_out);
    pa.flags = ctx->flags;
    pa.work = ctx->work;
    pa.nblocks = nb;
    pa.p0 = payload_start(nb);
    build_header(p, nb, pa.header);
    if (czk::launch_prep_fwd(pa, st) != hipSuccess)
        return CZ_ERR_HIP;

    if (nb) {
        const czk::KernelKey key{p->block, p->scheme, p->elem_bytes};
        czk::FwdArgs fa{};
        fa.field = d_field;
        fa.out = static_cast<uint8_t *>(d_out);
        fa.offsets = reinterpret_cast<uint64_t *>(fa.out + HDR);
        fa.flags = ctx->flags;
        fa.work = ctx->work;
        fa.nx = p->nx;
        fa.ny = p->ny;
        fa.nbx = p->nx / p->block;
        fa.nby = p->ny / p->block;
        fa.nblocks = nb;
        fa.p0 = pa.p0;
        fa.eps = p->epsilon;
        fa.eps_f = (float)p->epsilon;  // round to nearest, then up if it fell below
        if ((double)fa.eps_f < p->epsilon)
            fa.eps_f = std::nextafter(fa.eps_f, INFINITY);
        int grid = (int)nb;  // one workgroup per block up to 32^3
        if (p->block == 64) {  // persistent, one scratch slot per workgroup
            grid = grid_for(ctx, key, false, nb);
            if ((rc = ensure_scratch(ctx, (size_t)grid * 64 * 64 * 64 * p->elem_bytes)) != CZ_OK)
                return rc;
            fa.scratch = ctx->scratch;
        }
        if (czk::launch_fwd(key, fa, grid, st) != hipSuccess)
            return CZ_ERR_HIP;
    }
    if (d_out_bytes &&
        hipMemcpyAsync(d_out_bytes, &ctx->work->total, sizeof(uint64_t), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (h_out_bytes) {
        if ((rc = read_work(ctx, st)) != CZ_OK)
            return rc;
        *h_out_bytes = (size_t)ctx->pinned->total;
        return take_status(ctx, st);
    }
    return CZ_OK;
}

int cz_read_header(const void *h_hdr, size_t n, cz_params *out, uint64_t *nblocks, uint64_t *total_bytes)
{
    if (!h_hdr || !out || n < HDR)
        return CZ_ERR_ARG;
    uint32_t w[16];
    std::memcpy(w, h_hdr, 64);
    if (w[0] != MAGIC || w[1] != 1)
        return CZ_ERR_FORMAT;
    cz_params p{};
    p.scheme = w[2];
    p.elem_bytes = w[3];
    p.block = w[4];
    p.nx = w[6];
    p.ny = w[7];
    p.nz = w[8];
    std::memcpy(&p.epsilon, &w[10], 8);
    uint64_t nb_hdr = 0, payload = 0;
    std::memcpy(&nb_hdr, &w[12], 8);
    std::memcpy(&payload, &w[14], 8);
    uint64_t nb = 0;
    if (check_params(&p, &nb) != CZ_OK || nb != nb_hdr || w[5] != (uint32_t)(ilog2(p.block) - 2) || w[9] != 0)
        return CZ_ERR_FORMAT;
    *out = p;
    if (nblocks)
        *nblocks = nb;
    if (total_bytes)
        *total_bytes = payload_start(nb) + payload;
    return CZ_OK;
}

int cz_decompress(cz_ctx *ctx, const cz_params *expected, const void *d_in, size_t in_bytes, void *d_field,
                  size_t field_cap, void *stream)
{
    if (!ctx || !d_in)
        return CZ_ERR_ARG;
    DeviceGuard guard(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    cz_params p{};
    uint64_t nb = 0, total = 0;
    const bool sync = expected == nullptr;
    int rc;
    if (sync) {
        if (in_bytes < HDR)
            return CZ_ERR_FORMAT;
        uint8_t hdr[64];
        if (hipMemcpyAsync(hdr, d_in, 64, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return CZ_ERR_HIP;
        if ((rc = cz_read_header(hdr, 64, &p, &nb, &total)) != CZ_OK)
            return rc;
        if (total > in_bytes)
            return CZ_ERR_FORMAT;
    } else {
        p = *expected;
        if ((rc = check_params(&p, &nb)) != CZ_OK)
            return rc;
        total = in_bytes;
    }
    const uint64_t p0 = payload_start(nb);
    if (p0 > in_bytes || total < p0)
        return CZ_ERR_FORMAT;
    if ((uint64_t)p.nx * p.ny * p.nz * p.elem_bytes > field_cap)
        return CZ_ERR_CAPACITY;
    if (nb && !d_field)
        return CZ_ERR_ARG;
    if (czk::launch_prep_inv(ctx->work, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (nb) {
        const czk::KernelKey key{p.block, p.scheme, p.elem_bytes};
        czk::InvArgs ia{};
        ia.in = static_cast<const uint8_t *>(d_in);
        ia.field = d_field;
        ia.work = ctx->work;
        ia.nx = p.nx;
        ia.ny = p.ny;
        ia.nbx = p.nx / p.block;
        ia.nby = p.ny / p.block;
        ia.nblocks = nb;
        ia.p0 = p0;
        ia.payload = total - p0;
        const int grid = grid_for(ctx, key, true, nb);
        if (p.block == 64) {
            if ((rc = ensure_scratch(ctx, (size_t)grid * 64 * 64 * 64 * p.elem_bytes)) != CZ_OK)
                return rc;
            ia.scratch = ctx->scratch;
        }
        if (czk::launch_inv(key, ia, grid, st) != hipSuccess)
            return CZ_ERR_HIP;
    }
    if (sync) {
        if ((rc = read_work(ctx, st)) != CZ_OK)
            return rc;
        return take_status(ctx, st);
    }
    return CZ_OK;
}

int cz_get_status(cz_ctx *ctx, void *stream)
{
    if (!ctx)
        return CZ_ERR_ARG;
    DeviceGuard guard(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = read_work(ctx, st);
    if (rc != CZ_OK)
        return rc;
    rc = status_to_error(ctx->pinned->status);
    if (czk::launch_prep_inv(ctx->work, st) != hipSuccess)  // clears ticket and status
        return CZ_ERR_HIP;
    return rc;
}

const char *cz_strerror(int code)
{
    switch (code) {
    case CZ_OK: return "ok";
    case CZ_ERR_ARG: return "invalid argument";
    case CZ_ERR_SHAPE: return "unsupported block size or grid not a multiple of the block";
    case CZ_ERR_CAPACITY: return "buffer too small";
    case CZ_ERR_NONFINITE: return "non-finite input or coefficient";
    case CZ_ERR_FORMAT: return "corrupt or inconsistent stream";
    case CZ_ERR_HIP: return "HIP runtime error";
    case CZ_ERR_BUDGET: return "request exceeds the memory budget";
    case CZ_ERR_TIMEOUT: return "device-side wait exceeded its bound";
    default: return "unknown error";
    }
}

}  // extern "C"
