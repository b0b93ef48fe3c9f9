// Random access to a compressed stream (the paper's Sec. 2.3, "Data
// decompression"): decompression works block by block, so a reader that
// needs part of the field fetches only the records of the blocks it touches
// through the offsets table, and keeps recently decoded blocks in a cache so
// that neighbouring requests do not decode them again.
//
// Decoding runs the ordinary inverse kernels with a selection list: ticket k
// decodes record sel[2k] into output block sel[2k+1] of a dense pool of N^3
// blocks.  The cache is a pool of such blocks with least-recently-used
// replacement (host-side bookkeeping); a region request fetches the blocks
// its box touches and gathers the box from the pool.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "cz_host.h"

namespace {

constexpr int THREADS = 256;

// Decode the selected records (pairs already uploaded to d_sel) of a stream
// with parameters p into the pool `dst` of N^3 blocks, on the context's work
// queue (its ticket and status words, its published descriptor slot).
int decode_selected(cz_ctx *ctx, const cz_params &p, uint64_t stream_blocks, const void *d_in, size_t in_bytes,
                    const uint32_t *d_sel, uint64_t n, void *dst, czh::DevBuf &scratch, hipStream_t st)
{
    czk::Queue q = czh::work_queue(ctx);
    q.ntickets = n;
    q.fields = q.publish = ctx->one;
    q.one = czh::describe(p, stream_blocks, false);
    q.one.src = d_in;
    q.one.dst = dst;
    q.one.nx = p.block;  // output: a column of N^3 blocks, block k at k N^3
    q.one.ny = p.block;
    q.one.nbx = 1;
    q.one.nby = 1;
    q.one.nblocks = n;
    q.one.sel = d_sel;
    q.one.payload = in_bytes - q.one.p0;
    if (czk::launch_prep(q, false, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (n == 0)
        return CZ_OK;
    const czk::KernelKey key = czh::key_of(ctx, p);
    const int grid = czh::grid_for(ctx, key, true, n);
    int rc = scratch.ensure(std::max<size_t>(czh::scratch_need(key, grid), 1));
    if (rc != CZ_OK)
        return rc;
    q.scratch = scratch.ptr;
    return czk::launch_inv(key, q, grid, st) == hipSuccess ? CZ_OK : CZ_ERR_HIP;
}

int check_stream(const cz_params *p, size_t in_bytes, const void *d_in, uint64_t *nb)
{
    if (!p || !d_in)
        return CZ_ERR_ARG;
    int rc = czh::check_params(p, nb);
    if (rc != CZ_OK)
        return rc;
    return czh::payload_start(*nb) <= in_bytes ? CZ_OK : CZ_ERR_FORMAT;
}

// Gather the box [x0, x0+ex) x [y0, y0+ey) x [z0, z0+ez) from cached blocks:
// slot[] maps the box's blocks (x fastest, from block (bx0, by0, bz0)) to
// pool blocks.
template <typename T, int N>
__global__ __launch_bounds__(THREADS) void region_kernel(const T *__restrict__ pool, const uint32_t *__restrict__ slot,
                                                         uint32_t rbx, uint32_t rby, uint32_t x0, uint32_t y0,
                                                         uint32_t z0, uint32_t ex, uint32_t ey, uint32_t ez,
                                                         T *__restrict__ out)
{
    const uint64_t total = (uint64_t)ex * ey * ez;
    for (uint64_t e = (uint64_t)blockIdx.x * THREADS + threadIdx.x; e < total; e += (uint64_t)gridDim.x * THREADS) {
        const uint32_t x = (uint32_t)(e % ex), y = (uint32_t)((e / ex) % ey), z = (uint32_t)(e / ((uint64_t)ex * ey));
        const uint32_t gx = x0 + x, gy = y0 + y, gz = z0 + z;
        const uint32_t bx = gx / N - x0 / N, by = gy / N - y0 / N, bz = gz / N - z0 / N;
        const uint64_t s = slot[bx + rbx * (by + rby * bz)];
        out[e] = pool[s * N * N * N + (uint64_t)(gz % N) * N * N + (gy % N) * N + gx % N];
    }
}

}  // namespace

struct cz_cache {
    cz_ctx *ctx = nullptr;
    cz_params p{};
    uint64_t nblocks = 0;
    size_t cap = 0;                     // blocks the pool holds
    czh::DevBuf pool, scratch;
    czh::Staging sel, table;
    std::vector<int64_t> slot_of;       // per block of the stream: pool slot or -1
    std::vector<int64_t> block_of;      // per slot: block or -1
    std::vector<uint64_t> last_use;     // per slot: request stamp
    uint64_t stamp = 0;
    const void *stream = nullptr;       // the stream the pool holds blocks of
    size_t stream_bytes = 0;
    uint64_t hits = 0, misses = 0;
};

namespace {

// Make every block of blocks[0, n) resident; slots[i] receives its slot.
int cache_fetch(cz_cache *c, const void *d_in, size_t in_bytes, const uint32_t *blocks, size_t n, uint32_t *slots,
                hipStream_t st)
{
    if (n > c->cap)
        return CZ_ERR_ARG;
    if (in_bytes < czh::payload_start(c->nblocks))
        return CZ_ERR_FORMAT;
    for (size_t i = 0; i < n; ++i)
        if (blocks[i] >= c->nblocks)
            return CZ_ERR_ARG;
    if (d_in != c->stream || in_bytes != c->stream_bytes) {  // another stream: forget everything
        std::fill(c->slot_of.begin(), c->slot_of.end(), -1);
        std::fill(c->block_of.begin(), c->block_of.end(), -1);
        c->stream = d_in;
        c->stream_bytes = in_bytes;
    }
    const uint64_t now = ++c->stamp;
    std::vector<uint32_t> pairs;
    // hits first, so that they are protected from eviction by this request
    for (size_t i = 0; i < n; ++i) {
        const int64_t s = c->slot_of[blocks[i]];
        if (s >= 0)
            c->last_use[s] = now;
    }
    for (size_t i = 0; i < n; ++i) {
        const int64_t s = c->slot_of[blocks[i]];
        if (s >= 0) {  // resident (or decoded earlier in this request)
            ++c->hits;
            slots[i] = (uint32_t)s;
            continue;
        }
        // least recently used slot not used by this request (free slots have stamp 0)
        size_t best = c->cap;
        for (size_t k = 0; k < c->cap; ++k)
            if (c->last_use[k] != now && (best == c->cap || c->last_use[k] < c->last_use[best]))
                best = k;
        if (best == c->cap)
            return CZ_ERR_ARG;  // cannot happen with n <= cap
        if (c->block_of[best] >= 0)
            c->slot_of[c->block_of[best]] = -1;
        c->block_of[best] = blocks[i];
        c->slot_of[blocks[i]] = (int64_t)best;
        c->last_use[best] = now;
        pairs.push_back(blocks[i]);
        pairs.push_back((uint32_t)best);
        slots[i] = (uint32_t)best;
        ++c->misses;
    }
    if (pairs.empty())
        return CZ_OK;
    int rc = c->sel.upload(pairs.data(), pairs.size() * sizeof(uint32_t), st);
    if (rc != CZ_OK)
        return rc;
    return decode_selected(c->ctx, c->p, c->nblocks, d_in, in_bytes, static_cast<const uint32_t *>(c->sel.dev.ptr),
                           pairs.size() / 2, c->pool.ptr, c->scratch, st);
}

}  // namespace

extern "C" {

int cz_decompress_blocks(cz_ctx *ctx, const cz_params *p, const void *d_in, size_t in_bytes, const uint32_t *h_blocks,
                         size_t n, void *d_out, size_t out_cap, void *stream)
{
    if (!ctx || (n && (!h_blocks || !d_out)))
        return CZ_ERR_ARG;
    uint64_t nb = 0;
    int rc = check_stream(p, in_bytes, d_in, &nb);
    if (rc != CZ_OK)
        return rc;
    const uint64_t n3 = (uint64_t)p->block * p->block * p->block;
    if ((uint64_t)n * n3 * p->elem_bytes > out_cap)
        return CZ_ERR_CAPACITY;
    if (n >= (1ull << 31))
        return CZ_ERR_ARG;
    std::vector<uint32_t> pairs(2 * n);
    for (size_t k = 0; k < n; ++k) {
        if (h_blocks[k] >= nb)
            return CZ_ERR_ARG;
        pairs[2 * k] = h_blocks[k];
        pairs[2 * k + 1] = (uint32_t)k;
    }
    if (n == 0)
        return CZ_OK;
    czh::DeviceGuard guard(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = ctx->sel.upload(pairs.data(), pairs.size() * sizeof(uint32_t), st)) != CZ_OK)
        return rc;
    return decode_selected(ctx, *p, nb, d_in, in_bytes, static_cast<const uint32_t *>(ctx->sel.dev.ptr), n, d_out,
                           ctx->scratch, st);
}

int cz_cache_create(cz_ctx *ctx, const cz_params *p, size_t capacity_blocks, cz_cache **out)
{
    if (!ctx || !out || capacity_blocks == 0 || capacity_blocks >= (1ull << 31))
        return CZ_ERR_ARG;
    *out = nullptr;
    uint64_t nb = 0;
    int rc = p ? czh::check_params(p, &nb) : CZ_ERR_ARG;
    if (rc != CZ_OK)
        return rc;
    czh::DeviceGuard guard(ctx->device);
    cz_cache *c = new (std::nothrow) cz_cache();
    if (!c)
        return CZ_ERR_ARG;
    c->ctx = ctx;
    c->p = *p;
    c->nblocks = nb;
    c->cap = capacity_blocks;
    const size_t block_bytes = (size_t)p->block * p->block * p->block * p->elem_bytes;
    rc = c->pool.ensure(capacity_blocks * block_bytes);
    if (rc == CZ_OK)
        rc = c->sel.init();
    if (rc == CZ_OK)
        rc = c->table.init();
    if (rc != CZ_OK) {
        cz_cache_destroy(c);
        return rc;
    }
    c->slot_of.assign(nb, -1);
    c->block_of.assign(capacity_blocks, -1);
    c->last_use.assign(capacity_blocks, 0);
    *out = c;
    return CZ_OK;
}

int cz_cache_fetch(cz_cache *c, const void *d_in, size_t in_bytes, const uint32_t *h_blocks, size_t n,
                   void **h_ptrs, void *stream)
{
    if (!c || !d_in || (n && (!h_blocks || !h_ptrs)))
        return CZ_ERR_ARG;
    czh::DeviceGuard guard(c->ctx->device);
    std::vector<uint32_t> slots(n);
    int rc = cache_fetch(c, d_in, in_bytes, h_blocks, n, slots.data(), static_cast<hipStream_t>(stream));
    if (rc != CZ_OK)
        return rc;
    const size_t block_bytes = (size_t)c->p.block * c->p.block * c->p.block * c->p.elem_bytes;
    for (size_t i = 0; i < n; ++i)
        h_ptrs[i] = static_cast<uint8_t *>(c->pool.ptr) + slots[i] * block_bytes;
    return CZ_OK;
}

int cz_cache_region(cz_cache *c, const void *d_in, size_t in_bytes, const uint32_t origin[3], const uint32_t extent[3],
                    void *d_out, size_t out_cap, void *stream)
{
    if (!c || !d_in || !origin || !extent || !d_out)
        return CZ_ERR_ARG;
    const cz_params &p = c->p;
    const uint32_t dims[3] = {p.nx, p.ny, p.nz};
    for (int a = 0; a < 3; ++a)
        if (extent[a] == 0 || origin[a] >= dims[a] || extent[a] > dims[a] - origin[a])
            return CZ_ERR_ARG;
    const uint64_t cells = (uint64_t)extent[0] * extent[1] * extent[2];
    if (cells * p.elem_bytes > out_cap)
        return CZ_ERR_CAPACITY;
    const uint32_t N = p.block;
    uint32_t b0[3], nbr[3];
    for (int a = 0; a < 3; ++a) {
        b0[a] = origin[a] / N;
        nbr[a] = (origin[a] + extent[a] - 1) / N - b0[a] + 1;
    }
    const uint64_t nreg = (uint64_t)nbr[0] * nbr[1] * nbr[2];
    if (nreg > c->cap)
        return CZ_ERR_ARG;
    std::vector<uint32_t> blocks(nreg), slots(nreg);
    const uint32_t nbx = p.nx / N, nby = p.ny / N;
    for (uint32_t k = 0; k < nreg; ++k) {
        const uint32_t bx = b0[0] + k % nbr[0], by = b0[1] + (k / nbr[0]) % nbr[1], bz = b0[2] + k / (nbr[0] * nbr[1]);
        blocks[k] = bx + nbx * (by + nby * bz);
    }
    czh::DeviceGuard guard(c->ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = cache_fetch(c, d_in, in_bytes, blocks.data(), nreg, slots.data(), st);
    if (rc != CZ_OK)
        return rc;
    if ((rc = c->table.upload(slots.data(), slots.size() * sizeof(uint32_t), st)) != CZ_OK)
        return rc;
    const uint64_t g = std::min<uint64_t>((cells + THREADS - 1) / THREADS, 65536);
    const uint32_t *tab = static_cast<const uint32_t *>(c->table.dev.ptr);
#define CZ_REGION(T, NN)                                                                                     \
    hipLaunchKernelGGL((region_kernel<T, NN>), dim3((unsigned)g), dim3(THREADS), 0, st,                      \
                       static_cast<const T *>(c->pool.ptr), tab, nbr[0], nbr[1], origin[0], origin[1], origin[2], \
                       extent[0], extent[1], extent[2], static_cast<T *>(d_out))
#define CZ_REGION_N(T)                                                                                       \
    switch (N) {                                                                                             \
    case 8: CZ_REGION(T, 8); break;                                                                          \
    case 16: CZ_REGION(T, 16); break;                                                                        \
    case 32: CZ_REGION(T, 32); break;                                                                        \
    default: CZ_REGION(T, 64); break;                                                                        \
    }
    if (p.elem_bytes == 4) {
        CZ_REGION_N(float)
    } else {
        CZ_REGION_N(double)
    }
#undef CZ_REGION_N
#undef CZ_REGION
    return hipGetLastError() == hipSuccess ? CZ_OK : CZ_ERR_HIP;
}

int cz_cache_stats(cz_cache *c, uint64_t *hits, uint64_t *misses)
{
    if (!c)
        return CZ_ERR_ARG;
    if (hits)
        *hits = c->hits;
    if (misses)
        *misses = c->misses;
    return CZ_OK;
}

void cz_cache_destroy(cz_cache *c)
{
    if (!c)
        return;
    czh::DeviceGuard guard(c->ctx->device);
    (void)hipDeviceSynchronize();
    c->pool.release();
    c->scratch.release();
    c->sel.release();
    c->table.release();
    delete c;
}

}  // extern "C"
