// Host side of the C ABI declared in include/cz.h: parameter validation,
// stream layout arithmetic, workspace ownership, work queues and launches.
//
// The problem statement (arXiv 1903.07761, Sec. 2.1-2.3): a grid of equal
// cubic blocks of power-of-two edge, one scalar quantity at a time, a wavelet
// scheme, a precision and a decimation threshold.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "cz_host.h"

using namespace czh;

// Fixed device scratch of cz_compress_noalloc: the call's (ticket, status,
// size) words, its one-field descriptor table and one look-back flag per
// block.  Host code never passes `scratch` itself (on the host it is only a
// stand-in for the symbol): it passes the device address that
// hipGetSymbolAddress returned for the current device.
namespace {
constexpr size_t NA_WORK = 0;      // czk::CzWork
constexpr size_t NA_DESC = 256;    // czk::FieldDesc
constexpr size_t NA_FLAGS = 1024;  // CZ_NOALLOC_MAX_BLOCKS x u64
constexpr size_t NA_BYTES = NA_FLAGS + (size_t)CZ_NOALLOC_MAX_BLOCKS * sizeof(uint64_t);
static_assert(sizeof(czk::CzWork) <= NA_DESC - NA_WORK, "work words overlap the descriptor");
static_assert(sizeof(czk::FieldDesc) <= NA_FLAGS - NA_DESC, "descriptor overlaps the flags");
constexpr int NA_MAX_DEVICES = 64;
std::mutex na_mutex;
void *na_ptr[NA_MAX_DEVICES] = {};
}  // namespace

static __device__ __align__(256) uint8_t scratch[NA_BYTES];

namespace {
// Device address of `scratch` on `device`, looked up once per device with
// that device current (the caller holds a DeviceGuard for it).
int noalloc_scratch(int device, void **out)
{
    std::lock_guard<std::mutex> lock(na_mutex);
    if (device < 0 || device >= NA_MAX_DEVICES)
        return CZ_ERR_HIP;
    if (!na_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return CZ_ERR_HIP;
        na_ptr[device] = p;
    }
    *out = na_ptr[device];
    return CZ_OK;
}
}  // namespace

struct cz_plan {
    cz_ctx *ctx = nullptr;
    std::vector<cz_params> params;
    Layout layout;
    BatchWork work;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;  // the last run has finished with the staging
};

namespace czh {

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

uint64_t bound_of(const cz_params &p, uint64_t nb) { return payload_start(nb) + nb * record_bound(p.block, p.elem_bytes); }

void build_header(const cz_params &p, uint64_t nblocks, uint32_t out[16])
{
    std::memset(out, 0, 64);
    out[0] = MAGIC;
    out[1] = 1;
    out[2] = p.scheme;
    out[3] = p.elem_bytes;
    out[4] = p.block;
    out[5] = (uint32_t)(ilog2(p.block) - 2);
    out[6] = p.nx;
    out[7] = p.ny;
    out[8] = p.nz;
    out[9] = 0;
    std::memcpy(&out[10], &p.epsilon, 8);
    std::memcpy(&out[12], &nblocks, 8);
    // out[14..15] payload bytes: written by the last block
}

float eps_float(double eps)
{
    float f = (float)eps;  // round to nearest, then up if it fell below
    if ((double)f < eps)
        f = std::nextafter(f, INFINITY);
    return f;
}

int block_index(uint32_t N) { return N == 8 ? 0 : N == 16 ? 1 : N == 32 ? 2 : 3; }

czk::KernelKey key_of(const cz_ctx *ctx, const cz_params &p)
{
    czk::KernelKey k{p.block, p.scheme, p.elem_bytes, 0};
    k.variant = ctx->variant[block_index(p.block)][p.elem_bytes == 8][p.scheme];
    return k;
}

// Descriptor of one field (pointers and ticket base filled by the caller).
czk::FieldDesc describe(const cz_params &p, uint64_t nb, bool forward)
{
    czk::FieldDesc d{};
    d.nx = p.nx;
    d.ny = p.ny;
    d.nbx = p.nx / p.block;
    d.nby = p.ny / p.block;
    d.nblocks = nb;
    d.p0 = payload_start(nb);
    d.rblocks = nb;
    d.cstride = 1;
    d.eps = p.epsilon;
    d.eps_f = eps_float(p.epsilon);
    if (forward)
        build_header(p, nb, d.header);
    return d;
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

czk::Queue work_queue(cz_ctx *ctx)
{
    czk::Queue q{};
    q.nfields = 1;
    q.ticket = &ctx->work->ticket;
    q.status = &ctx->work->status;
    return q;
}

// Synchronous calls report their device-side error and consume it.
int take_status(cz_ctx *ctx, hipStream_t st)
{
    const int rc = status_to_error(ctx->pinned->status);
    if (ctx->pinned->status != 0 && czk::launch_prep(work_queue(ctx), false, st) != hipSuccess)
        return CZ_ERR_HIP;
    return rc;
}

// Workgroups of a launch over `tickets` blocks: one per block for the
// on-chip forward kernel, else enough persistent workgroups to fill the chip.
int grid_for(const cz_ctx *ctx, const czk::KernelKey &key, bool inverse, uint64_t tickets)
{
    if (!inverse && czk::fwd_one_block_per_workgroup(key))
        return (int)std::max<uint64_t>(tickets, 1);
    int per_cu = czk::occupancy(key, inverse);
    if (per_cu < 1)
        per_cu = 1;
    uint64_t g = (uint64_t)per_cu * (uint64_t)ctx->num_cu;
    const int cap = czk::grid_cap(key);
    if (cap > 0 && g > (uint64_t)cap)
        g = (uint64_t)cap;
    if (g > tickets)
        g = tickets;
    return (int)(g ? g : 1);
}

// Forward tickets of a field of nb blocks (small blocks go in groups).
uint64_t fwd_tickets(const czk::KernelKey &key, uint64_t nb)
{
    const uint64_t g = czk::fwd_blocks_per_ticket(key);
    return (nb + g - 1) / g;
}

size_t scratch_need(const czk::KernelKey &key, int grid) { return czk::scratch_bytes(key, grid); }

// Group the fields of a batch into classes (block size, precision, scheme,
// variant), each with a ticket range, a grid and its own 64^3 scratch slots.
int layout_batch(const cz_ctx *ctx, bool forward, int n, const cz_params *ps, Layout *L)
{
    std::map<ClassKey, std::vector<int>> by;
    L->forward = forward;
    L->n = n;
    L->nblocks.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        int rc = check_params(&ps[i], &L->nblocks[i]);
        if (rc != CZ_OK)
            return rc;
        const czk::KernelKey k = key_of(ctx, ps[i]);
        by[ClassKey(k.block, k.elem_bytes, k.scheme, k.variant)].push_back(i);
    }
    if ((int)by.size() > MAX_CLASSES)
        return CZ_ERR_ARG;
    L->flag_base.assign(n, 0);
    for (auto &kv : by) {
        const czk::KernelKey key{std::get<0>(kv.first), std::get<2>(kv.first), std::get<1>(kv.first),
                                 std::get<3>(kv.first)};
        L->keys.push_back(key);
        L->first.push_back((uint32_t)L->order.size());
        L->count.push_back((uint32_t)kv.second.size());
        uint64_t t = 0;
        for (int i : kv.second) {
            L->order.push_back(i);
            L->flag_base[i] = L->flags_total;
            L->flags_total += std::max<uint64_t>(L->nblocks[i], 1);
            t += forward ? fwd_tickets(key, L->nblocks[i]) : L->nblocks[i];
        }
        L->tickets.push_back(t);
        const int g = grid_for(ctx, key, !forward, t);
        L->grids.push_back(g);
        L->scratch_off.push_back(L->scratch_bytes);
        L->scratch_bytes += scratch_need(key, g);
    }
    return CZ_OK;
}

int size_work(BatchWork &w, const Layout &L)
{
    int rc;
    if ((rc = w.desc.ensure(std::max(L.n, 1) * sizeof(czk::FieldDesc))) != CZ_OK ||
        (rc = w.flags.ensure(std::max<uint64_t>(L.flags_total, 1) * sizeof(uint64_t))) != CZ_OK ||
        (rc = w.counters.ensure(2 * MAX_CLASSES * sizeof(uint32_t))) != CZ_OK ||
        (rc = w.totals.ensure(std::max(L.n, 1) * sizeof(uint64_t))) != CZ_OK ||
        (rc = w.fstat.ensure(std::max(L.n, 1) * sizeof(uint32_t))) != CZ_OK ||
        (rc = w.scratch.ensure(std::max<size_t>(L.scratch_bytes, 1))) != CZ_OK || (rc = w.pinned(L.n)) != CZ_OK ||
        (rc = w.lanes_for(L.keys.size())) != CZ_OK)
        return rc;
    return CZ_OK;
}

// Fill the pinned descriptor table for buffers srcs -> dsts (class order).
void stage_batch(BatchWork &w, const Layout &L, const cz_params *ps, const void *const *srcs,
                 const size_t *src_bytes, void *const *dsts)
{
    uint64_t *flags = static_cast<uint64_t *>(w.flags.ptr);
    uint64_t *totals = static_cast<uint64_t *>(w.totals.ptr);
    for (size_t c = 0; c < L.keys.size(); ++c) {
        uint64_t t = 0;
        for (uint32_t k = 0; k < L.count[c]; ++k) {
            const int i = L.order[L.first[c] + k];
            czk::FieldDesc d = describe(ps[i], L.nblocks[i], L.forward);
            d.src = srcs[i];
            d.dst = dsts[i];
            d.first = t;
            t += L.forward ? fwd_tickets(L.keys[c], L.nblocks[i]) : L.nblocks[i];
            if (L.forward) {
                d.flags = flags + L.flag_base[i];
                d.total = totals + i;
            } else {
                d.payload = src_bytes[i] - d.p0;
            }
            w.stage[L.first[c] + k] = d;
        }
    }
}

// Enqueue a staged batch on st: upload the descriptors, then every class on
// its own lane (forked from st, joined back), then fold the class status
// words into *status and copy the stream sizes to pinned memory.
int enqueue_batch(BatchWork &w, const Layout &L, uint32_t *status, bool per_field, hipStream_t st)
{
    czk::FieldDesc *desc = static_cast<czk::FieldDesc *>(w.desc.ptr);
    uint32_t *counters = static_cast<uint32_t *>(w.counters.ptr);
    if (hipMemcpyAsync(desc, w.stage, L.n * sizeof(czk::FieldDesc), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipEventRecord(w.fork, st) != hipSuccess)
        return CZ_ERR_HIP;
    for (size_t c = 0; c < L.keys.size(); ++c) {
        hipStream_t lane = w.lanes[c];
        if (hipStreamWaitEvent(lane, w.fork, 0) != hipSuccess)
            return CZ_ERR_HIP;
        czk::Queue q{};
        q.fields = desc + L.first[c];
        q.nfields = L.count[c];
        q.ntickets = L.tickets[c];
        q.ticket = counters + 2 * c;
        q.status = counters + 2 * c + 1;
        q.fstatus = static_cast<uint32_t *>(w.fstat.ptr) + L.first[c];
        q.scratch = static_cast<uint8_t *>(w.scratch.ptr) + L.scratch_off[c];
        if (czk::launch_prep(q, L.forward, lane) != hipSuccess)
            return CZ_ERR_HIP;
        if (L.tickets[c]) {
            const hipError_t e = L.forward ? czk::launch_fwd(L.keys[c], q, L.grids[c], lane)
                                           : czk::launch_inv(L.keys[c], q, L.grids[c], lane);
            if (e != hipSuccess)
                return CZ_ERR_HIP;
        }
        if (hipEventRecord(w.joins[c], lane) != hipSuccess || hipStreamWaitEvent(st, w.joins[c], 0) != hipSuccess)
            return CZ_ERR_HIP;
    }
    if (status && czk::launch_fold_status(counters, (int)L.keys.size(), status, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (per_field && hipMemcpyAsync(w.fstat_host, w.fstat.ptr, L.n * sizeof(uint32_t), hipMemcpyDeviceToHost,
                                    st) != hipSuccess)
        return CZ_ERR_HIP;
    if (L.forward &&
        hipMemcpyAsync(w.totals_host, w.totals.ptr, L.n * sizeof(uint64_t), hipMemcpyDeviceToHost, st) != hipSuccess)
        return CZ_ERR_HIP;
    return CZ_OK;
}

int check_batch_buffers(const Layout &L, const cz_params *ps, const void *const *srcs, const size_t *src_bytes,
                        void *const *dsts, const size_t *dst_caps, size_t *need)
{
    for (int i = 0; i < L.n; ++i) {
        const uint64_t nb = L.nblocks[i];
        if (L.forward) {
            if (dst_caps[i] < bound_of(ps[i], nb)) {
                if (need)
                    need[i] = (size_t)bound_of(ps[i], nb);
                return CZ_ERR_CAPACITY;
            }
            if (!dsts[i] || (nb && !srcs[i]))
                return CZ_ERR_ARG;
        } else {
            if (!srcs[i] || payload_start(nb) > src_bytes[i])
                return CZ_ERR_FORMAT;
            if ((uint64_t)ps[i].nx * ps[i].ny * ps[i].nz * ps[i].elem_bytes > dst_caps[i])
                return CZ_ERR_CAPACITY;
            if (nb && !dsts[i])
                return CZ_ERR_ARG;
        }
    }
    return CZ_OK;
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
    const bool ok = hipDeviceGetAttribute(&ctx->num_cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
                    hipMalloc(&ctx->work, sizeof(czk::CzWork)) == hipSuccess &&
                    hipMalloc(&ctx->one, sizeof(czk::FieldDesc)) == hipSuccess &&
                    hipMemset(ctx->work, 0, sizeof(czk::CzWork)) == hipSuccess &&
                    hipHostMalloc(&ctx->pinned, sizeof(czk::CzWork), hipHostMallocDefault) == hipSuccess &&
                    ctx->flags.ensure(4096 * sizeof(uint64_t)) == CZ_OK && ctx->batch.init() == CZ_OK &&
                    ctx->sel.init() == CZ_OK && ctx->huff_stage.init() == CZ_OK &&
                    noalloc_scratch(device, &ctx->noalloc) == CZ_OK;
    if (!ok) {
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
    ctx->flags.release();
    ctx->scratch.release();
    ctx->defer.release();
    ctx->dsizes.release();
    ctx->batch.release();
    ctx->sel.release();
    ctx->huff.release();
    ctx->huff_stage.release();
    if (ctx->work)
        (void)hipFree(ctx->work);
    if (ctx->one)
        (void)hipFree(ctx->one);
    if (ctx->pinned)
        (void)hipHostFree(ctx->pinned);
    delete ctx;
}

int cz_reserve(cz_ctx *ctx, uint64_t max_blocks)
{
    if (!ctx)
        return CZ_ERR_ARG;
    if (max_blocks >= MAX_BLOCKS)
        return CZ_ERR_SHAPE;
    DeviceGuard guard(ctx->device);
    const uint64_t nb = std::max<uint64_t>(max_blocks, 1);
    int rc = ctx->flags.ensure(nb * sizeof(uint64_t));
    if (rc == CZ_OK)
        rc = ctx->defer.ensure((size_t)nb * czk::DEFER_SLOT);
    if (rc == CZ_OK)
        rc = ctx->dsizes.ensure(czk::defer_sizes_bytes(nb));
    return rc;
}

size_t cz_compress_bound(const cz_params *p)
{
    uint64_t nb = 0;
    if (check_params(p, &nb) != CZ_OK)
        return 0;
    return (size_t)bound_of(*p, nb);
}

int cz_variant_count(uint32_t block, uint32_t elem_bytes)
{
    if (!supported_block(block) || (elem_bytes != 4 && elem_bytes != 8))
        return 0;
    return czk::variant_count(block, elem_bytes);
}

int cz_set_variant(cz_ctx *ctx, uint32_t block, uint32_t elem_bytes, uint32_t scheme, int variant)
{
    if (!ctx || scheme > 2 || variant < 0 || variant >= cz_variant_count(block, elem_bytes))
        return CZ_ERR_ARG;
    ctx->variant[block_index(block)][elem_bytes == 8][scheme] = (uint8_t)variant;
    return CZ_OK;
}

static int compress_impl(cz_ctx *ctx, const cz_params *p, const void *d_field, uint32_t cs, void *d_out,
                         size_t out_cap, uint64_t *d_out_bytes, size_t *h_out_bytes, void *stream)
{
    if (!ctx)
        return CZ_ERR_ARG;
    uint64_t nb = 0;
    int rc = check_params(p, &nb);
    if (rc != CZ_OK)
        return rc;
    const uint64_t bound = bound_of(*p, nb);
    if (out_cap < bound) {
        if (h_out_bytes)
            *h_out_bytes = (size_t)bound;
        return CZ_ERR_CAPACITY;
    }
    if (!d_out || (nb && !d_field))
        return CZ_ERR_ARG;
    DeviceGuard guard(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if ((rc = ctx->flags.ensure(std::max<uint64_t>(nb, 1) * sizeof(uint64_t))) != CZ_OK)
        return rc;

    const czk::KernelKey key = key_of(ctx, *p);
    czk::Queue q = work_queue(ctx);
    q.ntickets = fwd_tickets(key, nb);
    q.fields = q.publish = ctx->one;
    q.one = describe(*p, nb, true);
    q.one.src = d_field;
    q.one.cstride = cs;
    q.one.dst = d_out;
    q.one.flags = static_cast<uint64_t *>(ctx->flags.ptr);
    q.one.total = &ctx->work->total;
    // 32^3 blocks whose record fits a slot skip the look-back (fix-up below)
    const bool defer = nb && p->block == 32;
    if (defer) {
        if ((rc = ctx->defer.ensure((size_t)nb * czk::DEFER_SLOT)) != CZ_OK ||
            (rc = ctx->dsizes.ensure(czk::defer_sizes_bytes(nb))) != CZ_OK)
            return rc;
        q.one.defer = static_cast<uint8_t *>(ctx->defer.ptr);
        q.one.sizes = static_cast<uint32_t *>(ctx->dsizes.ptr);
    }
    if (czk::launch_prep(q, true, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (nb) {
        const int grid = grid_for(ctx, key, false, q.ntickets);
        if ((rc = ctx->scratch.ensure(scratch_need(key, grid))) != CZ_OK)
            return rc;
        q.scratch = ctx->scratch.ptr;
        if (czk::launch_fwd(key, q, grid, st) != hipSuccess)
            return CZ_ERR_HIP;
        if (defer && czk::launch_defer_fix(q, st) != hipSuccess)
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

int cz_compress(cz_ctx *ctx, const cz_params *p, const void *d_field, void *d_out, size_t out_cap,
                uint64_t *d_out_bytes, size_t *h_out_bytes, void *stream)
{
    return compress_impl(ctx, p, d_field, 1, d_out, out_cap, d_out_bytes, h_out_bytes, stream);
}

int cz_compress_noalloc(cz_ctx *ctx, const cz_params *p, const void *d_field, void *d_out, size_t out_cap,
                        uint64_t *d_out_bytes, size_t *h_out_bytes, void *stream)
{
    if (!ctx)
        return CZ_ERR_ARG;
    uint64_t nb = 0;
    int rc = check_params(p, &nb);
    if (rc != CZ_OK)
        return rc;
    // 64^3 blocks need a 1-2 MiB slot per resident workgroup: not in the fixed array
    if (p->block > 32 || nb > CZ_NOALLOC_MAX_BLOCKS)
        return CZ_ERR_SCRATCH;
    const uint64_t bound = bound_of(*p, nb);
    if (out_cap < bound) {
        if (h_out_bytes)
            *h_out_bytes = (size_t)bound;
        return CZ_ERR_CAPACITY;
    }
    if (!d_out || (nb && !d_field))
        return CZ_ERR_ARG;
    if (!ctx->noalloc)
        return CZ_ERR_HIP;
    DeviceGuard guard(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *base = static_cast<uint8_t *>(ctx->noalloc);
    czk::CzWork *w = reinterpret_cast<czk::CzWork *>(base + NA_WORK);
    czk::FieldDesc *desc = reinterpret_cast<czk::FieldDesc *>(base + NA_DESC);

    // the prep kernel zeroes the ticket, the status and this field's flags and
    // publishes the descriptor; the block kernels take the array's addresses
    const czk::KernelKey key = key_of(ctx, *p);
    czk::Queue q{};
    q.nfields = 1;
    q.ticket = &w->ticket;
    q.status = &w->status;
    q.ntickets = fwd_tickets(key, nb);
    q.fields = q.publish = desc;
    q.one = describe(*p, nb, true);
    q.one.src = d_field;
    q.one.cstride = 1;
    q.one.dst = d_out;
    q.one.flags = reinterpret_cast<uint64_t *>(base + NA_FLAGS);
    q.one.total = &w->total;
    if (czk::launch_prep(q, true, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (nb && czk::launch_fwd(key, q, grid_for(ctx, key, false, q.ntickets), st) != hipSuccess)
        return CZ_ERR_HIP;
    if (d_out_bytes &&
        hipMemcpyAsync(d_out_bytes, &w->total, sizeof(uint64_t), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (h_out_bytes) {
        if (hipMemcpyAsync(ctx->pinned, w, sizeof(czk::CzWork), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return CZ_ERR_HIP;
        *h_out_bytes = (size_t)ctx->pinned->total;
        return status_to_error(ctx->pinned->status);
    }
    // asynchronous: this call's device error joins the context's status word
    if (czk::launch_fold_status(&w->ticket, 1, &ctx->work->status, st) != hipSuccess)
        return CZ_ERR_HIP;
    return CZ_OK;
}

int cz_compress_strided(cz_ctx *ctx, const cz_params *p, const void *d_state, uint32_t ncomp, uint32_t comp,
                        void *d_out, size_t out_cap, uint64_t *d_out_bytes, size_t *h_out_bytes, void *stream)
{
    if (!p || ncomp == 0 || comp >= ncomp)
        return CZ_ERR_ARG;
    // a block row span of the state is addressed with 32-bit offsets
    if ((uint64_t)p->nx * p->block * p->elem_bytes * ncomp >= (1ull << 31))
        return CZ_ERR_SHAPE;
    const uint8_t *src = d_state ? static_cast<const uint8_t *>(d_state) + (size_t)comp * p->elem_bytes : nullptr;
    return compress_impl(ctx, p, src, ncomp, d_out, out_cap, d_out_bytes, h_out_bytes, stream);
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
    czk::Queue q = work_queue(ctx);
    q.ntickets = nb;
    q.fields = q.publish = ctx->one;
    q.one = describe(p, nb, false);
    q.one.src = d_in;
    q.one.dst = d_field;
    q.one.payload = total - p0;
    if (czk::launch_prep(q, false, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (nb) {
        const czk::KernelKey key = key_of(ctx, p);
        const int grid = grid_for(ctx, key, true, nb);
        if ((rc = ctx->scratch.ensure(scratch_need(key, grid))) != CZ_OK)
            return rc;
        q.scratch = ctx->scratch.ptr;
        if (czk::launch_inv(key, q, grid, st) != hipSuccess)
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
    if (czk::launch_prep(work_queue(ctx), false, st) != hipSuccess)  // clears ticket and status
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
    case CZ_ERR_SCRATCH: return "field exceeds the fixed scratch of the non-allocating compress (N > 32 or too many blocks)";
    default: return "unknown error";
    }
}

// ----------------------------------------------------------------- batches

static int run_batch(cz_ctx *ctx, bool forward, int n, const cz_params *ps, const void *const *srcs,
                     const size_t *src_bytes, void *const *dsts, const size_t *dst_caps, uint64_t *d_out_bytes,
                     size_t *h_out_bytes, void *stream)
{
    if (!ctx || n < 0 || (n && (!ps || !srcs || !dsts || !dst_caps || (!forward && !src_bytes))))
        return CZ_ERR_ARG;
    if (n == 0)
        return CZ_OK;
    Layout L;
    int rc = layout_batch(ctx, forward, n, ps, &L);
    if (rc != CZ_OK)
        return rc;
    if ((rc = check_batch_buffers(L, ps, srcs, src_bytes, dsts, dst_caps, h_out_bytes)) != CZ_OK)
        return rc;
    DeviceGuard guard(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    BatchWork &w = ctx->batch;
    if ((rc = size_work(w, L)) != CZ_OK)
        return rc;
    if (hipEventSynchronize(w.staged) != hipSuccess)  // the previous upload has left the staging
        return CZ_ERR_HIP;
    stage_batch(w, L, ps, srcs, src_bytes, dsts);
    if ((rc = enqueue_batch(w, L, &ctx->work->status, false, st)) != CZ_OK)
        return rc;
    if (hipEventRecord(w.staged, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (forward && d_out_bytes &&
        hipMemcpyAsync(d_out_bytes, w.totals.ptr, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (forward && h_out_bytes) {
        if ((rc = read_work(ctx, st)) != CZ_OK)
            return rc;
        for (int i = 0; i < n; ++i)
            h_out_bytes[i] = (size_t)w.totals_host[i];
        return take_status(ctx, st);
    }
    return CZ_OK;
}

int cz_compress_batch(cz_ctx *ctx, int n, const cz_params *ps, const void *const *d_fields, void *const *d_outs,
                      const size_t *caps, uint64_t *d_out_bytes, size_t *h_out_bytes, void *stream)
{
    return run_batch(ctx, true, n, ps, d_fields, nullptr, d_outs, caps, d_out_bytes, h_out_bytes, stream);
}

int cz_decompress_batch(cz_ctx *ctx, int n, const cz_params *ps, const void *const *d_ins, const size_t *in_bytes,
                        void *const *d_fields, const size_t *caps, void *stream)
{
    return run_batch(ctx, false, n, ps, d_ins, in_bytes, d_fields, caps, nullptr, nullptr, stream);
}

// -------------------------------------------------------- captured plans

int cz_plan_create(cz_ctx *ctx, int op, int n, const cz_params *ps, cz_plan **out)
{
    if (!ctx || !out || (op != 0 && op != 1) || n <= 0 || !ps)
        return CZ_ERR_ARG;
    *out = nullptr;
    DeviceGuard guard(ctx->device);
    cz_plan *plan = new (std::nothrow) cz_plan();
    if (!plan)
        return CZ_ERR_ARG;
    plan->ctx = ctx;
    plan->params.assign(ps, ps + n);
    int rc = layout_batch(ctx, op == 0, n, ps, &plan->layout);
    if (rc == CZ_OK)
        rc = plan->work.init();
    if (rc == CZ_OK)
        rc = size_work(plan->work, plan->layout);
    if (rc == CZ_OK && (hipEventCreateWithFlags(&plan->done, hipEventDisableTiming) != hipSuccess ||
                        hipEventRecord(plan->done, nullptr) != hipSuccess))
        rc = CZ_ERR_HIP;
    if (rc != CZ_OK) {
        cz_plan_destroy(plan);
        return rc;
    }
    *out = plan;
    return CZ_OK;
}

int cz_plan_run(cz_plan *plan, const void *const *srcs, const size_t *src_bytes, void *const *dsts,
                const size_t *dst_caps, void *stream)
{
    if (!plan || !srcs || !dsts || !dst_caps || (!plan->layout.forward && !src_bytes))
        return CZ_ERR_ARG;
    const Layout &L = plan->layout;
    int rc = check_batch_buffers(L, plan->params.data(), srcs, src_bytes, dsts, dst_caps, nullptr);
    if (rc != CZ_OK)
        return rc;
    DeviceGuard guard(plan->ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (hipEventSynchronize(plan->done) != hipSuccess)  // the previous run has read the staging
        return CZ_ERR_HIP;
    stage_batch(plan->work, L, plan->params.data(), srcs, src_bytes, dsts);
    if (!plan->exec) {
        // capture on a private stream: upload, per-class lanes, join, status, sizes
        hipStream_t cap = nullptr;
        if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess)
            return CZ_ERR_HIP;
        rc = CZ_OK;
        if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
            rc = CZ_ERR_HIP;
        if (rc == CZ_OK)
            rc = enqueue_batch(plan->work, L, &plan->ctx->work->status, false, cap);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(cap, &g);
        if (rc == CZ_OK && e != hipSuccess)
            rc = CZ_ERR_HIP;
        if (rc == CZ_OK && hipGraphInstantiate(&plan->exec, g, nullptr, nullptr, 0) != hipSuccess)
            rc = CZ_ERR_HIP;
        plan->graph = g;
        (void)hipStreamDestroy(cap);
        if (rc != CZ_OK)
            return rc;
    }
    if (hipGraphLaunch(plan->exec, st) != hipSuccess || hipEventRecord(plan->done, st) != hipSuccess)
        return CZ_ERR_HIP;
    return CZ_OK;
}

int cz_plan_result(cz_plan *plan, void *stream, size_t *h_out_bytes)
{
    if (!plan)
        return CZ_ERR_ARG;
    DeviceGuard guard(plan->ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = read_work(plan->ctx, st);
    if (rc != CZ_OK)
        return rc;
    if (h_out_bytes && plan->layout.forward)
        for (int i = 0; i < plan->layout.n; ++i)
            h_out_bytes[i] = (size_t)plan->work.totals_host[i];
    return take_status(plan->ctx, st);
}

void cz_plan_destroy(cz_plan *plan)
{
    if (!plan)
        return;
    DeviceGuard guard(plan->ctx->device);
    (void)hipDeviceSynchronize();
    if (plan->exec)
        (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph)
        (void)hipGraphDestroy(plan->graph);
    if (plan->done)
        (void)hipEventDestroy(plan->done);
    plan->work.release();
    delete plan;
}

}  // extern "C"
