// Host-side machinery shared by the C ABI calls and the serving scheduler:
// workspace buffers, batch layout (fields grouped into kernel classes), the
// staging of device descriptor tables and the enqueue of a batch on forked
// streams.  Internal to libcz.
#ifndef CZ_HOST_H
#define CZ_HOST_H

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <tuple>
#include <vector>

#include "../../include/cz.h"
#include "cz_kernels.h"

namespace czh {

constexpr uint32_t MAGIC = 0x31425A43u;  // "CZB1" little-endian
constexpr uint64_t MAX_BLOCKS = 1ull << 31;
constexpr uint64_t HDR = 64;
constexpr int MAX_CLASSES = 24;  // 4 block sizes x 2 precisions x 3 schemes

// Device memory that grows on demand (freed with its owner).
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t want)
    {
        if (want <= bytes)
            return CZ_OK;
        void *fresh = nullptr;
        if (hipMalloc(&fresh, want) != hipSuccess)
            return CZ_ERR_HIP;
        if (ptr) {
            (void)hipDeviceSynchronize();  // earlier work may still use the old buffer
            (void)hipFree(ptr);
        }
        ptr = fresh;
        bytes = want;
        return CZ_OK;
    }
    void release()
    {
        if (ptr)
            (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
};

// Workspace of a batch: the device descriptor table and its pinned staging,
// look-back flags, per-class (ticket, status) counters, stream sizes, 64^3
// scratch, and the lanes the classes run on concurrently.
struct BatchWork {
    DevBuf desc, flags, counters, totals, scratch, fstat;
    czk::FieldDesc *stage = nullptr;  // pinned, uploaded in stream order
    uint64_t *totals_host = nullptr;  // pinned readback of stream sizes (by field)
    uint32_t *fstat_host = nullptr;   // pinned readback of per-field status (class order)
    size_t cap = 0;                   // fields the pinned buffers hold
    hipEvent_t staged = nullptr;      // the staging may be rewritten once this fired
    hipStream_t lanes[MAX_CLASSES] = {};
    hipEvent_t fork = nullptr, joins[MAX_CLASSES] = {};

    int init()
    {
        if (hipEventCreateWithFlags(&staged, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(staged, nullptr) != hipSuccess)
            return CZ_ERR_HIP;
        return CZ_OK;
    }
    // Streams (default priority) and join events for the first n lanes.
    int lanes_for(size_t n)
    {
        for (size_t i = 0; i < n && i < (size_t)MAX_CLASSES; ++i) {
            if (!lanes[i] && hipStreamCreateWithFlags(&lanes[i], hipStreamNonBlocking) != hipSuccess)
                return CZ_ERR_HIP;
            if (!joins[i] && hipEventCreateWithFlags(&joins[i], hipEventDisableTiming) != hipSuccess)
                return CZ_ERR_HIP;
        }
        return CZ_OK;
    }
    int pinned(size_t n)
    {
        if (n <= cap)
            return CZ_OK;
        if (staged)
            (void)hipEventSynchronize(staged);
        if (stage)
            (void)hipHostFree(stage);
        if (totals_host)
            (void)hipHostFree(totals_host);
        if (fstat_host)
            (void)hipHostFree(fstat_host);
        stage = nullptr;
        totals_host = nullptr;
        fstat_host = nullptr;
        cap = 0;
        if (hipHostMalloc(&stage, n * sizeof(czk::FieldDesc), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&totals_host, n * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&fstat_host, n * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess)
            return CZ_ERR_HIP;
        cap = n;
        return CZ_OK;
    }
    void release()
    {
        desc.release();
        flags.release();
        counters.release();
        totals.release();
        scratch.release();
        fstat.release();
        if (stage)
            (void)hipHostFree(stage);
        if (totals_host)
            (void)hipHostFree(totals_host);
        if (fstat_host)
            (void)hipHostFree(fstat_host);
        if (staged)
            (void)hipEventDestroy(staged);
        if (fork)
            (void)hipEventDestroy(fork);
        for (int i = 0; i < MAX_CLASSES; ++i) {
            if (lanes[i])
                (void)hipStreamDestroy(lanes[i]);
            if (joins[i])
                (void)hipEventDestroy(joins[i]);
        }
    }
};



// Class of a field: fields of one class share a kernel and one queue.
using ClassKey = std::tuple<uint32_t, uint32_t, uint32_t, uint32_t>;

struct Layout {
    bool forward = true;
    int n = 0;
    std::vector<uint64_t> nblocks;      // per field
    std::vector<int> order;             // field indices grouped by class
    std::vector<czk::KernelKey> keys;   // per class
    std::vector<uint32_t> first, count; // per class: its range in `order`
    std::vector<uint64_t> tickets;      // per class
    std::vector<int> grids;             // per class
    std::vector<size_t> scratch_off;    // per class: its 64^3 slots
    size_t scratch_bytes = 0;
    std::vector<uint64_t> flag_base;    // per field (forward): offset into the flags
    uint64_t flags_total = 0;
};


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

// A pinned host array uploaded in stream order to a device array; the host
// side is rewritten only after the previous upload has left it.
struct Staging {
    DevBuf dev;
    void *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;

    int init()
    {
        if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(done, nullptr) != hipSuccess)
            return CZ_ERR_HIP;
        return CZ_OK;
    }
    int upload(const void *src, size_t bytes, hipStream_t st)
    {
        if (hipEventSynchronize(done) != hipSuccess)
            return CZ_ERR_HIP;
        if (bytes > cap) {
            if (host)
                (void)hipHostFree(host);
            host = nullptr;
            cap = 0;
            if (hipHostMalloc(&host, bytes, hipHostMallocDefault) != hipSuccess)
                return CZ_ERR_HIP;
            cap = bytes;
        }
        int rc = dev.ensure(bytes);
        if (rc != CZ_OK)
            return rc;
        std::memcpy(host, src, bytes);
        if (hipMemcpyAsync(dev.ptr, host, bytes, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipEventRecord(done, st) != hipSuccess)
            return CZ_ERR_HIP;
        return CZ_OK;
    }
    void release()
    {
        if (done)
            (void)hipEventSynchronize(done);
        dev.release();
        if (host)
            (void)hipHostFree(host);
        if (done)
            (void)hipEventDestroy(done);
        host = nullptr;
        done = nullptr;
        cap = 0;
    }
};

int check_params(const cz_params *p, uint64_t *nblocks);
uint64_t payload_start(uint64_t nblocks);
uint64_t bound_of(const cz_params &p, uint64_t nb);
int status_to_error(uint32_t st);
int layout_batch(const cz_ctx *ctx, bool forward, int n, const cz_params *ps, Layout *L);
int size_work(BatchWork &w, const Layout &L);
void stage_batch(BatchWork &w, const Layout &L, const cz_params *ps, const void *const *srcs,
                 const size_t *src_bytes, void *const *dsts);
// status: device word the class status bits are folded into (may be null);
// per_field: also copy the per-field status words to w.fstat_host.
int enqueue_batch(BatchWork &w, const Layout &L, uint32_t *status, bool per_field, hipStream_t st);
int check_batch_buffers(const Layout &L, const cz_params *ps, const void *const *srcs, const size_t *src_bytes,
                        void *const *dsts, const size_t *dst_caps, size_t *need);
czk::KernelKey key_of(const cz_ctx *ctx, const cz_params &p);
czk::FieldDesc describe(const cz_params &p, uint64_t nb, bool forward);
int grid_for(const cz_ctx *ctx, const czk::KernelKey &key, bool inverse, uint64_t tickets);
size_t scratch_need(const czk::KernelKey &key, int grid);
czk::Queue work_queue(cz_ctx *ctx);

}  // namespace czh

struct cz_ctx {
    int device = 0;
    int num_cu = 0;
    czk::CzWork *work = nullptr;    // device: ticket, status, total of plain calls
    czk::CzWork *pinned = nullptr;  // host-pinned mirror for synchronous reads
    czh::DevBuf flags;                   // plain calls: look-back flags
    czh::DevBuf scratch;                 // plain calls on 64^3 blocks: two slots per resident workgroup
    czh::DevBuf defer;                   // plain 32^3 compress: a record slot per block (deferred records)
    czh::DevBuf dsizes;                  // plain 32^3 compress: record sizes and the fix-up's chunk flags
    czk::FieldDesc *one = nullptr;  // device: the descriptor of a plain call (published by its prep kernel)
    uint8_t variant[4][2][3] = {};  // tuned kernel variant per (N, precision, scheme)
    czh::BatchWork batch;                // batch calls
    czh::Staging sel;                    // selected-block decoding: (record, output block) pairs
    czh::DevBuf huff;                    // lossless stage: histogram, code table, chunk sizes
    czh::Staging huff_stage;             // lossless stage: header and code / decode tables
    void *noalloc = nullptr;             // device address of this device's cz_compress_noalloc scratch
};

#endif  // CZ_HOST_H
