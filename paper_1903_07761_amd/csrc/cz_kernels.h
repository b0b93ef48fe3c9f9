// Kernel-side interface of the wavelet-stage library: the device work queue,
// the per-field descriptors it points to, and the launchers (internal; the
// public ABI is include/cz.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace czk {

// Threads per workgroup of the scratch-staged (N = 64) kernels.
constexpr int SCRATCH_THREADS = 512;

// Status bits latched by the kernels.
enum : uint32_t { STATUS_NONFINITE = 1u, STATUS_FORMAT = 2u, STATUS_TIMEOUT = 4u };

// Deferred records (32^3 forward of a single field): a block whose record
// fits DEFER_SLOT bytes writes it to slot b of the field's defer area instead
// of waiting for its predecessors' sizes; a fix-up launch places it.
constexpr uint32_t DEFER_SLOT = 8192;
constexpr uint32_t DEFER_BIT = 1u << 31;  // in sizes[b]: the record sits in its slot
constexpr uint32_t FIX_CHUNK = 1024;      // blocks per workgroup of the fix-up

// Per-context device workspace header (plain calls use its counters).
struct CzWork {
    uint32_t ticket;  // next block ticket
    uint32_t status;  // STATUS_* bits of the current call
    uint64_t total;   // stream bytes written by the last compress
    uint64_t reserved[6];
};

// One field of a work queue.  Forward: src = field, dst = stream; inverse:
// src = stream, dst = field.
struct FieldDesc {
    const void *src;
    void *dst;
    uint64_t *flags;      // forward: look-back flags, nblocks entries
    uint64_t *total;      // forward: stream bytes, written by the last block (may be null)
    uint32_t nx, ny, nbx, nby;
    uint64_t nblocks;
    uint64_t p0;          // payload start
    uint64_t payload;     // inverse: payload bytes available
    uint64_t first;       // the field's first ticket in its queue
    const uint32_t *sel;  // inverse, optional: ticket k decodes record sel[k] (else record k)
    uint64_t rblocks;     // inverse: records in the stream (sel entries must be below)
    double eps;
    float eps_f;          // smallest float >= eps (the same test for float data)
    uint32_t cstride;     // forward: elements between consecutive cells of src (1 = a plain field)
    uint32_t header[16];  // forward: the 64-byte header, payload size 0
    uint8_t *defer;       // forward, optional: nblocks slots of DEFER_SLOT bytes (32^3 blocks)
    uint32_t *sizes;      // with defer: nblocks record sizes, then the fix-up's chunk flags (u64)
};

// A device work queue: tickets [0, ntickets) map, in order, onto the blocks
// of the fields (field f owns tickets [first_f, first_f + nblocks_f)).  A
// single-field call passes its descriptor inline (`one`) with `publish` ==
// `fields` pointing at a device slot; its prep kernel copies the descriptor
// there before the block kernel runs.
struct Queue {
    const FieldDesc *fields;  // the block kernels read every descriptor from here
    uint32_t nfields;
    uint32_t reserved;
    uint64_t ntickets;
    uint32_t *ticket;     // device ticket counter
    uint32_t *status;     // device STATUS_* bits
    uint32_t *fstatus;    // optional: STATUS_* bits per field, indexed like fields
    void *scratch;        // N = 64: one N^3 slot of the field type per workgroup
    FieldDesc *publish;   // optional: the prep kernel copies `one` here (a one-field table)
    FieldDesc one;
};

struct KernelKey {
    uint32_t block;       // N
    uint32_t scheme;      // W4 | W4LI | W3AI
    uint32_t elem_bytes;  // 4 | 8
    uint32_t variant;     // tuning variant (see variant_count)
};

hipError_t launch_fwd(const KernelKey &key, const Queue &q, int grid, hipStream_t st);
hipError_t launch_inv(const KernelKey &key, const Queue &q, int grid, hipStream_t st);
// Reset the queue's ticket and status; forward: clear each field's flags and
// write its header, offset 0 and the pad before its payload.
hipError_t launch_prep(const Queue &q, bool forward, hipStream_t st);
// After a single-field forward with deferred records: offsets of every block
// (chunked scan of sizes[]), deferred records moved from their slots into the
// stream, the payload size in the header and *total.
hipError_t launch_defer_fix(const Queue &q, hipStream_t st);
// Bytes of the sizes area (sizes, then 8-byte-aligned chunk flags) for nblocks.
size_t defer_sizes_bytes(uint64_t nblocks);
// OR the status words of nclass (ticket, status) counter pairs into *status.
hipError_t launch_fold_status(const uint32_t *counters, int nclass, uint32_t *status, hipStream_t st);
// Resident workgroups per CU of the (fwd or inv) kernel for key.
int occupancy(const KernelKey &key, bool inverse);
// Forward launches one workgroup per ticket up to 32^3 (grid = tickets).
bool fwd_one_block_per_workgroup(const KernelKey &key);
// Blocks a forward ticket covers: a group of consecutive blocks of one field
// for 8^3 and 16^3 (one per wavefront), else one.  A field of nb blocks owns
// ceil(nb / this) forward tickets, and its look-back flags are per ticket.
uint32_t fwd_blocks_per_ticket(const KernelKey &key);
// Number of compiled shape variants for (block, elem_bytes).
int variant_count(uint32_t block, uint32_t elem_bytes);
// Upper bound on the workgroups of a launch (0: none).
int grid_cap(const KernelKey &key);
// Scratch bytes a launch of grid workgroups needs (N = 64; else 0).
size_t scratch_bytes(const KernelKey &key, int grid);

}  // namespace czk
