// Kernel-side interface of the wavelet-stage library: argument blocks, the
// device workspace layout and the launchers (internal; the public ABI is
// include/cz.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace czk {

// Threads per workgroup of the scratch-staged (N = 64) kernels.
constexpr int SCRATCH_THREADS = 512;

// Status bits latched by the kernels in CzWork::status.
enum : uint32_t { STATUS_NONFINITE = 1u, STATUS_FORMAT = 2u, STATUS_TIMEOUT = 4u };

// Per-context device workspace header; the look-back flags follow it.
struct CzWork {
    uint32_t ticket;  // next block ticket
    uint32_t status;  // STATUS_* bits of the current call
    uint64_t total;   // stream bytes written by the last compress
    uint64_t reserved[6];
};

struct KernelKey {
    uint32_t block;       // N
    uint32_t scheme;      // W4 | W4LI | W3AI
    uint32_t elem_bytes;  // 4 | 8
};

struct FwdArgs {
    const void *field;   // [nz][ny][nx] of T
    uint8_t *out;        // stream
    uint64_t *offsets;   // out + 64
    uint64_t *flags;     // look-back flags, nblocks entries, zeroed
    CzWork *work;
    uint32_t nx, ny, nbx, nby;
    uint64_t nblocks;
    uint64_t p0;         // payload start
    double eps;
    float eps_f;         // smallest float >= eps (the same test for float data)
    void *scratch;       // N = 64: one N^3 slot of T per workgroup of the grid
};

struct InvArgs {
    const uint8_t *in;   // stream
    void *field;         // [nz][ny][nx] of T
    CzWork *work;
    uint32_t nx, ny, nbx, nby;
    uint64_t nblocks;
    uint64_t p0;
    uint64_t payload;    // payload bytes from the header
    void *scratch;       // N = 64: one N^3 slot of T per workgroup of the grid
};

struct PrepArgs {
    uint8_t *out;
    uint64_t *flags;
    CzWork *work;
    uint64_t nblocks;
    uint64_t p0;
    uint32_t header[16];  // the 64-byte header, payload size 0
};

hipError_t launch_fwd(const KernelKey &key, const FwdArgs &a, int grid, hipStream_t st);
hipError_t launch_inv(const KernelKey &key, const InvArgs &a, int grid, hipStream_t st);
hipError_t launch_prep_fwd(const PrepArgs &a, hipStream_t st);
hipError_t launch_prep_inv(CzWork *work, hipStream_t st);
// Resident workgroups per CU of the (fwd or inv) kernel for key.
int occupancy(const KernelKey &key, bool inverse);
int threads_per_block(const KernelKey &key);

}  // namespace czk
