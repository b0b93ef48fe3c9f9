// Preconditioning of a packed stream for the host lossless coder (the paper's
// Sec. 2.3, "Lossless compression" and "Wavelet types", and Sec. 4.1, Exp. 2):
//   * byte shuffle with element size k: byte j of element i goes to
//     position j * n + i (n whole elements), the tail bytes stay at the end;
//   * Z-zeroing: clear the low bits of every stored detail coefficient
//     (values outside the 4^3 coarse corner), after decimation.
// Both are bandwidth-bound passes over the stream: one thread per element
// for the shuffle (k-byte loads, byte stores that coalesce into 64-byte runs
// per plane), one workgroup per record for the zeroing.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cz_host.h"

namespace {

constexpr int THREADS = 256;

template <int K>
struct Word;
template <>
struct Word<4> {
    using type = uint32_t;
};
template <>
struct Word<8> {
    using type = uint64_t;
};

template <int K>
__global__ __launch_bounds__(THREADS) void shuffle_kernel(const uint8_t *__restrict__ in, uint8_t *__restrict__ out,
                                                          uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * THREADS + threadIdx.x; i < n; i += (uint64_t)gridDim.x * THREADS) {
        using W = typename Word<K>::type;
        const W w = *reinterpret_cast<const W *>(in + i * K);  // the element, one aligned load
#pragma unroll
        for (int j = 0; j < K; ++j)
            out[(uint64_t)j * n + i] = (uint8_t)(w >> (8 * j));
    }
}

template <int K>
__global__ __launch_bounds__(THREADS) void unshuffle_kernel(const uint8_t *__restrict__ in, uint8_t *__restrict__ out,
                                                            uint64_t n)
{
    for (uint64_t i = (uint64_t)blockIdx.x * THREADS + threadIdx.x; i < n; i += (uint64_t)gridDim.x * THREADS) {
        using W = typename Word<K>::type;
        W w = 0;
#pragma unroll
        for (int j = 0; j < K; ++j)
            w |= (W)in[(uint64_t)j * n + i] << (8 * j);
        *reinterpret_cast<W *>(out + i * K) = w;  // the element, one aligned store
    }
}

// Zero the low bits of the detail values of record b.  The 64 coarse values
// sit at q = x + N (y + N z) with x, y, z < 4: sixteen runs of four kept
// values (corner bits are always set), whose first ranks are the popcounts of
// the mask below q.  Records are validated against the offsets first; an
// inconsistent one is left alone and flagged.
template <typename U, int N>
__global__ __launch_bounds__(THREADS) void zero_kernel(uint8_t *stream, uint64_t nblocks, uint64_t p0,
                                                       uint64_t payload, U clear, uint32_t *status)
{
    constexpr uint32_t MASK_BYTES = N * N * N / 8;
    __shared__ uint32_t s_run[16];
    __shared__ uint32_t s_ok;
    const uint64_t b = blockIdx.x;
    const uint64_t *offs = reinterpret_cast<const uint64_t *>(stream + 64);
    if (threadIdx.x == 0) {
        const uint64_t o0 = offs[b], o1 = offs[b + 1];
        uint32_t ok = o1 >= o0 && o1 <= payload && o1 - o0 >= 8ull + MASK_BYTES;
        if (ok) {
            const uint32_t nnz = *reinterpret_cast<const uint32_t *>(stream + p0 + o0);
            const uint64_t used = 8ull + MASK_BYTES + (uint64_t)nnz * sizeof(U);
            ok = nnz <= (uint32_t)(N * N * N) && ((used + 15ull) & ~15ull) == o1 - o0;
        }
        if (!ok)
            atomicOr(status, czk::STATUS_FORMAT);
        s_ok = ok;
    }
    __syncthreads();
    if (!s_ok)
        return;
    uint8_t *rec = stream + p0 + offs[b];
    const uint32_t nnz = *reinterpret_cast<const uint32_t *>(rec);
    const uint64_t *mask = reinterpret_cast<const uint64_t *>(rec + 8);
    if (threadIdx.x < 16) {
        const int y = threadIdx.x % 4, z = threadIdx.x / 4;
        const uint32_t q0 = (uint32_t)(N * (y + N * z));
        uint32_t r = 0;
        for (uint32_t w = 0; w < q0 / 64; ++w)
            r += (uint32_t)__popcll(mask[w]);
        const uint32_t below = q0 % 64;
        if (below)
            r += (uint32_t)__popcll(mask[q0 / 64] & ((1ull << below) - 1ull));
        s_run[threadIdx.x] = r;
    }
    __syncthreads();
    U *vals = reinterpret_cast<U *>(rec + 8 + MASK_BYTES);
    for (uint32_t r = threadIdx.x; r < nnz; r += THREADS) {
        bool coarse = false;
#pragma unroll
        for (int k = 0; k < 16; ++k)
            coarse |= r - s_run[k] < 4u;
        if (!coarse)
            vals[r] &= clear;
    }
}

int grid_for(uint64_t n)
{
    uint64_t g = (n + THREADS - 1) / THREADS;
    return (int)(g > 65536 ? 65536 : g < 1 ? 1 : g);
}

}  // namespace

extern "C" {

int cz_shuffle(const void *d_in, size_t nbytes, uint32_t elem, void *d_out, void *stream)
{
    if (elem != 4 && elem != 8)
        return CZ_ERR_ARG;
    if (nbytes == 0)
        return CZ_OK;
    if (!d_in || !d_out || d_in == d_out || reinterpret_cast<uintptr_t>(d_in) % elem)
        return CZ_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint64_t n = nbytes / elem;
    const uint8_t *in = static_cast<const uint8_t *>(d_in);
    uint8_t *out = static_cast<uint8_t *>(d_out);
    if (n) {
        if (elem == 4)
            hipLaunchKernelGGL(shuffle_kernel<4>, dim3(grid_for(n)), dim3(THREADS), 0, st, in, out, n);
        else
            hipLaunchKernelGGL(shuffle_kernel<8>, dim3(grid_for(n)), dim3(THREADS), 0, st, in, out, n);
        if (hipGetLastError() != hipSuccess)
            return CZ_ERR_HIP;
    }
    const size_t tail = nbytes - n * elem;
    if (tail && hipMemcpyAsync(out + n * elem, in + n * elem, tail, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return CZ_ERR_HIP;
    return CZ_OK;
}

int cz_unshuffle(const void *d_in, size_t nbytes, uint32_t elem, void *d_out, void *stream)
{
    if (elem != 4 && elem != 8)
        return CZ_ERR_ARG;
    if (nbytes == 0)
        return CZ_OK;
    if (!d_in || !d_out || d_in == d_out || reinterpret_cast<uintptr_t>(d_out) % elem)
        return CZ_ERR_ARG;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint64_t n = nbytes / elem;
    const uint8_t *in = static_cast<const uint8_t *>(d_in);
    uint8_t *out = static_cast<uint8_t *>(d_out);
    if (n) {
        if (elem == 4)
            hipLaunchKernelGGL(unshuffle_kernel<4>, dim3(grid_for(n)), dim3(THREADS), 0, st, in, out, n);
        else
            hipLaunchKernelGGL(unshuffle_kernel<8>, dim3(grid_for(n)), dim3(THREADS), 0, st, in, out, n);
        if (hipGetLastError() != hipSuccess)
            return CZ_ERR_HIP;
    }
    const size_t tail = nbytes - n * elem;
    if (tail && hipMemcpyAsync(out + n * elem, in + n * elem, tail, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return CZ_ERR_HIP;
    return CZ_OK;
}

int cz_zero_details(cz_ctx *ctx, const cz_params *p, void *d_stream, size_t nbytes, uint32_t bits, void *stream)
{
    if (!ctx || !p || !d_stream)
        return CZ_ERR_ARG;
    uint64_t nb = 0;
    int rc = czh::check_params(p, &nb);
    if (rc != CZ_OK)
        return rc;
    const uint32_t maxbits = p->elem_bytes == 4 ? 23u : 52u;
    if (bits > maxbits)
        return CZ_ERR_ARG;
    const uint64_t p0 = czh::payload_start(nb);
    if (nbytes < p0)
        return CZ_ERR_FORMAT;
    if (bits == 0 || nb == 0)
        return CZ_OK;
    czh::DeviceGuard guard(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t *s = static_cast<uint8_t *>(d_stream);
    uint32_t *status = &ctx->work->status;
    const uint64_t payload = nbytes - p0;
    const dim3 grid((unsigned)nb), block(THREADS);
#define CZ_ZERO(U, NN)                                                                                       \
    hipLaunchKernelGGL((zero_kernel<U, NN>), grid, block, 0, st, s, nb, p0, payload,                         \
                       (U)~((((U)1) << bits) - (U)1), status)
    if (p->elem_bytes == 4) {
        switch (p->block) {
        case 8: CZ_ZERO(uint32_t, 8); break;
        case 16: CZ_ZERO(uint32_t, 16); break;
        case 32: CZ_ZERO(uint32_t, 32); break;
        default: CZ_ZERO(uint32_t, 64); break;
        }
    } else {
        switch (p->block) {
        case 8: CZ_ZERO(uint64_t, 8); break;
        case 16: CZ_ZERO(uint64_t, 16); break;
        case 32: CZ_ZERO(uint64_t, 32); break;
        default: CZ_ZERO(uint64_t, 64); break;
        }
    }
#undef CZ_ZERO
    return hipGetLastError() == hipSuccess ? CZ_OK : CZ_ERR_HIP;
}

}  // extern "C"
