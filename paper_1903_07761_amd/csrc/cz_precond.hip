// Preconditioning of a packed stream for the host lossless coder (the paper's
// Sec. 2.3, "Lossless compression" and "Wavelet types", and Sec. 4.1, Exp. 2):
//   * byte shuffle with element size k: byte j of element i goes to
//     position j * n + i (n whole elements), the tail bytes stay at the end;
//   * Z-zeroing: clear the low bits of every stored detail coefficient
//     (values outside the 4^3 coarse corner), after decimation.
// Both are bandwidth-bound passes over the stream: one thread per four
// elements for the shuffle (16-byte loads, one 4-byte word into every plane),
// one workgroup per record for the zeroing.
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

// Byte j of element i, for four consecutive elements, as one 32-bit word
// (element i in the low byte): the four bytes they put into plane j.
template <int K, typename W>
__device__ __forceinline__ uint32_t plane_word(const W (&e)[4], int j)
{
    return (uint32_t)((e[0] >> (8 * j)) & 0xFF) | (uint32_t)((e[1] >> (8 * j)) & 0xFF) << 8 |
           (uint32_t)((e[2] >> (8 * j)) & 0xFF) << 16 | (uint32_t)((e[3] >> (8 * j)) & 0xFF) << 24;
}

// Store the 4 bytes of v at p with the widest stores p's alignment allows
// (align = p's address mod 4, the same for every thread writing one plane,
// since the planes start at out + j n and threads step by 4 bytes).
__device__ __forceinline__ void store4(uint8_t *p, uint32_t v, uint32_t align)
{
    if (align % 4 == 0) {
        *reinterpret_cast<uint32_t *>(p) = v;
    } else if (align % 2 == 0) {
        reinterpret_cast<uint16_t *>(p)[0] = (uint16_t)v;
        reinterpret_cast<uint16_t *>(p)[1] = (uint16_t)(v >> 16);
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k)
            p[k] = (uint8_t)(v >> (8 * k));
    }
}

__device__ __forceinline__ uint32_t load4(const uint8_t *p, uint32_t align)
{
    if (align % 4 == 0)
        return *reinterpret_cast<const uint32_t *>(p);
    if (align % 2 == 0)
        return (uint32_t)reinterpret_cast<const uint16_t *>(p)[0] |
               (uint32_t)reinterpret_cast<const uint16_t *>(p)[1] << 16;
    return (uint32_t)p[0] | (uint32_t)p[1] << 8 | (uint32_t)p[2] << 16 | (uint32_t)p[3] << 24;
}

// One thread per four consecutive elements: their 4 K bytes are read in one
// or two 16-byte loads (element loads when the input is not 16-byte aligned),
// and each plane receives one 4-byte word, so a wavefront writes 256
// consecutive bytes of every plane.  The last n % 4 elements go byte by byte.
template <int K>
__global__ __launch_bounds__(THREADS) void shuffle_kernel(const uint8_t *__restrict__ in, uint8_t *__restrict__ out,
                                                          uint64_t n, int wide)
{
    using W = typename Word<K>::type;
    const uint64_t groups = n / 4;
    for (uint64_t g = (uint64_t)blockIdx.x * THREADS + threadIdx.x; g < groups; g += (uint64_t)gridDim.x * THREADS) {
        const uint64_t i = 4 * g;
        W e[4];
        if (wide) {
            const uint4 *src = reinterpret_cast<const uint4 *>(in + i * K);
            if constexpr (K == 4) {
                const uint4 v = src[0];
                e[0] = v.x;
                e[1] = v.y;
                e[2] = v.z;
                e[3] = v.w;
            } else {
                const uint4 v0 = src[0], v1 = src[1];
                e[0] = (W)v0.x | (W)v0.y << 32;
                e[1] = (W)v0.z | (W)v0.w << 32;
                e[2] = (W)v1.x | (W)v1.y << 32;
                e[3] = (W)v1.z | (W)v1.w << 32;
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                e[k] = reinterpret_cast<const W *>(in + i * K)[k];
        }
#pragma unroll
        for (int j = 0; j < K; ++j)
            store4(out + (uint64_t)j * n + i, plane_word<K>(e, j),
                   (uint32_t)((reinterpret_cast<uintptr_t>(out) + (uint64_t)j * n) % 4));
    }
    if (blockIdx.x == 0 && threadIdx.x < (n % 4) * K) {
        const uint64_t i = 4 * groups + threadIdx.x / K;
        const int j = (int)(threadIdx.x % K);
        out[(uint64_t)j * n + i] = in[i * K + j];
    }
}

// The inverse: each thread gathers one 4-byte word from every plane and
// writes its four elements with one or two 16-byte stores.
template <int K>
__global__ __launch_bounds__(THREADS) void unshuffle_kernel(const uint8_t *__restrict__ in, uint8_t *__restrict__ out,
                                                            uint64_t n, int wide)
{
    using W = typename Word<K>::type;
    const uint64_t groups = n / 4;
    for (uint64_t g = (uint64_t)blockIdx.x * THREADS + threadIdx.x; g < groups; g += (uint64_t)gridDim.x * THREADS) {
        const uint64_t i = 4 * g;
        W e[4] = {0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const uint32_t v =
                load4(in + (uint64_t)j * n + i, (uint32_t)((reinterpret_cast<uintptr_t>(in) + (uint64_t)j * n) % 4));
#pragma unroll
            for (int k = 0; k < 4; ++k)
                e[k] |= (W)((v >> (8 * k)) & 0xFF) << (8 * j);
        }
        if (wide) {
            uint4 *dst = reinterpret_cast<uint4 *>(out + i * K);
            if constexpr (K == 4) {
                dst[0] = uint4{e[0], e[1], e[2], e[3]};
            } else {
                dst[0] = uint4{(uint32_t)e[0], (uint32_t)(e[0] >> 32), (uint32_t)e[1], (uint32_t)(e[1] >> 32)};
                dst[1] = uint4{(uint32_t)e[2], (uint32_t)(e[2] >> 32), (uint32_t)e[3], (uint32_t)(e[3] >> 32)};
            }
        } else {
#pragma unroll
            for (int k = 0; k < 4; ++k)
                reinterpret_cast<W *>(out + i * K)[k] = e[k];
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < (n % 4) * K) {
        const uint64_t i = 4 * groups + threadIdx.x / K;
        const int j = (int)(threadIdx.x % K);
        out[i * K + j] = in[(uint64_t)j * n + i];
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

// Workgroups for n elements handled four at a time (at least one, for the
// last n % 4 elements).
int grid_for(uint64_t n)
{
    uint64_t g = (n / 4 + THREADS - 1) / THREADS;
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
    const int wide = reinterpret_cast<uintptr_t>(in) % 16 == 0;
    if (n) {
        if (elem == 4)
            hipLaunchKernelGGL(shuffle_kernel<4>, dim3(grid_for(n)), dim3(THREADS), 0, st, in, out, n, wide);
        else
            hipLaunchKernelGGL(shuffle_kernel<8>, dim3(grid_for(n)), dim3(THREADS), 0, st, in, out, n, wide);
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
    const int wide = reinterpret_cast<uintptr_t>(out) % 16 == 0;
    if (n) {
        if (elem == 4)
            hipLaunchKernelGGL(unshuffle_kernel<4>, dim3(grid_for(n)), dim3(THREADS), 0, st, in, out, n, wide);
        else
            hipLaunchKernelGGL(unshuffle_kernel<8>, dim3(grid_for(n)), dim3(THREADS), 0, st, in, out, n, wide);
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
