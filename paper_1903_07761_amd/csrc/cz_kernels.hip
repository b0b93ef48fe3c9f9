// HIP kernels of the CubismZ wavelet stage for MI355X (gfx950).
//
// Paper: arXiv 1903.07761.  Sec. 2.3 ("Wavelet-based compression", "Wavelet
// types", "Data decompression") defines the per-block 3D transform, the
// decimation at eps and the mask + coefficient stream; Sec. 2.2 places each
// compressed piece with an exclusive prefix scan of the sizes.
//
// Design (one workgroup per N^3 block at a time, persistent over a block
// ticket counter):
//   * the workgroup has N*N threads; thread (x, y) owns the z-column of the
//     block in VGPRs, so the global load and store of a block are coalesced
//     rows (consecutive x in consecutive lanes);
//   * the finest level runs its x- and y-lines through LDS one group of Z
//     z-slabs at a time (Z = N keeps a 32^3 float block whole in LDS; double
//     blocks, 256 KiB at N = 32, are staged by slab), each line transformed
//     in registers by one thread, then the z-lines in registers;
//   * the coarser levels (at most (N/2)^3): x- and y-lines in LDS, z-lines in
//     the registers of the columns that hold them;
//   * decimation: one wavefront ballot per 64 consecutive coefficients gives a
//     mask word directly in the stream's bit order; word popcounts are scanned
//     across the workgroup, and each kept value's rank is the word prefix plus
//     mbcnt of its lanes below;
//   * record offsets: a single-pass decoupled look-back over block tickets
//     (each block publishes its record size as soon as its nnz is known, then
//     accumulates predecessors until it meets an inclusive prefix);
//   * the inverse mirrors the forward: mask words to LDS, ranks by prefix
//     popcount, gather, coarse levels, z-lines in registers, y and x
//     lines by slab group through LDS, coalesced store.
// The path is a short stencil plus a scan: bound by HBM bandwidth, no MFMA.
#pragma clang fp contract(off)

#include <hip/hip_runtime.h>

#include <cstdint>

#include "cz_lines.h"
#include "cz_kernels.h"
#include "cz_lookback.h"

namespace czk {

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Workgroup barrier that orders LDS only.  __syncthreads() also releases
// global memory, which costs a wait for every load and store still in flight;
// all communication between the threads of a workgroup here goes through LDS,
// so in-flight global accesses may stay in flight across this barrier.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Orders LDS accesses among the lanes of one wavefront (a wavefront's LDS
// instructions execute in program order; the fences keep the compiler from
// moving one lane's access across another lane's).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Exclusive scan of one u32 per thread over a workgroup of NT threads.
// s_w must hold NT/64 + 1 words; the total lands in s_w[NT/64].
template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_w)
{
    constexpr int NW = NT / 64;
    const uint32_t lane = lane_id();
    const uint32_t wave = threadIdx.x / 64;
    uint32_t inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(inc, off, 64);
        if (lane >= (uint32_t)off)
            inc += t;
    }
    if constexpr (NW == 1) {
        if (lane == 63)
            s_w[1] = inc;
        lds_barrier();
        return inc - v;
    } else {
        if (lane == 63)
            s_w[wave] = inc;
        lds_barrier();
        if (wave == 0) {
            uint32_t w = lane < (uint32_t)NW ? s_w[lane] : 0u;
            uint32_t wi = w;
#pragma unroll
            for (int off = 1; off < NW; off <<= 1) {
                uint32_t t = __shfl_up(wi, off, 64);
                if (lane >= (uint32_t)off)
                    wi += t;
            }
            if (lane < (uint32_t)NW)
                s_w[lane] = wi - w;
            if (lane == (uint32_t)NW - 1)
                s_w[NW] = wi;
        }
        lds_barrier();
        return inc - v + s_w[wave];
    }
}

// ------------------------------------------------------------------ LDS lines

// Transform (fwd or inv) every line along `axis` of the region [0,n)^3 of an
// LDS array with pitches (1, PY, PZ), one line per thread for the first n*n
// threads.  Lanes run along the fastest of the two other axes.
template <typename T, int S, int n, int AXIS, bool INV, int PY, int PZ>
__device__ __forceinline__ void lds_lines(T *lds)
{
    const int t = threadIdx.x;
    if (t < n * n) {
        const int i = t % n, j = t / n;
        int base, stride;
        if constexpr (AXIS == 0) {
            base = i * PY + j * PZ;
            stride = 1;
        } else if constexpr (AXIS == 1) {
            base = i + j * PZ;
            stride = PY;
        } else {
            base = i + j * PY;
            stride = PZ;
        }
        T v[n];
#pragma unroll
        for (int k = 0; k < n; ++k)
            v[k] = lds[base + k * stride];
        if constexpr (INV)
            line_inv<T, S, n>(v);
        else
            line_fwd<T, S, n>(v);
#pragma unroll
        for (int k = 0; k < n; ++k)
            lds[base + k * stride] = v[k];
    }
}

// Forward levels n, n/2, ..., 8 of the coarse region [0, n)^3 (LDS pitches
// PY, PZ), which is in LDS on entry: x- and y-lines in LDS, z-lines in the
// registers of the columns' owners (the thread of column (x, y), x, y < n,
// holds z in [0, n) in c[r], y = yq + r YR); on return the region's final
// coefficients are in c.  Each level's z-lines need no LDS pass.
template <typename T, int S, int n, int PY, int PZ, int R, int YR, int NC>
__device__ __forceinline__ void coarse_fwd(T (&c)[R][NC], T *lds, int x, int yq)
{
    lds_lines<T, S, n, 0, false, PY, PZ>(lds);
    lds_barrier();
    lds_lines<T, S, n, 1, false, PY, PZ>(lds);
    lds_barrier();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = yq + r * YR;
        if (r * YR < n && x < n && y < n) {
#pragma unroll
            for (int z = 0; z < n; ++z)
                c[r][z] = lds[z * PZ + y * PY + x];
            line_fwd<T, S, n>(c[r]);
        }
    }
    if constexpr (n / 2 >= 8) {
        // the next level's region back to LDS (each owner its own column)
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = yq + r * YR;
            if (r * YR < n / 2 && x < n / 2 && y < n / 2) {
#pragma unroll
                for (int z = 0; z < n / 2; ++z)
                    lds[z * PZ + y * PY + x] = c[r][z];
            }
        }
        lds_barrier();
        coarse_fwd<T, S, n / 2, PY, PZ, R, YR, NC>(c, lds, x, yq);
    }
}

// Inverse levels 8, 16, ..., n of the coarse region [0, n)^3, which is in
// the owners' registers on entry (as coarse_fwd leaves it) and on return:
// each level's z-lines there, its y- and x-lines in LDS.
template <typename T, int S, int n, int PY, int PZ, int R, int YR, int NC>
__device__ __forceinline__ void coarse_inv(T (&c)[R][NC], T *lds, int x, int yq)
{
    if constexpr (n / 2 >= 8)
        coarse_inv<T, S, n / 2, PY, PZ, R, YR, NC>(c, lds, x, yq);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = yq + r * YR;
        if (r * YR < n && x < n && y < n) {
            line_inv<T, S, n>(c[r]);
#pragma unroll
            for (int z = 0; z < n; ++z)
                lds[z * PZ + y * PY + x] = c[r][z];
        }
    }
    lds_barrier();
    lds_lines<T, S, n, 1, true, PY, PZ>(lds);
    lds_barrier();
    lds_lines<T, S, n, 0, true, PY, PZ>(lds);
    lds_barrier();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = yq + r * YR;
        if (r * YR < n && x < n && y < n) {
#pragma unroll
            for (int z = 0; z < n; ++z)
                c[r][z] = lds[z * PZ + y * PY + x];
        }
    }
}

template <typename T>
__device__ __forceinline__ bool finite(T v)
{
    return __builtin_isfinite(v);
}

// ------------------------------------------------------- buffer addressing
// Raw buffer accesses: a wave-uniform 128-bit resource (base, byte extent)
// in SGPRs plus a 32-bit per-lane byte offset, so a row access costs one VGPR
// of address instead of a 64-bit pair; accesses past the extent read 0 and
// drop writes.  Cache policy NT (non-temporal) for data streamed once.

using rsrc_t = __amdgpu_buffer_rsrc_t;
static constexpr int RSRC_DWORD3 = 0x00020000;  // raw buffer, gfx9 family
static constexpr int CPOL_NT = 2;

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, RSRC_DWORD3);
}

template <typename T>
__device__ __forceinline__ T buf_load(rsrc_t r, uint32_t voff);
template <>
__device__ __forceinline__ float buf_load<float>(rsrc_t r, uint32_t voff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, CPOL_NT));
}
template <>
__device__ __forceinline__ double buf_load<double>(rsrc_t r, uint32_t voff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, CPOL_NT));
}

__device__ __forceinline__ void buf_store(float v, rsrc_t r, uint32_t voff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, 0, CPOL_NT);
}
__device__ __forceinline__ void buf_store(double v, rsrc_t r, uint32_t voff)
{
    using u2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, 0, CPOL_NT);
}

// --------------------------------------------------------------- geometry

// N^3 block, Z z-slabs staged in LDS at a time, R z-columns per thread, and
// (forward) ZP z-planes kept in VGPRs after the finest level: planes
// [ZP, N) -- final level-1 details -- are parked in the LDS the staging
// frees, behind the coarse region.
// Thread t owns the columns (x, y_r) with x = t % N and
// y_r = t / N + r N / R, r = 0..R-1; for a fixed z and r the workgroup's
// threads hold N^2 / R consecutive coefficients q = x + N (y + N z), so each
// wavefront holds 64 consecutive q: one mask word.
template <typename T, int N, int Z, int R, int ZP = N>
struct Geom {
    static constexpr int NT = N * N / R;      // threads per workgroup
    static constexpr int YR = N / R;          // row stride between a thread's columns
    static constexpr int H = N / 2;
    static constexpr int PX = N + 1;          // finest-level staging: row pitch
    static constexpr int PS = N * PX;         //                       slab pitch
    static constexpr int QX = H + 1;          // coarse levels: row pitch
    static constexpr int QS = H * QX;         //                slab pitch
    static constexpr int STAGE = Z * PS;
    static constexpr int COARSE = H * QS;
    static constexpr int PARK = (N - ZP) * PS;  // parked planes, staging pitches
    static constexpr int LDS_ELEMS = STAGE > COARSE + PARK ? STAGE : COARSE + PARK;
    static constexpr int WAVES = NT / 64;     // wavefronts per workgroup
    static constexpr int WORDS = N * N * N / 64;  // mask words per block
    static constexpr uint32_t MASK_BYTES = (uint32_t)(N * N * N / 8);
    static_assert(N % Z == 0 && Z >= 1, "slab depth must divide the block edge");
    static_assert(NT % 64 == 0 && N % R == 0, "a workgroup is whole wavefronts");
    static_assert(WORDS <= NT, "one mask word per thread at most");
    static_assert(COARSE * sizeof(T) >= WORDS * sizeof(uint32_t), "coarse area reused for word prefixes");
    static_assert(ZP >= H && ZP <= N, "the coarse region stays in VGPRs");
    // mask word of (z, r) for wavefront w
    static __device__ __forceinline__ int word(int z, int r, int w) { return (z * R + r) * WAVES + w; }
};

// Finest level, one slab group: every line along x (AXIS 0) or y (AXIS 1) of
// the Z staged slabs, one line per thread per step, lanes along the other
// in-slab axis (row pitch PX is odd, so neither access pattern conflicts).
template <typename T, int S, int N, int Z, int NT, int PX, int PS, int AXIS, bool INV>
__device__ __forceinline__ void stage_lines(T *lds)
{
#pragma unroll 1
    for (int l = threadIdx.x; l < Z * N; l += NT) {
        const int i = l % N, j = l / N;
        const int base = j * PS + (AXIS == 0 ? i * PX : i);
        constexpr int stride = AXIS == 0 ? 1 : PX;
        T v[N];
#pragma unroll
        for (int k = 0; k < N; ++k)
            v[k] = lds[base + k * stride];
        if constexpr (INV)
            line_inv<T, S, N>(v);
        else
            line_fwd<T, S, N>(v);
#pragma unroll
        for (int k = 0; k < N; ++k)
            lds[base + k * stride] = v[k];
    }
}

// ------------------------------------------------------------------ forward

// Decimation test |c| >= eps in double.  For float data this equals
// |c| >= eps_f with eps_f the smallest float >= eps (computed on the host).
// What a block kernel needs of its field (see field_view).
struct FieldView {
    const void *src;
    void *dst;
    uint64_t *flags;
    uint64_t *total;
    uint32_t nx, ny, nbx, nby;
    uint64_t nblocks, p0, payload, first;
    const uint32_t *sel;
    uint64_t rblocks;
    double eps;
    float eps_f;
    uint32_t cs;  // element stride of the source (interleaved state), 1 for a plain field
};

template <typename T>
__device__ __forceinline__ bool keep_test(T v, const FieldView &a);
template <>
__device__ __forceinline__ bool keep_test<float>(float v, const FieldView &a)
{
    return __builtin_fabsf(v) >= a.eps_f;
}
template <>
__device__ __forceinline__ bool keep_test<double>(double v, const FieldView &a)
{
    return __builtin_fabs(v) >= a.eps;
}

// Issue the loads of slab group g of block b: planes [g Z, g Z + Z), one
// coalesced row segment per plane and column.
template <typename T, int N, int Z, int R>
__device__ __forceinline__ void load_planes(const FieldView &a, uint64_t b, int g, uint32_t lane_off, T (*dst)[N])
{
    using G = Geom<T, N, Z, R>;
    // source strides in elements (a.cs > 1: one quantity of an interleaved state)
    const uint32_t row = a.nx * a.cs;
    const size_t plane = (size_t)row * a.ny;
    const uint32_t bx = (uint32_t)(b % a.nbx);
    const uint32_t by = (uint32_t)((b / a.nbx) % a.nby);
    const uint32_t bz = (uint32_t)(b / ((uint64_t)a.nbx * a.nby));
    const T *blk = static_cast<const T *>(a.src) + ((size_t)bz * N * plane + (size_t)by * N * row + (size_t)bx * N * a.cs);
    const uint32_t slab_bytes = ((uint32_t)(N - 1) * row + N * a.cs) * (uint32_t)sizeof(T);
#pragma unroll
    for (int j = 0; j < Z; ++j) {
        const rsrc_t zr = make_rsrc(blk + (size_t)(g * Z + j) * plane, slab_bytes);
#pragma unroll
        for (int r = 0; r < R; ++r)
            dst[r][g * Z + j] = buf_load<T>(zr, (lane_off + (uint32_t)(r * G::YR) * row) * (uint32_t)sizeof(T));
    }
}

// The field that owns ticket t (fields hold consecutive ticket ranges).
__device__ __forceinline__ uint32_t field_of_ticket(const Queue &q, uint64_t t)
{
    uint32_t lo = 0, hi = q.nfields - 1;  // last field whose range starts at or before t
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (q.fields[mid].first <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

// The descriptor of field f as the prep kernel sees it: a one-field queue
// carries it inline until the prep kernel publishes it to q.fields.
__device__ __forceinline__ const FieldDesc &field_desc(const Queue &q, uint32_t f)
{
    return q.publish ? q.one : q.fields[f];
}

// The per-field values the block kernels read.  The field index is made
// wave-uniform first, so the descriptor is fetched from the table with scalar
// loads into SGPRs instead of occupying VGPRs for the whole block.  (One
// source only: choosing between two descriptor sources costs SGPRs for the
// whole kernel and measurably slows the forward transform.)
__device__ __forceinline__ FieldView view_of(const FieldDesc &d)
{
    return FieldView{d.src, d.dst, d.flags, d.total, d.nx, d.ny, d.nbx, d.nby, d.nblocks, d.p0, d.payload, d.first,
                     d.sel, d.rblocks, d.eps, d.eps_f, d.cstride};
}

// The table is read through the constant address space: it is written before
// the launch (host copy or the prep kernel) and never during it, and only
// loads from that space become scalar loads through the scalar cache; a
// generic pointer would make them vector loads, each a full memory round trip
// on the path to the block's first load.
using ConstDesc = const __attribute__((address_space(4))) FieldDesc;

__device__ __forceinline__ FieldView field_view(const Queue &q, uint32_t f)
{
    f = __builtin_amdgcn_readfirstlane(f);
    ConstDesc *d = (ConstDesc *)q.fields + f;
    return FieldView{d->src, d->dst, d->flags, d->total, d->nx, d->ny, d->nbx, d->nby, d->nblocks, d->p0,
                     d->payload, d->first, d->sel, d->rblocks, d->eps, d->eps_f, d->cstride};
}

// Latch STATUS_* bits for the queue and, when per-field words exist, for
// field f.
__device__ __forceinline__ void report(const Queue &q, uint32_t f, uint32_t bits)
{
    atomicOr(q.status, bits);
    if (q.fstatus)
        atomicOr(q.fstatus + f, bits);
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// One workgroup per block: the block's ticket is taken at workgroup start,
// so every smaller ticket belongs to a workgroup that is resident or done and
// the look-back always completes.
// Waves per SIMD the forward kernel's registers must leave room for: what
// one workgroup implies, except for float 32^3 blocks with two columns a
// thread and ZP = 18 (76 KiB of LDS), which run two workgroups a CU.
template <typename T, int N, int Z, int R, int ZP>
struct FwdWaves {
    static constexpr int one = N * N / R / 256 > 0 ? N * N / R / 256 : 1;
    static constexpr int value = sizeof(T) == 4 && N == 32 && Z == 16 && R == 2 && ZP == 18 ? 2 * one : one;
};

template <typename T, int N, int S, int Z, int R, int ZP>
__global__ __launch_bounds__(N *N / R, (FwdWaves<T, N, Z, R, ZP>::value)) void fwd_kernel(Queue q)
{
    using G = Geom<T, N, Z, R, ZP>;
    __shared__ T lds[G::LDS_ELEMS];
    __shared__ uint64_t s_words[G::WORDS];
    __shared__ uint32_t s_scan[G::WAVES + 1];
    __shared__ uint64_t s_block;
    __shared__ uint32_t s_field;
    __shared__ uint64_t s_off;

    const int tid = threadIdx.x;
    const int x = tid % N, yq = tid / N;
    const uint32_t lane = lane_id();
    const int wave = tid / 64;

    if (tid == 0) {
        const uint64_t t = atomicAdd(q.ticket, 1u);
        s_block = t;
        s_field = t < q.ntickets ? field_of_ticket(q, t) : 0u;
    }
    lds_barrier();
    const uint64_t t = uniform64(s_block);
    if (t >= q.ntickets)
        return;
    const FieldView a = field_view(q, s_field);
    const uint64_t b = t - a.first;
    const uint32_t lane_off = ((uint32_t)yq * a.nx + (uint32_t)x) * a.cs;  // element offset of (x, yq) in a z-plane
    // the defer area (read now, so the scalar loads overlap the block's loads)
    ConstDesc *desc = (ConstDesc *)q.fields + __builtin_amdgcn_readfirstlane(s_field);
    uint8_t *const slots = desc->defer;
    uint32_t *const sizes = desc->sizes;

    // load: for each z and r one coalesced row segment of N elements; the
    // rows of slab group g+1 stay in flight while group g is transformed
    T c[R][N];
    bool bad = false;
    load_planes<T, N, Z, R>(a, b, 0, lane_off, c);

    // finest level: x- and y-lines per slab group in LDS, z in VGPRs
#pragma unroll
    for (int g = 0; g < N / Z; ++g) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int j = 0; j < Z; ++j)
                lds[j * G::PS + (yq + r * G::YR) * G::PX + x] = c[r][g * Z + j];
        if (g + 1 < N / Z)
            load_planes<T, N, Z, R>(a, b, g + 1, lane_off, c);
        lds_barrier();
        stage_lines<T, S, N, Z, G::NT, G::PX, G::PS, 0, false>(lds);
        lds_barrier();
        stage_lines<T, S, N, Z, G::NT, G::PX, G::PS, 1, false>(lds);
        lds_barrier();
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int j = 0; j < Z; ++j)
                c[r][g * Z + j] = lds[j * G::PS + (yq + r * G::YR) * G::PX + x];
        lds_barrier();
    }
    // z-lines of the finest level, one column at a time; planes [ZP, N)
    // (final level-1 details) are parked in LDS right away
    T *park = lds + G::COARSE;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        __builtin_amdgcn_sched_barrier(0);
        line_fwd<T, S, N>(c[r]);
#pragma unroll
        for (int z = ZP; z < N; ++z)
            park[(z - ZP) * G::PS + (yq + r * G::YR) * G::PX + x] = c[r][z];
    }
    __builtin_amdgcn_sched_barrier(0);

    // coarser levels: [0, N/2)^3 (only columns with x, y < N/2 take part)
    if constexpr (N / 2 >= 8) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (r * G::YR < G::H) {
                const int y = yq + r * G::YR;
                if (x < G::H && y < G::H) {
#pragma unroll
                    for (int z = 0; z < G::H; ++z)
                        lds[z * G::QS + y * G::QX + x] = c[r][z];
                }
            }
        }
        lds_barrier();
        coarse_fwd<T, S, G::H, G::QX, G::QS, R, G::YR, N>(c, lds, x, yq);
    }

    // decimation: keep the 4^3 corner and |c| >= eps (compared in double).
    // Every input sample reaches some coefficient with a non-zero weight, so a
    // non-finite input always leaves a non-finite coefficient: checking the
    // coefficients covers the input too (and keeps the loaded values from
    // staying live until here).
    uint32_t keepbits[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int y = yq + r * G::YR;
        uint32_t kb = 0;
#pragma unroll
        for (int z = 0; z < ZP; ++z) {
            const T v = c[r][z];
            bad |= !finite(v);
            const bool keep = (z < 4 && x < 4 && y < 4) || keep_test<T>(v, a);
            kb |= (uint32_t)keep << z;
        }
        const T *pk = park + y * G::PX + x;
#pragma unroll
        for (int z = ZP; z < N; ++z) {
            const T v = pk[(z - ZP) * G::PS];
            bad |= !finite(v);
            kb |= (uint32_t)keep_test<T>(v, a) << z;
        }
        keepbits[r] = kb;
    }
    if (bad)
        report(q, s_field, STATUS_NONFINITE);
    // mask words: lane z R + r of each wavefront keeps the ballot of (z, r)
    uint64_t myword = 0;
#pragma unroll
    for (int z = 0; z < N; ++z) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const uint64_t m = __ballot((keepbits[r] >> z) & 1u);
            myword = lane == (uint32_t)(z * R + r) ? m : myword;
        }
    }
    if (lane < (uint32_t)(N * R))
        s_words[(int)lane * G::WAVES + wave] = myword;
    lds_barrier();

    // word popcounts -> exclusive prefix in q order
    const uint32_t cnt = tid < G::WORDS ? (uint32_t)__popcll(s_words[tid]) : 0u;
    const uint32_t pre = block_exclusive_scan<G::NT>(cnt, s_scan);
    const uint32_t nnz = s_scan[G::WAVES];
    uint32_t *s_pre = reinterpret_cast<uint32_t *>(lds);  // coarse data already read back
    if (tid < G::WORDS)
        s_pre[tid] = pre;

    const uint64_t used = 8ull + G::MASK_BYTES + (uint64_t)nnz * sizeof(T);
    const uint64_t rbytes = (used + 15ull) & ~15ull;
    // a record that fits a slot of the field's defer area goes there without
    // waiting for the predecessors' sizes (its own size is published for the
    // blocks that do look back); the fix-up launch places it
    const bool deferred = slots != nullptr && rbytes <= DEFER_SLOT;
    uint64_t off = 0;
    if (deferred) {
        if (tid == 0) {
            atomic_store_u64(&a.flags[b], FLAG_AGG | rbytes);
            sizes[b] = (uint32_t)rbytes | DEFER_BIT;
        }
    } else {
        if (tid < 64) {
            const uint64_t o = lookback_wave(a.flags, b, rbytes, q.status, q.fstatus ? q.fstatus + s_field : nullptr);
            if (tid == 0)
                s_off = o;
        }
        lds_barrier();
        off = s_off;
        if (tid == 0 && sizes)
            sizes[b] = (uint32_t)rbytes;
    }
    uint8_t *out = static_cast<uint8_t *>(a.dst);
    uint8_t *rec = deferred ? slots + b * DEFER_SLOT : out + a.p0 + off;

    if (tid == 0) {
        reinterpret_cast<uint32_t *>(rec)[0] = nnz;
        reinterpret_cast<uint32_t *>(rec)[1] = 0u;
        for (uint64_t p = used; p < rbytes; p += 4)
            *reinterpret_cast<uint32_t *>(rec + p) = 0u;
        if (!deferred) {
            reinterpret_cast<uint64_t *>(out + 64)[b + 1] = off + rbytes;
            if (b + 1 == a.nblocks) {
                *reinterpret_cast<uint64_t *>(out + 56) = off + rbytes;
                if (a.total)
                    *a.total = a.p0 + off + rbytes;
            }
        }
    }
    uint64_t *mask = reinterpret_cast<uint64_t *>(rec + 8);
    if (tid < G::WORDS)
        mask[tid] = s_words[tid];
    const rsrc_t vr = make_rsrc(rec + 8 + G::MASK_BYTES, nnz * (uint32_t)sizeof(T));
#pragma unroll
    for (int z = 0; z < ZP; ++z) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if ((keepbits[r] >> z) & 1u) {
                const int wi = G::word(z, r, wave);
                buf_store(c[r][z], vr, (s_pre[wi] + mbcnt(s_words[wi])) * (uint32_t)sizeof(T));
            }
        }
    }
#pragma unroll
    for (int z = ZP; z < N; ++z) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if ((keepbits[r] >> z) & 1u) {
                const int wi = G::word(z, r, wave);
                const T v = park[(z - ZP) * G::PS + (yq + r * G::YR) * G::PX + x];
                buf_store(v, vr, (s_pre[wi] + mbcnt(s_words[wi])) * (uint32_t)sizeof(T));
            }
        }
    }
}

// ------------------------------------------------- forward, small blocks

// Blocks of 8^3 and 16^3 transform in well under a microsecond each; with one
// block per workgroup the single ticket counter (one atomic per block, which
// the L2 serialises) and the per-block look-back set the pace.  Here a
// workgroup takes one ticket for a group of SG consecutive blocks and runs
// them side by side, one block per wavefront: each wavefront holds its
// block's z-columns in VGPRs (lane (x, yq) owns columns y = yq + r N/R),
// transforms its x- and y-lines through its own LDS region by slab groups of
// SZ planes (one line per lane per pass), decimates with one ballot per mask
// word, and scans its word counts with cross-lane shuffles.  The group then
// publishes one size and runs one look-back over group-indexed flags; each
// record lands at the group's offset plus the sizes of the group's earlier
// blocks, the exclusive scan of Sec. 2.2 taken in two levels.
template <typename T, int N>
struct SmallGeom {
    static constexpr int R = N * N / 64;        // columns per lane: 1 (8^3), 4 (16^3)
    static constexpr int YR = N / R;            // row stride between a lane's columns
    static constexpr int SZ = 64 / N;           // planes per slab group: a pass is 64 lines
    static constexpr int PX = N + 1;            // staging row pitch (odd)
    static constexpr int PS = N * PX;           // staging slab pitch
    static constexpr int REGION = SZ * PS;      // LDS elements per wavefront
    static constexpr int WORDS = N * R;         // mask words per block (= N^3 / 64)
    static constexpr uint32_t MASK_BYTES = (uint32_t)(N * N * N / 8);
    static_assert(N == 8 || N == 16, "one block per wavefront: 8^3 or 16^3");
    static_assert(WORDS <= 64, "one mask word per lane at most");
    // the coarse level of a 16^3 block (8^3, pitches 9 and 72) reuses the region
    static_assert(N == 8 || REGION >= 8 * 72, "coarse cube fits the region");
};

// Blocks per workgroup (= wavefronts): 16 for 8^3; 8 for float and 4 for
// double 16^3 (measured on 512^3 fields: 8 float / 4 double 16^3 blocks a
// group beat 16 and 4 / 8, and 16 8^3 blocks beat 8).
template <typename T, int N>
struct SmallGroup {
    static constexpr int value = N == 8 ? 16 : sizeof(T) == 8 ? 4 : 8;
};

// Every line along AXIS of the n^3 cube at the start of an LDS region with
// pitches (1, PY, PZ): n*n lines, one per lane for the first n*n lanes.
template <typename T, int S, int n, int AXIS, int PY, int PZ>
__device__ __forceinline__ void wave_lines(T *reg, int lane)
{
    if (lane < n * n) {
        const int i = lane % n, j = lane / n;
        int base, stride;
        if constexpr (AXIS == 0) {
            base = i * PY + j * PZ;
            stride = 1;
        } else if constexpr (AXIS == 1) {
            base = i + j * PZ;
            stride = PY;
        } else {
            base = i + j * PY;
            stride = PZ;
        }
        T v[n];
#pragma unroll
        for (int k = 0; k < n; ++k)
            v[k] = reg[base + k * stride];
        line_fwd<T, S, n>(v);
#pragma unroll
        for (int k = 0; k < n; ++k)
            reg[base + k * stride] = v[k];
    }
}

// The 64 lines along x (AXIS 0) or y (AXIS 1) of SZ = 64 / N staged planes
// (pitches 1, PX, PS), one per lane: lane = i + N j, i the other in-plane
// coordinate, j the plane.
template <typename T, int S, int N, int AXIS, int PX, int PS, bool INV = false>
__device__ __forceinline__ void slab_lines(T *reg, int lane)
{
    const int i = lane % N, j = lane / N;
    const int base = j * PS + (AXIS == 0 ? i * PX : i);
    constexpr int stride = AXIS == 0 ? 1 : PX;
    T v[N];
#pragma unroll
    for (int k = 0; k < N; ++k)
        v[k] = reg[base + k * stride];
    if constexpr (INV)
        line_inv<T, S, N>(v);
    else
        line_fwd<T, S, N>(v);
#pragma unroll
    for (int k = 0; k < N; ++k)
        reg[base + k * stride] = v[k];
}

template <typename T, int N, int S>
__global__ __launch_bounds__((64 * SmallGroup<T, N>::value)) void fwd_small_kernel(Queue q)
{
    using G = SmallGeom<T, N>;
    constexpr int SG = SmallGroup<T, N>::value;
    constexpr int R = G::R;
    __shared__ T lds[SG * G::REGION];
    __shared__ uint64_t s_ticket;
    __shared__ uint32_t s_field;
    __shared__ uint64_t s_size[SG];
    __shared__ uint64_t s_goff;

    const int tid = threadIdx.x;
    const int lane = (int)lane_id();
    const int w = tid / 64;  // this wavefront's block within the group
    const int x = lane % N, yq = lane / N;
    T *reg = lds + w * G::REGION;

    if (tid == 0) {
        const uint64_t t = atomicAdd(q.ticket, 1u);
        s_ticket = t;
        s_field = t < q.ntickets ? field_of_ticket(q, t) : 0u;
    }
    lds_barrier();
    const uint64_t t = uniform64(s_ticket);
    if (t >= q.ntickets)
        return;
    const FieldView a = field_view(q, s_field);
    const uint64_t g = t - a.first;  // the group within the field
    const uint64_t b = g * SG + (uint64_t)w;
    const bool live = b < a.nblocks;  // the field's last group may be short

    T c[R][N];
    if (live) {
        const uint32_t lane_off = ((uint32_t)yq * a.nx + (uint32_t)x) * a.cs;
        load_planes<T, N, N, R>(a, b, 0, lane_off, c);
    } else {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int z = 0; z < N; ++z)
                c[r][z] = T(0);
    }

    // finest level: x- and y-lines by slab groups of SZ planes, z in VGPRs
#pragma unroll
    for (int sg = 0; sg < N / G::SZ; ++sg) {
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int j = 0; j < G::SZ; ++j)
                reg[j * G::PS + (yq + r * G::YR) * G::PX + x] = c[r][sg * G::SZ + j];
        wave_lds_sync();
        slab_lines<T, S, N, 0, G::PX, G::PS>(reg, lane);  // x-lines of the SZ planes
        wave_lds_sync();
        slab_lines<T, S, N, 1, G::PX, G::PS>(reg, lane);  // y-lines
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int j = 0; j < G::SZ; ++j)
                c[r][sg * G::SZ + j] = reg[j * G::PS + (yq + r * G::YR) * G::PX + x];
        wave_lds_sync();
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
        line_fwd<T, S, N>(c[r]);

    // 16^3: the level at n = 8 on the coarse cube, every pass in LDS
    if constexpr (N == 16) {
        constexpr int QX = 9, QS = 72;
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int y = yq + r * G::YR;
            if (x < 8) {
#pragma unroll
                for (int z = 0; z < 8; ++z)
                    reg[z * QS + y * QX + x] = c[r][z];
            }
        }
        wave_lds_sync();
        wave_lines<T, S, 8, 0, QX, QS>(reg, lane);
        wave_lds_sync();
        wave_lines<T, S, 8, 1, QX, QS>(reg, lane);
        wave_lds_sync();
        wave_lines<T, S, 8, 2, QX, QS>(reg, lane);
        wave_lds_sync();
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int y = yq + r * G::YR;
            if (x < 8) {
#pragma unroll
                for (int z = 0; z < 8; ++z)
                    c[r][z] = reg[z * QS + y * QX + x];
            }
        }
    }

    // decimation: the 4^3 corner and |c| >= eps; word (z, r) is the ballot of
    // 64 consecutive q, kept by lane z R + r
    bool bad = false;
    uint64_t myword = 0;
#pragma unroll
    for (int z = 0; z < N; ++z) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int y = yq + r * G::YR;
            const T v = c[r][z];
            bad |= !finite(v);
            const bool keep = (z < 4 && x < 4 && y < 4) || keep_test<T>(v, a);
            const uint64_t m = __ballot(keep);
            myword = lane == z * R + r ? m : myword;
        }
    }
    if (live && bad)
        report(q, s_field, STATUS_NONFINITE);
    const uint32_t cnt = lane < G::WORDS ? (uint32_t)__popcll(myword) : 0u;
    uint32_t inc = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t o = __shfl_up(inc, off, 64);
        if (lane >= off)
            inc += o;
    }
    const uint32_t pre = inc - cnt;  // kept values before word `lane`
    const uint32_t nnz = __builtin_amdgcn_readlane(inc, 63);
    const uint64_t used = 8ull + G::MASK_BYTES + (uint64_t)nnz * sizeof(T);
    const uint64_t rbytes = live ? (used + 15ull) & ~15ull : 0ull;

    // one size and one look-back for the group
    if (lane == 0)
        s_size[w] = rbytes;
    lds_barrier();
    if (w == 0) {
        uint64_t total = 0;
#pragma unroll
        for (int k = 0; k < SG; ++k)
            total += s_size[k];
        const uint64_t o = lookback_wave(a.flags, g, total, q.status, q.fstatus ? q.fstatus + s_field : nullptr);
        if (lane == 0)
            s_goff = o;
    }
    lds_barrier();
    if (!live)
        return;
    uint64_t off = s_goff;
    for (int k = 0; k < w; ++k)
        off += s_size[k];

    uint8_t *out = static_cast<uint8_t *>(a.dst);
    uint8_t *rec = out + a.p0 + off;
    if (lane == 0) {
        reinterpret_cast<uint32_t *>(rec)[0] = nnz;
        reinterpret_cast<uint32_t *>(rec)[1] = 0u;
        reinterpret_cast<uint64_t *>(out + 64)[b + 1] = off + rbytes;
        for (uint64_t p = used; p < rbytes; p += 4)
            *reinterpret_cast<uint32_t *>(rec + p) = 0u;
        if (b + 1 == a.nblocks) {
            *reinterpret_cast<uint64_t *>(out + 56) = off + rbytes;
            if (a.total)
                *a.total = a.p0 + off + rbytes;
        }
    }
    if (lane < G::WORDS)
        reinterpret_cast<uint64_t *>(rec + 8)[lane] = myword;
    const rsrc_t vr = make_rsrc(rec + 8 + G::MASK_BYTES, nnz * (uint32_t)sizeof(T));
#pragma unroll
    for (int z = 0; z < N; ++z) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int wi = z * R + r;
            const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)myword, wi);
            const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(myword >> 32), wi);
            const uint64_t word = ((uint64_t)hi << 32) | lo;
            if ((word >> lane) & 1u) {
                const uint32_t rank = __builtin_amdgcn_readlane(pre, wi) + mbcnt(word);
                buf_store(c[r][z], vr, rank * (uint32_t)sizeof(T));
            }
        }
    }
}

// ------------------------------------------------- inverse, 8^3 blocks

// An 8^3 block decodes in well under a microsecond of work but through three
// dependent memory round trips (record offsets, then its header and mask,
// then its values), so a wavefront that decodes one block at a time mostly
// waits.  Here each wavefront keeps IK blocks in flight: lane (x, y) owns the
// z-column of every block, the offsets, nnz and the 8 mask words of a block
// are uniform and come through scalar loads (the stream is read-only during
// the call), so the prefix of each mask word is a scalar sum and needs no
// LDS, and the value gathers of all IK blocks are issued together.  The
// transforms then run one block after another through the wavefront's LDS
// region (z-lines in VGPRs, y- then x-lines in LDS).  Blocks are independent:
// wavefront w takes the ticket groups w, w + W, ... (W wavefronts in the
// grid), with no counter.
constexpr int IK = 4;             // 8^3 blocks in flight per wavefront
constexpr int INV8_WAVES = 4;     // wavefronts per workgroup

template <typename T, int S>
__global__ __launch_bounds__(64 * INV8_WAVES) void inv_small8_kernel(Queue q)
{
    constexpr int N = 8, PX = 9, PS = 72;
    constexpr uint32_t MASK_BYTES = 64;
    using CU64 = const __attribute__((address_space(4))) uint64_t;
    using CU32 = const __attribute__((address_space(4))) uint32_t;
    // float: the group's blocks are stored together, row by row (an 8^3
    // float block's rows are 32 bytes, and written one block at a time they
    // ran at a third of the double blocks' rate); double rows are 64 bytes and
    // the LDS of four regions a wavefront would halve the resident groups
    constexpr bool ROWS = sizeof(T) == 4;
    constexpr int REGIONS = ROWS ? IK : 1;
    __shared__ T lds[INV8_WAVES * REGIONS * N * PS];
    const int lane = (int)lane_id();
    const int wave = threadIdx.x / 64;
    const int x = lane % N, y = lane / N;
    T *reg = lds + wave * REGIONS * N * PS;
    const uint64_t nw = (uint64_t)gridDim.x * INV8_WAVES;
    for (uint64_t g = (uint64_t)blockIdx.x * INV8_WAVES + wave; g * IK < q.ntickets; g += nw) {
        bool ok[IK];
        uint32_t fld[IK];
        uint64_t ob[IK];
        CU64 *mk[IK];
        const uint8_t *vals[IK];
        uint32_t nnz[IK];
        // headers: record offsets, then nnz and the mask, of every block
#pragma unroll
        for (int j = 0; j < IK; ++j) {
            const uint64_t t = g * IK + j;
            ok[j] = t < q.ntickets;
            fld[j] = 0;
            ob[j] = 0;
            mk[j] = nullptr;
            vals[j] = nullptr;
            nnz[j] = 0;
            if (ok[j]) {
                fld[j] = __builtin_amdgcn_readfirstlane(field_of_ticket(q, t));
                const FieldView a = field_view(q, fld[j]);
                const uint64_t k = t - a.first;
                const uint64_t b = uniform64(a.sel ? a.sel[2 * k] : k);  // the record this ticket decodes
                ob[j] = uniform64(a.sel ? a.sel[2 * k + 1] : k);       // and the output block it fills
                const uint8_t *in = static_cast<const uint8_t *>(a.src);
                CU64 *offs = (CU64 *)(in + 64);
                ok[j] = b < a.rblocks;
                const uint64_t o0 = ok[j] ? offs[b] : 0, o1 = ok[j] ? offs[b + 1] : 0;
                ok[j] = ok[j] && o1 >= o0 && o1 <= a.payload && o1 - o0 >= 8ull + MASK_BYTES;
                if (ok[j]) {
                    const uint8_t *rec = in + a.p0 + o0;
                    nnz[j] = *(CU32 *)rec;
                    const uint64_t used = 8ull + MASK_BYTES + (uint64_t)nnz[j] * sizeof(T);
                    ok[j] = nnz[j] <= (uint32_t)(N * N * N) && ((used + 15ull) & ~15ull) == o1 - o0;
                    mk[j] = (CU64 *)(rec + 8);
                    vals[j] = rec + 8 + MASK_BYTES;
                }
                if (!ok[j] && lane == 0)
                    report(q, fld[j], STATUS_FORMAT);
            }
        }
        // gathers of every block: plane z's word is uniform, its prefix a scalar sum
        T c[IK][N];
#pragma unroll
        for (int j = 0; j < IK; ++j) {
            uint64_t w[N];
            uint32_t pre = 0;
#pragma unroll
            for (int z = 0; z < N; ++z) {
                w[z] = ok[j] ? mk[j][z] : 0ull;
                pre += (uint32_t)__popcll(w[z]);
            }
            if (ok[j] && pre != nnz[j]) {
                ok[j] = false;
                if (lane == 0)
                    report(q, fld[j], STATUS_FORMAT);
            }
            const rsrc_t vr = make_rsrc(vals[j], ok[j] ? nnz[j] * (uint32_t)sizeof(T) : 0u);
            pre = 0;
#pragma unroll
            for (int z = 0; z < N; ++z) {
                c[j][z] = T(0);
                if ((w[z] >> lane) & 1ull)
                    c[j][z] = buf_load<T>(vr, (pre + mbcnt(w[z])) * (uint32_t)sizeof(T));
                pre += (uint32_t)__popcll(w[z]);
            }
        }
        if constexpr (!ROWS) {
            // transforms and stores, one block after another
#pragma unroll
            for (int j = 0; j < IK; ++j) {
                if (!ok[j])
                    continue;
                line_inv<T, S, N>(c[j]);
#pragma unroll
                for (int z = 0; z < N; ++z)
                    reg[z * PS + y * PX + x] = c[j][z];
                wave_lds_sync();
                slab_lines<T, S, N, 1, PX, PS, true>(reg, lane);  // y-lines
                wave_lds_sync();
                slab_lines<T, S, N, 0, PX, PS, true>(reg, lane);  // x-lines
                wave_lds_sync();
                const FieldView a = field_view(q, fld[j]);
                const uint64_t b = ob[j];
                const size_t plane = (size_t)a.nx * a.ny;
                const uint32_t bx = (uint32_t)(b % a.nbx);
                const uint32_t by = (uint32_t)((b / a.nbx) % a.nby);
                const uint32_t bz = (uint32_t)(b / ((uint64_t)a.nbx * a.nby));
                T *blk = static_cast<T *>(a.dst) + ((size_t)bz * N * plane + (size_t)by * N * a.nx + (size_t)bx * N);
                const uint32_t slab_bytes = ((uint32_t)(N - 1) * a.nx + N) * (uint32_t)sizeof(T);
                const uint32_t lane_off = ((uint32_t)y * a.nx + (uint32_t)x) * (uint32_t)sizeof(T);
#pragma unroll
                for (int z = 0; z < N; ++z)
                    buf_store(reg[z * PS + y * PX + x], make_rsrc(blk + (size_t)z * plane, slab_bytes), lane_off);
                wave_lds_sync();  // the region is rewritten by the next block
            }
        } else {
            // transforms, one block after another, each in its own LDS region
#pragma unroll
            for (int j = 0; j < IK; ++j) {
                if (!ok[j])
                    continue;
                T *rj = reg + j * N * PS;
                line_inv<T, S, N>(c[j]);
#pragma unroll
                for (int z = 0; z < N; ++z)
                    rj[z * PS + y * PX + x] = c[j][z];
                wave_lds_sync();
                slab_lines<T, S, N, 1, PX, PS, true>(rj, lane);  // y-lines
                wave_lds_sync();
                slab_lines<T, S, N, 0, PX, PS, true>(rj, lane);  // x-lines
            }
            wave_lds_sync();
            // stores of the whole group: its blocks are consecutive, usually
            // x-neighbours in one row of blocks, so a plane's rows of all IK
            // blocks go out together (lane l of a store takes element x' = l mod
            // IK N of row y of the group's plane, block x' / N), whole cache lines
            // instead of one N-element segment per block and row
            T *base[IK];
            size_t pl[IK];
            uint32_t rowp[IK];
#pragma unroll
            for (int j = 0; j < IK; ++j) {
                const FieldView a = field_view(q, fld[j]);
                const uint64_t b = ob[j];
                pl[j] = (size_t)a.nx * a.ny;
                rowp[j] = a.nx;
                const uint32_t bx = (uint32_t)(b % a.nbx);
                const uint32_t by = (uint32_t)((b / a.nbx) % a.nby);
                const uint32_t bz = (uint32_t)(b / ((uint64_t)a.nbx * a.nby));
                base[j] = static_cast<T *>(a.dst) + ((size_t)bz * N * pl[j] + (size_t)by * N * a.nx + (size_t)bx * N);
            }
            constexpr int W = IK * N;                  // elements of a group row
            constexpr int STORES = IK * N * N / 64;    // store instructions per plane
            static_assert((IK * N * N) % 64 == 0 && 64 % W == 0, "whole group rows per store");
#pragma unroll
            for (int z = 0; z < N; ++z) {
#pragma unroll
                for (int k = 0; k < STORES; ++k) {
                    const int e = k * 64 + lane;
                    const int yy = e / W, xx = e % W, j = xx / N, xj = xx % N;
                    bool okj = false;
                    T *bj = nullptr;
                    size_t plj = 0;
                    uint32_t rpj = 0;
#pragma unroll
                    for (int i = 0; i < IK; ++i) {
                        if (j == i) {
                            okj = ok[i];
                            bj = base[i];
                            plj = pl[i];
                            rpj = rowp[i];
                        }
                    }
                    if (okj)
                        bj[(size_t)z * plj + (size_t)yy * rpj + xj] = reg[j * N * PS + z * PS + yy * PX + xj];
                }
            }
            wave_lds_sync();  // the regions are rewritten by the next group
        }
    }
}

// ------------------------------------------------------------------ inverse

// The same for the inverse: float 32^3 blocks with two columns a thread and
// 16-slab staging (72 KiB of LDS) fit two workgroups a CU when the
// registers do.
template <typename T, int N, int Z, int R>
struct InvWaves {
    static constexpr int one = N * N / R / 256 > 0 ? N * N / R / 256 : 1;
    static constexpr int value = sizeof(T) == 4 && N == 32 && Z == 16 && R == 2 ? 2 * one : one;
};

template <typename T, int N, int S, int Z, int R>
__global__ __launch_bounds__(N *N / R, (InvWaves<T, N, Z, R>::value)) void inv_kernel(Queue q)
{
    using G = Geom<T, N, Z, R>;
    __shared__ T lds[G::LDS_ELEMS];
    __shared__ uint64_t s_words[G::WORDS];
    __shared__ uint32_t s_pre[G::WORDS];
    __shared__ uint32_t s_scan[G::WAVES + 1];
    __shared__ uint64_t s_block;
    __shared__ uint32_t s_field;
    __shared__ uint32_t s_ok;
    __shared__ uint64_t s_rec, s_out;

    const int tid = threadIdx.x;
    const int x = tid % N, yq = tid / N;
    const uint32_t lane = lane_id();
    const int wave = tid / 64;

    // Small blocks take their tickets TB at a time: they decode in well under
    // a microsecond, and one atomic per block on the single counter (which
    // the L2 serialises) would set the pace.  Any order is correct here:
    // blocks are independent.  (The surplus grid x TB on the counter is far
    // from its 32-bit range.)
    constexpr uint32_t TB = N <= 8 ? 8 : N <= 16 ? 4 : 1;
    uint32_t next = 0, end = 0;  // thread 0's batch [next, end)
    while (true) {
        if (tid == 0) {
            uint64_t t;
            if constexpr (TB == 1) {
                t = atomicAdd(q.ticket, 1u);
            } else {
                if (next == end) {
                    next = atomicAdd(q.ticket, TB);
                    end = next + TB;
                }
                t = next++;
            }
            uint32_t ok = 0, f = 0;
            uint64_t rb = 0, ob = 0;
            if (t < q.ntickets) {
                f = field_of_ticket(q, t);
                const FieldView a = field_view(q, f);
                const uint8_t *in = static_cast<const uint8_t *>(a.src);
                const uint64_t *offs = reinterpret_cast<const uint64_t *>(in + 64);
                const uint64_t k = t - a.first;
                const uint64_t b = a.sel ? a.sel[2 * k] : k;  // the record this ticket decodes
                rb = b;
                ob = a.sel ? a.sel[2 * k + 1] : k;          // and the output block it fills
                ok = b < a.rblocks;
                const uint64_t o0 = ok ? offs[b] : 0, o1 = ok ? offs[b + 1] : 0;
                ok = ok && o1 >= o0 && o1 <= a.payload && o1 - o0 >= 8ull + G::MASK_BYTES;
                if (ok) {
                    const uint32_t nnz = *reinterpret_cast<const uint32_t *>(in + a.p0 + o0);
                    const uint64_t used = 8ull + G::MASK_BYTES + (uint64_t)nnz * sizeof(T);
                    ok = nnz <= (uint32_t)(N * N * N) && ((used + 15ull) & ~15ull) == o1 - o0;
                }
                if (!ok)
                    report(q, f, STATUS_FORMAT);
            }
            s_block = t;
            s_field = f;
            s_ok = ok;
            s_rec = rb;
            s_out = ob;
        }
        lds_barrier();
        const uint64_t t = uniform64(s_block);
        if (t >= q.ntickets)
            break;
        if (!s_ok) {
            lds_barrier();
            continue;
        }
        const FieldView a = field_view(q, s_field);
        const uint64_t b = uniform64(s_out);  // output block (the field's block index unless selected)
        const size_t plane = (size_t)a.nx * a.ny;
        const uint32_t lane_off = (uint32_t)yq * a.nx + (uint32_t)x;
        const uint32_t slab_bytes = ((uint32_t)(N - 1) * a.nx + N) * (uint32_t)sizeof(T);
        const uint8_t *in = static_cast<const uint8_t *>(a.src);
        const uint64_t *offs = reinterpret_cast<const uint64_t *>(in + 64);
        const uint8_t *rec = in + a.p0 + offs[uniform64(s_rec)];
        const uint32_t nnz = *reinterpret_cast<const uint32_t *>(rec);
        const uint64_t *mask = reinterpret_cast<const uint64_t *>(rec + 8);
        const rsrc_t vr = make_rsrc(rec + 8 + G::MASK_BYTES, nnz * (uint32_t)sizeof(T));

        if (tid < G::WORDS)
            s_words[tid] = mask[tid];
        lds_barrier();
        const uint32_t cnt = tid < G::WORDS ? (uint32_t)__popcll(s_words[tid]) : 0u;
        const uint32_t pre = block_exclusive_scan<G::NT>(cnt, s_scan);
        if (tid < G::WORDS)
            s_pre[tid] = pre;
        lds_barrier();
        if (s_scan[G::WAVES] != nnz) {
            if (tid == 0)
                report(q, s_field, STATUS_FORMAT);
            lds_barrier();
            continue;
        }

        // gather: kept coefficient q -> vals[rank(q)], dropped -> +0
        T c[R][N];
#pragma unroll
        for (int z = 0; z < N; ++z) {
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int wi = G::word(z, r, wave);
                const uint64_t m = s_words[wi];
                c[r][z] = T(0);
                if ((m >> lane) & 1ull)
                    c[r][z] = buf_load<T>(vr, (s_pre[wi] + mbcnt(m)) * (uint32_t)sizeof(T));
            }
        }

        // coarser levels 8 .. N/2: z-lines in VGPRs, y- and x-lines in LDS
        if constexpr (N / 2 >= 8) {
            coarse_inv<T, S, G::H, G::QX, G::QS, R, G::YR, N>(c, lds, x, yq);
            lds_barrier();  // the staging below reuses the coarse area
        }

        // finest level: z in VGPRs, then y- and x-lines per slab group
#pragma unroll
        for (int r = 0; r < R; ++r)
            line_inv<T, S, N>(c[r]);
        const uint32_t bx = (uint32_t)(b % a.nbx);
        const uint32_t by = (uint32_t)((b / a.nbx) % a.nby);
        const uint32_t bz = (uint32_t)(b / ((uint64_t)a.nbx * a.nby));
        T *blk = static_cast<T *>(a.dst) + ((size_t)bz * N * plane + (size_t)by * N * a.nx + (size_t)bx * N);
#pragma unroll
        for (int g = 0; g < N / Z; ++g) {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int j = 0; j < Z; ++j)
                    lds[j * G::PS + (yq + r * G::YR) * G::PX + x] = c[r][g * Z + j];
            lds_barrier();
            stage_lines<T, S, N, Z, G::NT, G::PX, G::PS, 1, true>(lds);
            lds_barrier();
            stage_lines<T, S, N, Z, G::NT, G::PX, G::PS, 0, true>(lds);
            lds_barrier();
#pragma unroll
            for (int j = 0; j < Z; ++j) {
                const rsrc_t zr = make_rsrc(blk + (size_t)(g * Z + j) * plane, slab_bytes);
#pragma unroll
                for (int r = 0; r < R; ++r)
                    buf_store(lds[j * G::PS + (yq + r * G::YR) * G::PX + x], zr,
                              (lane_off + (uint32_t)(r * G::YR) * a.nx) * (uint32_t)sizeof(T));
            }
            lds_barrier();
        }
    }
}

// ------------------------------------------------- scratch-staged blocks
// Blocks too large for a CU (N = 64: 1 MiB float, 2 MiB double) live in
// per-workgroup scratch slots in global memory between passes (one a
// workgroup in the inverse, two in the forward).  Each level's
// x- and y-lines run on chunks of z-planes staged through LDS (row pitch
// n + 1), the finest level reading its rows straight from the field (forward)
// or writing them straight to it (inverse); the z-lines run in registers,
// one column per thread at a time, lanes along x; the levels from (N/4)^3
// down run entirely in LDS.  The finest z-pass also decimates the finest
// details (forward) or gathers them from the record (inverse), so the slot
// never holds a dropped detail.  Full workgroup barriers separate passes that
// communicate through the scratch slot (they must order global memory).

template <int NT>
__device__ __forceinline__ void gbarrier() { __syncthreads(); }

// Elements a thread moves at once between global memory and LDS in the
// scratch kernels' x/y passes and LDS-resident levels.
constexpr int XY_U = 8;

// Consecutive mask words a wavefront handles at once in the scratch kernels'
// per-word loops (decimation, record values, gather), their loads all in flight.
constexpr int DEC_U = 16;

template <typename T, int N>
struct Big {
    static constexpr int NT = SCRATCH_THREADS;
    static constexpr int TAIL = N / 4;  // edge of the LDS-resident levels
    // mask words and their prefixes sit above the coarse levels' staging
    // while the finest z-pass and the coarse levels run
    static constexpr size_t WORDS_AT = 81920;
    static constexpr int WORDS = N * N * N / 64;
    static constexpr size_t CHUNK_BYTES = (sizeof(T) == 4 ? 8 : 4) * (size_t)N * (N + 1) * sizeof(T);
    static constexpr size_t WORD_BYTES = (size_t)WORDS * (sizeof(uint64_t) + sizeof(uint32_t));
    static constexpr size_t LDS_BYTES = CHUNK_BYTES > WORDS_AT + WORD_BYTES ? CHUNK_BYTES : WORDS_AT + WORD_BYTES;
    // planes per LDS chunk at level n: the largest power of two that fits
    static constexpr int chunk(int n)
    {
        int z = n;
        while (z > 1 && (size_t)z * n * (n + 1) * sizeof(T) > CHUNK_BYTES)
            z /= 2;
        return z;
    }
};

// x- and y-lines of one level (forward: x then y; inverse: y then x) on the
// planes [0, n) of [0, n)^2, ZC planes at a time through LDS.  Rows are read
// from src and written to dst (strides in elements; src may equal dst).
template <typename T, int S, int n, int ZC, bool INV, int NT>
__device__ __forceinline__ void xy_level(const T *src, size_t sps, size_t srs, uint32_t ses, T *dst, size_t dps,
                                         size_t drs, T *lds)
{
    constexpr int PX = n + 1, PS = n * PX;
    static_assert(ZC * n * n % (NT * XY_U) == 0, "whole batches of elements per thread");
    for (int z0 = 0; z0 < n; z0 += ZC) {
        if constexpr (!INV) {
            // forward: XY_U loads in flight, then their LDS writes (the
            // scheduling barrier keeps the compiler from pairing each load
            // with its write, one round trip per element, when the kernel's
            // registers look scarce)
            for (int e0 = threadIdx.x; e0 < ZC * n * n; e0 += NT * XY_U) {
                T t[XY_U];
#pragma unroll
                for (int u = 0; u < XY_U; ++u) {
                    const int e = e0 + u * NT;
                    const int x = e % n, y = (e / n) % n, j = e / (n * n);
                    t[u] = src[(size_t)(z0 + j) * sps + (size_t)y * srs + (size_t)x * ses];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < XY_U; ++u) {
                    const int e = e0 + u * NT;
                    const int x = e % n, y = (e / n) % n, j = e / (n * n);
                    lds[j * PS + y * PX + x] = t[u];
                }
            }
        } else {
#pragma unroll 8
            for (int e = threadIdx.x; e < ZC * n * n; e += NT) {
                const int x = e % n, y = (e / n) % n, j = e / (n * n);
                lds[j * PS + y * PX + x] = src[(size_t)(z0 + j) * sps + (size_t)y * srs + (size_t)x * ses];
            }
        }
        lds_barrier();
        if constexpr (!INV) {
            stage_lines<T, S, n, ZC, NT, PX, PS, 0, false>(lds);
            lds_barrier();
            stage_lines<T, S, n, ZC, NT, PX, PS, 1, false>(lds);
        } else {
            stage_lines<T, S, n, ZC, NT, PX, PS, 1, true>(lds);
            lds_barrier();
            stage_lines<T, S, n, ZC, NT, PX, PS, 0, true>(lds);
        }
        lds_barrier();
#pragma unroll 8
        for (int e = threadIdx.x; e < ZC * n * n; e += NT) {
            const int x = e % n, y = (e / n) % n, j = e / (n * n);
            dst[(size_t)(z0 + j) * dps + (size_t)y * drs + x] = lds[j * PS + y * PX + x];
        }
        lds_barrier();
    }
}

// z-lines of one level on the columns of [0, n)^2 of the scratch block.
template <typename T, int S, int N, int n, bool INV, int NT>
__device__ __forceinline__ void z_level(T *blk)
{
#pragma unroll 1
    for (int l = threadIdx.x; l < n * n; l += NT) {
        const int x = l % n, y = l / n;
        T v[n];
#pragma unroll
        for (int k = 0; k < n; ++k)
            v[k] = blk[(size_t)k * N * N + y * N + x];
        if constexpr (INV)
            line_inv<T, S, n>(v);
        else
            line_fwd<T, S, n>(v);
#pragma unroll
        for (int k = 0; k < n; ++k)
            blk[(size_t)k * N * N + y * N + x] = v[k];
    }
}

// All lines of one axis of [0, n)^3 in LDS (row pitch PY, slab pitch PZ),
// NT threads, each taking lines until none is left.
template <typename T, int S, int n, int AXIS, bool INV, int PY, int PZ, int NT>
__device__ __forceinline__ void lds_lines_all(T *lds)
{
#pragma unroll 1
    for (int t = threadIdx.x; t < n * n; t += NT) {
        const int i = t % n, j = t / n;
        const int base = AXIS == 0 ? i * PY + j * PZ : AXIS == 1 ? i + j * PZ : i + j * PY;
        constexpr int stride = AXIS == 0 ? 1 : AXIS == 1 ? PY : PZ;
        T v[n];
#pragma unroll
        for (int k = 0; k < n; ++k)
            v[k] = lds[base + k * stride];
        if constexpr (INV)
            line_inv<T, S, n>(v);
        else
            line_fwd<T, S, n>(v);
#pragma unroll
        for (int k = 0; k < n; ++k)
            lds[base + k * stride] = v[k];
    }
}

template <typename T, int S, int n, int PY, int PZ, int NT>
__device__ __forceinline__ void tail_fwd(T *lds)
{
    lds_lines_all<T, S, n, 0, false, PY, PZ, NT>(lds);
    lds_barrier();
    lds_lines_all<T, S, n, 1, false, PY, PZ, NT>(lds);
    lds_barrier();
    lds_lines_all<T, S, n, 2, false, PY, PZ, NT>(lds);
    lds_barrier();
    if constexpr (n / 2 >= 8)
        tail_fwd<T, S, n / 2, PY, PZ, NT>(lds);
}

template <typename T, int S, int n, int PY, int PZ, int NT>
__device__ __forceinline__ void tail_inv(T *lds)
{
    if constexpr (n / 2 >= 8)
        tail_inv<T, S, n / 2, PY, PZ, NT>(lds);
    lds_lines_all<T, S, n, 2, true, PY, PZ, NT>(lds);
    lds_barrier();
    lds_lines_all<T, S, n, 1, true, PY, PZ, NT>(lds);
    lds_barrier();
    lds_lines_all<T, S, n, 0, true, PY, PZ, NT>(lds);
    lds_barrier();
}

// Levels m, m/2, ..., 8 of the region [0, m)^3 of the scratch block, in LDS.
template <typename T, int S, int N, int m, bool INV, int NT>
__device__ __forceinline__ void tail_levels(T *blk, T *lds)
{
    constexpr int QX = m + 1, QS = m * QX;
#pragma unroll 8
    for (int e = threadIdx.x; e < m * m * m; e += NT) {
        const int x = e % m, y = (e / m) % m, z = e / (m * m);
        lds[z * QS + y * QX + x] = blk[(size_t)z * N * N + y * N + x];
    }
    lds_barrier();
    if constexpr (INV)
        tail_inv<T, S, m, QX, QS, NT>(lds);
    else
        tail_fwd<T, S, m, QX, QS, NT>(lds);
#pragma unroll 8
    for (int e = threadIdx.x; e < m * m * m; e += NT) {
        const int x = e % m, y = (e / m) % m, z = e / (m * m);
        blk[(size_t)z * N * N + y * N + x] = lds[z * QS + y * QX + x];
    }
}

// The finest z-lines of the forward with the decimation of the finest
// details: once a column's z-line is transformed, every coefficient outside
// the coarse octant [0, N/2)^3 is final, so its keep bit is taken here.  A
// wavefront holds one row y (x = lane) of each plane, so one ballot per plane
// gives the mask word of (z, y) (bits of the octant's x < N/2 left for the
// coarse pass).  Only coefficients still needed go back to the slot: the
// octant (the next level's input) and kept details.
template <typename T, int S, int N, int NT>
__device__ __forceinline__ void z_finest_dec(T *blk, const FieldView &a, uint64_t *s_words, bool &bad)
{
    static_assert(N == 64, "one row of a plane per wavefront");
    constexpr int H = N / 2;
    const uint32_t lane = lane_id();
#pragma unroll 1
    for (int l = threadIdx.x; l < N * N; l += NT) {
        const int x = l % N, y = l / N;
        T v[N];
#pragma unroll
        for (int k = 0; k < N; ++k)
            v[k] = blk[(size_t)k * N * N + y * N + x];
        line_fwd<T, S, N>(v);
#pragma unroll
        for (int z = 0; z < N; ++z) {
            const bool fin = x >= H || y >= H || z >= H;
            const bool keep = fin && keep_test<T>(v[z], a);
            bad |= fin && !finite(v[z]);
            const uint64_t m = __ballot(keep);
            if (lane == 0)
                s_words[z * N + y] = m;
            if (!fin || keep)
                blk[(size_t)z * N * N + y * N + x] = v[z];
        }
    }
}

template <typename T, int N>
__device__ __forceinline__ constexpr bool coarse_staging_below_words()
{
    using B = Big<T, N>;
    return (size_t)B::chunk(N / 2) * (N / 2) * (N / 2 + 1) * sizeof(T) <= B::WORDS_AT &&
           (size_t)B::TAIL * B::TAIL * (B::TAIL + 1) * sizeof(T) <= B::WORDS_AT && B::TAIL == N / 4;
}

// Forward transform of a 64^3 block: field rows -> scratch slot, the finest
// details decimated on the way (mask words of them in s_words).
template <typename T, int S, int N, int NT>
__device__ __forceinline__ void big_fwd(const T *src, size_t plane, size_t row, uint32_t cs, T *blk, T *lds,
                                        const FieldView &a, uint64_t *s_words, bool &bad)
{
    using B = Big<T, N>;
    static_assert(coarse_staging_below_words<T, N>(), "the coarse levels' staging stays below the mask words");
    xy_level<T, S, N, B::chunk(N), false, NT>(src, plane, row, cs, blk, (size_t)N * N, N, lds);
    gbarrier<NT>();
    z_finest_dec<T, S, N, NT>(blk, a, s_words, bad);
    gbarrier<NT>();
    xy_level<T, S, N / 2, B::chunk(N / 2), false, NT>(blk, (size_t)N * N, N, 1, blk, (size_t)N * N, N, lds);
    gbarrier<NT>();
    z_level<T, S, N, N / 2, false, NT>(blk);
    gbarrier<NT>();
    tail_levels<T, S, N, B::TAIL, false, NT>(blk, lds);
    gbarrier<NT>();
}

// The finest z-lines of the inverse with the gather of the finest details
// fused in: the coarse octant [0, N/2)^3 comes from the slot (the coarse
// levels' output), every other coefficient straight from the record (kept:
// its value at the rank that the mask word's prefix and the bits below it
// give; dropped: 0).  The transformed columns go back to the slot whole.
template <typename T, int S, int N, int NT>
__device__ __forceinline__ void z_finest_gather(T *blk, rsrc_t vr, const uint64_t *s_words, const uint32_t *s_pre)
{
    static_assert(N == 64, "one row of a plane per wavefront");
    constexpr int H = N / 2;
    const uint32_t lane = lane_id();
#pragma unroll 1
    for (int l = threadIdx.x; l < N * N; l += NT) {
        const int x = l % N, y = l / N;
        T v[N];
#pragma unroll
        for (int z = 0; z < N; ++z) {
            const uint64_t m = s_words[z * N + y];
            v[z] = T(0);
            if (z < H && y < H && x < H)
                v[z] = blk[(size_t)z * N * N + y * N + x];
            else if ((m >> lane) & 1ull)
                v[z] = buf_load<T>(vr, (s_pre[z * N + y] + mbcnt(m)) * (uint32_t)sizeof(T));
        }
        line_inv<T, S, N>(v);
#pragma unroll
        for (int z = 0; z < N; ++z)
            blk[(size_t)z * N * N + y * N + x] = v[z];
    }
}

// Inverse transform of a 64^3 block whose coarse octant has been gathered
// into the scratch slot: slot -> field rows (the finest details from the
// record, mask words and prefixes in s_words / s_pre).
template <typename T, int S, int N, int NT>
__device__ __forceinline__ void big_inv(T *blk, T *dst, size_t plane, size_t row, T *lds, rsrc_t vr,
                                        const uint64_t *s_words, const uint32_t *s_pre)
{
    using B = Big<T, N>;
    static_assert(coarse_staging_below_words<T, N>(), "the coarse levels' staging stays below the mask words");
    tail_levels<T, S, N, B::TAIL, true, NT>(blk, lds);
    gbarrier<NT>();
    z_level<T, S, N, N / 2, true, NT>(blk);
    gbarrier<NT>();
    xy_level<T, S, N / 2, B::chunk(N / 2), true, NT>(blk, (size_t)N * N, N, 1, blk, (size_t)N * N, N, lds);
    gbarrier<NT>();
    z_finest_gather<T, S, N, NT>(blk, vr, s_words, s_pre);
    gbarrier<NT>();
    xy_level<T, S, N, B::chunk(N), true, NT>(blk, (size_t)N * N, N, 1, dst, plane, row, lds);
}

// Workgroup-wide exclusive scan of W word counts (W a multiple of NT): thread
// t owns words [t K, t K + K).  Returns the total; s_pre receives prefixes.
template <int NT, int W>
__device__ __forceinline__ uint32_t scan_words(const uint64_t *s_words, uint32_t *s_pre, uint32_t *s_w)
{
    constexpr int K = W / NT;
    static_assert(W % NT == 0, "words per thread must be whole");
    uint32_t local[K];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        local[k] = (uint32_t)__popcll(s_words[threadIdx.x * K + k]);
        sum += local[k];
    }
    const uint32_t pre = block_exclusive_scan<NT>(sum, s_w);
    uint32_t run = pre;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        s_pre[threadIdx.x * K + k] = run;
        run += local[k];
    }
    return s_w[NT / 64];
}

// The 64^3 forward is persistent with two blocks in flight per workgroup:
// block k is transformed, decimated and its record size published in one
// slot, then block k-1's look-back is resolved and its record written from
// the other slot.  A record's offset waits for every earlier block's size;
// resolving it one block later gives those blocks a whole block's time to
// publish instead of exposing the spread of their finishing times.  Mask
// words and prefixes of a block wait in a side area beside its slot while the
// next block's transform uses the LDS.  No wait is on a later ticket: every
// earlier ticket's size is published before its holder waits on anything.
template <typename T, int N, int S>
__global__ __launch_bounds__(SCRATCH_THREADS) void fwd_scratch_kernel(Queue q)
{
    using B = Big<T, N>;
    constexpr int NT = SCRATCH_THREADS;
    constexpr int WORDS = N * N * N / 64;
    constexpr uint32_t MASK_BYTES = (uint32_t)(N * N * N / 8);
    constexpr int WAVES = NT / 64;
    static_assert(WORDS % (WAVES * DEC_U) == 0 && WORDS % NT == 0, "whole runs of words per wavefront");
    static_assert(B::WORD_BYTES <= B::WORDS_AT, "two blocks' mask words fit the LDS side by side");
    constexpr int H = N / 2;
    constexpr int K = WORDS / NT;  // words per thread in scan_words' layout
    constexpr size_t SLOT = (size_t)N * N * N;
    // LDS: line staging during the transform; the current block's mask words
    // and prefixes above the coarse levels' staging (the finest level's
    // staging is done with before the first word is written); the previous
    // block's, reloaded for its record, at the bottom
    __shared__ __align__(16) uint8_t lds_raw[B::LDS_BYTES];
    T *lds = reinterpret_cast<T *>(lds_raw);
    uint64_t *s_words = reinterpret_cast<uint64_t *>(lds_raw + B::WORDS_AT);
    uint32_t *s_pre = reinterpret_cast<uint32_t *>(lds_raw + B::WORDS_AT + WORDS * sizeof(uint64_t));
    uint64_t *p_words = reinterpret_cast<uint64_t *>(lds_raw);
    uint32_t *p_pre = reinterpret_cast<uint32_t *>(lds_raw + WORDS * sizeof(uint64_t));
    __shared__ uint32_t s_scan[WAVES + 1];
    __shared__ uint64_t s_block;
    __shared__ uint32_t s_field;
    __shared__ uint64_t s_off;
    __shared__ uint32_t s_bad;

    const int tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const int wave = tid / 64;
    // two slots per workgroup, then (after every workgroup's slots) a side
    // area per slot for its block's mask words and prefixes
    T *slots = static_cast<T *>(q.scratch) + (size_t)blockIdx.x * 2 * SLOT;
    uint8_t *sides = reinterpret_cast<uint8_t *>(static_cast<T *>(q.scratch) + (size_t)gridDim.x * 2 * SLOT) +
                     (size_t)blockIdx.x * 2 * B::WORD_BYTES;

    int cur = 0;             // slot of the block taken this iteration
    bool have_prev = false;  // a block waits in the other slot for its record
    uint32_t pf = 0, pnnz = 0;
    uint64_t pb = 0;
    while (true) {
        if (tid == 0) {
            const uint64_t t = atomicAdd(q.ticket, 1u);
            s_block = t;
            s_field = t < q.ntickets ? field_of_ticket(q, t) : 0u;
            s_bad = 0;
        }
        gbarrier<NT>();
        const uint64_t t = uniform64(s_block);
        const bool more = t < q.ntickets;
        const uint32_t f = s_field;
        uint64_t b = 0;
        uint32_t nnz = 0;
        if (more) {
            if (have_prev) {
                // this block's transform reuses the LDS: the waiting block's
                // mask words and prefixes go to its side area first
                uint64_t *sw = reinterpret_cast<uint64_t *>(sides + (size_t)(cur ^ 1) * B::WORD_BYTES);
                uint32_t *sp = reinterpret_cast<uint32_t *>(sw + WORDS);
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    sw[tid * K + k] = s_words[tid * K + k];
                    sp[tid * K + k] = s_pre[tid * K + k];
                }
                gbarrier<NT>();
            }
            const FieldView a = field_view(q, f);
            b = t - a.first;
            T *blkS = slots + (size_t)cur * SLOT;
            const size_t row = (size_t)a.nx * a.cs, plane = row * a.ny;
            const uint32_t bx = (uint32_t)(b % a.nbx);
            const uint32_t by = (uint32_t)((b / a.nbx) % a.nby);
            const uint32_t bz = (uint32_t)(b / ((uint64_t)a.nbx * a.nby));
            const T *src = static_cast<const T *>(a.src) +
                           ((size_t)bz * N * plane + (size_t)by * N * row + (size_t)bx * N * a.cs);
            bool bad = false;
            big_fwd<T, S, N, NT>(src, plane, row, a.cs, blkS, lds, a, s_words, bad);

            // decimation of the coarse octant (x, y, z < N/2; the 4^3 corner
            // always kept): row (z, y) of it is the low half of word z N + y.
            // Wavefront w takes the runs of U consecutive rows starting at
            // U w, U (w + WAVES), ..., all U loads of a run in flight together.
            static_assert(N == 64 && (H * H) % (WAVES * DEC_U) == 0, "whole runs of octant rows");
            for (int r0 = wave * DEC_U; r0 < H * H; r0 += WAVES * DEC_U) {
                T v[DEC_U];
#pragma unroll
                for (int u = 0; u < DEC_U; ++u) {
                    const int z = (r0 + u) / H, y = (r0 + u) % H;
                    v[u] = T(0);
                    if ((int)lane < H)
                        v[u] = blkS[(size_t)z * N * N + y * N + (int)lane];
                }
#pragma unroll
                for (int u = 0; u < DEC_U; ++u) {
                    const int z = (r0 + u) / H, y = (r0 + u) % H, x = (int)lane;
                    const bool in = x < H;
                    bad |= in && !finite(v[u]);
                    const bool keep = in && ((x < 4 && y < 4 && z < 4) || keep_test<T>(v[u], a));
                    const uint64_t m = __ballot(keep);
                    if (lane == 0)
                        s_words[z * N + y] |= m;
                }
            }
            if (bad)
                s_bad = 1;
            gbarrier<NT>();
            if (tid == 0 && s_bad)
                report(q, f, STATUS_NONFINITE);
            nnz = scan_words<NT, WORDS>(s_words, s_pre, s_scan);
            const uint64_t rbytes = (8ull + MASK_BYTES + (uint64_t)nnz * sizeof(T) + 15ull) & ~15ull;
            if (tid < 64)
                lookback_publish(a.flags, b, rbytes);
        }
        if (have_prev) {
            // the previous block: its words and prefixes (back in LDS from
            // its side area if a transform ran since, else still in place),
            // its offset from the look-back, then its record
            const uint64_t *pw = s_words;
            const uint32_t *pp = s_pre;
            if (more) {
                const uint64_t *sw = reinterpret_cast<const uint64_t *>(sides + (size_t)(cur ^ 1) * B::WORD_BYTES);
                const uint32_t *sp = reinterpret_cast<const uint32_t *>(sw + WORDS);
                uint64_t mw[K];
                uint32_t mp[K];
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    mw[k] = sw[tid * K + k];
                    mp[k] = sp[tid * K + k];
                }
                gbarrier<NT>();  // every thread is done with the LDS below
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    p_words[tid * K + k] = mw[k];
                    p_pre[tid * K + k] = mp[k];
                }
                pw = p_words;
                pp = p_pre;
            }
            const FieldView a = field_view(q, pf);
            const uint64_t used = 8ull + MASK_BYTES + (uint64_t)pnnz * sizeof(T);
            const uint64_t rbytes = (used + 15ull) & ~15ull;
            if (tid < 64) {
                const uint64_t o =
                    lookback_resolve(a.flags, pb, rbytes, q.status, q.fstatus ? q.fstatus + pf : nullptr);
                if (tid == 0)
                    s_off = o;
            }
            gbarrier<NT>();
            const uint64_t off = s_off;
            const T *blkP = slots + (size_t)(cur ^ 1) * SLOT;
            uint8_t *out = static_cast<uint8_t *>(a.dst);
            uint8_t *rec = out + a.p0 + off;
            if (tid == 0) {
                reinterpret_cast<uint32_t *>(rec)[0] = pnnz;
                reinterpret_cast<uint32_t *>(rec)[1] = 0u;
                reinterpret_cast<uint64_t *>(out + 64)[pb + 1] = off + rbytes;
                for (uint64_t p = used; p < rbytes; p += 4)
                    *reinterpret_cast<uint32_t *>(rec + p) = 0u;
                if (pb + 1 == a.nblocks) {
                    *reinterpret_cast<uint64_t *>(out + 56) = off + rbytes;
                    if (a.total)
                        *a.total = a.p0 + off + rbytes;
                }
            }
            uint64_t *mask = reinterpret_cast<uint64_t *>(rec + 8);
            for (int w = tid; w < WORDS; w += NT)
                mask[w] = pw[w];
            const rsrc_t vr = make_rsrc(rec + 8 + MASK_BYTES, pnnz * (uint32_t)sizeof(T));
            // kept values from the slot into the record, runs of U words a
            // wavefront, all U loads of a run in flight together
            for (int w0 = wave * DEC_U; w0 < WORDS; w0 += WAVES * DEC_U) {
                uint64_t m[DEC_U];
                T v[DEC_U];
#pragma unroll
                for (int u = 0; u < DEC_U; ++u) {
                    m[u] = pw[w0 + u];
                    v[u] = T(0);
                    if ((m[u] >> lane) & 1ull)
                        v[u] = blkP[(w0 + u) * 64 + (int)lane];
                }
#pragma unroll
                for (int u = 0; u < DEC_U; ++u)
                    if ((m[u] >> lane) & 1ull)
                        buf_store(v[u], vr, (pp[w0 + u] + mbcnt(m[u])) * (uint32_t)sizeof(T));
            }
        }
        gbarrier<NT>();
        if (!more)
            break;
        have_prev = true;
        pf = f;
        pb = b;
        pnnz = nnz;
        cur ^= 1;
    }
}

template <typename T, int N, int S>
__global__ __launch_bounds__(SCRATCH_THREADS) void inv_scratch_kernel(Queue q)
{
    constexpr int NT = SCRATCH_THREADS;
    constexpr int WORDS = N * N * N / 64;
    constexpr uint32_t MASK_BYTES = (uint32_t)(N * N * N / 8);
    constexpr int WAVES = NT / 64;
    static_assert(WORDS % (WAVES * DEC_U) == 0 && WORDS % NT == 0, "whole runs of words per wavefront");
    constexpr int H = N / 2;
    // LDS: line staging; mask words and prefixes above the coarse levels'
    // staging until the finest z-pass has read them
    __shared__ __align__(16) uint8_t lds_raw[Big<T, N>::LDS_BYTES];
    T *lds = reinterpret_cast<T *>(lds_raw);
    uint64_t *s_words = reinterpret_cast<uint64_t *>(lds_raw + Big<T, N>::WORDS_AT);
    uint32_t *s_pre = reinterpret_cast<uint32_t *>(lds_raw + Big<T, N>::WORDS_AT + WORDS * sizeof(uint64_t));
    __shared__ uint32_t s_scan[WAVES + 1];
    __shared__ uint64_t s_block;
    __shared__ uint32_t s_field;
    __shared__ uint32_t s_ok;
    __shared__ uint64_t s_rec, s_out;

    const int tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const int wave = tid / 64;
    T *blkS = static_cast<T *>(q.scratch) + (size_t)blockIdx.x * N * N * N;

    while (true) {
        if (tid == 0) {
            const uint64_t t = atomicAdd(q.ticket, 1u);
            uint32_t ok = 0, f = 0;
            uint64_t rb = 0, ob = 0;
            if (t < q.ntickets) {
                f = field_of_ticket(q, t);
                const FieldView a = field_view(q, f);
                const uint8_t *in = static_cast<const uint8_t *>(a.src);
                const uint64_t *offs = reinterpret_cast<const uint64_t *>(in + 64);
                const uint64_t k = t - a.first;
                const uint64_t b = a.sel ? a.sel[2 * k] : k;  // the record this ticket decodes
                rb = b;
                ob = a.sel ? a.sel[2 * k + 1] : k;          // and the output block it fills
                ok = b < a.rblocks;
                const uint64_t o0 = ok ? offs[b] : 0, o1 = ok ? offs[b + 1] : 0;
                ok = ok && o1 >= o0 && o1 <= a.payload && o1 - o0 >= 8ull + MASK_BYTES;
                if (ok) {
                    const uint32_t nnz = *reinterpret_cast<const uint32_t *>(in + a.p0 + o0);
                    const uint64_t used = 8ull + MASK_BYTES + (uint64_t)nnz * sizeof(T);
                    ok = nnz <= (uint32_t)(N * N * N) && ((used + 15ull) & ~15ull) == o1 - o0;
                }
                if (!ok)
                    report(q, f, STATUS_FORMAT);
            }
            s_block = t;
            s_field = f;
            s_ok = ok;
            s_rec = rb;
            s_out = ob;
        }
        gbarrier<NT>();
        const uint64_t t = uniform64(s_block);
        if (t >= q.ntickets)
            break;
        if (!s_ok) {
            gbarrier<NT>();
            continue;
        }
        const FieldView a = field_view(q, s_field);
        const uint64_t b = uniform64(s_out);  // output block (the field's block index unless selected)
        const size_t plane = (size_t)a.nx * a.ny;
        const uint8_t *in = static_cast<const uint8_t *>(a.src);
        const uint64_t *offs = reinterpret_cast<const uint64_t *>(in + 64);
        const uint8_t *rec = in + a.p0 + offs[uniform64(s_rec)];
        const uint32_t nnz = *reinterpret_cast<const uint32_t *>(rec);
        const uint64_t *mask = reinterpret_cast<const uint64_t *>(rec + 8);
        const rsrc_t vr = make_rsrc(rec + 8 + MASK_BYTES, nnz * (uint32_t)sizeof(T));
        {
            uint64_t mw[WORDS / NT];
#pragma unroll
            for (int k = 0; k < WORDS / NT; ++k)
                mw[k] = mask[tid + k * NT];
#pragma unroll
            for (int k = 0; k < WORDS / NT; ++k)
                s_words[tid + k * NT] = mw[k];
        }
        gbarrier<NT>();
        const uint32_t total = scan_words<NT, WORDS>(s_words, s_pre, s_scan);
        gbarrier<NT>();
        if (total != nnz) {
            if (tid == 0)
                report(q, s_field, STATUS_FORMAT);
            gbarrier<NT>();
            continue;
        }
        // gather of the coarse octant: row (z, y) of it (x = lane < N/2) is
        // the low half of word z N + y; runs of U rows a wavefront, their
        // loads in flight together
        static_assert(N == 64 && (H * H) % (WAVES * DEC_U) == 0, "whole runs of octant rows");
        for (int r0 = wave * DEC_U; r0 < H * H; r0 += WAVES * DEC_U) {
            T v[DEC_U];
#pragma unroll
            for (int u = 0; u < DEC_U; ++u) {
                const int w = ((r0 + u) / H) * N + (r0 + u) % H;
                const uint64_t m = s_words[w];
                v[u] = T(0);
                if ((int)lane < H && ((m >> lane) & 1ull))
                    v[u] = buf_load<T>(vr, (s_pre[w] + mbcnt(m)) * (uint32_t)sizeof(T));
            }
#pragma unroll
            for (int u = 0; u < DEC_U; ++u) {
                const int z = (r0 + u) / H, y = (r0 + u) % H;
                if ((int)lane < H)
                    blkS[(size_t)z * N * N + y * N + (int)lane] = v[u];
            }
        }
        gbarrier<NT>();
        const uint32_t bx = (uint32_t)(b % a.nbx);
        const uint32_t by = (uint32_t)((b / a.nbx) % a.nby);
        const uint32_t bz = (uint32_t)(b / ((uint64_t)a.nbx * a.nby));
        T *dst = static_cast<T *>(a.dst) + ((size_t)bz * N * plane + (size_t)by * N * a.nx + (size_t)bx * N);
        big_inv<T, S, N, NT>(blkS, dst, plane, a.nx, lds, vr, s_words, s_pre);
        gbarrier<NT>();
    }
}

// ------------------------------------------------------------- bookkeeping

// Reset the queue's ticket and status, publish an inline descriptor and
// clear the per-field status words.  Forward: for every field (y index of
// the grid) clear its look-back flags and write its header (payload size 0
// until its last block fills it), offset 0 and the zero pad between its
// offset table and payload; a field without blocks gets its total here.
// Fix-up after a forward with deferred records (one field): chunk c of
// FIX_CHUNK blocks scans its record sizes, takes the sizes of all earlier
// chunks by a look-back over chunk flags, writes the offsets of its blocks
// and moves its deferred records from their slots into the stream.  Chunks
// take tickets from a counter behind the flags, so every smaller chunk is
// resident or done.
size_t defer_sizes_bytes(uint64_t nblocks)
{
    const uint64_t nch = (nblocks + FIX_CHUNK - 1) / FIX_CHUNK;
    return (size_t)(((nblocks * 4 + 7) & ~7ull) + 8 * (nch + 1));
}

__device__ __forceinline__ uint64_t *chunk_flags(uint32_t *sizes, uint64_t nblocks)
{
    return reinterpret_cast<uint64_t *>(reinterpret_cast<uint8_t *>(sizes) + ((nblocks * 4 + 7) & ~7ull));
}

__global__ __launch_bounds__(256) void defer_scan_kernel(Queue q)
{
    constexpr int NT = 256, PER = FIX_CHUNK / NT;
    __shared__ uint32_t s_scan[NT / 64 + 1];
    __shared__ uint64_t s_chunk, s_base;
    const FieldView a = field_view(q, 0);
    ConstDesc *desc = (ConstDesc *)q.fields;
    uint32_t *sizes = desc->sizes;
    const uint64_t nb = a.nblocks;
    const uint64_t nch = (nb + FIX_CHUNK - 1) / FIX_CHUNK;
    uint64_t *cflags = chunk_flags(sizes, nb);
    uint8_t *out = static_cast<uint8_t *>(a.dst);
    const int tid = threadIdx.x;
    while (true) {
        if (tid == 0)
            s_chunk = atomicAdd(reinterpret_cast<unsigned long long *>(cflags + nch), 1ull);
        lds_barrier();
        const uint64_t c = uniform64(s_chunk);
        if (c >= nch)
            break;
        const uint64_t b0 = c * FIX_CHUNK + (uint64_t)tid * PER;
        uint32_t sz[PER];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            sz[k] = b0 + k < nb ? sizes[b0 + k] & ~DEFER_BIT : 0u;
            sum += sz[k];
        }
        const uint32_t pre = block_exclusive_scan<NT>(sum, s_scan);  // a chunk's records stay below 2^32 bytes
        if (tid < 64) {
            const uint64_t o = lookback_wave(cflags, c, s_scan[NT / 64], q.status, nullptr);
            if (tid == 0)
                s_base = o;
        }
        lds_barrier();
        uint64_t run = s_base + pre;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const uint64_t b = b0 + k;
            if (b < nb) {
                run += sz[k];
                reinterpret_cast<uint64_t *>(out + 64)[b + 1] = run;
                if (b + 1 == nb) {
                    *reinterpret_cast<uint64_t *>(out + 56) = run;
                    if (a.total)
                        *a.total = a.p0 + run;
                }
            }
        }
        lds_barrier();  // s_chunk, s_base are rewritten for the next chunk
    }
}

// One wavefront per block: a deferred record moves from its slot to the
// offset the scan wrote, 16 bytes a lane (4 when the stream is not 16-byte
// aligned), every load issued before the stores.
__global__ __launch_bounds__(256) void defer_copy_kernel(Queue q)
{
    const FieldView a = field_view(q, 0);
    ConstDesc *desc = (ConstDesc *)q.fields;
    const uint8_t *slots = desc->defer;
    const uint32_t *sizes = desc->sizes;
    const uint64_t b = (uint64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (b >= a.nblocks)
        return;
    const uint32_t r = sizes[b];
    if (!(r & DEFER_BIT))
        return;
    const uint32_t sz = r & ~DEFER_BIT;
    const uint32_t lane = threadIdx.x % 64;
    uint8_t *out = static_cast<uint8_t *>(a.dst);
    const uint64_t off = reinterpret_cast<const uint64_t *>(out + 64)[b];
    const uint8_t *src = slots + b * DEFER_SLOT;
    uint8_t *dst = out + a.p0 + off;
    if (((reinterpret_cast<uintptr_t>(out) | (uintptr_t)a.p0) & 15u) == 0) {
        using u4 = uint32_t __attribute__((ext_vector_type(4)));
        constexpr int K = DEFER_SLOT / (64 * 16);
        u4 v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {  // offsets past the record re-read its first bytes (the slot is whole)
            const uint32_t o = (uint32_t)(k * 64 + lane) * 16u;
            v[k] = *reinterpret_cast<const u4 *>(src + (o < sz ? o : 0u));
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const uint32_t o = (uint32_t)(k * 64 + lane) * 16u;
            if (o < sz)
                *reinterpret_cast<u4 *>(dst + o) = v[k];
        }
    } else {
        for (uint32_t o = lane * 4u; o < sz; o += 64u * 4u)
            *reinterpret_cast<uint32_t *>(dst + o) = *reinterpret_cast<const uint32_t *>(src + o);
    }
}

__global__ void prep_kernel(Queue q, int forward)
{
    const uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    if (i0 == 0 && blockIdx.y == 0) {
        *q.ticket = 0;
        *q.status = 0;
        if (q.publish)
            *q.publish = q.one;
    }
    if (i0 == 0 && q.fstatus)
        q.fstatus[blockIdx.y] = 0;
    if (!forward)
        return;
    const FieldDesc &a = field_desc(q, blockIdx.y);
    uint8_t *out = static_cast<uint8_t *>(a.dst);
    for (uint64_t i = i0; i < a.nblocks; i += stride)
        a.flags[i] = 0;
    if (i0 == 0) {
        uint32_t *h = reinterpret_cast<uint32_t *>(out);
        for (int k = 0; k < 16; ++k)
            h[k] = a.header[k];
        reinterpret_cast<uint64_t *>(out + 64)[0] = 0;
        if (a.nblocks == 0 && a.total)
            *a.total = a.p0;
    }
    const uint64_t pad0 = 64 + 8 * (a.nblocks + 1);
    for (uint64_t p = pad0 + 4 * i0; p < a.p0; p += 4 * stride)
        *reinterpret_cast<uint32_t *>(out + p) = 0u;
    if (a.sizes) {  // the fix-up's chunk flags and chunk counter
        uint64_t *cf = chunk_flags(a.sizes, a.nblocks);
        const uint64_t nch = (a.nblocks + FIX_CHUNK - 1) / FIX_CHUNK;
        for (uint64_t i = i0; i <= nch; i += stride)
            cf[i] = 0;
    }
}

// OR the status words of a batch's classes (ticket, status pairs) into one.
__global__ void fold_status_kernel(const uint32_t *counters, int nclass, uint32_t *status)
{
    if (threadIdx.x == 0) {
        uint32_t bits = 0;
        for (int c = 0; c < nclass; ++c)
            bits |= counters[2 * c + 1];
        if (bits)
            atomicOr(status, bits);
    }
}

// ----------------------------------------------------------------- dispatch

// Shape per (precision, N, variant): slab depth Z, columns per thread R and
// (forward) planes kept in VGPRs ZP.
//   variant 0: float blocks and double blocks up to 16^3 staged whole in LDS,
//     one column per thread.  A double 32^3 block (256 KiB) is staged 16 slabs
//     at a time (132 KiB of LDS), one column per thread (1024 threads, 128
//     VGPRs a lane); after the finest level 14 planes of details are parked in
//     LDS (118 KiB + the 35 KiB coarse region).  Float 32^3 parks 16 planes.
//   variant 1: half the slab depth (N = 16, 32); two columns per thread at
//     N = 32.
//   variant 2 (double 32^3 only): 16 slabs at a time, two columns per thread
//     (512 threads, 256 VGPRs a lane).
template <typename T, int N, int V>
struct Shape {
    static constexpr bool big = sizeof(T) == 8 && N >= 32;
    // float 32^3, variant 2: the variant-1 tiling with two planes fewer parked
    // (76 KiB of LDS) so that two workgroups share a CU
    static constexpr bool pair = !big && N == 32 && V == 2;
    static constexpr int Z = (V == 1 && N >= 16) || pair ? (big ? N / 4 : N / 2) : (big ? N / 2 : N);
    static constexpr int R = (V == 2 && big) || (V == 1 && N == 32) || pair ? 2 : 1;
    static constexpr int ZP = N < 32 ? N : (big || pair ? N / 2 + 2 : N / 2);
    static constexpr int NT = N * N / R;
};

template <typename T, int N, int S, int V>
static hipError_t launch_fwd_t(const Queue &q, int grid, hipStream_t st)
{
    using P = Shape<T, N, V>;
    hipLaunchKernelGGL((fwd_kernel<T, N, S, P::Z, P::R, P::ZP>), dim3(grid), dim3(P::NT), 0, st, q);
    return hipGetLastError();
}

template <typename T, int N, int S, int V>
static hipError_t launch_inv_t(const Queue &q, int grid, hipStream_t st)
{
    using P = Shape<T, N, V>;
    hipLaunchKernelGGL((inv_kernel<T, N, S, P::Z, P::R>), dim3(grid), dim3(P::NT), 0, st, q);
    return hipGetLastError();
}

template <typename T, int N, int S, int V>
static int occupancy_t(bool inverse)
{
    using P = Shape<T, N, V>;
    int nb = 0;
    hipError_t e;
    if constexpr (N == 32)
        e = inverse ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, inv_kernel<T, N, S, P::Z, P::R>, P::NT, 0)
                    : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fwd_kernel<T, N, S, P::Z, P::R, P::ZP>,
                                                                   P::NT, 0);
    else  // smaller blocks: only the inverse uses this tiling
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, inv_kernel<T, N, S, P::Z, P::R>, P::NT, 0);
    return e == hipSuccess ? nb : 0;
}

template <typename T, int S>
static hipError_t launch_fwd_scratch_t(const Queue &q, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((fwd_scratch_kernel<T, 64, S>), dim3(grid), dim3(SCRATCH_THREADS), 0, st, q);
    return hipGetLastError();
}

template <typename T, int S>
static hipError_t launch_inv_scratch_t(const Queue &q, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((inv_scratch_kernel<T, 64, S>), dim3(grid), dim3(SCRATCH_THREADS), 0, st, q);
    return hipGetLastError();
}

template <typename T, int S>
static hipError_t scratch_dispatch(bool inverse, const Queue &q, int grid, hipStream_t st)
{
    return inverse ? launch_inv_scratch_t<T, S>(q, grid, st) : launch_fwd_scratch_t<T, S>(q, grid, st);
}

// (T, N, S, V) -> OP<T, N, S, V> ARGS for the on-chip block sizes.
#define CZ_SCHEMES(T, N, V, OP, ARGS)                                                                         \
    switch (key.scheme) {                                                                                    \
    case W4: return OP<T, N, W4, V> ARGS;                                                                    \
    case W4LI: return OP<T, N, W4LI, V> ARGS;                                                                \
    default: return OP<T, N, W3AI, V> ARGS;                                                                  \
    }
#define CZ_VARIANTS(T, N, OP, ARGS)                                                                           \
    if (key.variant == 1) {                                                                                  \
        CZ_SCHEMES(T, N, 1, OP, ARGS)                                                                        \
    }                                                                                                        \
    if constexpr (N == 32) {                                                                                 \
        if (key.variant == 2) {                                                                              \
            CZ_SCHEMES(T, N, 2, OP, ARGS)                                                                    \
        }                                                                                                    \
    }                                                                                                        \
    CZ_SCHEMES(T, N, 0, OP, ARGS)
#define CZ_DISPATCH(T, OP, ARGS)                                                                              \
    switch (key.block) {                                                                                     \
    case 8: CZ_SCHEMES(T, 8, 0, OP, ARGS)                                                                    \
    case 16: CZ_VARIANTS(T, 16, OP, ARGS)                                                                    \
    default: CZ_VARIANTS(T, 32, OP, ARGS)                                                                    \
    }

template <typename T, int N, int S>
static hipError_t launch_fwd_small_t(const Queue &q, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((fwd_small_kernel<T, N, S>), dim3(grid), dim3(64 * SmallGroup<T, N>::value), 0, st, q);
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_fwd_small(const KernelKey &key, const Queue &q, int grid, hipStream_t st)
{
    if (key.block == 8) {
        switch (key.scheme) {
        case W4: return launch_fwd_small_t<T, 8, W4>(q, grid, st);
        case W4LI: return launch_fwd_small_t<T, 8, W4LI>(q, grid, st);
        default: return launch_fwd_small_t<T, 8, W3AI>(q, grid, st);
        }
    }
    switch (key.scheme) {
    case W4: return launch_fwd_small_t<T, 16, W4>(q, grid, st);
    case W4LI: return launch_fwd_small_t<T, 16, W4LI>(q, grid, st);
    default: return launch_fwd_small_t<T, 16, W3AI>(q, grid, st);
    }
}

hipError_t launch_fwd(const KernelKey &key, const Queue &q, int grid, hipStream_t st)
{
    if (key.block <= 16)
        return key.elem_bytes == 4 ? launch_fwd_small<float>(key, q, grid, st)
                                   : launch_fwd_small<double>(key, q, grid, st);
    if (key.block == 64) {
        if (key.elem_bytes == 4) {
            switch (key.scheme) {
            case W4: return scratch_dispatch<float, W4>(false, q, grid, st);
            case W4LI: return scratch_dispatch<float, W4LI>(false, q, grid, st);
            default: return scratch_dispatch<float, W3AI>(false, q, grid, st);
            }
        }
        switch (key.scheme) {
        case W4: return scratch_dispatch<double, W4>(false, q, grid, st);
        case W4LI: return scratch_dispatch<double, W4LI>(false, q, grid, st);
        default: return scratch_dispatch<double, W3AI>(false, q, grid, st);
        }
    }
    if (key.elem_bytes == 4) {
        CZ_VARIANTS(float, 32, launch_fwd_t, (q, grid, st))
    } else {
        CZ_VARIANTS(double, 32, launch_fwd_t, (q, grid, st))
    }
}

template <typename T, int S>
static hipError_t launch_inv8_t(const Queue &q, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((inv_small8_kernel<T, S>), dim3(grid), dim3(64 * INV8_WAVES), 0, st, q);
    return hipGetLastError();
}

hipError_t launch_inv(const KernelKey &key, const Queue &q, int grid, hipStream_t st)
{
    if (key.block == 8) {
        if (key.elem_bytes == 4)
            return key.scheme == W4 ? launch_inv8_t<float, W4>(q, grid, st)
                 : key.scheme == W4LI ? launch_inv8_t<float, W4LI>(q, grid, st)
                                      : launch_inv8_t<float, W3AI>(q, grid, st);
        return key.scheme == W4 ? launch_inv8_t<double, W4>(q, grid, st)
             : key.scheme == W4LI ? launch_inv8_t<double, W4LI>(q, grid, st)
                                  : launch_inv8_t<double, W3AI>(q, grid, st);
    }
    if (key.block == 64) {
        if (key.elem_bytes == 4) {
            switch (key.scheme) {
            case W4: return scratch_dispatch<float, W4>(true, q, grid, st);
            case W4LI: return scratch_dispatch<float, W4LI>(true, q, grid, st);
            default: return scratch_dispatch<float, W3AI>(true, q, grid, st);
            }
        }
        switch (key.scheme) {
        case W4: return scratch_dispatch<double, W4>(true, q, grid, st);
        case W4LI: return scratch_dispatch<double, W4LI>(true, q, grid, st);
        default: return scratch_dispatch<double, W3AI>(true, q, grid, st);
        }
    }
    if (key.elem_bytes == 4) {
        CZ_DISPATCH(float, launch_inv_t, (q, grid, st))
    } else {
        CZ_DISPATCH(double, launch_inv_t, (q, grid, st))
    }
}

template <typename T, int N, int S>
static int occupancy_small_t()
{
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fwd_small_kernel<T, N, S>,
                                                                      64 * SmallGroup<T, N>::value, 0);
    return e == hipSuccess ? nb : 0;
}

int occupancy(const KernelKey &key, bool inverse)
{
    if (key.block == 64)
        return 1;  // one workgroup per CU, its blocks staged in its scratch slots
    if (!inverse && key.block <= 16) {
        const bool f = key.elem_bytes == 4;
        if (key.block == 8)
            return key.scheme == W4 ? (f ? occupancy_small_t<float, 8, W4>() : occupancy_small_t<double, 8, W4>())
                 : key.scheme == W4LI ? (f ? occupancy_small_t<float, 8, W4LI>() : occupancy_small_t<double, 8, W4LI>())
                 : (f ? occupancy_small_t<float, 8, W3AI>() : occupancy_small_t<double, 8, W3AI>());
        return key.scheme == W4 ? (f ? occupancy_small_t<float, 16, W4>() : occupancy_small_t<double, 16, W4>())
             : key.scheme == W4LI ? (f ? occupancy_small_t<float, 16, W4LI>() : occupancy_small_t<double, 16, W4LI>())
             : (f ? occupancy_small_t<float, 16, W3AI>() : occupancy_small_t<double, 16, W3AI>());
    }
    if (!inverse) {
        if (key.elem_bytes == 4) {
            CZ_VARIANTS(float, 32, occupancy_t, (inverse))
        } else {
            CZ_VARIANTS(double, 32, occupancy_t, (inverse))
        }
    }
    if (key.block == 8) {
        int nb = 0;
        const hipError_t e =
            key.elem_bytes == 4
                ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, inv_small8_kernel<float, W3AI>, 64 * INV8_WAVES, 0)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, inv_small8_kernel<double, W3AI>, 64 * INV8_WAVES, 0);
        return e == hipSuccess ? nb : 0;
    }
    if (key.elem_bytes == 4) {
        CZ_DISPATCH(float, occupancy_t, (inverse))
    } else {
        CZ_DISPATCH(double, occupancy_t, (inverse))
    }
}

bool fwd_one_block_per_workgroup(const KernelKey &key) { return key.block <= 32; }

uint32_t fwd_blocks_per_ticket(const KernelKey &key)
{
    if (key.block == 8)
        return key.elem_bytes == 8 ? SmallGroup<double, 8>::value : SmallGroup<float, 8>::value;
    if (key.block == 16)
        return key.elem_bytes == 8 ? SmallGroup<double, 16>::value : SmallGroup<float, 16>::value;
    return 1u;
}

// 64^3 variants differ only in how many workgroups (each with its scratch
// slot) are resident at once: 256, 128 or 64.  Fewer slots keep the scratch
// working set in the last-level cache at the price of idle CUs.
int variant_count(uint32_t block, uint32_t elem_bytes)
{
    if (block == 32)
        return 3;
    return block == 16 ? 2 : block == 64 ? 3 : 1;
}

size_t scratch_bytes(const KernelKey &key, int grid)
{
    if (key.block != 64)
        return 0;
    // forward: two slots and two side areas (mask words and prefixes) per
    // workgroup; the inverse uses the first grid slots
    const size_t words = (size_t)64 * 64 * 64 / 64;
    return (size_t)grid * 2 * ((size_t)64 * 64 * 64 * key.elem_bytes + words * (sizeof(uint64_t) + sizeof(uint32_t)));
}

int grid_cap(const KernelKey &key)
{
    return key.block == 64 ? 256 >> (key.variant < 3 ? key.variant : 0) : 0;
}

hipError_t launch_fold_status(const uint32_t *counters, int nclass, uint32_t *status, hipStream_t st)
{
    hipLaunchKernelGGL(fold_status_kernel, dim3(1), dim3(64), 0, st, counters, nclass, status);
    return hipGetLastError();
}

hipError_t launch_defer_fix(const Queue &q, hipStream_t st)
{
    const uint64_t nb = q.one.nblocks;
    const uint64_t nch = (nb + FIX_CHUNK - 1) / FIX_CHUNK;
    if (nch == 0)
        return hipSuccess;
    const uint64_t g = nch < 2048 ? nch : 2048;  // workgroups loop over chunk tickets
    hipLaunchKernelGGL(defer_scan_kernel, dim3((uint32_t)g), dim3(256), 0, st, q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(defer_copy_kernel, dim3((uint32_t)((nb + 3) / 4)), dim3(256), 0, st, q);
    return hipGetLastError();
}

hipError_t launch_prep(const Queue &q, bool forward, hipStream_t st)
{
    // enough threads in x to clear the largest field's flags in a few passes
    const uint64_t most = forward && q.ntickets > 0 ? q.ntickets : 1;
    int gx = (int)((most + 255) / 256);
    if (gx > 1024)
        gx = 1024;
    const uint32_t gy = forward || q.fstatus ? q.nfields : 1;
    hipLaunchKernelGGL(prep_kernel, dim3(gx, gy), dim3(256), 0, st, q, forward ? 1 : 0);
    return hipGetLastError();
}

}  // namespace czk
