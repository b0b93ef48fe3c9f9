// GPU lossless stage: byte-oriented canonical Huffman coding in
// independently decodable chunks.  The paper's second substage is a
// general-purpose lossless coder over the (optionally shuffled) output of the
// wavelet stage (Sec. 2.2-2.3); on the GPU it runs next to the data instead of
// after a device-to-host copy.
//
// Code lengths: optimal under a 12-bit limit (package-merge, Larmore and
// Hirschberg 1990: leaves sorted by (count, symbol); L - 1 rounds of pairing
// the previous list into packages and merging them with the leaves by weight,
// a leaf before a package of equal weight; the first 2n - 2 items give the
// lengths).  Codes: canonical (RFC 1951, Sec. 3.2.2), written bit-reversed,
// least significant bit first, into little-endian 32-bit words; each chunk of
// 4 KiB of input is padded to whole words.  Container: 32-byte header
// {"CZH1", version 1, u64 raw bytes, u32 chunk bytes, u32 chunks, u32 max
// length, u32 0}, 256 code lengths, (chunks + 1) u64 chunk offsets relative to
// the payload, zero pad to 16 bytes, the chunks.
//
// Encoding: a histogram kernel, the code built on the host from the 256
// counts, and one encoding kernel (one workgroup a group of chunks, codes
// packed with LDS atomics, the group placed by a decoupled look-back over the
// group sizes and copied out whole): two reads of the input.  Decoding: one thread
// a chunk with a 4096-entry lookup table in LDS, the lanes of a wavefront in
// lockstep, the chunk's words read ahead into an LDS ring and the decoded
// words staged in LDS and written by the whole wavefront.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "cz_host.h"
#include "cz_lookback.h"

namespace {

constexpr uint32_t MAGIC = 0x31485A43u;  // "CZH1"
constexpr int MAXLEN = 12;
constexpr uint32_t CHUNK = 4096;
constexpr int ENC_THREADS = 256;
constexpr int BYTES_PER_THREAD = CHUNK / ENC_THREADS;
constexpr uint32_t CHUNK_WORDS = (CHUNK * MAXLEN + 31) / 32;
constexpr size_t HEAD = 32 + 256;

size_t payload_start(uint64_t nchunks) { return (HEAD + 8 * (nchunks + 1) + 15) & ~size_t(15); }

// Byte histogram.  Each workgroup counts into HIST_COPIES interleaved copies
// of the 256 bins (lane l uses copy l % HIST_COPIES), so a run of equal bytes
// -- the zero bytes of a shuffled stream -- spreads over several LDS words
// instead of serializing on one.  The 16-byte-aligned middle of the input is
// read 16 bytes a thread; the unaligned ends byte by byte.
constexpr int HIST_THREADS = 256;
constexpr int HIST_COPIES = 16;

__global__ __launch_bounds__(HIST_THREADS) void hist_kernel(const uint8_t *__restrict__ in, uint64_t n,
                                                            unsigned long long *hist)
{
    __shared__ uint32_t h[256 * HIST_COPIES];
    for (int k = threadIdx.x; k < 256 * HIST_COPIES; k += HIST_THREADS)
        h[k] = 0;
    __syncthreads();
    const uint32_t copy = threadIdx.x % HIST_COPIES;
    const uint64_t head = min<uint64_t>(n, (16 - (reinterpret_cast<uintptr_t>(in) & 15)) & 15);
    const uint64_t units = (n - head) / 16;
    const uint64_t tail = head + units * 16;
    const uint64_t gid = (uint64_t)blockIdx.x * HIST_THREADS + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * HIST_THREADS;
    const uint4 *mid = reinterpret_cast<const uint4 *>(in + head);
    for (uint64_t u = gid; u < units; u += stride) {
        const uint4 v = mid[u];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int k = 0; k < 16; ++k)
            atomicAdd(&h[((w[k / 4] >> (8 * (k % 4))) & 0xFFu) * HIST_COPIES + copy], 1u);
    }
    // the unaligned head and the tail: at most 15 bytes each
    if (gid < head)
        atomicAdd(&h[in[gid] * HIST_COPIES + copy], 1u);
    if (gid < n - tail)
        atomicAdd(&h[in[tail + gid] * HIST_COPIES + copy], 1u);
    __syncthreads();
    for (int bin = threadIdx.x; bin < 256; bin += HIST_THREADS) {
        uint32_t t = 0;
#pragma unroll
        for (int k = 0; k < HIST_COPIES; ++k)
            t += h[bin * HIST_COPIES + k];
        if (t)
            atomicAdd(&hist[bin], (unsigned long long)t);
    }
}

// One workgroup a group of CPG consecutive chunks, groups in ticket order.
// Thread t codes bytes [16 t, 16 t + 16) of every chunk of the group; a
// workgroup scan of the threads' bit counts (one per chunk) places every code
// in its chunk's words, packed in LDS with atomic ORs.  The group's byte size
// goes through a decoupled look-back over the groups (the same single-pass
// exclusive scan that places the block records), which gives the group's
// offset in the payload; its chunks are then copied out whole, back to back.
constexpr int CPG = 8;

// WORDS: the input is 16-byte aligned, and every thread reads its 16 bytes
// of each chunk through a buffer resource whose extent is the group's input
// rounded up to 16 bytes (a read is wholly inside it or wholly past it and
// then reads 0; bytes past the input lie in its last 16-byte block, on its
// last page, and are not used), issued by every thread for every chunk
// before any is used -- all eight chunks' reads in flight together.
// Otherwise 16-byte loads where aligned, bytes elsewhere.
template <bool WORDS>
__global__ __launch_bounds__(ENC_THREADS) void encode_kernel(const uint8_t *__restrict__ in, uint64_t n,
                                                             const uint32_t *__restrict__ code, uint64_t nchunks,
                                                             uint64_t *flags, uint32_t *ticket, uint64_t *offs,
                                                             uint8_t *payload, uint64_t *total, uint32_t *status)
{
    constexpr int NW = ENC_THREADS / 64;
    __shared__ uint32_t s_code[256];
    __shared__ uint32_t s_words[CPG][CHUNK_WORDS];
    __shared__ uint32_t s_scan[CPG][NW + 1];  // per chunk: wave prefixes, then the chunk's bits
    __shared__ uint32_t s_cw[CPG + 1];        // word offsets of the chunks within the group
    __shared__ uint64_t s_g, s_off;
    if (threadIdx.x == 0)
        s_g = atomicAdd(ticket, 1u);
    s_code[threadIdx.x] = code[threadIdx.x];
    for (uint32_t w = threadIdx.x; w < CPG * CHUNK_WORDS; w += ENC_THREADS)
        (&s_words[0][0])[w] = 0;
    __syncthreads();
    const uint64_t g = s_g;
    const uint64_t c0 = g * CPG;
    if (c0 >= nchunks)
        return;
    const int nc = (int)min<uint64_t>(CPG, nchunks - c0);
    const uint32_t lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    uint32_t data[CPG][4];
    int cnt[CPG];
    uint32_t mybits[CPG], incl[CPG];
#pragma unroll
    for (int j = 0; j < CPG; ++j) {
        const uint64_t base = (c0 + j) * CHUNK + (uint64_t)threadIdx.x * BYTES_PER_THREAD;
        cnt[j] = j < nc ? (int)min<uint64_t>(BYTES_PER_THREAD, base < n ? n - base : 0) : 0;
    }
    if constexpr (WORDS) {
        const uint64_t gbase = c0 * CHUNK;  // < n: the group has a chunk
        const uint64_t span = min<uint64_t>(n - gbase, (uint64_t)CPG * CHUNK);
        const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<uint8_t *>(in + gbase), (short)0, (int)((span + 15) & ~15ull), 0x00020000);
#pragma unroll
        for (int j = 0; j < CPG; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                data[j][q] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(
                    r, (uint32_t)(j * CHUNK + threadIdx.x * BYTES_PER_THREAD + 4 * q), 0, 0);
    }
#pragma unroll
    for (int j = 0; j < CPG; ++j) {
        if constexpr (!WORDS) {
            const uint64_t base = (c0 + j) * CHUNK + (uint64_t)threadIdx.x * BYTES_PER_THREAD;
            if (cnt[j] == BYTES_PER_THREAD && (reinterpret_cast<uintptr_t>(in + base) & 15) == 0) {
                const uint4 v = *reinterpret_cast<const uint4 *>(in + base);
                data[j][0] = v.x;
                data[j][1] = v.y;
                data[j][2] = v.z;
                data[j][3] = v.w;
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    uint32_t w = 0;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        w |= (4 * q + k < cnt[j] ? (uint32_t)in[base + 4 * q + k] : 0u) << (8 * k);
                    data[j][q] = w;
                }
            }
        }
        uint32_t bits = 0;
#pragma unroll
        for (int k = 0; k < BYTES_PER_THREAD; ++k)
            bits += k < cnt[j] ? s_code[(data[j][k / 4] >> (8 * (k % 4))) & 0xFFu] >> 16 : 0u;
        mybits[j] = bits;
        incl[j] = bits;
    }
    // exclusive scans of the threads' bit counts, one per chunk
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
        for (int j = 0; j < CPG; ++j) {
            const uint32_t v = __shfl_up(incl[j], o);
            if (lane >= (uint32_t)o)
                incl[j] += v;
        }
    }
    if (lane == 63) {
#pragma unroll
        for (int j = 0; j < CPG; ++j)
            s_scan[j][wave] = incl[j];
    }
    __syncthreads();
    if (threadIdx.x < CPG) {
        const int j = threadIdx.x;
        uint32_t run = 0;
        for (int w = 0; w < NW; ++w) {
            const uint32_t v = s_scan[j][w];
            s_scan[j][w] = run;
            run += v;
        }
        s_scan[j][NW] = run;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int j = 0; j < CPG; ++j) {
            s_cw[j] = run;
            run += (s_scan[j][NW] + 31) / 32;
        }
        s_cw[CPG] = run;
    }
#pragma unroll
    for (int j = 0; j < CPG; ++j) {
        uint32_t pos = s_scan[j][wave] + incl[j] - mybits[j];
#pragma unroll
        for (int k = 0; k < BYTES_PER_THREAD; ++k) {
            if (k < cnt[j]) {
                const uint32_t e = s_code[(data[j][k / 4] >> (8 * (k % 4))) & 0xFFu];
                const uint32_t l = e >> 16, r = e & 0xFFFFu;
                const uint32_t w = pos / 32, sh = pos % 32;
                atomicOr(&s_words[j][w], r << sh);
                if (sh + l > 32)
                    atomicOr(&s_words[j][w + 1], r >> (32 - sh));
                pos += l;
            }
        }
    }
    __syncthreads();
    const uint64_t bytes = (uint64_t)s_cw[CPG] * 4;
    if (threadIdx.x < 64) {
        const uint64_t o = czk::lookback_wave(flags, g, bytes, status, nullptr);
        if (threadIdx.x == 0)
            s_off = o;
    }
    __syncthreads();
    const uint64_t off = s_off;
    if (threadIdx.x <= (uint32_t)nc) {
        const int j = threadIdx.x;
        if (j > 0 || g == 0)
            offs[c0 + j] = off + (uint64_t)s_cw[j] * 4;  // chunk c0 + j starts here (c0 + nc: the end)
    }
    if (threadIdx.x == 0 && c0 + nc == nchunks)
        *total = off + bytes;
    uint32_t *dst = reinterpret_cast<uint32_t *>(payload + off);
    for (int j = 0; j < nc; ++j) {
        const uint32_t w0 = s_cw[j], nw = s_cw[j + 1] - w0;
        for (uint32_t w = threadIdx.x; w < nw; w += ENC_THREADS)
            dst[w0 + w] = s_words[j][w];
    }
}

// Decoder workgroups: one wavefront for short streams (few chunks: every
// CU should get some), four for long ones (they share one copy of the table
// in LDS, so more wavefronts fit a CU).  Each wavefront runs its own lockstep
// loop and synchronizes only within itself.
constexpr uint64_t DEC_WIDE_CHUNKS = 256ull * 64 * 16;  // chunks from which a group has four wavefronts

// Decoding: one thread a chunk, table[k] = symbol | length << 8 for the next
// 12 bits k (in LDS), one symbol a step on every lane, and every vector
// memory access issued by all lanes at fixed steps (a lane with nothing to
// move uses an offset past the buffer's extent: its load returns 0 and its
// store is dropped).  The waits for them then count exactly, and no wait
// covers another access still in flight -- a load issued under a divergent
// branch, or a store every few symbols, would make every refill wait for
// all of them.
//   * input: each lane's next words wait in an LDS ring of LS_RING words, fed
//     every LS_PERIOD steps from two sets of four word loads, each set in
//     flight for two periods; a lane whose ring is empty before its chunk's
//     words are all in skips the step;
//   * output: every fourth symbol's word goes to an LDS ring of out_words
//     words; every 4 out_words steps the wave writes all lanes' new words,
//     out_words consecutive words of a chunk per group of lanes of a store
//     instruction.
constexpr int LS_RING = 16;
constexpr int LS_RP = LS_RING + 1;  // odd pitches: lanes on different banks
constexpr int LS_PERIOD = 8;
constexpr uint32_t LS_OOR = 0xFFFFFFF0u;  // an offset past every buffer's extent
constexpr int out_words(int waves) { return waves > 1 ? 8 : 16; }

using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ rsrc_t ls_rsrc(const void *base, uint32_t bytes)
{
    // raw buffer (stride 0): accesses at or past `bytes` read 0 and drop writes
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ uint32_t ls_load(rsrc_t r, uint32_t off)
{
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
}

__device__ __forceinline__ uint64_t ls_min(uint64_t a, uint64_t b) { return a < b ? a : b; }

struct LsSet {
    uint32_t v[4];
    uint32_t n;  // words of this set that carry data
};

// Ordering of LDS accesses between the lanes of one wavefront: they run in
// program order, so a compiler-level fence suffices.  A one-wavefront group
// uses the workgroup barrier, which is the same there and compiles tighter.
template <int WAVES>
__device__ __forceinline__ void wave_sync()
{
    if constexpr (WAVES == 1) {
        __syncthreads();
    } else {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
}

template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void decode_kernel(const uint8_t *__restrict__ payload,
                                                             uint64_t payload_bytes,
                                                             const uint64_t *__restrict__ offs,
                                                             const uint16_t *__restrict__ table, uint64_t nchunks,
                                                             uint64_t raw, uint8_t *out, uint32_t *status)
{
    constexpr int NT = 64 * WAVES;
    constexpr int LS_OUT = out_words(WAVES), LS_OP = LS_OUT + 1, LS_FLUSH = 4 * LS_OUT;
    __shared__ uint16_t s_tab[1u << MAXLEN];
    __shared__ uint32_t s_in[NT * LS_RP];  // a row per thread
    __shared__ uint32_t s_out[NT * LS_OP];
    __shared__ uint32_t s_from[NT], s_to[NT];
    for (uint32_t k = threadIdx.x; k < (1u << MAXLEN); k += NT)
        s_tab[k] = table[k];
    const uint32_t t = threadIdx.x;
    const uint32_t lane = WAVES > 1 ? t % 64 : t;
    const uint32_t w64 = WAVES > 1 ? t - lane : 0u;  // the wavefront's first thread
    const uint64_t c0 = ((uint64_t)blockIdx.x * WAVES + t / 64) * 64;  // the wavefront's first chunk
    const uint64_t c = c0 + lane;
    bool err = false;
    bool live = c < nchunks;
    uint64_t o0 = 0, o1 = 0;
    if (live) {
        o0 = offs[c];
        o1 = offs[c + 1];
        if (o1 < o0 || o1 > payload_bytes || (o0 | o1) % 4 || o1 == o0) {
            err = true;  // a chunk with symbols needs words inside the payload
            live = false;
        }
    }
    // the workgroup's input window: from the smallest chunk start
    uint64_t base = live ? o0 : ~0ull;
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)base, m, 64);
        const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(base >> 32), m, 64);
        const uint64_t o = ((uint64_t)hi << 32) | lo;
        base = o < base ? o : base;
    }
    if (base == ~0ull)
        base = 0;
    {  // equal on every lane: make it scalar (readfirstlane returns a signed 32-bit value)
        const uint32_t bhi = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
        const uint32_t blo = (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)base);
        base = ((uint64_t)bhi << 32) | blo;
    }
    if (live && o1 - base > 0x7FFFFFF0ull) {  // a valid container's group spans a few hundred KiB
        err = true;
        live = false;
    }
    const rsrc_t rin = ls_rsrc(payload + base, (uint32_t)(ls_min(payload_bytes - base, 0x7FFFFFF0ull) & ~3ull));
    const uint64_t obase = c0 * CHUNK;  // below raw unless the wavefront has no chunk (then unused)
    const rsrc_t rout = ls_rsrc(out + obase, (uint32_t)(ls_min(raw - obase, 64ull * CHUNK) & ~3ull));
    const uint32_t w0 = live ? (uint32_t)((o0 - base) / 4) : 0u;  // first word, in the window
    const uint32_t nw = live ? (uint32_t)((o1 - o0) / 4) : 0u;    // the chunk's words
    const uint32_t nbits = nw * 32u;
    const uint32_t n = live ? (uint32_t)ls_min(CHUNK, raw - c * CHUNK) : 0u;
    uint32_t issued = 0, tail = 0, head = 0;
    auto issue = [&](LsSet &s) {
        s.n = (issued < nw && issued + 4 <= head + LS_RING) ? min(4u, nw - issued) : 0u;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            s.v[k] = ls_load(rin, (uint32_t)k < s.n ? (w0 + issued + (uint32_t)k) * 4u : LS_OOR);
        issued += s.n;
    };
    uint32_t nxt = 0;  // the ring's word at head, once head < tail
    auto land = [&](const LsSet &s) {
        // words past the set's count go to the row's pad word
#pragma unroll
        for (int k = 0; k < 4; ++k)
            s_in[t * LS_RP + ((uint32_t)k < s.n ? (tail + (uint32_t)k) % LS_RING : LS_RING)] = s.v[k];
        nxt = head == tail && s.n ? s.v[0] : nxt;
        tail += s.n;
    };
    LsSet A, B;
    issue(A);
    issue(B);
    land(A);
    land(B);
    issue(A);
    issue(B);
    __syncthreads();  // the table; from here on each wavefront keeps to itself
    if (c0 >= nchunks)
        return;

    uint64_t window = 0;
    uint32_t avail = 0, used = 0, pack = 0, i = 0, flushed = 0;
    // one step, without branches: the lanes of a wavefront run one
    // instruction stream, and a branch per condition would cost every lane
    // the exec-mask bookkeeping of all of them
    auto step = [&]() {
        const bool go = live && i < n;
        const bool need = go && avail < (uint32_t)MAXLEN && head < tail;
        window |= need ? (uint64_t)nxt << avail : 0ull;  // avail < 44: the shift is defined
        avail += need ? 32u : 0u;
        head += need ? 1u : 0u;
        const uint32_t ahead = s_in[t * LS_RP + head % LS_RING];  // needed two steps later at the earliest
        nxt = need ? ahead : nxt;
        // decode unless more words are due than have landed
        const bool dec = go && (avail >= (uint32_t)MAXLEN || tail == nw);
        const uint32_t e = s_tab[window & ((1u << MAXLEN) - 1)];
        const uint32_t l = e >> 8;
        const bool bad = dec && (l == 0 || used + l > nbits);  // no such code, or past the chunk's bits
        const bool ok = dec && !bad;
        err = err || bad;
        live = live && !bad;
        used += ok ? l : 0u;
        window = ok ? window >> l : window;
        avail -= ok ? l : 0u;
        pack |= ok ? (e & 0xFFu) << (8 * (i % 4)) : 0u;
        // a completed word goes to the ring, anything else to the row's pad word
        const bool full = ok && i % 4 == 3;
        s_out[t * LS_OP + (full ? (i / 4) % LS_OUT : LS_OUT)] = pack;
        pack = full ? 0u : pack;
        i += ok ? 1u : 0u;
    };
    auto flush = [&]() {
        // rows r of the wavefront: words [s_from, s_to) of chunk c0 + r,
        // LS_OUT a row at most
        s_from[t] = flushed;
        s_to[t] = i / 4;
        wave_sync<WAVES>();
#pragma unroll 4
        for (int k = 0; k < LS_OUT; ++k) {
            const uint32_t r = (64u / LS_OUT) * (uint32_t)k + lane / LS_OUT;
            const uint32_t w = s_from[w64 + r] + lane % LS_OUT;
            const bool ok = w < s_to[w64 + r];
            const uint32_t v = s_out[(w64 + r) * LS_OP + w % LS_OUT];
            __builtin_amdgcn_raw_buffer_store_b32(v, rout, ok ? r * CHUNK + w * 4u : LS_OOR, 0, 0);
        }
        flushed = i / 4;
        wave_sync<WAVES>();
    };
    uint32_t s = 0;
    while (__ballot(live && i < n)) {
#pragma unroll
        for (int k = 0; k < LS_PERIOD; ++k)
            step();
        land(A);
        issue(A);
#pragma unroll
        for (int k = 0; k < LS_PERIOD; ++k)
            step();
        land(B);
        issue(B);
        s += 2 * LS_PERIOD;
        if (s % LS_FLUSH == 0)
            flush();
    }
    flush();
    // the last chunk's trailing bytes
    if (live && n % 4)
        for (uint32_t k = 0; k < n % 4; ++k)
            out[c * CHUNK + n - n % 4 + k] = (uint8_t)(pack >> (8 * k));
    if (err)
        atomicOr(status, czk::STATUS_FORMAT);
}

// Package-merge: length-limited optimal code lengths (see the file header).
void package_merge(const uint64_t counts[256], uint8_t lengths[256])
{
    std::memset(lengths, 0, 256);
    std::vector<int> used;
    for (int s = 0; s < 256; ++s)
        if (counts[s])
            used.push_back(s);
    if (used.empty())
        return;
    if (used.size() == 1) {
        lengths[used[0]] = 1;
        return;
    }
    const int n = (int)used.size();
    std::stable_sort(used.begin(), used.end(), [&](int a, int b) { return counts[a] < counts[b]; });
    // list[l]: the leaves merged with the packages of list[l - 1] (package j
    // pairs its items 2 j and 2 j + 1).  An item is a leaf position (>= 0) or
    // -1 - j for package j.
    struct Item {
        uint64_t w;
        int what;
    };
    std::vector<std::vector<Item>> list(MAXLEN);
    for (int i = 0; i < n; ++i)
        list[0].push_back({counts[used[i]], i});
    for (int l = 1; l < MAXLEN; ++l) {
        const std::vector<Item> &prev = list[l - 1];
        std::vector<Item> &cur = list[l];
        const int np = (int)prev.size() / 2;
        int i = 0, j = 0;
        while (i < n || j < np) {
            const uint64_t pw = j < np ? prev[2 * j].w + prev[2 * j + 1].w : 0;
            if (j >= np || (i < n && list[0][i].w <= pw)) {
                cur.push_back(list[0][i]);
                ++i;
            } else {
                cur.push_back({pw, -1 - j});
                ++j;
            }
        }
    }
    // The first 2 n - 2 items of the last list are chosen; the packages in a
    // chosen prefix are packages 0 .. p - 1, which choose the first 2 p items
    // of the list below.  A leaf's length is the number of lists in whose
    // chosen prefix it appears.
    std::vector<int> len(n, 0);
    int sel = 2 * n - 2;
    for (int l = MAXLEN - 1; l >= 0; --l) {
        int p = 0;
        for (int k = 0; k < sel; ++k) {
            if (list[l][k].what >= 0)
                ++len[list[l][k].what];
            else
                ++p;
        }
        sel = 2 * p;
    }
    for (int k = 0; k < n; ++k)
        lengths[used[k]] = (uint8_t)len[k];
}

// Canonical codes, bit-reversed: code[s] = reversed code | length << 16.
void canonical(const uint8_t lengths[256], uint32_t code[256])
{
    int bl_count[MAXLEN + 2] = {0};
    for (int s = 0; s < 256; ++s)
        if (lengths[s])
            ++bl_count[lengths[s]];
    uint32_t next[MAXLEN + 2] = {0};
    uint32_t c = 0;
    for (int bits = 1; bits <= MAXLEN; ++bits) {
        c = (c + (uint32_t)bl_count[bits - 1]) << 1;
        if (bits == 1)
            c = 0;
        next[bits] = c;
    }
    for (int s = 0; s < 256; ++s) {
        const int l = lengths[s];
        code[s] = 0;
        if (!l)
            continue;
        uint32_t v = next[l]++, r = 0;
        for (int k = 0; k < l; ++k) {
            r = (r << 1) | (v & 1u);
            v >>= 1;
        }
        code[s] = r | ((uint32_t)l << 16);
    }
}

}  // namespace

extern "C" {

size_t cz_huff_bound(size_t nbytes)
{
    const uint64_t nchunks = (nbytes + CHUNK - 1) / CHUNK;
    return payload_start(nchunks) + nchunks * (size_t)CHUNK_WORDS * 4;
}

int cz_huff_encode(cz_ctx *ctx, const void *d_in, size_t nbytes, void *d_out, size_t out_cap, size_t *h_out_bytes,
                   void *stream)
{
    if (!ctx || !d_out || !h_out_bytes || (nbytes && !d_in) || nbytes >= (1ull << 40) ||
        reinterpret_cast<uintptr_t>(d_out) % 8)
        return CZ_ERR_ARG;
    const uint64_t nchunks = (nbytes + CHUNK - 1) / CHUNK;
    if (out_cap < cz_huff_bound(nbytes)) {
        *h_out_bytes = cz_huff_bound(nbytes);
        return CZ_ERR_CAPACITY;
    }
    czh::DeviceGuard guard(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint8_t *in = static_cast<const uint8_t *>(d_in);
    uint8_t *out = static_cast<uint8_t *>(d_out);
    // workspace: histogram (256 u64), code table (256 u32), ticket, status,
    // payload size, then the look-back flags (one u64 a group of chunks)
    constexpr size_t W_HIST = 0, W_CODE = 2048, W_TICKET = 3072, W_STATUS = 3076, W_TOTAL = 3080, W_FLAGS = 3088;
    const uint64_t ngroups = (nchunks + CPG - 1) / CPG;
    int rc = ctx->huff.ensure(W_FLAGS + ngroups * 8);
    if (rc != CZ_OK)
        return rc;
    uint8_t *w = static_cast<uint8_t *>(ctx->huff.ptr);
    unsigned long long *hist = reinterpret_cast<unsigned long long *>(w + W_HIST);
    uint32_t *code = reinterpret_cast<uint32_t *>(w + W_CODE);
    uint64_t *total = reinterpret_cast<uint64_t *>(w + W_TOTAL);
    uint64_t counts[256] = {0};
    if (hipMemsetAsync(hist, 0, 2048, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (nbytes) {
        const int g = (int)std::min<uint64_t>((nbytes / 16 + HIST_THREADS - 1) / HIST_THREADS + 1, 4096);
        hipLaunchKernelGGL(hist_kernel, dim3(g), dim3(HIST_THREADS), 0, st, in, (uint64_t)nbytes, hist);
        if (hipGetLastError() != hipSuccess)
            return CZ_ERR_HIP;
    }
    if (hipMemcpyAsync(counts, hist, 2048, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return CZ_ERR_HIP;
    uint8_t head[HEAD];
    std::memset(head, 0, HEAD);
    uint8_t *lengths = head + 32;
    package_merge(counts, lengths);
    uint32_t table[256];
    canonical(lengths, table);
    const uint32_t h32[8] = {MAGIC, 1, (uint32_t)nbytes, (uint32_t)((uint64_t)nbytes >> 32), CHUNK, (uint32_t)nchunks,
                             (uint32_t)MAXLEN, 0};
    std::memcpy(head, h32, 32);
    const size_t p0 = payload_start(nchunks);
    // header + code table through pinned staging; the pad between offsets and
    // payload, the ticket, status and total, and the flags start at zero
    std::vector<uint8_t> stage(HEAD + 1024);
    std::memcpy(stage.data(), head, HEAD);
    std::memcpy(stage.data() + HEAD, table, 1024);
    if ((rc = ctx->huff_stage.upload(stage.data(), stage.size(), st)) != CZ_OK)
        return rc;
    const uint8_t *staged = static_cast<const uint8_t *>(ctx->huff_stage.dev.ptr);
    if (hipMemcpyAsync(out, staged, HEAD, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(code, staged + HEAD, 1024, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemsetAsync(out + HEAD + 8 * (nchunks + 1), 0, p0 - (HEAD + 8 * (nchunks + 1)), st) != hipSuccess ||
        hipMemsetAsync(w + W_TICKET, 0, W_FLAGS - W_TICKET + ngroups * 8, st) != hipSuccess)
        return CZ_ERR_HIP;
    uint64_t *offs = reinterpret_cast<uint64_t *>(out + HEAD);
    if (nchunks) {
        if (reinterpret_cast<uintptr_t>(in) % 16 == 0)
            hipLaunchKernelGGL(encode_kernel<true>, dim3((unsigned)ngroups), dim3(ENC_THREADS), 0, st, in,
                               (uint64_t)nbytes, code, nchunks, reinterpret_cast<uint64_t *>(w + W_FLAGS),
                               reinterpret_cast<uint32_t *>(w + W_TICKET), offs, out + p0, total,
                               reinterpret_cast<uint32_t *>(w + W_STATUS));
        else
            hipLaunchKernelGGL(encode_kernel<false>, dim3((unsigned)ngroups), dim3(ENC_THREADS), 0, st, in,
                               (uint64_t)nbytes, code, nchunks, reinterpret_cast<uint64_t *>(w + W_FLAGS),
                               reinterpret_cast<uint32_t *>(w + W_TICKET), offs, out + p0, total,
                               reinterpret_cast<uint32_t *>(w + W_STATUS));
        if (hipGetLastError() != hipSuccess)
            return CZ_ERR_HIP;
    } else if (hipMemsetAsync(offs, 0, 8, st) != hipSuccess) {
        return CZ_ERR_HIP;
    }
    uint64_t back[2] = {0, 0};  // status word (low half), payload size
    if (hipMemcpyAsync(back, w + W_TICKET, 16, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return CZ_ERR_HIP;
    if ((uint32_t)(back[0] >> 32) != 0)
        return CZ_ERR_TIMEOUT;
    *h_out_bytes = p0 + back[1];
    return CZ_OK;
}

int cz_huff_decode(cz_ctx *ctx, const void *d_in, size_t in_bytes, void *d_out, size_t out_cap, void *stream)
{
    if (!ctx || !d_in || in_bytes < HEAD || reinterpret_cast<uintptr_t>(d_in) % 16)
        return CZ_ERR_ARG;
    czh::DeviceGuard guard(ctx->device);
    hipStream_t st = static_cast<hipStream_t>(stream);
    uint8_t head[HEAD];
    if (hipMemcpyAsync(head, d_in, HEAD, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return CZ_ERR_HIP;
    uint32_t h32[8];
    std::memcpy(h32, head, 32);
    const uint64_t raw = h32[2] | ((uint64_t)h32[3] << 32);
    const uint64_t nchunks = h32[5];
    if (h32[0] != MAGIC || h32[1] != 1 || h32[4] != CHUNK || h32[6] != MAXLEN || h32[7] != 0 ||
        nchunks != (raw + CHUNK - 1) / CHUNK)
        return CZ_ERR_FORMAT;
    const size_t p0 = payload_start(nchunks);
    if (p0 > in_bytes)
        return CZ_ERR_FORMAT;
    if (raw > out_cap)
        return CZ_ERR_CAPACITY;
    if (raw == 0)
        return CZ_OK;
    if (!d_out || reinterpret_cast<uintptr_t>(d_out) % 4)
        return CZ_ERR_ARG;
    // the lengths must form a complete or single-code prefix code within the limit
    const uint8_t *lengths = head + 32;
    double kraft = 0;
    int nused = 0;
    for (int s = 0; s < 256; ++s) {
        if (lengths[s] > MAXLEN)
            return CZ_ERR_FORMAT;
        if (lengths[s]) {
            kraft += 1.0 / (double)(1u << lengths[s]);
            ++nused;
        }
    }
    if (nused == 0 || kraft > 1.0 || (nused > 1 && kraft < 1.0))
        return CZ_ERR_FORMAT;
    uint32_t code[256];
    canonical(lengths, code);
    std::vector<uint16_t> table(1u << MAXLEN, 0);
    for (int s = 0; s < 256; ++s) {
        const uint32_t l = code[s] >> 16, r = code[s] & 0xFFFFu;
        if (!l)
            continue;
        for (uint32_t k = 0; k < (1u << (MAXLEN - l)); ++k)
            table[r | (k << l)] = (uint16_t)(s | (l << 8));
    }
    int rc = ctx->huff_stage.upload(table.data(), table.size() * 2, st);
    if (rc != CZ_OK)
        return rc;
    const uint8_t *in = static_cast<const uint8_t *>(d_in);
    const uint8_t *payload = in + p0;
    const uint64_t pbytes = in_bytes - p0;
    const uint64_t *offs = reinterpret_cast<const uint64_t *>(in + HEAD);
    const uint16_t *tab = static_cast<const uint16_t *>(ctx->huff_stage.dev.ptr);
    uint8_t *dst = static_cast<uint8_t *>(d_out);
    if (nchunks >= DEC_WIDE_CHUNKS)
        hipLaunchKernelGGL(decode_kernel<4>, dim3((unsigned)((nchunks + 255) / 256)), dim3(256), 0, st, payload,
                           pbytes, offs, tab, nchunks, raw, dst, &ctx->work->status);
    else
        hipLaunchKernelGGL(decode_kernel<1>, dim3((unsigned)((nchunks + 63) / 64)), dim3(64), 0, st, payload,
                           pbytes, offs, tab, nchunks, raw, dst, &ctx->work->status);
    return hipGetLastError() == hipSuccess ? CZ_OK : CZ_ERR_HIP;
}

}  // extern "C"
