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
// a chunk with a 4096-entry lookup table in LDS, the chunk's words read
// ahead in 16-byte blocks (two loop shapes, by the stream's mean code length).
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

// One thread a chunk; table[k] = symbol | length << 8 for the next 12 bits k.
// The chunk's words come from 16-byte blocks of the payload, read ahead.
// Blocks may extend past the chunk's words (into the next chunk, or zeros
// past the payload): a prefix code decides each symbol by its own bits, and
// the bits the chunk's symbols use must lie within its words.  Two loop
// shapes, chosen per stream by its mean code length:
//   * GROUPED (mean >= 4 bits): groups of GB blocks, the next group in
//     flight; each word enters a 64-bit window and the window is emptied
//     symbol by symbol.  With long codes every lane takes about as many
//     symbols per word, so the lanes stay together.
//   * FLAT (short codes, skewed streams): every iteration decodes one symbol
//     on every lane, refilling a lane's window from the next word when it
//     holds fewer than 12 bits; a lane whose words are mostly 1-bit codes no
//     longer holds back the others word by word.
constexpr int DEC_THREADS = 64;  // small workgroups: a short stream has few chunks
constexpr int GB = 4;            // 16-byte blocks a group

template <bool FLAT>
__global__ __launch_bounds__(DEC_THREADS) void decode_kernel(const uint8_t *__restrict__ payload,
                                                             uint64_t payload_bytes,
                                                             const uint64_t *__restrict__ offs,
                                                             const uint16_t *__restrict__ table, uint64_t nchunks,
                                                             uint64_t raw, uint8_t *out, uint32_t *status)
{
    __shared__ uint16_t s_tab[1u << MAXLEN];
    for (uint32_t k = threadIdx.x; k < (1u << MAXLEN); k += DEC_THREADS)
        s_tab[k] = table[k];
    __syncthreads();
    const uint64_t c = (uint64_t)blockIdx.x * DEC_THREADS + threadIdx.x;
    if (c >= nchunks)
        return;
    const uint64_t o0 = offs[c], o1 = offs[c + 1];
    if (o1 < o0 || o1 > payload_bytes || (o0 | o1) % 4) {
        atomicOr(status, czk::STATUS_FORMAT);
        return;
    }
    const uint64_t start = c * CHUNK;
    const uint32_t n = (uint32_t)min<uint64_t>(CHUNK, raw - start);  // >= 1 for c < nchunks
    if (o1 == o0) {
        atomicOr(status, czk::STATUS_FORMAT);  // symbols but no bits
        return;
    }
    const uint32_t nbits = (uint32_t)min<uint64_t>((o1 - o0) * 8, 1u << 31);  // a chunk needs < 2^16
    const uint4 *pb = reinterpret_cast<const uint4 *>(payload);  // 16-byte aligned
    const uint32_t *pw = reinterpret_cast<const uint32_t *>(payload);
    const uint64_t nblk = payload_bytes / 16, nwords = payload_bytes / 4;
    auto block = [&](uint64_t bi) -> uint4 {
        if (bi < nblk)
            return pb[bi];
        uint4 v{0u, 0u, 0u, 0u};  // the payload's partial last block, zeros past its end
        const uint64_t w = bi * 4;
        if (w < nwords)
            v.x = pw[w];
        if (w + 1 < nwords)
            v.y = pw[w + 1];
        if (w + 2 < nwords)
            v.z = pw[w + 2];
        return v;
    };
    uint64_t window = 0;
    uint32_t avail = 0, used = 0, pack = 0, i = 0;
    uint32_t *o32 = reinterpret_cast<uint32_t *>(out + start);
    // decode one symbol from the window (at least MAXLEN bits in it); false on a bad code
    auto one = [&]() -> bool {
        const uint16_t e = s_tab[window & ((1u << MAXLEN) - 1)];
        const uint32_t l = e >> 8;
        used += l;
        if (l == 0 || used > nbits)  // no such code, or past the chunk's bits
            return false;
        window >>= l;
        avail -= l;
        pack |= (uint32_t)(e & 0xFF) << (8 * (i % 4));
        if (i % 4 == 3) {
            o32[i / 4] = pack;
            pack = 0;
        }
        ++i;
        return true;
    };
    if constexpr (FLAT) {
        uint64_t bi = o0 / 16;
        uint32_t wi = (uint32_t)(o0 / 4) % 4;  // next word of cur
        uint4 cur = block(bi), n1 = block(bi + 1), n2 = block(bi + 2);
        while (i < n) {
            if (avail < (uint32_t)MAXLEN) {
                const uint32_t w = wi == 0 ? cur.x : wi == 1 ? cur.y : wi == 2 ? cur.z : cur.w;
                window |= (uint64_t)w << avail;
                avail += 32;
                if (++wi == 4) {
                    wi = 0;
                    cur = n1;
                    n1 = n2;
                    n2 = block(++bi + 2);
                }
            }
            if (!one()) {
                atomicOr(status, czk::STATUS_FORMAT);
                return;
            }
        }
    } else {
        const uint64_t b0 = o0 / 16;     // block holding the chunk's first word
        int skip = (int)((o0 / 4) % 4);  // words of that block before the chunk
        uint4 cur[GB], nxt[GB];
#pragma unroll
        for (int k = 0; k < GB; ++k)
            cur[k] = block(b0 + k);
#pragma unroll
        for (int k = 0; k < GB; ++k)
            nxt[k] = block(b0 + GB + k);
        uint64_t g = 0;
        while (i < n) {
#pragma unroll
            for (int k = 0; k < 4 * GB; ++k) {
                if (k < skip)
                    continue;
                if (i >= n)
                    break;
                const uint4 v = cur[k / 4];
                const uint32_t w = k % 4 == 0 ? v.x : k % 4 == 1 ? v.y : k % 4 == 2 ? v.z : v.w;
                window |= (uint64_t)w << avail;  // avail < MAXLEN here
                avail += 32;
                while (avail >= (uint32_t)MAXLEN && i < n) {
                    if (!one()) {
                        atomicOr(status, czk::STATUS_FORMAT);
                        return;
                    }
                }
            }
            skip = 0;
            // the next group becomes current; the one after it is requested
            ++g;
#pragma unroll
            for (int k = 0; k < GB; ++k)
                cur[k] = nxt[k];
#pragma unroll
            for (int k = 0; k < GB; ++k)
                nxt[k] = block(b0 + (g + 1) * GB + k);
        }
    }
    if (n % 4)
        for (uint32_t k = 0; k < n % 4; ++k)
            out[start + n - n % 4 + k] = (uint8_t)(pack >> (8 * k));
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
        hipLaunchKernelGGL(encode_kernel, dim3((unsigned)ngroups), dim3(ENC_THREADS), 0, st, in, (uint64_t)nbytes,
                           code, nchunks, reinterpret_cast<uint64_t *>(w + W_FLAGS),
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
    // mean code length from the payload size: short codes take the flat loop
    const dim3 grid((unsigned)((nchunks + DEC_THREADS - 1) / DEC_THREADS)), threads(DEC_THREADS);
    if (pbytes * 8 < 4 * raw)
        hipLaunchKernelGGL(decode_kernel<true>, grid, threads, 0, st, payload, pbytes, offs, tab, nchunks, raw, dst,
                           &ctx->work->status);
    else
        hipLaunchKernelGGL(decode_kernel<false>, grid, threads, 0, st, payload, pbytes, offs, tab, nchunks, raw, dst,
                           &ctx->work->status);
    return hipGetLastError() == hipSuccess ? CZ_OK : CZ_ERR_HIP;
}

}  // extern "C"
