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
// 16 KiB of input is padded to whole words.  Container: 32-byte header
// {"CZH1", version 1, u64 raw bytes, u32 chunk bytes, u32 chunks, u32 max
// length, u32 0}, 256 code lengths, (chunks + 1) u64 chunk offsets relative to
// the payload, zero pad to 16 bytes, the chunks.
//
// Encoding: a histogram kernel, the code built on the host from the 256
// counts, a kernel for each chunk's encoded size, a one-workgroup scan that
// writes the offsets, and an encoding kernel (one workgroup a chunk, codes
// packed with LDS atomics, the chunk copied out whole).  Decoding: one thread
// a chunk with a 4096-entry lookup table in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "cz_host.h"

namespace {

constexpr uint32_t MAGIC = 0x31485A43u;  // "CZH1"
constexpr int MAXLEN = 12;
constexpr uint32_t CHUNK = 16384;
constexpr int ENC_THREADS = 256;
constexpr int BYTES_PER_THREAD = CHUNK / ENC_THREADS;
constexpr uint32_t CHUNK_WORDS = (CHUNK * MAXLEN + 31) / 32;
constexpr size_t HEAD = 32 + 256;

size_t payload_start(uint64_t nchunks) { return (HEAD + 8 * (nchunks + 1) + 15) & ~size_t(15); }

__global__ __launch_bounds__(256) void hist_kernel(const uint8_t *__restrict__ in, uint64_t n,
                                                   unsigned long long *hist)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256)
        atomicAdd(&h[in[i]], 1u);
    __syncthreads();
    if (h[threadIdx.x])
        atomicAdd(&hist[threadIdx.x], (unsigned long long)h[threadIdx.x]);
}

// Encoded bits of each chunk.
__global__ __launch_bounds__(ENC_THREADS) void chunk_bits_kernel(const uint8_t *__restrict__ in, uint64_t n,
                                                                 const uint32_t *__restrict__ code,
                                                                 uint32_t *bits)
{
    __shared__ uint32_t s_len[256];
    __shared__ uint32_t s_sum[ENC_THREADS / 64];
    s_len[threadIdx.x] = code[threadIdx.x] >> 16;
    __syncthreads();
    const uint64_t c = blockIdx.x;
    const uint64_t base = c * CHUNK;
    const uint64_t end = min(n, base + CHUNK);
    uint32_t sum = 0;
    for (uint64_t i = base + threadIdx.x; i < end; i += ENC_THREADS)
        sum += s_len[in[i]];
    for (int o = 32; o > 0; o >>= 1)
        sum += __shfl_xor(sum, o);
    if (threadIdx.x % 64 == 0)
        s_sum[threadIdx.x / 64] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < ENC_THREADS / 64; ++w)
            t += s_sum[w];
        bits[c] = t;
    }
}

// Chunk offsets (bytes, whole words) into the container, and the payload size.
__global__ __launch_bounds__(1024) void scan_kernel(const uint32_t *__restrict__ bits, uint64_t nchunks,
                                                    uint64_t *offs, uint64_t *total)
{
    __shared__ uint64_t s_part[1024];
    const uint64_t per = (nchunks + 1023) / 1024;
    const uint64_t b0 = threadIdx.x * per, b1 = min(nchunks, b0 + per);
    uint64_t sum = 0;
    for (uint64_t c = b0; c < b1; ++c)
        sum += (uint64_t)((bits[c] + 31) / 32) * 4;
    s_part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t run = 0;
        for (int t = 0; t < 1024; ++t) {
            const uint64_t v = s_part[t];
            s_part[t] = run;
            run += v;
        }
        *total = run;
        offs[nchunks] = run;
    }
    __syncthreads();
    uint64_t run = s_part[threadIdx.x];
    for (uint64_t c = b0; c < b1; ++c) {
        offs[c] = run;
        run += (uint64_t)((bits[c] + 31) / 32) * 4;
    }
}

__global__ __launch_bounds__(ENC_THREADS) void encode_kernel(const uint8_t *__restrict__ in, uint64_t n,
                                                             const uint32_t *__restrict__ code,
                                                             const uint64_t *__restrict__ offs, uint8_t *payload)
{
    __shared__ uint32_t s_code[256];
    __shared__ uint32_t s_words[CHUNK_WORDS];
    __shared__ uint32_t s_scan[ENC_THREADS / 64 + 1];
    s_code[threadIdx.x] = code[threadIdx.x];
    for (uint32_t w = threadIdx.x; w < CHUNK_WORDS; w += ENC_THREADS)
        s_words[w] = 0;
    __syncthreads();
    const uint64_t c = blockIdx.x;
    const uint64_t base = c * CHUNK + (uint64_t)threadIdx.x * BYTES_PER_THREAD;
    const int cnt = (int)min<uint64_t>(BYTES_PER_THREAD, base < n ? n - base : 0);
    uint32_t mybits = 0;
    for (int i = 0; i < cnt; ++i)
        mybits += s_code[in[base + i]] >> 16;
    // exclusive scan of the threads' bit counts
    const uint32_t lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    uint32_t incl = mybits;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(incl, o);
        if (lane >= (uint32_t)o)
            incl += v;
    }
    if (lane == 63)
        s_scan[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < ENC_THREADS / 64; ++w) {
            const uint32_t v = s_scan[w];
            s_scan[w] = run;
            run += v;
        }
        s_scan[ENC_THREADS / 64] = run;
    }
    __syncthreads();
    uint32_t pos = s_scan[wave] + incl - mybits;
    for (int i = 0; i < cnt; ++i) {
        const uint32_t e = s_code[in[base + i]];
        const uint32_t l = e >> 16, r = e & 0xFFFFu;
        const uint32_t w = pos / 32, sh = pos % 32;
        atomicOr(&s_words[w], r << sh);
        if (sh + l > 32)
            atomicOr(&s_words[w + 1], r >> (32 - sh));
        pos += l;
    }
    __syncthreads();
    const uint32_t words = (s_scan[ENC_THREADS / 64] + 31) / 32;
    uint32_t *dst = reinterpret_cast<uint32_t *>(payload + offs[c]);
    for (uint32_t w = threadIdx.x; w < words; w += ENC_THREADS)
        dst[w] = s_words[w];
}

// One thread a chunk; table[k] = symbol | length << 8 for the next 12 bits k.
__global__ __launch_bounds__(64) void decode_kernel(const uint8_t *__restrict__ payload, uint64_t payload_bytes,
                                                    const uint64_t *__restrict__ offs, const uint16_t *__restrict__ table,
                                                    uint64_t nchunks, uint64_t raw, uint8_t *out, uint32_t *status)
{
    __shared__ uint16_t s_tab[1u << MAXLEN];
    for (uint32_t k = threadIdx.x; k < (1u << MAXLEN); k += 64)
        s_tab[k] = table[k];
    __syncthreads();
    const uint64_t c = (uint64_t)blockIdx.x * 64 + threadIdx.x;
    if (c >= nchunks)
        return;
    const uint64_t o0 = offs[c], o1 = offs[c + 1];
    if (o1 < o0 || o1 > payload_bytes || (o0 | o1) % 4) {
        atomicOr(status, czk::STATUS_FORMAT);
        return;
    }
    const uint32_t *w = reinterpret_cast<const uint32_t *>(payload + o0);
    const uint64_t nwords = (o1 - o0) / 4;
    const uint64_t start = c * CHUNK;
    const uint32_t n = (uint32_t)min<uint64_t>(CHUNK, raw - start);
    uint64_t window = 0;  // the next bits, lowest first
    uint32_t avail = 0;
    uint64_t next = 0, used = 0;
    uint32_t pack = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (avail < MAXLEN) {
            const uint64_t v = next < nwords ? w[next] : 0u;  // zeros past the chunk's words
            ++next;
            window |= v << avail;
            avail += 32;
        }
        const uint16_t e = s_tab[window & ((1u << MAXLEN) - 1)];
        const uint32_t l = e >> 8;
        used += l;
        if (l == 0 || used > nwords * 32) {  // no such code, or the chunk's bits ran out
            atomicOr(status, czk::STATUS_FORMAT);
            return;
        }
        window >>= l;
        avail -= l;
        pack |= (uint32_t)(e & 0xFF) << (8 * (i % 4));
        if (i % 4 == 3 || i + 1 == n) {
            if (i % 4 == 3)
                *reinterpret_cast<uint32_t *>(out + start + i - 3) = pack;
            else
                for (uint32_t k = 0; k <= i % 4; ++k)
                    out[start + i - i % 4 + k] = (uint8_t)(pack >> (8 * k));
            pack = 0;
        }
    }
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
    struct Item {
        uint64_t w;
        std::vector<uint16_t> mult;  // per leaf position
    };
    std::vector<Item> leaves(n);
    for (int i = 0; i < n; ++i) {
        leaves[i].w = counts[used[i]];
        leaves[i].mult.assign(n, 0);
        leaves[i].mult[i] = 1;
    }
    std::vector<Item> cur = leaves;
    for (int round = 0; round < MAXLEN - 1; ++round) {
        std::vector<Item> packages;
        for (size_t i = 0; i + 1 < cur.size(); i += 2) {
            Item p;
            p.w = cur[i].w + cur[i + 1].w;
            p.mult = cur[i].mult;
            for (int k = 0; k < n; ++k)
                p.mult[k] += cur[i + 1].mult[k];
            packages.push_back(std::move(p));
        }
        std::vector<Item> out;
        size_t i = 0, j = 0;
        while (i < leaves.size() || j < packages.size()) {
            if (j >= packages.size() || (i < leaves.size() && leaves[i].w <= packages[j].w))
                out.push_back(leaves[i++]);
            else
                out.push_back(std::move(packages[j++]));
        }
        cur = std::move(out);
    }
    std::vector<int> len(n, 0);
    for (int i = 0; i < 2 * n - 2; ++i)
        for (int k = 0; k < n; ++k)
            len[k] += cur[i].mult[k];
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
    // workspace: histogram (256 u64), code table (256 u32), chunk bits, payload size
    const size_t bits_bytes = (nchunks * 4 + 7) & ~uint64_t(7);
    const size_t ws = 256 * 8 + 256 * 4 + bits_bytes + 8;
    int rc = ctx->huff.ensure(ws);
    if (rc != CZ_OK)
        return rc;
    uint8_t *w = static_cast<uint8_t *>(ctx->huff.ptr);
    unsigned long long *hist = reinterpret_cast<unsigned long long *>(w);
    uint32_t *code = reinterpret_cast<uint32_t *>(w + 2048);
    uint32_t *bits = reinterpret_cast<uint32_t *>(w + 3072);
    uint64_t *total = reinterpret_cast<uint64_t *>(w + 3072 + bits_bytes);
    uint64_t counts[256] = {0};
    if (hipMemsetAsync(hist, 0, 2048, st) != hipSuccess)
        return CZ_ERR_HIP;
    if (nbytes) {
        const int g = (int)std::min<uint64_t>((nbytes + 255) / 256, 8192);
        hipLaunchKernelGGL(hist_kernel, dim3(g), dim3(256), 0, st, in, (uint64_t)nbytes, hist);
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
    // header + code table through pinned staging; the pad between offsets and payload zeroed
    std::vector<uint8_t> stage(HEAD + 1024);
    std::memcpy(stage.data(), head, HEAD);
    std::memcpy(stage.data() + HEAD, table, 1024);
    if ((rc = ctx->huff_stage.upload(stage.data(), stage.size(), st)) != CZ_OK)
        return rc;
    const uint8_t *staged = static_cast<const uint8_t *>(ctx->huff_stage.dev.ptr);
    if (hipMemcpyAsync(out, staged, HEAD, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(code, staged + HEAD, 1024, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemsetAsync(out + HEAD + 8 * (nchunks + 1), 0, p0 - (HEAD + 8 * (nchunks + 1)), st) != hipSuccess)
        return CZ_ERR_HIP;
    uint64_t *offs = reinterpret_cast<uint64_t *>(out + HEAD);
    if (nchunks) {
        hipLaunchKernelGGL(chunk_bits_kernel, dim3((unsigned)nchunks), dim3(ENC_THREADS), 0, st, in, (uint64_t)nbytes,
                           code, bits);
        hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, st, bits, nchunks, offs, total);
        hipLaunchKernelGGL(encode_kernel, dim3((unsigned)nchunks), dim3(ENC_THREADS), 0, st, in, (uint64_t)nbytes,
                           code, offs, out + p0);
        if (hipGetLastError() != hipSuccess)
            return CZ_ERR_HIP;
    } else if (hipMemsetAsync(offs, 0, 8, st) != hipSuccess || hipMemsetAsync(total, 0, 8, st) != hipSuccess) {
        return CZ_ERR_HIP;
    }
    uint64_t payload = 0;
    if (hipMemcpyAsync(&payload, total, 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return CZ_ERR_HIP;
    *h_out_bytes = p0 + payload;
    return CZ_OK;
}

int cz_huff_decode(cz_ctx *ctx, const void *d_in, size_t in_bytes, void *d_out, size_t out_cap, void *stream)
{
    if (!ctx || !d_in || in_bytes < HEAD || reinterpret_cast<uintptr_t>(d_in) % 8)
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
    const unsigned g = (unsigned)((nchunks + 63) / 64);
    hipLaunchKernelGGL(decode_kernel, dim3(g), dim3(64), 0, st, in + p0, (uint64_t)(in_bytes - p0),
                       reinterpret_cast<const uint64_t *>(in + HEAD),
                       static_cast<const uint16_t *>(ctx->huff_stage.dev.ptr), nchunks, raw,
                       static_cast<uint8_t *>(d_out), &ctx->work->status);
    return hipGetLastError() == hipSuccess ? CZ_OK : CZ_ERR_HIP;
}

}  // extern "C"
