"""Oracle of the GPU lossless stage -- TEST INFRASTRUCTURE ONLY.

Only the test suite and the benchmark's CPU leg may import this module; the
product library never does, and the two share no code.

The paper's second substage is a general-purpose lossless coder applied to
the (optionally shuffled) output of the wavelet stage (Sec. 2.2-2.3).  The
GPU stage built here is a byte-oriented canonical Huffman coder whose stream
is cut into independently decodable chunks, so that decoding, like the
paper's block-level decompression, can start anywhere.  Definitions:

  * code lengths: optimal lengths under a maximum length L (= 12), computed
    with the package-merge algorithm of Larmore and Hirschberg (1990):
    leaves sorted by (count, symbol); at each of the L - 1 merge steps the
    previous list is paired in order into packages, and packages and leaves
    are merged by weight, a leaf before a package of equal weight; the first
    2 n - 2 items of the final list give every symbol its length (the number
    of items containing it).  One used symbol gets length 1; none: no code.
  * codes: canonical, as in RFC 1951 (Sec. 3.2.2): codes of equal length are
    consecutive in symbol order, shorter codes first.
  * bits: each code is written bit-reversed, least significant bit first,
    into little-endian 32-bit words (the first code bit is the lowest bit of
    the first word); each chunk's bits are padded with zeros to a whole word.
  * container: header {char[4] "CZH1", u32 version 1, u64 raw bytes,
    u32 chunk bytes, u32 chunks, u32 max length, u32 0}, 256 code lengths
    (u8), (chunks + 1) u64 chunk offsets relative to the payload (offset 0 =
    0), zero pad to 16 bytes, then the chunks' words.
"""
from __future__ import annotations

import struct

import numpy as np

MAGIC = b"CZH1"
MAX_LEN = 12
CHUNK = 4096
_HDR = struct.Struct("<4sIQIIII")  # 32 bytes


def package_merge(counts, max_len: int = MAX_LEN):
    """Length-limited optimal code lengths for the 256 byte counts."""
    counts = [int(c) for c in counts]
    used = [s for s in range(len(counts)) if counts[s] > 0]
    lengths = [0] * len(counts)
    if not used:
        return lengths
    if len(used) == 1:
        lengths[used[0]] = 1
        return lengths
    n = len(used)
    if n > (1 << max_len):
        raise ValueError("too many symbols for the length limit")
    leaves = sorted(used, key=lambda s: (counts[s], s))
    # an item: (weight, tuple of per-leaf multiplicities as a dict symbol -> count, is_leaf)
    leaf_items = [(counts[s], {s: 1}, True) for s in leaves]
    cur = list(leaf_items)
    for _ in range(max_len - 1):
        packages = []
        for i in range(0, len(cur) - 1, 2):
            a, b = cur[i], cur[i + 1]
            merged = dict(a[1])
            for k, v in b[1].items():
                merged[k] = merged.get(k, 0) + v
            packages.append((a[0] + b[0], merged, False))
        # merge two lists sorted by weight; a leaf precedes a package of equal weight
        out, i, j = [], 0, 0
        while i < len(leaf_items) or j < len(packages):
            if j >= len(packages) or (i < len(leaf_items) and leaf_items[i][0] <= packages[j][0]):
                out.append(leaf_items[i])
                i += 1
            else:
                out.append(packages[j])
                j += 1
        cur = out
    for item in cur[: 2 * n - 2]:
        for s, k in item[1].items():
            lengths[s] += k
    return lengths


def canonical_codes(lengths):
    """RFC 1951 canonical codes: list of (code, length) per symbol."""
    max_len = max(lengths) if any(lengths) else 0
    bl_count = [0] * (max_len + 1)
    for l in lengths:
        if l:
            bl_count[l] += 1
    next_code = [0] * (max_len + 2)
    code = 0
    for bits in range(1, max_len + 1):
        code = (code + bl_count[bits - 1]) << 1 if bits > 1 else 0
        next_code[bits] = code
    out = [(0, 0)] * len(lengths)
    for s, l in enumerate(lengths):
        if l:
            out[s] = (next_code[l], l)
            next_code[l] += 1
    return out


def _reverse(code: int, length: int) -> int:
    r = 0
    for _ in range(length):
        r = (r << 1) | (code & 1)
        code >>= 1
    return r


def encode_chunk(data: bytes, codes) -> bytes:
    acc, nbits, words = 0, 0, []
    for b in data:
        c, l = codes[b]
        acc |= _reverse(c, l) << nbits
        nbits += l
        while nbits >= 32:
            words.append(acc & 0xFFFFFFFF)
            acc >>= 32
            nbits -= 32
    if nbits:
        words.append(acc & 0xFFFFFFFF)
    return struct.pack(f"<{len(words)}I", *words)


def encode(data: bytes, chunk: int = CHUNK, max_len: int = MAX_LEN) -> bytes:
    counts = np.bincount(np.frombuffer(data, dtype=np.uint8), minlength=256) if data else np.zeros(256, np.int64)
    lengths = package_merge(counts, max_len)
    codes = canonical_codes(lengths)
    nchunks = (len(data) + chunk - 1) // chunk
    payload = [encode_chunk(data[k * chunk:(k + 1) * chunk], codes) for k in range(nchunks)]
    offs = [0]
    for p in payload:
        offs.append(offs[-1] + len(p))
    head = _HDR.pack(MAGIC, 1, len(data), chunk, nchunks, max_len, 0) + bytes(lengths)
    head += struct.pack(f"<{nchunks + 1}Q", *offs)
    head += bytes((-len(head)) % 16)
    return head + b"".join(payload)


def decode(blob: bytes) -> bytes:
    magic, version, raw, chunk, nchunks, max_len, _ = _HDR.unpack_from(blob, 0)
    if magic != MAGIC or version != 1:
        raise ValueError("not a CZH1 container")
    lengths = list(blob[32:32 + 256])
    offs = struct.unpack_from(f"<{nchunks + 1}Q", blob, 288)
    p0 = 288 + 8 * (nchunks + 1)
    p0 += (-p0) % 16
    codes = canonical_codes(lengths)
    table = {(_reverse(c, l), l): s for s, (c, l) in enumerate(codes) if l}
    out = bytearray()
    for k in range(nchunks):
        n = min(chunk, raw - k * chunk)
        words = list(struct.unpack_from(f"<{(offs[k + 1] - offs[k]) // 4}I", blob, p0 + offs[k])) + [0, 0]
        pos = 0
        for _ in range(n):
            w = pos // 32
            window = (words[w] | (words[w + 1] << 32)) >> (pos % 32)  # the next bits, lowest first
            for l in range(1, max_len + 1):
                key = window & ((1 << l) - 1)
                if (key, l) in table:
                    out.append(table[(key, l)])
                    pos += l
                    break
            else:
                raise ValueError("invalid code")
    return bytes(out)
