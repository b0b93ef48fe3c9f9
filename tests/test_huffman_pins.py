"""Pins of the lossless-stage oracle (length-limited canonical Huffman):
brute force over all length vectors for small alphabets, the worked example
of RFC 1951, the Kraft equality, and round trips."""
import itertools
import struct

import numpy as np
import pytest

from oracle import huffman as H


def brute_force_cost(counts, max_len):
    """Minimum sum of count * length over length vectors satisfying Kraft."""
    used = [c for c in counts if c > 0]
    best = None
    for ls in itertools.product(range(1, max_len + 1), repeat=len(used)):
        if sum(2.0 ** -l for l in ls) <= 1.0:
            cost = sum(c * l for c, l in zip(used, ls))
            best = cost if best is None else min(best, cost)
    return best


@pytest.mark.parametrize("counts,max_len", [
    ([1, 1, 2, 3, 5, 8, 13], 6), ([1, 1, 2, 3, 5, 8, 13], 4), ([1, 1, 2, 3, 5, 8, 13], 3),
    ([5, 5, 5, 5], 2), ([100, 1, 1, 1, 1], 3), ([7, 3, 3, 1, 1, 1], 4), ([2, 9, 4, 4, 1, 1, 6], 3)])
def test_package_merge_is_optimal(counts, max_len):
    lengths = H.package_merge(counts + [0] * (256 - len(counts)), max_len)[:len(counts)]
    assert max(lengths) <= max_len
    assert sum(2.0 ** -l for l in lengths) == 1.0  # a complete prefix code
    assert sum(c * l for c, l in zip(counts, lengths)) == brute_force_cost(counts, max_len)


def test_package_merge_unlimited_matches_huffman_example():
    # Fibonacci weights: Huffman's tree is a chain, lengths 6,6,5,4,3,2,1
    lengths = H.package_merge([1, 1, 2, 3, 5, 8, 13] + [0] * 249, 12)[:7]
    assert lengths == [6, 6, 5, 4, 3, 2, 1]


def test_canonical_codes_rfc1951_example():
    # RFC 1951 Sec. 3.2.2: lengths (3,3,3,3,3,2,4,4) for A..H
    codes = H.canonical_codes([3, 3, 3, 3, 3, 2, 4, 4])
    assert codes == [(0b010, 3), (0b011, 3), (0b100, 3), (0b101, 3), (0b110, 3), (0b00, 2), (0b1110, 4), (0b1111, 4)]


def test_degenerate_alphabets():
    assert H.package_merge([0] * 256) == [0] * 256
    one = H.package_merge([0] * 7 + [42] + [0] * 248)
    assert one[7] == 1 and sum(one) == 1


def test_bit_order_worked_example():
    # two symbols, lengths 1 each: codes 0 and 1; "\x01\x00\x01" -> bits 1,0,1 LSB first = 0b101
    blob = H.encode(b"\x01\x00\x01")
    magic, version, raw, chunk, nchunks, max_len, _ = struct.unpack_from("<4sIQIIII", blob, 0)
    assert (magic, raw, nchunks) == (b"CZH1", 3, 1)
    p0 = 288 + 16
    assert struct.unpack_from("<I", blob, p0)[0] == 0b101
    assert H.decode(blob) == b"\x01\x00\x01"


@pytest.mark.parametrize("n", [0, 1, 100, H.CHUNK, H.CHUNK + 1, 3 * H.CHUNK + 77])
def test_roundtrip_and_size(n):
    rng = np.random.default_rng(n)
    data = (rng.geometric(0.3, n) % 256).astype(np.uint8).tobytes()  # skewed bytes
    blob = H.encode(data)
    assert H.decode(blob) == data
    if n:
        counts = np.bincount(np.frombuffer(data, dtype=np.uint8), minlength=256)
        lengths = list(blob[32:288])
        bits = int(sum(int(c) * l for c, l in zip(counts, lengths)))
        nchunks = (n + H.CHUNK - 1) // H.CHUNK
        payload = len(blob) - (288 + 8 * (nchunks + 1) + (-(288 + 8 * (nchunks + 1)) % 16))
        assert bits <= payload * 8 < bits + 32 * nchunks  # whole words per chunk
