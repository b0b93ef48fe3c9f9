"""Oracle of the lossless-stage preconditioning -- TEST INFRASTRUCTURE ONLY.

Only the test suite and the benchmark's CPU leg may import this module; the
product library never does, and the two share no code.

What it computes (arXiv 1903.07761):
  * Sec. 2.3 ("Lossless compression" and "Wavelet types") and Sec. 4.1
    (Exp. 2): before the lossless coder, the aggregate output of the first
    substage may be byte-shuffled; the experiments shuffle at byte level with
    an element size of 4 bytes (single precision).  A byte shuffle with
    element size k sends byte j of element i to position j * n + i, where n is
    the number of whole elements; the bytes after the last whole element are
    kept in place at the end (the usual convention of shuffling codecs).
  * Same passages: Z4 / Z8 zero the 4 / 8 least significant bits of the
    wavelet detail coefficients.  Readings: the detail coefficients are the
    stored values outside the 4^3 coarse corner (the 64 coarse values are
    left untouched); zeroing is applied to the packed stream after
    decimation, so the keep decisions are those of the exact coefficients;
    at most the mantissa may be zeroed (23 bits float, 52 bits double).
"""
from __future__ import annotations

import struct

import numpy as np

_HDR = struct.Struct("<4s9I d Q Q")


def shuffle(buf: bytes, elem: int) -> bytes:
    """Byte shuffle: the k byte planes of the n whole elements, then the tail."""
    if elem < 1:
        raise ValueError("element size must be positive")
    n = len(buf) // elem
    body = np.frombuffer(buf, dtype=np.uint8, count=n * elem).reshape(n, elem)
    return body.T.tobytes() + bytes(buf[n * elem:])


def unshuffle(buf: bytes, elem: int) -> bytes:
    """Inverse of shuffle."""
    if elem < 1:
        raise ValueError("element size must be positive")
    n = len(buf) // elem
    planes = np.frombuffer(buf, dtype=np.uint8, count=n * elem).reshape(elem, n)
    return planes.T.tobytes() + bytes(buf[n * elem:])


def max_zero_bits(elem_bytes: int) -> int:
    return 23 if elem_bytes == 4 else 52


def zero_details(stream: bytes, bits: int) -> bytes:
    """Zero the `bits` least significant bits of every stored detail
    coefficient of a stream (values outside the 4^3 coarse corner), walking
    each record's mask in ascending q to find which stored value is which."""
    (magic, version, scheme, elem, N, levels, nx, ny, nz, reserved, eps, nblocks,
     payload) = _HDR.unpack_from(stream, 0)
    if not 0 <= bits <= max_zero_bits(elem):
        raise ValueError("bits out of range")
    out = bytearray(stream)
    if bits == 0:
        return bytes(out)
    p0 = (64 + 8 * (nblocks + 1) + 15) // 16 * 16
    off = struct.unpack_from(f"<{nblocks + 1}Q", stream, 64)
    uint = np.uint32 if elem == 4 else np.uint64
    keep_high = ~uint((1 << bits) - 1)
    n3 = N ** 3
    for b in range(nblocks):
        rec = p0 + off[b]
        nnz = struct.unpack_from("<I", stream, rec)[0]
        mask = np.unpackbits(np.frombuffer(stream, dtype=np.uint8, count=n3 // 8, offset=rec + 8),
                             bitorder="little")
        kept_q = np.nonzero(mask)[0]
        assert kept_q.size == nnz
        vstart = rec + 8 + n3 // 8
        vals = np.frombuffer(bytes(out[vstart:vstart + nnz * elem]), dtype=uint).copy()
        x, y, z = kept_q % N, (kept_q // N) % N, kept_q // (N * N)
        detail = ~((x < 4) & (y < 4) & (z < 4))
        vals[detail] &= keep_high
        out[vstart:vstart + nnz * elem] = vals.tobytes()
    return bytes(out)
