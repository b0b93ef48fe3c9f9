"""Independent reader of the compressed stream, for tests.

Layout (little-endian): 64-byte header {magic "CZB1", u32 version, scheme,
elem_bytes, N, levels, nx, ny, nz, reserved; f64 epsilon; u64 nblocks,
payload_bytes}; (nblocks+1) u64 record offsets relative to the payload; zero
pad to 16 bytes; per block a record {u32 nnz, u32 flags, N^3/8 mask bytes with
bit q = bit (q & 7) of byte q >> 3, nnz values in ascending q, zero pad to 16}.
"""
from __future__ import annotations

import struct
from dataclasses import dataclass

import numpy as np

HDR = struct.Struct("<4s9I d Q Q")
assert HDR.size == 64


@dataclass
class Header:
    magic: bytes
    version: int
    scheme: int
    elem_bytes: int
    block: int
    levels: int
    nx: int
    ny: int
    nz: int
    reserved: int
    epsilon: float
    nblocks: int
    payload_bytes: int

    @property
    def payload_start(self) -> int:
        return (64 + 8 * (self.nblocks + 1) + 15) // 16 * 16

    @property
    def dtype(self):
        return np.float32 if self.elem_bytes == 4 else np.float64


def header(stream: bytes) -> Header:
    return Header(*HDR.unpack_from(stream, 0))


def offsets(stream: bytes, h: Header | None = None) -> np.ndarray:
    h = h or header(stream)
    return np.frombuffer(stream, dtype="<u8", count=h.nblocks + 1, offset=64)


@dataclass
class Record:
    nnz: int
    flags: int
    mask: np.ndarray  # bool[N^3], q order
    values: np.ndarray  # kept values, ascending q
    raw: bytes  # the full record bytes, padding included


def record(stream: bytes, b: int, h: Header | None = None) -> Record:
    h = h or header(stream)
    off = offsets(stream, h)
    start = h.payload_start + int(off[b])
    end = h.payload_start + int(off[b + 1])
    raw = stream[start:end]
    n3 = h.block ** 3
    nnz, flags = struct.unpack_from("<II", raw, 0)
    mbytes = np.frombuffer(raw, dtype=np.uint8, count=n3 // 8, offset=8)
    mask = np.unpackbits(mbytes, bitorder="little").astype(bool)
    vals = np.frombuffer(raw, dtype=h.dtype, count=nnz, offset=8 + n3 // 8)
    return Record(nnz, flags, mask, vals, raw)


def coefficients(stream: bytes, b: int, h: Header | None = None) -> np.ndarray:
    """Dense decimated coefficient block [z, y, x] of record b (dropped = +0)."""
    h = h or header(stream)
    r = record(stream, b, h)
    c = np.zeros(h.block ** 3, dtype=h.dtype)
    c[r.mask] = r.values
    return c.reshape(h.block, h.block, h.block)


def validate(stream: bytes) -> Header:
    """Check every structural invariant of a stream; raise AssertionError."""
    h = header(stream)
    assert h.magic == b"CZB1" and h.version == 1 and h.reserved == 0
    assert h.scheme in (0, 1, 2) and h.elem_bytes in (4, 8)
    assert h.block in (8, 16, 32, 64) and h.levels == h.block.bit_length() - 3
    N = h.block
    assert h.nx % N == 0 and h.ny % N == 0 and h.nz % N == 0
    assert h.nblocks == (h.nx // N) * (h.ny // N) * (h.nz // N)
    p0 = h.payload_start
    assert len(stream) == p0 + h.payload_bytes, (len(stream), p0, h.payload_bytes)
    assert stream[64 + 8 * (h.nblocks + 1):p0] == bytes(p0 - 64 - 8 * (h.nblocks + 1))
    off = offsets(stream, h)
    assert off[0] == 0 and int(off[-1]) == h.payload_bytes
    n3 = N ** 3
    corner = np.zeros((N, N, N), dtype=bool)
    corner[:4, :4, :4] = True
    corner = corner.reshape(-1)
    for b in range(h.nblocks):
        r = record(stream, b, h)
        used = 8 + n3 // 8 + r.nnz * h.elem_bytes
        assert int(off[b + 1] - off[b]) == (used + 15) // 16 * 16
        assert r.flags == 0
        assert int(r.mask.sum()) == r.nnz
        assert r.mask[corner].all()
        assert r.raw[used:] == bytes(len(r.raw) - used)
    return h
