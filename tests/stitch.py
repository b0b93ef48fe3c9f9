"""Host-side assembly of one stream from pieces compressed apart, for tests.

Paper: arXiv 1903.07761, Sec. 2.2: every process compresses its own part of
the domain, the sizes of the compressed parts go through an exclusive prefix
scan, and each part is written at its prefix.  Here a part is a contiguous
range of blocks (a slab of whole block layers along z is one, since blocks
are numbered x fastest, then y, then z); its record offsets are rebased by
the exclusive scan of the parts' payload sizes and the payloads are
concatenated.  The layout arithmetic is that of the stream format (the
64-byte header, (nblocks + 1) u64 offsets, zero pad to 16 bytes, records).
"""
from __future__ import annotations

import numpy as np

import streamfmt as S


def _pack_header(h: S.Header, nz: int, nblocks: int, payload: int) -> bytes:
    return S.HDR.pack(h.magic, h.version, h.scheme, h.elem_bytes, h.block, h.levels, h.nx, h.ny, nz,
                      h.reserved, h.epsilon, nblocks, payload)


def exclusive_scan(sizes) -> np.ndarray:
    s = np.asarray(sizes, dtype=np.uint64)
    out = np.zeros(s.size + 1, dtype=np.uint64)
    np.cumsum(s, out=out[1:])
    return out


def stitch_slabs(parts: list[bytes]) -> bytes:
    """One stream from the streams of consecutive z-slabs of a field (same
    nx, ny, block, scheme, precision and epsilon; slab i above slab i - 1)."""
    hs = [S.header(p) for p in parts]
    h0 = hs[0]
    for h in hs[1:]:
        assert (h.nx, h.ny, h.block, h.scheme, h.elem_bytes, h.epsilon) == \
            (h0.nx, h0.ny, h0.block, h0.scheme, h0.elem_bytes, h0.epsilon)
    nb = sum(h.nblocks for h in hs)
    nz = sum(h.nz for h in hs)
    prefix = exclusive_scan([h.payload_bytes for h in hs])  # where each part's payload starts
    offs = [np.zeros(1, dtype=np.uint64)]
    for h, p, base in zip(hs, parts, prefix[:-1]):
        offs.append(S.offsets(p, h)[1:] + base)
    off = np.concatenate(offs)
    assert off.size == nb + 1
    p0 = (64 + 8 * (nb + 1) + 15) // 16 * 16
    out = bytearray(_pack_header(h0, nz, nb, int(prefix[-1])))
    out += off.astype("<u8").tobytes()
    out += bytes(p0 - len(out))
    for h, p in zip(hs, parts):
        out += p[h.payload_start:h.payload_start + h.payload_bytes]
    return bytes(out)


def stream_from_records(template: bytes, ranges: list[tuple[int, int, np.ndarray, np.ndarray]],
                        nz: int | None = None) -> bytes:
    """One stream from block ranges [b0, b1) whose records sit at fixed
    strides in `recs` with sizes `sizes` (the oracle's block-range entry
    point).  `template` is a stream of the same nx, ny, block, scheme,
    precision and epsilon (for example that of the field's first block
    layer); `nz` is the whole field's depth (default: the template's)."""
    h0 = S.header(template)
    nz = h0.nz if nz is None else nz
    ranges = sorted(ranges, key=lambda r: r[0])
    nb = ranges[-1][1]
    assert nb == (h0.nx // h0.block) * (h0.ny // h0.block) * (nz // h0.block)
    assert ranges[0][0] == 0
    for a, b in zip(ranges, ranges[1:]):
        assert a[1] == b[0], "block ranges must tile the field"
    sizes = np.concatenate([r[3] for r in ranges]).astype(np.uint64)
    off = exclusive_scan(sizes)
    p0 = (64 + 8 * (nb + 1) + 15) // 16 * 16
    out = bytearray(_pack_header(h0, nz, nb, int(off[-1])))
    out += off.astype("<u8").tobytes()
    out += bytes(p0 - len(out))
    for b0, b1, recs, sz in ranges:
        stride = recs.size // max(b1 - b0, 1)
        for k in range(b1 - b0):
            out += recs[k * stride:k * stride + int(sz[k])].tobytes()
    return bytes(out)


def split_slabs(stream: bytes, layers_per_part: int) -> list[bytes]:
    """The inverse of stitch_slabs: cut a stream into the streams of slabs of
    `layers_per_part` block layers along z (the last slab may be thinner),
    each with its offsets rebased to start at 0."""
    h = S.header(stream)
    N = h.block
    per_layer = (h.nx // N) * (h.ny // N)
    layers = h.nz // N
    off = S.offsets(stream, h)
    out = []
    for l0 in range(0, layers, layers_per_part):
        l1 = min(layers, l0 + layers_per_part)
        b0, b1 = l0 * per_layer, l1 * per_layer
        o = off[b0:b1 + 1] - off[b0]
        nb = b1 - b0
        p0 = (64 + 8 * (nb + 1) + 15) // 16 * 16
        part = bytearray(_pack_header(h, (l1 - l0) * N, nb, int(o[-1])))
        part += o.astype("<u8").tobytes()
        part += bytes(p0 - len(part))
        part += stream[h.payload_start + int(off[b0]):h.payload_start + int(off[b1])]
        out.append(bytes(part))
    return out
