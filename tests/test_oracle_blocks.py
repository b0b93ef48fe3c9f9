"""Pins of the oracle's block-range entry points against its whole-field ones.

Paper: arXiv 1903.07761, Sec. 2.1 and 2.3: blocks are compressed
independently (filters on the interval need no neighbour data), so the
record of a block does not depend on which other blocks are compressed in
the same call, and a block decodes from its record alone.  The block-range
entry points (used to time a bounded sample of a large field, and to split a
field across workers) must therefore produce exactly the records of the
whole-field call for the same blocks, and decode exactly the same blocks.
"""
import numpy as np
import pytest

import streamfmt as S
from stitch import stream_from_records

SCHEMES = ["W4", "W4_li", "W3_ai"]


def field_of(shape, dt, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    smooth = np.sin(0.2 * x) * np.cos(0.15 * y) + 0.01 * z
    return (smooth + 0.05 * rng.standard_normal(shape)).astype(dt)


CASES = [
    (8, (16, 24, 40)),   # 30 blocks, a ragged grid
    (16, (32, 48, 16)),  # 6 blocks
    (32, (64, 32, 96)),  # 6 blocks
]


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("N,shape", CASES)
def test_compress_blocks_records_equal_whole_field(oracle, N, shape, scheme, dt):
    f = field_of(shape, dt, 101 + N)
    eps = 2e-2 * float(f.max() - f.min())
    whole = oracle.compress(f, N, scheme, eps)
    h = S.header(whole)
    nb = h.nblocks
    # split points that cut the block order anywhere, including ranges of one block
    cuts = sorted({0, 1, nb // 3, nb // 2 + 1, nb - 1, nb})
    ranges = []
    for b0, b1 in zip(cuts, cuts[1:]):
        if b1 <= b0:
            continue
        recs, sizes = oracle.compress_blocks(f, N, scheme, eps, b0, b1)
        stride = oracle.record_bound(N, f.dtype.itemsize)
        assert recs.size == (b1 - b0) * stride
        for k in range(b1 - b0):
            r = S.record(whole, b0 + k, h)
            assert int(sizes[k]) == len(r.raw), (b0 + k)
            assert recs[k * stride:k * stride + len(r.raw)].tobytes() == r.raw, (b0 + k)
        ranges.append((b0, b1, recs, sizes))
    # the records, placed by an exclusive scan of their sizes, are the whole stream
    assert stream_from_records(whole, ranges) == whole


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("N,shape", CASES)
def test_decompress_blocks_equal_whole_field(oracle, N, shape, scheme, dt):
    f = field_of(shape, dt, 202 + N)
    eps = 1e-2 * float(f.max() - f.min())
    whole = oracle.compress(f, N, scheme, eps)
    want = oracle.decompress(whole)
    nb = S.header(whole).nblocks
    b0, b1 = 1, max(2, nb - 1)
    recs, sizes = oracle.compress_blocks(f, N, scheme, eps, b0, b1)
    sentinel = np.array(7.25, dtype=dt)
    out = np.full(f.shape, sentinel, dtype=dt)
    oracle.decompress_blocks(recs, sizes, f.shape, N, scheme, b0, b1, out)
    nz, ny, nx = f.shape
    nbx, nby = nx // N, ny // N
    for b in range(nb):
        bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
        sl = (slice(bz * N, bz * N + N), slice(by * N, by * N + N), slice(bx * N, bx * N + N))
        if b0 <= b < b1:
            assert out[sl].tobytes() == want[sl].tobytes(), b
        else:
            assert (out[sl] == sentinel).all(), f"block {b} outside the range was written"


def test_block_range_errors(oracle):
    f = np.zeros((16, 16, 24), np.float32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress_blocks(f, 16, "W4", 0.1, 0, 1)
    assert e.value.code == oracle.ERR_SHAPE
    g = f.copy()
    g[3, 4, 5] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.compress_blocks(g, 8, "W4", 0.1, 0, 6)
    assert e.value.code == oracle.ERR_NONFINITE
    # a record whose popcount disagrees with its nnz is rejected on decode
    recs, sizes = oracle.compress_blocks(f, 8, "W4", 0.1, 0, 2)
    bad = recs.copy()
    bad[8] ^= 0x80  # a mask bit outside the always-kept corner
    out = np.zeros_like(f)
    with pytest.raises(oracle.OracleError) as e:
        oracle.decompress_blocks(bad, sizes, f.shape, 8, "W4", 0, 2, out)
    assert e.value.code == oracle.ERR_FORMAT


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("N,shape", CASES)
def test_openmp_timing_build_equals_one_thread(oracle, N, shape, dt):
    """The all-cores timing build (OpenMP parallel-for over chunks of blocks,
    the node layer of Sec. 2.1) yields the records, sizes and decoded blocks
    of the single-threaded block-range call, for any thread count."""
    f = field_of(shape, dt, 303 + N)
    eps = 1e-2 * float(f.max() - f.min())
    nb = (shape[0] // N) * (shape[1] // N) * (shape[2] // N)
    b0, b1 = 1, nb
    recs, sizes = oracle.compress_blocks(f, N, "W4_li", eps, b0, b1)
    want = np.zeros_like(f)
    oracle.decompress_blocks(recs, sizes, f.shape, N, "W4_li", b0, b1, want)
    for threads in (1, 3, 8):
        pr, ps = oracle.compress_blocks_par(f, N, "W4_li", eps, b0, b1, threads)
        assert np.array_equal(ps, sizes) and np.array_equal(pr, recs), threads
        got = np.zeros_like(f)
        oracle.decompress_blocks_par(pr, ps, f.shape, N, "W4_li", b0, b1, got, threads)
        assert got.tobytes() == want.tobytes(), threads
