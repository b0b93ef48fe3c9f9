"""Pins of the preconditioning oracle (byte shuffle, Z4/Z8 zeroing) against
values written out by hand and an independent reading of the stream."""
import zlib

import numpy as np
import pytest
import torch

import streamfmt as S
from oracle import precond


def test_shuffle_worked_example():
    # three 4-byte elements and a 2-byte tail: planes of byte 0, 1, 2, 3, then the tail
    buf = bytes(range(14))
    assert precond.shuffle(buf, 4) == bytes([0, 4, 8, 1, 5, 9, 2, 6, 10, 3, 7, 11, 12, 13])
    assert precond.unshuffle(bytes([0, 4, 8, 1, 5, 9, 2, 6, 10, 3, 7, 11, 12, 13]), 4) == buf
    # 8-byte elements: two elements, no tail
    buf = bytes(range(16))
    assert precond.shuffle(buf, 8) == bytes([0, 8, 1, 9, 2, 10, 3, 11, 4, 12, 5, 13, 6, 14, 7, 15])


@pytest.mark.parametrize("elem", [1, 2, 4, 8])
def test_shuffle_roundtrip_and_size(elem):
    rng = np.random.default_rng(elem)
    for n in (0, 1, elem - 1, elem, 3 * elem + 1, 1000, 4099):
        buf = rng.integers(0, 256, n, dtype=np.uint8).tobytes()
        s = precond.shuffle(buf, elem)
        assert len(s) == n
        assert precond.unshuffle(s, elem) == buf
        assert sorted(s) == sorted(buf)  # a permutation of the bytes


def test_shuffle_of_float_array_groups_bytes():
    # little-endian floats: the first plane holds every element's lowest byte
    a = np.arange(1, 6, dtype=np.float32)
    s = np.frombuffer(precond.shuffle(a.tobytes(), 4), dtype=np.uint8)
    b = a.view(np.uint8).reshape(5, 4)
    for j in range(4):
        assert np.array_equal(s[5 * j:5 * (j + 1)], b[:, j])


def _stream(oracle, dtype, N, scheme, frac, seed=5):
    from paper_1903_07761_amd import fields

    n = max(2 * N, 32)
    f = fields.bubble_cloud(n, seed, nbubbles=20, dtype=torch.float32 if dtype == np.float32 else torch.float64)
    f = f.numpy()[:N, :, :].copy()
    return f, oracle.compress(f, N, scheme, frac * float(f.max() - f.min()))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("N", [8, 16, 32])
@pytest.mark.parametrize("bits", [4, 8])
def test_zero_details_against_dense_blocks(oracle, dtype, N, bits):
    """Independent reading: densify every record with the test stream reader,
    clear the low bits of every position outside the 4^3 corner, and compare
    with the oracle's rank walk."""
    f, s = _stream(oracle, dtype, N, "W3_ai", 1e-3)
    z = precond.zero_details(s, bits)
    h = S.validate(z)
    assert z[:h.payload_start] == s[:h.payload_start]  # header and offsets untouched
    uint = np.uint32 if dtype == np.float32 else np.uint64
    clear = ~uint((1 << bits) - 1)
    corner = np.zeros((N, N, N), dtype=bool)
    corner[:4, :4, :4] = True
    for b in range(h.nblocks):
        before = S.coefficients(s, b, h).view(uint)
        after = S.coefficients(z, b, h).view(uint)
        assert np.array_equal(after[corner], before[corner])
        assert np.array_equal(after[~corner], before[~corner] & clear)
        assert np.array_equal(S.record(z, b, h).mask, S.record(s, b, h).mask)


def test_zero_details_bounds_and_identity(oracle):
    f, s = _stream(oracle, np.float32, 16, "W4", 1e-3)
    assert precond.zero_details(s, 0) == s
    assert precond.max_zero_bits(4) == 23 and precond.max_zero_bits(8) == 52
    with pytest.raises(ValueError):
        precond.zero_details(s, 24)
    # zeroing never changes a value by 2^bits units in the last place or more
    z = precond.zero_details(s, 8)
    h = S.header(s)
    for b in range(h.nblocks):
        v0 = S.record(s, b, h).values.view(np.uint32).astype(np.int64)
        v1 = S.record(z, b, h).values.view(np.uint32).astype(np.int64)
        assert np.all(np.abs(v0 - v1) < 256)


def test_zeroing_and_shuffle_help_zlib(oracle):
    """The paper reports a higher ratio after zlib with shuffling (Table 2)
    and with Z8; at the PSNR of these thresholds the loss does not show."""
    f, s = _stream(oracle, np.float32, 32, "W3_ai", 1e-3, seed=7)
    plain = len(zlib.compress(s, 6))
    shuf = len(zlib.compress(precond.shuffle(s, 4), 6))
    z8 = precond.zero_details(s, 8)
    z8shuf = len(zlib.compress(precond.shuffle(z8, 4), 6))
    assert shuf < plain
    assert z8shuf < shuf
    # the decimation error at this threshold dwarfs 8 bits of float mantissa
    assert abs(oracle.psnr(f, oracle.decompress(z8)) - oracle.psnr(f, oracle.decompress(s))) < 0.05
