"""Random access: selected blocks, the decoded-block cache and boxes of the
field, each bit-identical to the same part of the oracle's full
decompression of the same stream."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu

TDT = {np.float32: torch.float32, np.float64: torch.float64}


@pytest.fixture(scope="module")
def codec():
    need_gpu()
    from paper_1903_07761_amd.codec import Codec

    return Codec(0)


def make_stream(codec, N, dt, shape, seed):
    from paper_1903_07761_amd import fields

    n = max(shape)
    f = fields.bubble_cloud(n, seed, nbubbles=20, dtype=TDT[dt])[: shape[0], : shape[1], : shape[2]].contiguous().cuda()
    eps = 1e-3 * float(f.max() - f.min())
    buf, nb = codec.compress(f, N, "W3_ai", eps)
    return f, buf, nb, codec.params(f, N, "W3_ai", eps)


def block_box(full, N, b, nbx, nby):
    bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
    return full[bz * N:(bz + 1) * N, by * N:(by + 1) * N, bx * N:(bx + 1) * N]


CASES = [(8, np.float32, (16, 24, 32)), (16, np.float64, (32, 48, 16)), (32, np.float32, (64, 32, 96)),
         (32, np.float64, (32, 64, 64)), (64, np.float32, (64, 64, 128))]


@pytest.mark.parametrize("N,dt,shape", CASES)
def test_decompress_blocks(codec, oracle, N, dt, shape):
    f, buf, nb, p = make_stream(codec, N, dt, shape, 41 + N)
    full = oracle.decompress(buf[:nb].cpu().numpy().tobytes())
    nbx, nby = shape[2] // N, shape[1] // N
    nblocks = full.size // N ** 3
    rng = np.random.default_rng(N)
    ids = list(rng.integers(0, nblocks, size=min(7, nblocks) + 2))  # repeats and any order
    ids[0] = nblocks - 1
    out = codec.decompress_blocks(buf, nb, p, ids)
    assert codec.status() == 0
    got = out.cpu().numpy()
    for k, b in enumerate(ids):
        assert np.array_equal(got[k], block_box(full, N, int(b), nbx, nby)), (k, b)
    say(f"[roi] blocks N={N} {np.dtype(dt).name}: {len(ids)} ok")


@pytest.mark.parametrize("N,dt,shape", CASES)
def test_regions_through_the_cache(codec, oracle, N, dt, shape):
    f, buf, nb, p = make_stream(codec, N, dt, shape, 51 + N)
    full = oracle.decompress(buf[:nb].cpu().numpy().tobytes())
    nz, ny, nx = shape
    cache = codec.cache(p, 16)
    rng = np.random.default_rng(N + 1)
    boxes = [((0, 0, 0), (nx, ny, nz)) if (nx // N) * (ny // N) * (nz // N) <= 16 else ((0, 0, 0), (N, N, N))]
    for _ in range(12):
        ext = [int(rng.integers(1, min(d, N) + 1)) for d in (nx, ny, nz)]  # at most 2 blocks an axis
        org = [int(rng.integers(0, d - e + 1)) for d, e in zip((nx, ny, nz), ext)]
        boxes.append((tuple(org), tuple(ext)))
    for org, ext in boxes:
        out = codec.region(cache, buf, nb, p, org, ext)
        torch.cuda.synchronize()
        ref = full[org[2]:org[2] + ext[2], org[1]:org[1] + ext[1], org[0]:org[0] + ext[0]]
        assert np.array_equal(out.cpu().numpy(), ref), (org, ext)
    hits, misses = cache.stats()
    assert misses >= 1 and hits >= 1
    assert codec.status() == 0
    say(f"[roi] regions N={N}: hits {hits} misses {misses}")
    cache.close()


def test_cache_reuse_and_eviction(codec, oracle):
    N, dt, shape = 16, np.float32, (32, 32, 64)  # 16 blocks
    f, buf, nb, p = make_stream(codec, N, dt, shape, 61)
    full = oracle.decompress(buf[:nb].cpu().numpy().tobytes())
    cache = codec.cache(p, 4)
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]

    def read(ptr):
        host = np.empty((N, N, N), dtype=dt)
        torch.cuda.synchronize()
        assert hip.hipMemcpy(host.ctypes.data, ptr, host.nbytes, 2) == 0  # device to host
        return host

    seq = [[0, 1, 2], [1, 2, 3], [0, 3], [9, 10, 11, 12], [12, 12, 9]]
    expect_hits = [0, 2, 2, 0, 3]
    for ids, eh in zip(seq, expect_hits):
        h0, m0 = cache.stats()
        ptrs = cache.fetch(buf.data_ptr(), nb, ids)
        h1, m1 = cache.stats()
        assert h1 - h0 == eh and (h1 - h0) + (m1 - m0) == len(ids), (ids, h1 - h0, m1 - m0)
        for b, ptr in zip(ids, ptrs):
            assert np.array_equal(read(ptr), block_box(full, N, b, 4, 2)), (ids, b)
    # another stream buffer empties the pool
    other = buf.clone()
    h0, m0 = cache.stats()
    cache.fetch(other.data_ptr(), nb, [9])
    assert cache.stats()[1] == m0 + 1
    cache.close()


def test_random_access_errors(codec):
    from paper_1903_07761_amd import _cz

    f, buf, nb, p = make_stream(codec, 16, np.float32, (32, 32, 32), 71)
    with pytest.raises(_cz.CzError) as e:
        codec.decompress_blocks(buf, nb, p, [8])
    assert e.value.code == _cz.ERR_ARG
    small = torch.empty(16 ** 3, dtype=torch.float32, device="cuda")
    with pytest.raises(_cz.CzError) as e:
        codec.decompress_blocks(buf, nb, p, [0, 1], out=small)
    assert e.value.code == _cz.ERR_CAPACITY
    cache = codec.cache(p, 2)
    with pytest.raises(_cz.CzError) as e:
        cache.fetch(buf.data_ptr(), nb, [0, 1, 2])
    assert e.value.code == _cz.ERR_ARG
    with pytest.raises(_cz.CzError) as e:
        codec.region(cache, buf, nb, p, (20, 0, 0), (16, 4, 4))
    assert e.value.code == _cz.ERR_ARG
    with pytest.raises(_cz.CzError) as e:
        codec.region(cache, buf, nb, p, (0, 0, 0), (32, 32, 1))  # touches 4 blocks > capacity
    assert e.value.code == _cz.ERR_ARG
    cache.close()
    assert codec.status() == 0
