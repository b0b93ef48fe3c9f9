"""Sharding a field by block ranges and placing the parts by an exclusive scan.

Paper: arXiv 1903.07761, Sec. 2.2: each process compresses its part of the
domain, an exclusive prefix scan of the compressed sizes gives every part
its place, and the parts together form the output.  Here the parts are
slabs of whole block layers along z (contiguous ranges of the block order),
compressed as separate fields -- as separate devices would -- and stitched
on the host; the result must be byte-identical to compressing the whole
field at once, on the oracle (CPU) and on libcz (GPU).
"""
import numpy as np
import pytest
import torch

import streamfmt as S
from stitch import stitch_slabs

SCHEMES = ["W4", "W4_li", "W3_ai"]


def bumps(shape, dt, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny, (np.arange(nx) + 0.5) / nx,
                          indexing="ij")
    f = 0.1 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    for _ in range(4):
        c = rng.random(3)
        s = rng.uniform(0.05, 0.2)
        f += rng.uniform(0.5, 2) * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * s * s))
    return (f * (1 + 0.001 * rng.standard_normal(shape))).astype(dt)


def slab_cuts(nz, N, parts):
    layers = nz // N
    cuts = sorted({0, layers} | {max(1, min(layers - 1, (layers * k) // parts)) for k in range(1, parts)})
    return [(a * N, b * N) for a, b in zip(cuts, cuts[1:]) if b > a]


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("N,shape,parts", [(8, (40, 16, 24), 3), (16, (64, 32, 48), 4), (32, (96, 64, 32), 3)])
def test_oracle_slabs_stitch_to_whole(oracle, N, shape, parts, scheme, dt):
    f = bumps(shape, dt, 300 + N)
    eps = 1e-3 * float(f.max() - f.min())
    whole = oracle.compress(f, N, scheme, eps)
    pieces = [oracle.compress(np.ascontiguousarray(f[z0:z1]), N, scheme, eps) for z0, z1 in slab_cuts(shape[0], N, parts)]
    assert len(pieces) >= 2
    stitched = stitch_slabs(pieces)
    S.validate(stitched)
    assert stitched == whole


def test_stitch_of_one_part_is_identity(oracle):
    f = bumps((32, 32, 32), np.float32, 5)
    s = oracle.compress(f, 16, "W4", 1e-3)
    assert stitch_slabs([s]) == s


@pytest.mark.gpu
@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("N,shape,parts", [(8, (40, 16, 24), 3), (16, (64, 32, 48), 4), (32, (160, 64, 96), 4),
                                           (64, (192, 64, 128), 3)])
def test_gpu_slabs_stitch_to_whole(oracle, N, shape, parts, scheme, dt):
    from gpu_common import need_gpu, say

    need_gpu()
    from paper_1903_07761_amd.codec import Codec

    codec = Codec(0)
    f = bumps(shape, dt, 400 + N)
    eps = 1e-3 * float(f.max() - f.min())
    t = torch.from_numpy(f).cuda()
    say(f"[shard] N={N} shape={shape} {scheme} {np.dtype(dt).name} parts={parts}")
    buf, n = codec.compress(t, N, scheme, eps)
    whole = buf[:n].cpu().numpy().tobytes()
    pieces = []
    for z0, z1 in slab_cuts(shape[0], N, parts):
        b, m = codec.compress(t[z0:z1].contiguous(), N, scheme, eps)
        pieces.append(b[:m].cpu().numpy().tobytes())
    stitched = stitch_slabs(pieces)
    assert stitched == whole
    assert whole == oracle.compress(f, N, scheme, eps)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_split_is_the_inverse_of_stitch(oracle, scheme):
    from stitch import split_slabs

    f = bumps((96, 32, 64), np.float64, 9)
    s = oracle.compress(f, 16, scheme, 1e-3)
    for per in (1, 2, 4, 6):
        parts = split_slabs(s, per)
        assert stitch_slabs(parts) == s
        z = 0
        for p in parts:
            h = S.header(p)
            want = oracle.compress(np.ascontiguousarray(f[z:z + h.nz]), 16, scheme, 1e-3)
            assert p == want
            z += h.nz


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_threaded_oracle_equals_single_call(oracle, dt):
    import oracle_par

    f = bumps((64, 64, 96), dt, 10)
    eps = 1e-3 * float(f.max() - f.min())
    for N, scheme in ((8, "W4"), (16, "W4_li"), (32, "W3_ai")):
        s = oracle.compress(f, N, scheme, eps)
        assert oracle_par.compress(oracle, f, N, scheme, eps) == s
        assert oracle_par.decompress(oracle, s).tobytes() == oracle.decompress(s).tobytes()
