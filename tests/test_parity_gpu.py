"""GPU <-> oracle parity of the wavelet stage through the C ABI.

Forward (transform + decimation + mask + compaction + offsets + header) and
inverse (unpack + inverse transform + store) of libcz against the CPU oracle
on the same seeded inputs: whole streams at small sizes (several blocks,
non-cubic grids, every scheme x precision x block size), sampled blocks at
the full workload sizes, and the edge cases.  Bar: streams byte-identical, or
the comparison rule (mask bits may differ only within 1e-6 eps of eps,
coefficients within 4 ulp; with equal masks the layout is byte-identical).
"""
import numpy as np
import pytest
import torch

import streamfmt as S
from gpu_common import assert_stream_parity, block_of, compare_records, need_gpu, ordinal, sample_blocks, say

pytestmark = pytest.mark.gpu

SCHEMES = ["W4", "W4_li", "W3_ai"]
TDT = {np.float32: torch.float32, np.float64: torch.float64}


@pytest.fixture(scope="module")
def codec():
    need_gpu()
    from paper_1903_07761_amd.codec import Codec

    return Codec(0)


def gpu_compress(codec, f: np.ndarray, N, scheme, eps):
    t = torch.from_numpy(np.ascontiguousarray(f)).cuda()
    buf, n = codec.compress(t, N, scheme, eps)
    return buf[:n].cpu().numpy().tobytes()


def gpu_decompress(codec, s: bytes) -> np.ndarray:
    t = torch.frombuffer(bytearray(s), dtype=torch.uint8).cuda()
    out = codec.decompress(t, len(s))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def small_field(kind, shape, dt, seed):
    from paper_1903_07761_amd import fields

    nz, ny, nx = shape
    if kind == "bumps":
        n = max(shape)
        return fields.gaussian_bumps(n, seed, dtype=TDT[dt]).numpy()[:nz, :ny, :nx].copy()
    if kind == "bubbles":
        n = max(shape)
        return fields.bubble_cloud(n, seed, nbubbles=30, dtype=TDT[dt]).numpy()[:nz, :ny, :nx].copy()
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape).astype(dt)


CASES = [
    # (N, shape [nz, ny, nx]) -- several blocks, non-cubic grids, ragged block counts
    (8, (16, 24, 40)),
    (16, (32, 48, 16)),
    (32, (32, 96, 64)),
    (32, (64, 32, 32)),
    (64, (64, 64, 128)),  # scratch-staged path
]


@pytest.mark.parametrize("kind", ["bumps", "noise", "bubbles"])
@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("N,shape", CASES)
def test_forward_parity(codec, oracle, N, shape, scheme, dt, kind):
    f = small_field(kind, shape, dt, 1903 + N)
    rng = float(f.max() - f.min())
    for frac in (0.0, 1e-3, 3e-2):
        eps = frac * rng
        say(f"[fwd] N={N} shape={shape} {scheme} {np.dtype(dt).name} {kind} eps={eps:.3g}")
        g = gpu_compress(codec, f, N, scheme, eps)
        o = oracle.compress(f, N, scheme, eps)
        S.validate(g)
        verdict = assert_stream_parity(g, o, eps)
        say("   ", verdict, len(g), "bytes")


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("N,shape", CASES)
def test_inverse_parity(codec, oracle, N, shape, scheme, dt):
    """The GPU inverse of the oracle's stream equals the oracle's inverse."""
    f = small_field("bumps", shape, dt, 7 + N)
    for frac in (0.0, 1e-3):
        eps = frac * float(f.max() - f.min())
        say(f"[inv] N={N} shape={shape} {scheme} {np.dtype(dt).name} eps={eps:.3g}")
        o = oracle.compress(f, N, scheme, eps)
        want = oracle.decompress(o)
        got = gpu_decompress(codec, o)
        d = np.abs(ordinal(got.reshape(-1)) - ordinal(want.reshape(-1))).max()
        assert d <= 4, f"inverse differs by {d} ulp"
        say("    max ulp", int(d), "psnr", oracle.psnr(f, got))


def test_roundtrip_and_determinism(codec, oracle):
    f = small_field("bubbles", (64, 64, 64), np.float32, 5)
    eps = 1e-3 * float(f.max() - f.min())
    say("[roundtrip] 64^3 f32 W3_ai N=32")
    a = gpu_compress(codec, f, 32, "W3_ai", eps)
    b = gpu_compress(codec, f, 32, "W3_ai", eps)
    assert a == b
    r = gpu_decompress(codec, a)
    assert np.array_equal(r, oracle.decompress(oracle.compress(f, 32, "W3_ai", eps)))


def test_async_path_and_device_size(codec, oracle):
    f = small_field("bumps", (32, 64, 96), np.float64, 11)
    eps = 1e-4 * float(f.max() - f.min())
    t = torch.from_numpy(f).cuda()
    nbytes = torch.zeros(1, dtype=torch.int64, device="cuda")
    say("[async] 32x64x96 f64 W4_li N=16")
    buf, n = codec.compress(t, 16, "W4_li", eps, sync=False, out_bytes=nbytes)
    assert n is None
    assert codec.status() == 0
    n = int(nbytes.item())
    o = oracle.compress(f, 16, "W4_li", eps)
    assert buf[:n].cpu().numpy().tobytes() == o
    out = torch.empty_like(t)
    codec.decompress(buf, n, out=out, expected=codec.params(t, 16, "W4_li", eps))
    assert codec.status() == 0
    assert np.array_equal(out.cpu().numpy(), oracle.decompress(o))


# ------------------------------------------------------------------ edges

def test_empty_field(codec, oracle):
    say("[edge] empty field")
    f = np.zeros((0, 32, 32), np.float32)
    t = torch.zeros((0, 32, 32), dtype=torch.float32, device="cuda")
    buf, n = codec.compress(t, 32, "W4", 0.1)
    assert buf[:n].cpu().numpy().tobytes() == oracle.compress(f, 32, "W4", 0.1)
    out = codec.decompress(buf, n)
    assert out.shape == (0, 32, 32)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_keep_all_and_keep_corner_only(codec, oracle, dt):
    f = small_field("noise", (32, 32, 64), dt, 3)
    for eps in (0.0, 1e30):
        say(f"[edge] eps={eps} {np.dtype(dt).name}")
        g = gpu_compress(codec, f, 32, "W4", eps)
        assert g == oracle.compress(f, 32, "W4", eps)
        h = S.header(g)
        for b in range(h.nblocks):
            assert S.record(g, b, h).nnz == (32 ** 3 if eps == 0 else 64)


def test_constant_field(codec, oracle):
    say("[edge] constant field")
    f = np.full((64, 64, 64), 3.25, np.float32)
    g = gpu_compress(codec, f, 32, "W3_ai", 1e-9)
    assert g == oracle.compress(f, 32, "W3_ai", 1e-9)
    assert len(g) == 144 + 8 * 4368


def test_threshold_tie(codec, oracle):
    """A coefficient exactly equal to eps is kept on both sides."""
    N = 8
    B = np.zeros((N, N, N), np.float32)
    B[0, 0, 1] = 1.0
    C = oracle.fwd_block("W4", B)
    c = float(np.abs(C[C != 0]).min())
    for eps in (c, float(np.nextafter(c, np.inf))):
        say(f"[edge] tie eps={eps!r}")
        assert gpu_compress(codec, B, N, "W4", eps) == oracle.compress(B, N, "W4", eps)


@pytest.mark.parametrize("N", [8, 16, 32, 64])
@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_nonfinite_input_is_an_error(codec, N, dt):
    from paper_1903_07761_amd import CzError, _cz

    say(f"[edge] NaN/inf input N={N} {dt}")
    t = torch.ones((64, 64, 64), dtype=dt, device="cuda")
    for pos in ((5, 6, 7), (63, 62, 61)):  # coarse corner / finest details of the last block
        for bad in (float("nan"), float("inf"), float("-inf")):
            t[pos] = bad
            with pytest.raises(CzError) as e:
                codec.compress(t, N, "W4", 0.1)
            assert e.value.code == _cz.ERR_NONFINITE
            t[pos] = 1.0
    codec.compress(t, N, "W4", 0.1)  # clean again: no error


def test_capacity_and_shape_errors(codec):
    from paper_1903_07761_amd import CzError, _cz

    say("[edge] capacity / shape")
    t = torch.ones((32, 32, 32), dtype=torch.float32, device="cuda")
    small = torch.empty(100, dtype=torch.uint8, device="cuda")
    with pytest.raises(CzError) as e:
        codec.compress(t, 32, "W4", 0.1, out=small)
    assert e.value.code == _cz.ERR_CAPACITY
    t2 = torch.ones((32, 32, 40), dtype=torch.float32, device="cuda")
    with pytest.raises(CzError) as e:
        codec.compress(t2, 32, "W4", 0.1)
    assert e.value.code == _cz.ERR_SHAPE


def test_corrupt_stream_is_rejected(codec, oracle):
    import struct

    from paper_1903_07761_amd import CzError, _cz

    f = small_field("bumps", (16, 16, 32), np.float32, 2)
    good = oracle.compress(f, 8, "W4", 1e-3)
    h = S.header(good)
    cases = {}
    bad = bytearray(good)
    struct.pack_into("<I", bad, h.payload_start + int(S.offsets(good, h)[3]), 99999)  # nnz of block 3
    cases["nnz"] = bytes(bad)
    bad = bytearray(good)
    struct.pack_into("<Q", bad, 64 + 8 * 2, 7)  # offsets not a valid record size
    cases["offset"] = bytes(bad)
    bad = bytearray(good)
    rec = h.payload_start + int(S.offsets(good, h)[1])
    bad[rec + 8 + 10] ^= 0x10  # a mask bit flipped: popcount != nnz
    cases["mask"] = bytes(bad)
    for name, s in cases.items():
        say(f"[edge] corrupt stream: {name}")
        t = torch.frombuffer(bytearray(s), dtype=torch.uint8).cuda()
        with pytest.raises(CzError) as e:
            codec.decompress(t, len(s))
        assert e.value.code == _cz.ERR_FORMAT
    assert codec.status() == 0


# ------------------------------------------------------- full-size workloads

def gpu_record_stream(buf: torch.Tensor, h, off, b: int, alone: bytes) -> bytes:
    """A one-block stream holding the GPU's record b, framed with the header
    and offsets of the oracle's single-block stream (same N, type, scheme)."""
    start = h.payload_start + int(off[b])
    rec = buf[start:h.payload_start + int(off[b + 1])].cpu().numpy().tobytes()
    ho = S.header(alone)
    frame = bytearray(alone[:ho.payload_start])
    import struct

    struct.pack_into("<Q", frame, 56, len(rec))
    struct.pack_into("<Q", frame, 64 + 8, len(rec))
    return bytes(frame) + rec


def check_sampled(codec, oracle, field_gpu: torch.Tensor, N, scheme, eps, k, seed, tag):
    """Compress the whole field on the GPU in the benchmark's launch
    configuration; check the offsets table; compare k sampled records with the
    oracle compressing those blocks alone (blocks are independent); decompress
    on the GPU and compare the sampled blocks with the oracle's inverse."""
    say(f"[{tag}] compress {tuple(field_gpu.shape)} {field_gpu.dtype} {scheme} N={N} eps={eps:.4g}")
    buf, n = codec.compress(field_gpu, N, scheme, eps)
    torch.cuda.synchronize()
    h = S.header(buf[:64].cpu().numpy().tobytes())
    off = buf[64:64 + 8 * (h.nblocks + 1)].cpu().numpy().view(np.uint64)
    assert off[0] == 0 and np.all(np.diff(off.astype(np.int64)) > 0) and int(off[-1]) == h.payload_bytes
    assert n == h.payload_start + h.payload_bytes
    say(f"[{tag}] decompress, CR_stage1 = {field_gpu.numel() * field_gpu.element_size() / n:.3f}")
    rec = codec.decompress(buf, n)
    torch.cuda.synchronize()
    nz, ny, nx = field_gpu.shape
    nbx, nby = nx // N, ny // N
    worst = 0
    for b in sample_blocks(h.nblocks, k, seed):
        bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
        sl = (slice(bz * N, (bz + 1) * N), slice(by * N, (by + 1) * N), slice(bx * N, (bx + 1) * N))
        blk = field_gpu[sl].cpu().numpy()
        alone = oracle.compress(blk, N, scheme, eps)
        g1 = gpu_record_stream(buf, h, off, b, alone)
        S.validate(g1)
        _, u = compare_records(g1, alone, 0, 0, eps)
        worst = max(worst, u)
        want = oracle.decompress(alone)
        got = rec[sl].cpu().numpy()
        d = int(np.abs(ordinal(got.reshape(-1)) - ordinal(want.reshape(-1))).max())
        assert d <= 4, f"block {b}: inverse differs by {d} ulp"
    say(f"[{tag}] sampled blocks agree (max {worst} ulp)")
    return buf, n, rec


def test_c1_full(codec, oracle):
    """128^3 float32 Gaussian bumps, W4, N = 32, eps = 1e-3 range: whole stream."""
    from paper_1903_07761_amd import fields

    f = fields.gaussian_bumps(128, 1903, dtype=torch.float32)
    eps = 1e-3 * fields.value_range(f)
    say("[C1] 128^3 f32 W4 N=32")
    g = gpu_compress(codec, f.numpy(), 32, "W4", eps)
    o = oracle.compress(f.numpy(), 32, "W4", eps)
    say("   ", assert_stream_parity(g, o, eps))
    r = gpu_decompress(codec, g)
    say("    PSNR", oracle.psnr(f.numpy(), r), "max err", float(np.abs(r - f.numpy()).max()))


@pytest.mark.parametrize("frac", [1e-2, 1e-3, 1e-4])
def test_c2_sampled(codec, oracle, frac):
    """512^3 float32 bubble cloud (pressure-like), W4_li, N = 32."""
    from paper_1903_07761_amd import fields

    f = fields.bubble_cloud(512, 1904, dtype=torch.float32, device="cuda")
    eps = frac * fields.value_range(f)
    check_sampled(codec, oracle, f, 32, "W4_li", eps, 24, 1904, f"C2 eps={frac}")


def test_c3_sampled(codec, oracle):
    """1024^3 float64 fields, W3_ai, N = 32, eps = 1e-4 range: density-like
    bubble cloud and one divergence-free velocity component."""
    from paper_1903_07761_amd import fields

    rho = fields.bubble_cloud(1024, 1905, v_in=0.016, dtype=torch.float64, device="cuda")
    check_sampled(codec, oracle, rho, 32, "W3_ai", 1e-4 * fields.value_range(rho), 12, 1905, "C3 rho")
    del rho
    torch.cuda.empty_cache()
    u = fields.div_free_velocity(1024, 1907, dtype=torch.float64, device="cuda")[0]
    check_sampled(codec, oracle, u, 32, "W3_ai", 1e-4 * fields.value_range(u), 12, 1907, "C3 u")
