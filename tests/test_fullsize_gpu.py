"""Whole-stream parity at the sizes the benchmark runs, and persistent
kernels that process several blocks per workgroup.

The oracle compresses the full fields here (in threads over disjoint block
ranges, placed by the exclusive scan of their sizes: tests/oracle_par.py),
so the whole stream -- header, every offset (and with it the look-back's
steps past the first 64 predecessors), every record -- is compared byte for
byte with libcz's, and the GPU inverse of the oracle's stream is compared
with the oracle's inverse over the whole field.
"""
import time

import numpy as np
import pytest
import torch

import oracle_par
from gpu_common import assert_stream_parity, need_gpu, ordinal, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def codec():
    need_gpu()
    from paper_1903_07761_amd.codec import Codec

    return Codec(0)


def whole_parity(codec, oracle, field_gpu: torch.Tensor, N: int, scheme: str, eps: float, tag: str):
    t0 = time.time()
    say(f"[{tag}] GPU compress {tuple(field_gpu.shape)} {field_gpu.dtype} {scheme} N={N} eps={eps:.4g}")
    buf, n = codec.compress(field_gpu, N, scheme, eps)
    torch.cuda.synchronize()
    g = buf[:n].cpu().numpy().tobytes()
    del buf
    f = field_gpu.cpu().numpy()
    say(f"[{tag}] oracle compress ({oracle_par.workers()} threads), GPU stream {n} bytes")
    o = oracle_par.compress(oracle, f, N, scheme, eps)
    verdict = assert_stream_parity(g, o, eps)
    say(f"[{tag}] stream: {verdict}, {time.time() - t0:.1f} s")
    del g
    # inverse of the oracle's stream on both sides, whole field
    dev = torch.frombuffer(bytearray(o), dtype=torch.uint8).cuda()
    got = codec.decompress(dev, len(o))
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    del dev
    want = oracle_par.decompress(oracle, o)
    if got.tobytes() != want.tobytes():
        d = int(np.abs(ordinal(got.reshape(-1)) - ordinal(want.reshape(-1))).max())
        assert d <= 4, f"{tag}: inverse differs by {d} ulp"
        say(f"[{tag}] inverse within {d} ulp")
    else:
        say(f"[{tag}] inverse bit-identical")
    say(f"[{tag}] PSNR {oracle.psnr(f, got):.2f} dB, CR_stage1 {f.nbytes / len(o):.3f}, {time.time() - t0:.1f} s")


@pytest.mark.parametrize("frac", [1e-2, 1e-3, 1e-4])
def test_c2_whole_stream(codec, oracle, frac):
    """512^3 float32 bubble cloud (pressure-like), W4_li, N = 32: 4096 blocks."""
    from paper_1903_07761_amd import fields

    f = fields.bubble_cloud(512, 1904, dtype=torch.float32, device="cuda")
    whole_parity(codec, oracle, f, 32, "W4_li", frac * fields.value_range(f), f"C2 eps={frac}")


@pytest.mark.parametrize("which", ["u", "rho"])
def test_c3_whole_stream(codec, oracle, which):
    """1024^3 float64, W3_ai, N = 32, eps = 1e-4 range: 32768 blocks.  u is a
    smooth velocity component (CR ~ 56), rho the noisy density-like cloud
    (every record near full size)."""
    from paper_1903_07761_amd import fields

    if which == "u":
        f = fields.div_free_velocity(1024, 1907, dtype=torch.float64, device="cuda")[0]
    else:
        f = fields.bubble_cloud(1024, 1905, v_in=0.016, dtype=torch.float64, device="cuda")
    whole_parity(codec, oracle, f, 32, "W3_ai", 1e-4 * fields.value_range(f), f"C3 {which}")
    del f
    torch.cuda.empty_cache()


@pytest.mark.parametrize("scheme", ["W4", "W4_li", "W3_ai"])
@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_64cubed_several_blocks_per_workgroup(oracle, dt, scheme):
    """The 64^3 kernels are persistent with one scratch slot per workgroup.
    With the 64-slot variant and 128 blocks every workgroup reuses its slot
    for a second block (and more, in the 216-block case), forward and
    inverse."""
    need_gpu()
    from paper_1903_07761_amd import _cz, fields
    from paper_1903_07761_amd.codec import Codec

    codec = Codec(0, tuned=False)
    elem = 4 if dt == torch.float32 else 8
    assert _cz.variant_count(64, elem) >= 3
    codec.set_variant(64, dt, scheme, 2)  # 64 resident workgroups, 64 scratch slots
    f = fields.bubble_cloud(512, 1906, nbubbles=60, dtype=dt, device="cuda")[:128].contiguous()
    whole_parity(codec, oracle, f, 64, scheme, 1e-3 * fields.value_range(f), f"64^3 x128 {dt} {scheme}")
    if dt == torch.float64 and scheme == "W3_ai":
        g = fields.gaussian_bumps(384, 1907, dtype=dt, device="cuda")
        whole_parity(codec, oracle, g, 64, scheme, 1e-3 * fields.value_range(g), "64^3 x216 f64 W3_ai")


def test_32cubed_inverse_persistent_many_blocks(oracle):
    """The 32^3 inverse is persistent (grid = resident workgroups); 1024
    blocks of a 256 x 512 x 256 float field on every variant."""
    need_gpu()
    from paper_1903_07761_amd import _cz, fields
    from paper_1903_07761_amd.codec import Codec

    codec = Codec(0, tuned=False)
    f = fields.bubble_cloud(512, 1908, nbubbles=80, dtype=torch.float32, device="cuda")[:256, :, :256].contiguous()
    eps = 1e-3 * fields.value_range(f)
    for v in range(_cz.variant_count(32, 4)):
        codec.set_variant(32, torch.float32, "W4_li", v)
        whole_parity(codec, oracle, f, 32, "W4_li", eps, f"32^3 f32 W4_li variant {v}")


@pytest.mark.parametrize("N,shape", [(8, (120, 200, 232)), (16, (144, 240, 208))])
@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_small_blocks_many_groups(codec, oracle, N, shape, dt):
    """8^3 and 16^3 blocks go in groups of one workgroup (one block per
    wavefront, one ticket and one look-back per group): 10875 8^3 blocks
    (680 groups of 16) and 1755 16^3 blocks, counts that leave the last group
    short, so the group look-back runs many steps past its first 64
    predecessors and each record's offset adds the sizes of the earlier
    blocks of its group."""
    from paper_1903_07761_amd import fields

    n = max(shape)
    f = fields.bubble_cloud(n, 1909, nbubbles=60, dtype=dt, device="cuda")[: shape[0], : shape[1], : shape[2]]
    f = f.contiguous()
    for scheme in ("W4", "W4_li", "W3_ai"):
        whole_parity(codec, oracle, f, N, scheme, 1e-3 * fields.value_range(f), f"{N}^3 {dt} {scheme}")


@pytest.mark.parametrize("layout", ["halves", "checker"])
@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_deferred_and_direct_records(codec, oracle, dt, layout):
    """32^3 blocks whose record fits a slot skip the look-back and are placed
    by the fix-up; larger records look back through the sizes the deferred
    ones published.  'halves': 320 smooth blocks (deferred) then 192 noisy
    ones (direct), so the first direct block walks back over 320 published
    sizes; 'checker': the two kinds alternate block by block."""
    from paper_1903_07761_amd import fields

    n = 256
    smooth = fields.gaussian_bumps(n, 1911, dtype=dt)
    rng = torch.Generator().manual_seed(1912)
    noisy = smooth + 0.05 * torch.randn(n, n, n, generator=rng, dtype=torch.float64).to(dt)
    if layout == "halves":
        f = torch.cat([smooth[:160], noisy[160:]], dim=0)
    else:
        z, y, x = torch.meshgrid(torch.arange(n) // 32, torch.arange(n) // 32, torch.arange(n) // 32, indexing="ij")
        f = torch.where(((x + y + z) % 2 == 0), smooth, noisy)
    f = f.contiguous().cuda()
    whole_parity(codec, oracle, f, 32, "W3_ai", 1e-3 * fields.value_range(f), f"deferred/direct {layout} {dt}")


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_deferred_records_into_an_offset_buffer(codec, oracle, dt):
    """The stream may start at any 4-byte-aligned address: with the output 4
    bytes into a buffer, the fix-up moves deferred records with 4-byte
    accesses; the stream equals the oracle's and the bytes around it are
    untouched."""
    from paper_1903_07761_amd import _cz, fields

    f = fields.gaussian_bumps(128, 1913, dtype=dt, device="cuda")  # smooth: records fit the slots
    eps = 1e-3 * fields.value_range(f)
    p = codec.params(f, 32, "W3_ai", eps)
    cap = _cz.compress_bound(p)
    buf = torch.full((cap + 32,), 0x5C, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    n = codec.ctx.compress(p, f.data_ptr(), buf.data_ptr() + 4, cap, stream=st)
    torch.cuda.synchronize()
    host = buf.cpu().numpy()
    assert host[:4].tobytes() == b"\x5c" * 4
    assert host[4 + n:].tobytes() == b"\x5c" * (cap + 28 - n)
    assert host[4:4 + n].tobytes() == oracle.compress(f.cpu().numpy(), 32, "W3_ai", eps)
