"""cz_compress_noalloc: the compress entry point for callers that cannot
allocate, whose scratch (ticket, status, size, descriptor, look-back flags)
lives in a fixed device array of the library instead of the context's
growable workspace.  Its streams must equal cz_compress's byte for byte (and
the oracle's, on these small fields), on consecutive calls that reuse the
array with a smaller field second, in the synchronous and the asynchronous
form; sizes beyond the array are refused before any work is issued."""
import numpy as np
import pytest
import torch

from gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu

ELEM = {torch.float32: 4, torch.float64: 8}


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    from paper_1903_07761_amd import _cz

    return _cz.Context(0)


def field(shape, dt, seed):
    from paper_1903_07761_amd import fields

    n = max(shape)
    f = fields.bubble_cloud(n, seed, nbubbles=40, dtype=dt)[: shape[0], : shape[1], : shape[2]].contiguous()
    return f


def params_of(f: torch.Tensor, N, scheme, eps):
    from paper_1903_07761_amd import _cz

    nz, ny, nx = f.shape
    return _cz.params(nx, ny, nz, N, scheme, ELEM[f.dtype], eps)


def both(ctx, f_cpu: torch.Tensor, N, scheme, frac):
    """(noalloc stream, cz_compress stream, oracle-ready eps) of one field."""
    from paper_1903_07761_amd import _cz, fields

    eps = frac * fields.value_range(f_cpu)
    f = f_cpu.cuda()
    p = params_of(f, N, scheme, eps)
    cap = _cz.lib().cz_compress_bound(p)
    a = torch.full((cap,), 0xA5, dtype=torch.uint8, device="cuda")
    b = torch.full((cap,), 0x5A, dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    na = ctx.compress_noalloc(p, f.data_ptr(), a.data_ptr(), cap, stream=st)
    nb = ctx.compress(p, f.data_ptr(), b.data_ptr(), cap, stream=st)
    torch.cuda.synchronize()
    return a[:na].cpu().numpy().tobytes(), b[:nb].cpu().numpy().tobytes(), eps


CASES = [
    # (first shape, second smaller shape, N, dtype, scheme)
    ((96, 64, 128), (32, 32, 64), 32, torch.float32, "W4_li"),
    ((64, 96, 64), (32, 64, 32), 32, torch.float64, "W3_ai"),
    ((64, 64, 48), (16, 32, 32), 16, torch.float32, "W4"),
    ((64, 64, 64), (8, 16, 24), 8, torch.float64, "W4_li"),
]


@pytest.mark.parametrize("first,second,N,dt,scheme", CASES)
def test_noalloc_equals_compress_on_two_calls(ctx, oracle, first, second, N, dt, scheme):
    for k, shape in enumerate((first, second)):
        f = field(shape, dt, 1910 + k)
        say(f"noalloc call {k}: {shape} {dt} N={N} {scheme}")
        g, ref, eps = both(ctx, f, N, scheme, 1e-3)
        assert g == ref, f"call {k}: cz_compress_noalloc differs from cz_compress"
        assert g == oracle.compress(f.numpy(), N, scheme, eps), f"call {k}: differs from the oracle"


def test_noalloc_async_size_and_status(ctx):
    """Asynchronous form: the size lands in the device word, a non-finite
    input is reported by cz_get_status, and the next call starts clean."""
    from paper_1903_07761_amd import _cz, fields

    f = field((64, 64, 64), torch.float32, 1912).cuda()
    p = params_of(f, 32, "W4", 1e-3 * fields.value_range(f.cpu()))
    cap = _cz.lib().cz_compress_bound(p)
    out = torch.zeros(cap, dtype=torch.uint8, device="cuda")
    word = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    assert ctx.get_status(st) == _cz.OK
    ctx.compress_noalloc(p, f.data_ptr(), out.data_ptr(), cap, stream=st, d_out_bytes=word.data_ptr(), sync=False)
    n_sync = ctx.compress_noalloc(p, f.data_ptr(), out.data_ptr(), cap, stream=st)
    torch.cuda.synchronize()
    assert int(word.item()) == n_sync
    assert ctx.get_status(st) == _cz.OK
    bad = f.clone()
    bad[5, 6, 7] = float("nan")
    ctx.compress_noalloc(p, bad.data_ptr(), out.data_ptr(), cap, stream=st, sync=False)
    assert ctx.get_status(st) == _cz.ERR_NONFINITE
    with pytest.raises(_cz.CzError) as e:
        ctx.compress_noalloc(p, bad.data_ptr(), out.data_ptr(), cap, stream=st)
    assert e.value.code == _cz.ERR_NONFINITE
    assert ctx.compress_noalloc(p, f.data_ptr(), out.data_ptr(), cap, stream=st) == n_sync


def test_noalloc_refuses_beyond_its_scratch(ctx):
    """N = 64, or more than CZ_NOALLOC_MAX_BLOCKS blocks: CZ_ERR_SCRATCH before
    any work (the real, small buffers would be refused by the capacity check
    too, were the scratch check missing)."""
    from paper_1903_07761_amd import _cz

    src = torch.zeros(64 ** 3, dtype=torch.float32, device="cuda")
    out = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    for p in (_cz.params(64, 64, 64, 64, "W4", 4, 0.1), _cz.params(1024, 1024, 1024, 8, "W4", 4, 0.1),
              _cz.params(1024, 1024, 1032, 8, "W4", 4, 0.1)):
        with pytest.raises(_cz.CzError) as e:
            ctx.compress_noalloc(p, src.data_ptr(), out.data_ptr(), out.numel())
        assert e.value.code == _cz.ERR_SCRATCH
    # the largest accepted count: 2^20 blocks of 8^3
    p = _cz.params(1024, 1024, 512, 8, "W4", 4, 0.1)
    with pytest.raises(_cz.CzError) as e:
        ctx.compress_noalloc(p, src.data_ptr(), out.data_ptr(), out.numel())
    assert e.value.code == _cz.ERR_CAPACITY


def test_noalloc_takes_no_device_memory(ctx):
    """A field far beyond the context's initial workspace (32768 blocks)
    leaves the device's free memory unchanged."""
    from paper_1903_07761_amd import _cz, fields

    fresh = _cz.Context(0)
    small = field((64, 64, 64), torch.float32, 1913).cuda()
    big = fields.gaussian_bumps(256, 1914, dtype=torch.float32, device="cuda")
    outs = []
    for f in (small, big):
        p = params_of(f, 8, "W3_ai", 1e-3 * float(f.max() - f.min()))
        cap = _cz.lib().cz_compress_bound(p)
        outs.append((f, p, cap, torch.empty(cap, dtype=torch.uint8, device="cuda")))
    st = torch.cuda.current_stream().cuda_stream
    f, p, cap, out = outs[0]
    fresh.compress_noalloc(p, f.data_ptr(), out.data_ptr(), cap, stream=st)  # warm the code object
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    f, p, cap, out = outs[1]
    n = fresh.compress_noalloc(p, f.data_ptr(), out.data_ptr(), cap, stream=st)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, f"free device memory moved by {free0 - free1} bytes"
    ref = torch.empty(cap, dtype=torch.uint8, device="cuda")
    assert fresh.compress(p, f.data_ptr(), ref.data_ptr(), cap, stream=st) == n
    torch.cuda.synchronize()
    assert torch.equal(out[:n], ref[:n])
    fresh.close()
