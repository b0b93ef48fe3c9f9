"""Batched launches: several fields in one call, captured plans, and the
kernel variants.

Each field of a batch is an independent compression problem (Sec. 2.2: one
quantity at a time), so every batched output must be byte-identical to the
single-field call with the same parameters, and that call is held to the
oracle by the parity tests; one case here also goes straight to the oracle.
Plans are replayed several times with eager work between the replays, each
replay checked against the eager result and against the oracle; the batched
forward and the batched inverse are also compared with the oracle directly.
"""
import numpy as np
import pytest
import torch

from gpu_common import assert_stream_parity, need_gpu, say

pytestmark = pytest.mark.gpu

TDT = {4: torch.float32, 8: torch.float64}


@pytest.fixture(scope="module")
def codec():
    need_gpu()
    from paper_1903_07761_amd.codec import Codec

    return Codec(0)


def mixed_fields(seed: int):
    """A mix of block sizes, precisions, schemes, grid shapes and thresholds,
    including a field without blocks and two fields that share a class."""
    from paper_1903_07761_amd import fields

    rng = np.random.default_rng(seed)
    spec = [
        # (N, elem, scheme, [nz, ny, nx])
        (32, 8, "W3_ai", (64, 32, 96)),
        (32, 8, "W3_ai", (32, 64, 32)),
        (16, 4, "W4_li", (48, 32, 16)),
        (8, 8, "W4", (16, 24, 8)),
        (64, 4, "W4", (64, 64, 128)),
        (32, 4, "W4", (32, 32, 64)),
        (16, 8, "W3_ai", (16, 16, 16)),
        (8, 4, "W4_li", (0, 8, 8)),
    ]
    out = []
    for i, (N, e, s, shape) in enumerate(spec):
        n = max(max(shape), 8)
        if 0 in shape:
            f = torch.empty(shape, dtype=TDT[e])
        elif i % 2:
            f = fields.gaussian_bumps(n, seed + i, dtype=TDT[e])[: shape[0], : shape[1], : shape[2]]
        else:
            f = fields.bubble_cloud(n, seed + i, nbubbles=20, dtype=TDT[e])[: shape[0], : shape[1], : shape[2]]
        f = f.contiguous()
        r = float(f.max() - f.min()) if f.numel() else 1.0
        eps = float(rng.choice([0.0, 1e-4, 1e-3, 1e-2])) * r
        out.append((f.cuda(), N, s, eps))
    return out


def plain_streams(codec, items):
    res = []
    for f, N, s, eps in items:
        buf, n = codec.compress(f, N, s, eps)
        res.append(buf[:n].cpu().numpy().tobytes())
    return res


def test_compress_batch_matches_single_calls(codec):
    items = mixed_fields(7001)
    ref = plain_streams(codec, items)
    outs, sizes = codec.compress_batch(*zip(*[(f, N, s, e) for f, N, s, e in items]))
    for i, (o, n) in enumerate(zip(outs, sizes)):
        say(f"[batch fwd] field {i}: N={items[i][1]} {items[i][2]} {items[i][0].dtype} bytes={n}")
        assert n == len(ref[i])
        assert o[:n].cpu().numpy().tobytes() == ref[i]


def test_compress_batch_async_sizes(codec):
    items = mixed_fields(7002)
    ref = plain_streams(codec, items)
    sizes = torch.zeros(len(items), dtype=torch.int64, device="cuda")
    outs, none = codec.compress_batch(*zip(*[(f, N, s, e) for f, N, s, e in items]), sync=False, out_bytes=sizes)
    assert none is None
    assert codec.status() == 0
    for i, o in enumerate(outs):
        n = int(sizes[i])
        assert n == len(ref[i])
        assert o[:n].cpu().numpy().tobytes() == ref[i]


def test_batch_against_oracle(codec, oracle):
    items = mixed_fields(7003)
    outs, sizes = codec.compress_batch(*zip(*[(f, N, s, e) for f, N, s, e in items]))
    for (f, N, s, eps), o, n in zip(items, outs, sizes):
        ref = oracle.compress(f.cpu().numpy(), N, s, eps)
        say(f"[batch vs oracle] N={N} {s} {f.dtype}: {assert_stream_parity(o[:n].cpu().numpy().tobytes(), ref, eps)}")


def test_decompress_batch_matches_single_calls(codec):
    items = mixed_fields(7004)
    outs, sizes = codec.compress_batch(*zip(*[(f, N, s, e) for f, N, s, e in items]))
    ps = [codec.params(f, N, s, e) for f, N, s, e in items]
    recs = codec.decompress_batch(outs, sizes, ps)
    assert codec.status() == 0
    for i, (o, n) in enumerate(zip(outs, sizes)):
        one = codec.decompress(o, n)
        torch.cuda.synchronize()
        assert recs[i].cpu().numpy().tobytes() == one.cpu().numpy().tobytes()


def test_decompress_batch_against_oracle(codec, oracle):
    """The batched inverse of the oracle's streams equals the oracle's inverse."""
    items = mixed_fields(7008)
    ps = [codec.params(f, N, s, e) for f, N, s, e in items]
    streams = [oracle.compress(f.cpu().numpy(), N, s, e) for f, N, s, e in items]
    bufs = [torch.frombuffer(bytearray(o), dtype=torch.uint8).cuda() if o else torch.empty(0, dtype=torch.uint8,
            device="cuda") for o in streams]
    recs = codec.decompress_batch(bufs, [len(o) for o in streams], ps)
    torch.cuda.synchronize()
    assert codec.status() == 0
    for i, (o, r) in enumerate(zip(streams, recs)):
        want = oracle.decompress(o)
        say(f"[batch inv vs oracle] field {i}: N={items[i][1]} {items[i][2]} {items[i][0].dtype}")
        assert r.cpu().numpy().tobytes() == want.tobytes(), i


def test_decompress_batch_reports_corrupt_stream(codec):
    items = mixed_fields(7005)[:3]
    outs, sizes = codec.compress_batch(*zip(*[(f, N, s, e) for f, N, s, e in items]))
    ps = [codec.params(f, N, s, e) for f, N, s, e in items]
    # point block 1's offset of field 1 beyond the payload: an inconsistent record
    h = outs[1][64 + 8: 64 + 16].clone()
    outs[1][64 + 8: 64 + 16] = torch.tensor([0xFF] * 8, dtype=torch.uint8, device="cuda")
    codec.decompress_batch(outs, sizes, ps)
    from paper_1903_07761_amd import _cz

    assert codec.status() == _cz.ERR_FORMAT
    outs[1][64 + 8: 64 + 16] = h
    codec.decompress_batch(outs, sizes, ps)
    assert codec.status() == 0


def test_compress_batch_nonfinite_and_capacity(codec):
    from paper_1903_07761_amd import _cz

    items = mixed_fields(7006)[:3]
    f1 = items[1][0].clone()
    f1.view(-1)[5] = float("nan")
    items[1] = (f1,) + items[1][1:]
    with pytest.raises(_cz.CzError) as e:
        codec.compress_batch(*zip(*[(f, N, s, eps) for f, N, s, eps in items]))
    assert e.value.code == _cz.ERR_NONFINITE
    assert codec.status() == 0  # the synchronous call consumed the error
    f, N, s, eps = items[0]
    small = [torch.empty(64, dtype=torch.uint8, device="cuda")]
    with pytest.raises(_cz.CzError) as e:
        codec.compress_batch([f], [N], [s], [eps], outs=small)
    assert e.value.code == _cz.ERR_CAPACITY


def test_plan_replays(codec, oracle):
    items = mixed_fields(7007)
    ps = [codec.params(f, N, s, e) for f, N, s, e in items]
    plan = codec.plan("compress", ps)
    inv = codec.plan("decompress", ps)
    from paper_1903_07761_amd import _cz

    bufs = [torch.empty(_cz.compress_bound(p), dtype=torch.uint8, device="cuda") for p in ps]
    recs = [torch.empty_like(f) for f, _, _, _ in items]
    st = torch.cuda.current_stream().cuda_stream
    for rep in range(4):
        # new field values each replay (same parameters), eager work in between
        fs = [(f * (1.0 + 0.25 * rep)).contiguous() for f, _, _, _ in items]
        cur = [(fs[i],) + items[i][1:] for i in range(len(items))]
        ref = plain_streams(codec, cur)
        plan.run([f.data_ptr() for f in fs], [b.data_ptr() for b in bufs], [b.numel() for b in bufs], stream=st)
        sizes = plan.result(stream=st)
        say(f"[plan] replay {rep}: sizes {sizes}")
        for i in range(len(items)):
            assert sizes[i] == len(ref[i])
            got = bufs[i][: sizes[i]].cpu().numpy().tobytes()
            assert got == ref[i], (rep, i)
            f, N, s, eps = cur[i]
            assert got == oracle.compress(f.cpu().numpy(), N, s, eps), ("oracle", rep, i)
        inv.run([b.data_ptr() for b in bufs], [r.data_ptr() for r in recs],
                [r.numel() * r.element_size() for r in recs], src_bytes=sizes, stream=st)
        assert inv.result(stream=st) is None
        for i in range(len(items)):
            one = codec.decompress(bufs[i], sizes[i])
            torch.cuda.synchronize()
            assert recs[i].cpu().numpy().tobytes() == one.cpu().numpy().tobytes(), (rep, i)
            want = oracle.decompress(bufs[i][: sizes[i]].cpu().numpy().tobytes()) if sizes[i] else None
            if want is not None:
                assert recs[i].cpu().numpy().tobytes() == want.tobytes(), ("oracle", rep, i)
    plan.close()
    inv.close()


@pytest.mark.parametrize("N,elem", [(8, 4), (8, 8), (16, 4), (16, 8), (32, 4), (32, 8), (64, 4), (64, 8)])
def test_variants_identical(codec, oracle, N, elem):
    from paper_1903_07761_amd import _cz, fields

    nv = _cz.variant_count(N, elem)
    assert nv >= 1
    n = max(2 * N, 64)
    f = fields.bubble_cloud(n, 7100 + N, nbubbles=20, dtype=TDT[elem])[:N, :, :].contiguous().cuda()
    for s in ("W4", "W4_li", "W3_ai"):
        eps = 1e-3 * float(f.max() - f.min())
        ref = oracle.compress(f.cpu().numpy(), N, s, eps)
        for v in range(nv):
            codec.set_variant(N, TDT[elem], s, v)
            buf, nb = codec.compress(f, N, s, eps)
            g = buf[:nb].cpu().numpy().tobytes()
            assert g == ref, (s, v)
            rec = codec.decompress(buf, nb)
            torch.cuda.synchronize()
            assert np.array_equal(rec.cpu().numpy(), oracle.decompress(ref)), (s, v)
        codec.set_variant(N, TDT[elem], s, 0)
    with pytest.raises(_cz.CzError):
        codec.set_variant(N, TDT[elem], "W4", nv)
