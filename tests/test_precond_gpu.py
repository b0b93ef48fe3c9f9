"""GPU preconditioning (byte shuffle, Z4/Z8 zeroing) against the oracle:
byte-identical outputs on the same inputs."""
import numpy as np
import pytest
import torch

from gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def codec():
    need_gpu()
    from paper_1903_07761_amd.codec import Codec

    return Codec(0)


@pytest.mark.parametrize("elem", [4, 8])
def test_shuffle_matches_oracle(codec, elem):
    from oracle import precond

    rng = np.random.default_rng(elem)
    for n in (0, 1, elem - 1, elem, 7 * elem + 3, 4099, 1 << 20, (1 << 20) + 5):
        host = rng.integers(0, 256, n, dtype=np.uint8)
        dev = torch.from_numpy(host).cuda()
        out = codec.shuffle(dev, n, elem)
        back = codec.unshuffle(out, n, elem)
        torch.cuda.synchronize()
        ref = precond.shuffle(host.tobytes(), elem)
        assert out.cpu().numpy().tobytes() == ref, n
        assert back.cpu().numpy().tobytes() == host.tobytes(), n
    say(f"[shuffle] elem {elem} ok")


@pytest.mark.parametrize("elem", [4, 8])
def test_shuffle_alignments(codec, elem):
    """Element counts of every residue mod 4 (planes starting at every
    alignment), inputs that are element- but not 16-byte-aligned, and outputs
    at odd addresses: the word-wide plane accesses fall back to narrower ones
    and the results stay byte-identical to the oracle's."""
    from oracle import precond
    from paper_1903_07761_amd import _cz

    rng = np.random.default_rng(100 + elem)
    for nel in (4097, 4098, 4099, 4100, 65541):
        nbytes = nel * elem + 3  # three tail bytes as well
        host = rng.integers(0, 256, nbytes, dtype=np.uint8)
        ref = precond.shuffle(host.tobytes(), elem)
        for in_off, out_off in ((0, 0), (elem, 1), (elem, 2), (0, 3)):
            src = torch.zeros(nbytes + 32, dtype=torch.uint8, device="cuda")
            src[in_off:in_off + nbytes] = torch.from_numpy(host).cuda()
            dst = torch.zeros(nbytes + 32, dtype=torch.uint8, device="cuda")
            _cz.shuffle(src.data_ptr() + in_off, nbytes, elem, dst.data_ptr() + out_off)
            torch.cuda.synchronize()
            got = dst[out_off:out_off + nbytes].cpu().numpy().tobytes()
            assert got == ref, (nel, in_off, out_off)
            # unshuffle from a plane buffer at an odd offset into an element-aligned output
            back = torch.zeros(nbytes + 32, dtype=torch.uint8, device="cuda")
            _cz.unshuffle(dst.data_ptr() + out_off, nbytes, elem, back.data_ptr() + in_off)
            torch.cuda.synchronize()
            assert back[in_off:in_off + nbytes].cpu().numpy().tobytes() == host.tobytes(), (nel, in_off, out_off)
    say(f"[shuffle] elem {elem} alignments ok")


def test_shuffle_rejects_bad_arguments(codec):
    from paper_1903_07761_amd import _cz

    a = torch.zeros(64, dtype=torch.uint8, device="cuda")
    b = torch.zeros(64, dtype=torch.uint8, device="cuda")
    for args in ((a.data_ptr(), 64, 3, b.data_ptr()), (a.data_ptr(), 64, 4, a.data_ptr()),
                 (a.data_ptr() + 1, 60, 4, b.data_ptr())):
        with pytest.raises(_cz.CzError) as e:
            _cz.shuffle(*args)
        assert e.value.code == _cz.ERR_ARG


@pytest.mark.parametrize("N,dt", [(8, np.float32), (16, np.float64), (32, np.float32), (32, np.float64),
                                  (64, np.float32)])
@pytest.mark.parametrize("bits", [4, 8])
def test_zero_details_matches_oracle(codec, oracle, N, dt, bits):
    from oracle import precond
    from paper_1903_07761_amd import fields

    n = max(2 * N, 64)
    f = fields.bubble_cloud(n, 31 + N, nbubbles=20, dtype=torch.float32 if dt == np.float32 else torch.float64)
    f = f[:N].contiguous().cuda()
    eps = 1e-3 * float(f.max() - f.min())
    buf, nb = codec.compress(f, N, "W3_ai", eps)
    stream = buf[:nb].cpu().numpy().tobytes()
    p = codec.params(f, N, "W3_ai", eps)
    codec.zero_details(buf, nb, p, bits)
    assert codec.status() == 0
    got = buf[:nb].cpu().numpy().tobytes()
    assert got == precond.zero_details(stream, bits)
    # the zeroed stream still decodes
    rec = codec.decompress(buf, nb)
    torch.cuda.synchronize()
    assert np.array_equal(rec.cpu().numpy(), oracle.decompress(got))


def test_zero_details_errors(codec):
    from paper_1903_07761_amd import _cz, fields

    f = fields.gaussian_bumps(32, 2, dtype=torch.float32).cuda()
    buf, nb = codec.compress(f, 16, "W4", 1e-3)
    p = codec.params(f, 16, "W4", 1e-3)
    with pytest.raises(_cz.CzError) as e:
        codec.zero_details(buf, nb, p, 24)
    assert e.value.code == _cz.ERR_ARG
    bad = buf.clone()
    bad[64 + 8: 64 + 16] = torch.tensor([0xFF] * 8, dtype=torch.uint8, device="cuda")
    codec.zero_details(bad, nb, p, 4)
    assert codec.status() == _cz.ERR_FORMAT
    assert codec.status() == 0
