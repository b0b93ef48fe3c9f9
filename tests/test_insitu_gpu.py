"""In-situ extraction: compressing one quantity straight from an interleaved
state with strided loads gives the stream of the extracted field, byte for
byte, and that stream is the oracle's."""
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


@pytest.mark.parametrize("N,dt,shape,ncomp", [(8, np.float64, (16, 8, 24), 3), (16, np.float32, (32, 16, 48), 5),
                                               (32, np.float32, (32, 64, 64), 7), (32, np.float64, (64, 32, 32), 5),
                                               (64, np.float64, (64, 64, 128), 4)])
def test_strided_matches_extracted_field(codec, oracle, N, dt, shape, ncomp):
    from paper_1903_07761_amd import fields

    n = max(shape)
    comps = []
    for k in range(ncomp):
        g = fields.bubble_cloud(n, 80 + k, nbubbles=15, dtype=TDT[dt]) if k % 2 else \
            fields.gaussian_bumps(n, 80 + k, dtype=TDT[dt])
        comps.append(g[: shape[0], : shape[1], : shape[2]])
    state = torch.stack(comps, dim=-1).contiguous().cuda()  # [nz, ny, nx, ncomp]
    for comp in (0, ncomp // 2, ncomp - 1):
        f = state[..., comp].contiguous()
        for scheme in ("W4", "W3_ai"):
            eps = 1e-3 * float(f.max() - f.min())
            a, na = codec.compress_component(state, comp, N, scheme, eps)
            b, nb = codec.compress(f, N, scheme, eps)
            assert na == nb and torch.equal(a[:na], b[:nb]), (comp, scheme)
            if comp == ncomp // 2 and scheme == "W3_ai":
                ref = oracle.compress(f.cpu().numpy(), N, scheme, eps)
                assert a[:na].cpu().numpy().tobytes() == ref
    say(f"[in situ] N={N} {np.dtype(dt).name} ncomp={ncomp} ok")


def test_strided_argument_errors(codec):
    from paper_1903_07761_amd import _cz

    state = torch.zeros((16, 16, 16, 3), dtype=torch.float32, device="cuda")
    for comp in (3, 7):
        with pytest.raises(_cz.CzError) as e:
            codec.compress_component(state, comp, 16, "W4", 0.0)
        assert e.value.code == _cz.ERR_ARG
