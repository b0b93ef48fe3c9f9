"""torch-facing wrapper of the libcz C ABI: tensors in, tensors out.

The tensors only carry device memory and the current HIP stream; every step
of compression and decompression runs in libcz's kernels.
"""
from __future__ import annotations

import torch

from . import _cz

_ELEM = {torch.float32: 4, torch.float64: 8}
_DTYPE = {4: torch.float32, 8: torch.float64}


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Codec:
    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the wavelet stage runs on a HIP device; none is available")
        self.device = torch.device("cuda", device)
        self.ctx = _cz.Context(device)

    def params(self, field: torch.Tensor, block: int, scheme, epsilon: float) -> _cz.cz_params:
        nz, ny, nx = field.shape
        return _cz.params(nx, ny, nz, block, scheme, _ELEM[field.dtype], epsilon)

    def bound(self, shape, dtype, block: int) -> int:
        nz, ny, nx = shape
        return _cz.compress_bound(_cz.params(nx, ny, nz, block, 0, _ELEM[dtype], 0.0))

    def compress(self, field: torch.Tensor, block: int, scheme, epsilon: float, out: torch.Tensor | None = None,
                 sync: bool = True, out_bytes: torch.Tensor | None = None):
        """Compress a contiguous [nz, ny, nx] device field.  Returns
        (stream buffer, size in bytes) when sync, else (buffer, None)."""
        assert field.is_cuda and field.is_contiguous() and field.dim() == 3
        p = self.params(field, block, scheme, epsilon)
        cap = _cz.compress_bound(p)
        if cap == 0:
            raise _cz.CzError(_cz.ERR_SHAPE, "cz_compress_bound")
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=field.device)
        n = self.ctx.compress(p, field.data_ptr(), out.data_ptr(), out.numel(), _stream_handle(field.device),
                              out_bytes.data_ptr() if out_bytes is not None else None, sync)
        return out, n

    def decompress(self, stream_buf: torch.Tensor, nbytes: int, out: torch.Tensor | None = None,
                   expected: _cz.cz_params | None = None) -> torch.Tensor:
        """Rebuild the field from a device stream (header read back unless
        `expected` gives its parameters)."""
        assert stream_buf.is_cuda and stream_buf.dtype == torch.uint8
        if out is None:
            if expected is None:
                hdr = stream_buf[:64].cpu().numpy().tobytes()
                p, _, _ = _cz.read_header(hdr)
            else:
                p = expected
            out = torch.empty((p.nz, p.ny, p.nx), dtype=_DTYPE[p.elem_bytes], device=stream_buf.device)
        self.ctx.decompress(stream_buf.data_ptr(), nbytes, out.data_ptr(), out.numel() * out.element_size(),
                            _stream_handle(stream_buf.device), expected)
        return out

    def status(self) -> int:
        return self.ctx.get_status(_stream_handle(self.device))
