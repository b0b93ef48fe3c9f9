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
    def __init__(self, device: int = 0, tuned: bool = True):
        """tuned: select the kernel variants recorded for this device's
        architecture by the autotuner, when a table exists (outputs do not
        depend on the variant)."""
        if not torch.cuda.is_available():
            raise RuntimeError("the wavelet stage runs on a HIP device; none is available")
        self.device = torch.device("cuda", device)
        self.ctx = _cz.Context(device)
        self.tuned = 0
        if tuned:
            from . import autotune

            self.tuned = autotune.apply(self)

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

    def compress_component(self, state: torch.Tensor, comp: int, block: int, scheme, epsilon: float,
                           out: torch.Tensor | None = None):
        """Compress quantity `comp` of a contiguous interleaved state
        [nz, ny, nx, ncomp] straight from the state.  Returns (buffer, size)."""
        assert state.is_cuda and state.is_contiguous() and state.dim() == 4
        nz, ny, nx, ncomp = state.shape
        p = _cz.params(nx, ny, nz, block, scheme, _ELEM[state.dtype], epsilon)
        cap = _cz.compress_bound(p)
        if out is None:
            out = torch.empty(cap, dtype=torch.uint8, device=state.device)
        n = self.ctx.compress_strided(p, state.data_ptr(), ncomp, comp, out.data_ptr(), out.numel(),
                                      _stream_handle(state.device))
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

    def set_variant(self, block: int, dtype, scheme, variant: int):
        self.ctx.set_variant(block, _ELEM[dtype], scheme, variant)

    def batch_params(self, fields, blocks, schemes, epsilons):
        return [self.params(f, b, s, e) for f, b, s, e in zip(fields, blocks, schemes, epsilons)]

    def compress_batch(self, fields, blocks, schemes, epsilons, outs=None, sync: bool = True,
                       out_bytes: torch.Tensor | None = None):
        """Compress several contiguous [nz, ny, nx] device fields in one call.
        Returns (stream buffers, sizes or None)."""
        for f in fields:
            assert f.is_cuda and f.is_contiguous() and f.dim() == 3
        ps = self.batch_params(fields, blocks, schemes, epsilons)
        if outs is None:
            outs = [torch.empty(_cz.compress_bound(p), dtype=torch.uint8, device=self.device) for p in ps]
        sizes = self.ctx.compress_batch(ps, [f.data_ptr() for f in fields], [o.data_ptr() for o in outs],
                                        [o.numel() for o in outs], _stream_handle(self.device),
                                        out_bytes.data_ptr() if out_bytes is not None else None, sync)
        return outs, sizes

    def decompress_batch(self, bufs, nbytes, ps, outs=None):
        """Rebuild several fields; ps[i] are the parameters the stream was made with."""
        if outs is None:
            outs = [torch.empty((p.nz, p.ny, p.nx), dtype=_DTYPE[p.elem_bytes], device=self.device) for p in ps]
        self.ctx.decompress_batch(ps, [b.data_ptr() for b in bufs], list(nbytes), [o.data_ptr() for o in outs],
                                  [o.numel() * o.element_size() for o in outs], _stream_handle(self.device))
        return outs

    def shuffle(self, buf: torch.Tensor, nbytes: int, elem: int = 4, out: torch.Tensor | None = None):
        """Byte-shuffle the first nbytes of a device buffer (element size elem)."""
        if out is None:
            out = torch.empty(nbytes, dtype=torch.uint8, device=buf.device)
        _cz.shuffle(buf.data_ptr(), nbytes, elem, out.data_ptr(), _stream_handle(buf.device))
        return out

    def unshuffle(self, buf: torch.Tensor, nbytes: int, elem: int = 4, out: torch.Tensor | None = None):
        if out is None:
            out = torch.empty(nbytes, dtype=torch.uint8, device=buf.device)
        _cz.unshuffle(buf.data_ptr(), nbytes, elem, out.data_ptr(), _stream_handle(buf.device))
        return out

    def zero_details(self, buf: torch.Tensor, nbytes: int, p: _cz.cz_params, bits: int):
        """Z-zeroing of the detail coefficients of a device stream, in place."""
        self.ctx.zero_details(p, buf.data_ptr(), nbytes, bits, _stream_handle(buf.device))
        return buf

    def decompress_blocks(self, buf: torch.Tensor, nbytes: int, p: _cz.cz_params, blocks,
                          out: torch.Tensor | None = None) -> torch.Tensor:
        """Decode the listed blocks of a device stream into [n, N, N, N]."""
        N = p.block
        if out is None:
            out = torch.empty((len(blocks), N, N, N), dtype=_DTYPE[p.elem_bytes], device=buf.device)
        self.ctx.decompress_blocks(p, buf.data_ptr(), nbytes, list(blocks), out.data_ptr(),
                                   out.numel() * out.element_size(), _stream_handle(buf.device))
        return out

    def cache(self, p: _cz.cz_params, capacity_blocks: int) -> _cz.Cache:
        return _cz.Cache(self.ctx, p, capacity_blocks)

    def region(self, cache: _cz.Cache, buf: torch.Tensor, nbytes: int, p: _cz.cz_params, origin, extent,
               out: torch.Tensor | None = None) -> torch.Tensor:
        """Decode the box origin (x, y, z) + extent of the field through a cache;
        returns [ez, ey, ex]."""
        ex, ey, ez = extent
        if out is None:
            out = torch.empty((ez, ey, ex), dtype=_DTYPE[p.elem_bytes], device=buf.device)
        cache.region(buf.data_ptr(), nbytes, list(origin), list(extent), out.data_ptr(),
                     out.numel() * out.element_size(), _stream_handle(buf.device))
        return out

    def huff_encode(self, buf: torch.Tensor, nbytes: int):
        """GPU lossless stage: returns (container buffer, size)."""
        out = torch.empty(_cz.huff_bound(nbytes), dtype=torch.uint8, device=buf.device)
        n = self.ctx.huff_encode(buf.data_ptr(), nbytes, out.data_ptr(), out.numel(), _stream_handle(buf.device))
        return out, n

    def huff_decode(self, buf: torch.Tensor, nbytes: int, raw_bytes: int, out: torch.Tensor | None = None):
        if out is None:
            out = torch.empty(max(raw_bytes, 1), dtype=torch.uint8, device=buf.device)
        self.ctx.huff_decode(buf.data_ptr(), nbytes, out.data_ptr(), out.numel(), _stream_handle(buf.device))
        return out

    def plan(self, op: str, ps) -> _cz.Plan:
        return _cz.Plan(self.ctx, op, ps)
