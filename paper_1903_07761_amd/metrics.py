"""Quality and size measures of a compressed field (measurement only).

PSNR follows Eq. (1) of the paper (Sec. 3): 20 log10((max_R - min_R) /
(2 sqrt(MSE))), with the mean square error accumulated in double; +inf when
the reconstruction is exact.  CR is raw bytes over compressed bytes, the
compressed size including all metadata (Sec. 3).
"""
from __future__ import annotations

import math

import torch


def error_stats(ref: torch.Tensor, dec: torch.Tensor, chunk: int = 1 << 26):
    """(PSNR in dB, max |ref - dec|) accumulated chunk by chunk in float64."""
    r = ref.reshape(-1)
    d = dec.reshape(-1)
    lo, hi, sse, mx = math.inf, -math.inf, 0.0, 0.0
    for i in range(0, r.numel(), chunk):
        a = r[i:i + chunk].to(torch.float64)
        b = d[i:i + chunk].to(torch.float64)
        lo = min(lo, float(a.min()))
        hi = max(hi, float(a.max()))
        e = a - b
        sse += float((e * e).sum())
        mx = max(mx, float(e.abs().max()))
    mse = sse / max(1, r.numel())
    psnr = math.inf if mse == 0.0 else 20.0 * math.log10((hi - lo) / (2.0 * math.sqrt(mse)))
    return psnr, mx


def compression_ratio(raw_bytes: int, compressed_bytes: int) -> float:
    return raw_bytes / compressed_bytes if compressed_bytes else math.inf
