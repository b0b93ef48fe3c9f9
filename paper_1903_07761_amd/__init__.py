"""MI355X-native wavelet stage of CubismZ (arXiv 1903.07761).

``codec`` wraps the C ABI of ``libcz.so`` (include/cz.h) for torch tensors:
per-block 3D W4 / W4_li / W3_ai forward transform, decimation at eps, bit
mask + packed coefficient stream, and the inverse; all of it in hand-written
HIP kernels for gfx950.  ``fields`` makes seeded synthetic inputs,
``metrics`` measures PSNR (Eq. 1) and compression ratios, ``lossless`` is the
host zlib back end.
"""
from ._cz import (SCHEMES, W3_AI, W4, W4_LI, Context, CzError, compress_bound, cz_params, params,  # noqa: F401
                  read_header)
