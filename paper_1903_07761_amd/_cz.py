"""ctypes binding of libcz (include/cz.h): argument marshalling only.

Every step of the wavelet stage runs in the HIP kernels of libcz.so; this
module passes device pointers, sizes and the HIP stream through, and raises
``CzError`` on a non-zero status.  It fails loudly when the library has not
been built (``python -m paper_1903_07761_amd.build``).
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libcz.so")

W4, W4_LI, W3_AI = 0, 1, 2
SCHEMES = {"W4": W4, "W4_li": W4_LI, "W3_ai": W3_AI}

OK, ERR_ARG, ERR_SHAPE, ERR_CAPACITY, ERR_NONFINITE, ERR_FORMAT, ERR_HIP, ERR_BUDGET, ERR_TIMEOUT = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)


class cz_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_uint32), ("ny", ctypes.c_uint32), ("nz", ctypes.c_uint32),
                ("block", ctypes.c_uint32), ("scheme", ctypes.c_uint32), ("elem_bytes", ctypes.c_uint32),
                ("epsilon", ctypes.c_double)]


class CzError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str = ""):
        super().__init__(f"{what}: {strerror(code)} ({code}){' ' + detail if detail else ''}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libcz.so is not built at {LIB_PATH}; run python -m paper_1903_07761_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32, u64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_uint64
        P = ctypes.POINTER(cz_params)
        L.cz_create.argtypes = [ctypes.POINTER(vp), i32]
        L.cz_create.restype = i32
        L.cz_destroy.argtypes = [vp]
        L.cz_destroy.restype = None
        L.cz_reserve.argtypes = [vp, u64]
        L.cz_reserve.restype = i32
        L.cz_compress_bound.argtypes = [P]
        L.cz_compress_bound.restype = sz
        L.cz_compress.argtypes = [vp, P, vp, vp, sz, vp, ctypes.POINTER(sz), vp]
        L.cz_compress.restype = i32
        L.cz_decompress.argtypes = [vp, P, vp, sz, vp, sz, vp]
        L.cz_decompress.restype = i32
        L.cz_get_status.argtypes = [vp, vp]
        L.cz_get_status.restype = i32
        L.cz_read_header.argtypes = [vp, sz, P, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.cz_read_header.restype = i32
        L.cz_strerror.argtypes = [i32]
        L.cz_strerror.restype = ctypes.c_char_p
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().cz_strerror(code).decode()
    except ImportError:
        return f"error {code}"


def _check(rc: int, what: str):
    if rc != OK:
        raise CzError(rc, what)


def params(nx, ny, nz, block, scheme, elem_bytes, epsilon) -> cz_params:
    s = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    return cz_params(nx, ny, nz, block, s, elem_bytes, float(epsilon))


class Context:
    """Owns a libcz context (device workspace) on one HIP device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().cz_create(ctypes.byref(h), device), "cz_create")
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().cz_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, max_blocks: int):
        _check(lib().cz_reserve(self.handle, max_blocks), "cz_reserve")

    def compress(self, p: cz_params, d_field: int, d_out: int, out_cap: int, stream: int = 0,
                 d_out_bytes: int | None = None, sync: bool = True) -> int | None:
        """cz_compress; returns the stream size when sync."""
        nbytes = ctypes.c_size_t(0)
        rc = lib().cz_compress(self.handle, ctypes.byref(p), d_field, d_out, out_cap, d_out_bytes,
                               ctypes.byref(nbytes) if sync else None, stream)
        if rc != OK:
            raise CzError(rc, "cz_compress", f"(required {nbytes.value} bytes)" if rc == ERR_CAPACITY else "")
        return nbytes.value if sync else None

    def decompress(self, d_in: int, in_bytes: int, d_field: int, field_cap: int, stream: int = 0,
                   expected: cz_params | None = None):
        rc = lib().cz_decompress(self.handle, ctypes.byref(expected) if expected is not None else None, d_in,
                                 in_bytes, d_field, field_cap, stream)
        _check(rc, "cz_decompress")

    def get_status(self, stream: int = 0) -> int:
        return lib().cz_get_status(self.handle, stream)


def compress_bound(p: cz_params) -> int:
    return int(lib().cz_compress_bound(ctypes.byref(p)))


def read_header(hdr: bytes):
    """Parse a host copy of a stream header -> (params, nblocks, total bytes)."""
    buf = ctypes.create_string_buffer(bytes(hdr[:64]), 64)
    p = cz_params()
    nb, tot = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(lib().cz_read_header(buf, 64, ctypes.byref(p), ctypes.byref(nb), ctypes.byref(tot)), "cz_read_header")
    return p, nb.value, tot.value
