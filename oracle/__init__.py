"""CPU oracle of the CubismZ wavelet stage -- TEST INFRASTRUCTURE ONLY.

Plain single-threaded C (``cz_oracle.c``) built with gcc, loaded through
ctypes.  Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` may import this package; the product library
(``paper_1903_07761_amd``) never does, and the two share no code.

The C source states, with citations of the paper (arXiv 1903.07761, Sec. 2.3
and Eq. 1), what each routine computes and which readings of the paper it
takes where the paper is silent.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libczoracle.so")
SOURCES = [os.path.join(HERE, "cz_oracle.c")]
DEPS = SOURCES + [os.path.join(HERE, "cz_oracle_t.h")]
# Timing build for the benchmark's all-cores CPU baseline: the same oracle
# routines under an OpenMP parallel-for over blocks (cz_oracle_omp.c).
PAR_LIB_PATH = os.path.join(HERE, "libczoracle_omp.so")
PAR_SOURCES = SOURCES + [os.path.join(HERE, "cz_oracle_omp.c")]

# gcc flags: IEEE arithmetic exactly as written (no contraction into FMA, no
# fast-math reassociation, no flush-to-zero).
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra"]

W4, W4LI, W3AI = 0, 1, 2
SCHEMES = {"W4": W4, "W4_li": W4LI, "W3_ai": W3AI}

OK, ERR_ARG, ERR_SHAPE, ERR_CAPACITY, ERR_NONFINITE, ERR_FORMAT = 0, -1, -2, -3, -4, -5


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile the oracle into ``libczoracle.so`` next to its source."""
    if not force and os.path.exists(LIB_PATH):
        newest = max(os.path.getmtime(p) for p in DEPS)
        if os.path.getmtime(LIB_PATH) >= newest:
            return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    subprocess.run(["gcc", *CFLAGS, *SOURCES, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, LIB_PATH)
    tmp = PAR_LIB_PATH + ".tmp"
    subprocess.run(["gcc", *CFLAGS, "-fopenmp", *PAR_SOURCES, "-o", tmp, "-lm"], check=True)
    os.replace(tmp, PAR_LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, u32, u64, i32, f64 = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32,
                                      ctypes.c_uint64, ctypes.c_int, ctypes.c_double)
        L.czo_compress_bound.argtypes = [u32, u32, u32, i32, i32]
        L.czo_compress_bound.restype = sz
        L.czo_psnr.argtypes = [vp, vp, sz, i32]
        L.czo_psnr.restype = f64
        for s in ("f32", "f64"):
            for fn in ("czo_fwd1", "czo_inv1"):
                f = getattr(L, f"{fn}_{s}")
                f.argtypes = [i32, i32, vp, vp]
                f.restype = None
            for fn in ("czo_fwd_line", "czo_inv_line", "czo_fwd_block", "czo_inv_block"):
                f = getattr(L, f"{fn}_{s}")
                f.argtypes = [i32, i32, vp]
                f.restype = None
            f = getattr(L, f"czo_compress_{s}")
            f.argtypes = [u32, u32, u32, i32, i32, f64, vp, vp, sz, ctypes.POINTER(sz)]
            f.restype = i32
            f = getattr(L, f"czo_decompress_{s}")
            f.argtypes = [vp, sz, vp, sz]
            f.restype = i32
            f = getattr(L, f"czo_compress_blocks_{s}")
            f.argtypes = [u32, u32, u32, i32, i32, f64, vp, u64, u64, vp, vp]
            f.restype = i32
            f = getattr(L, f"czo_decompress_blocks_{s}")
            f.argtypes = [u32, u32, u32, i32, i32, vp, vp, u64, u64, vp]
            f.restype = i32
        _lib = L
    return _lib


def _sfx(dtype) -> str:
    dt = np.dtype(dtype)
    if dt == np.float32:
        return "f32"
    if dt == np.float64:
        return "f64"
    raise TypeError(f"oracle supports float32/float64, not {dt}")


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _scheme(scheme) -> int:
    return SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)


def fwd1(scheme, v: np.ndarray) -> np.ndarray:
    """One forward level of a 1D line: returns [coarse | details]."""
    v = np.ascontiguousarray(v)
    out = np.empty_like(v)
    getattr(lib(), f"czo_fwd1_{_sfx(v.dtype)}")(_scheme(scheme), v.size, _ptr(v), _ptr(out))
    return out


def inv1(scheme, w: np.ndarray) -> np.ndarray:
    w = np.ascontiguousarray(w)
    out = np.empty_like(w)
    getattr(lib(), f"czo_inv1_{_sfx(w.dtype)}")(_scheme(scheme), w.size, _ptr(w), _ptr(out))
    return out


def fwd_line(scheme, v: np.ndarray) -> np.ndarray:
    """Full-depth 1D transform (levels n, n/2, ..., 8)."""
    v = np.array(v, copy=True, order="C")
    getattr(lib(), f"czo_fwd_line_{_sfx(v.dtype)}")(_scheme(scheme), v.size, _ptr(v))
    return v


def inv_line(scheme, w: np.ndarray) -> np.ndarray:
    w = np.array(w, copy=True, order="C")
    getattr(lib(), f"czo_inv_line_{_sfx(w.dtype)}")(_scheme(scheme), w.size, _ptr(w))
    return w


def fwd_block(scheme, block: np.ndarray) -> np.ndarray:
    """Forward 3D multilevel transform of one block indexed [z, y, x]."""
    b = np.array(block, copy=True, order="C")
    assert b.ndim == 3 and b.shape[0] == b.shape[1] == b.shape[2]
    getattr(lib(), f"czo_fwd_block_{_sfx(b.dtype)}")(_scheme(scheme), b.shape[0], _ptr(b))
    return b


def inv_block(scheme, coef: np.ndarray) -> np.ndarray:
    b = np.array(coef, copy=True, order="C")
    getattr(lib(), f"czo_inv_block_{_sfx(b.dtype)}")(_scheme(scheme), b.shape[0], _ptr(b))
    return b


def compress_bound(shape, block: int, elem_bytes: int) -> int:
    nz, ny, nx = shape
    return int(lib().czo_compress_bound(nx, ny, nz, block, elem_bytes))


def compress(field: np.ndarray, block: int, scheme, epsilon: float) -> bytes:
    """Compress a C-order [nz, ny, nx] field into a stream (bytes)."""
    f = np.ascontiguousarray(field)
    nz, ny, nx = f.shape
    cap = max(compress_bound(f.shape, block, f.dtype.itemsize), 64)
    out = np.full(cap, 0xA5, dtype=np.uint8)  # garbage: every byte must be written
    nbytes = ctypes.c_size_t(0)
    rc = getattr(lib(), f"czo_compress_{_sfx(f.dtype)}")(
        nx, ny, nz, block, _scheme(scheme), float(epsilon), _ptr(f), _ptr(out), cap, ctypes.byref(nbytes))
    if rc != OK:
        raise OracleError(rc, "compress")
    return out[: nbytes.value].tobytes()


def decompress(stream: bytes, dtype=None) -> np.ndarray:
    """Rebuild the [nz, ny, nx] field from a stream."""
    buf = np.frombuffer(stream, dtype=np.uint8)
    if buf.size < 64:
        raise OracleError(ERR_FORMAT, "decompress")
    hdr = buf[:64].view(np.uint32)
    elem = int(hdr[3])
    nx, ny, nz = int(hdr[6]), int(hdr[7]), int(hdr[8])
    dt = dtype or (np.float32 if elem == 4 else np.float64)
    field = np.zeros((nz, ny, nx), dtype=dt)
    rc = getattr(lib(), f"czo_decompress_{_sfx(dt)}")(_ptr(buf), buf.size, _ptr(field), field.size)
    if rc != OK:
        raise OracleError(rc, "decompress")
    return field


def record_bound(block: int, elem_bytes: int) -> int:
    n3 = block ** 3
    return (8 + n3 // 8 + n3 * elem_bytes + 15) // 16 * 16


def compress_blocks(field: np.ndarray, block: int, scheme, epsilon: float, b0: int, b1: int):
    """Records of blocks [b0, b1) of the field: (records array at record-bound
    strides, per-record byte counts)."""
    f = np.ascontiguousarray(field)
    nz, ny, nx = f.shape
    rb = record_bound(block, f.dtype.itemsize)
    recs = np.zeros((b1 - b0) * rb, dtype=np.uint8)
    sizes = np.zeros(b1 - b0, dtype=np.uint64)
    rc = getattr(lib(), f"czo_compress_blocks_{_sfx(f.dtype)}")(
        nx, ny, nz, block, _scheme(scheme), float(epsilon), _ptr(f), b0, b1, _ptr(recs), _ptr(sizes))
    if rc != OK:
        raise OracleError(rc, "compress_blocks")
    return recs, sizes


def decompress_blocks(recs: np.ndarray, sizes: np.ndarray, shape, block: int, scheme, b0: int, b1: int,
                      out: np.ndarray) -> np.ndarray:
    nz, ny, nx = shape
    rc = getattr(lib(), f"czo_decompress_blocks_{_sfx(out.dtype)}")(
        nx, ny, nz, block, _scheme(scheme), _ptr(recs), _ptr(sizes), b0, b1, _ptr(out))
    if rc != OK:
        raise OracleError(rc, "decompress_blocks")
    return out


_par = None


def par_lib() -> ctypes.CDLL:
    """The OpenMP timing build (built by build())."""
    global _par
    if _par is None:
        if not os.path.exists(PAR_LIB_PATH):
            build()
        L = ctypes.CDLL(PAR_LIB_PATH)
        vp, u32, u64, i32, f64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        L.czo_par_max_threads.argtypes = []
        L.czo_par_max_threads.restype = i32
        for s in ("f32", "f64"):
            f = getattr(L, f"czo_compress_blocks_par_{s}")
            f.argtypes = [u32, u32, u32, i32, i32, f64, vp, u64, u64, vp, vp, i32]
            f.restype = i32
            f = getattr(L, f"czo_decompress_blocks_par_{s}")
            f.argtypes = [u32, u32, u32, i32, i32, vp, vp, u64, u64, vp, i32]
            f.restype = i32
        _par = L
    return _par


def par_max_threads() -> int:
    """Threads an OpenMP region takes by default (OMP_NUM_THREADS, else the cores)."""
    return int(par_lib().czo_par_max_threads())


def compress_blocks_par(field: np.ndarray, block: int, scheme, epsilon: float, b0: int, b1: int, threads: int):
    """compress_blocks on `threads` OpenMP threads (chunks of blocks per
    thread); the same records and sizes."""
    f = np.ascontiguousarray(field)
    nz, ny, nx = f.shape
    rb = record_bound(block, f.dtype.itemsize)
    recs = np.zeros((b1 - b0) * rb, dtype=np.uint8)
    sizes = np.zeros(b1 - b0, dtype=np.uint64)
    rc = getattr(par_lib(), f"czo_compress_blocks_par_{_sfx(f.dtype)}")(
        nx, ny, nz, block, _scheme(scheme), float(epsilon), _ptr(f), b0, b1, _ptr(recs), _ptr(sizes), threads)
    if rc != OK:
        raise OracleError(rc, "compress_blocks_par")
    return recs, sizes


def decompress_blocks_par(recs: np.ndarray, sizes: np.ndarray, shape, block: int, scheme, b0: int, b1: int,
                          out: np.ndarray, threads: int) -> np.ndarray:
    nz, ny, nx = shape
    rc = getattr(par_lib(), f"czo_decompress_blocks_par_{_sfx(out.dtype)}")(
        nx, ny, nz, block, _scheme(scheme), _ptr(recs), _ptr(sizes), b0, b1, _ptr(out), threads)
    if rc != OK:
        raise OracleError(rc, "decompress_blocks_par")
    return out


def psnr(ref: np.ndarray, dec: np.ndarray) -> float:
    """Eq. (1) of the paper, accumulated in double."""
    r = np.ascontiguousarray(ref)
    d = np.ascontiguousarray(dec, dtype=r.dtype)
    return float(lib().czo_psnr(_ptr(r), _ptr(d), r.size, r.dtype.itemsize))
