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

OK, ERR_ARG, ERR_SHAPE, ERR_CAPACITY, ERR_NONFINITE, ERR_FORMAT, ERR_HIP, ERR_BUDGET, ERR_TIMEOUT, ERR_SCRATCH = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)
NOALLOC_MAX_BLOCKS = 1 << 20


class cz_params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_uint32), ("ny", ctypes.c_uint32), ("nz", ctypes.c_uint32),
                ("block", ctypes.c_uint32), ("scheme", ctypes.c_uint32), ("elem_bytes", ctypes.c_uint32),
                ("epsilon", ctypes.c_double)]


class cz_request(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int), ("p", cz_params), ("d_src", ctypes.c_void_p), ("src_bytes", ctypes.c_size_t),
                ("d_dst", ctypes.c_void_p), ("dst_cap", ctypes.c_size_t), ("user_tag", ctypes.c_uint64)]


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
        L.cz_compress_noalloc.argtypes = [vp, P, vp, vp, sz, vp, ctypes.POINTER(sz), vp]
        L.cz_compress_noalloc.restype = i32
        L.cz_compress_strided.argtypes = [vp, P, vp, ctypes.c_uint32, ctypes.c_uint32, vp, sz, vp,
                                          ctypes.POINTER(sz), vp]
        L.cz_compress_strided.restype = i32
        L.cz_decompress.argtypes = [vp, P, vp, sz, vp, sz, vp]
        L.cz_decompress.restype = i32
        L.cz_get_status.argtypes = [vp, vp]
        L.cz_get_status.restype = i32
        L.cz_read_header.argtypes = [vp, sz, P, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.cz_read_header.restype = i32
        L.cz_strerror.argtypes = [i32]
        L.cz_strerror.restype = ctypes.c_char_p
        u32, PP = ctypes.c_uint32, ctypes.POINTER(vp)
        PS = ctypes.POINTER(sz)
        L.cz_variant_count.argtypes = [u32, u32]
        L.cz_variant_count.restype = i32
        L.cz_set_variant.argtypes = [vp, u32, u32, u32, i32]
        L.cz_set_variant.restype = i32
        L.cz_compress_batch.argtypes = [vp, i32, P, PP, PP, PS, vp, PS, vp]
        L.cz_compress_batch.restype = i32
        L.cz_decompress_batch.argtypes = [vp, i32, P, PP, PS, PP, PS, vp]
        L.cz_decompress_batch.restype = i32
        L.cz_plan_create.argtypes = [vp, i32, i32, P, PP]
        L.cz_plan_create.restype = i32
        L.cz_plan_run.argtypes = [vp, PP, PS, PP, PS, vp]
        L.cz_plan_run.restype = i32
        L.cz_plan_result.argtypes = [vp, vp, PS]
        L.cz_plan_result.restype = i32
        L.cz_plan_destroy.argtypes = [vp]
        L.cz_plan_destroy.restype = None
        L.cz_shuffle.argtypes = [vp, sz, u32, vp, vp]
        L.cz_shuffle.restype = i32
        L.cz_unshuffle.argtypes = [vp, sz, u32, vp, vp]
        L.cz_unshuffle.restype = i32
        L.cz_zero_details.argtypes = [vp, P, vp, sz, u32, vp]
        L.cz_zero_details.restype = i32
        L.cz_huff_bound.argtypes = [sz]
        L.cz_huff_bound.restype = sz
        L.cz_huff_encode.argtypes = [vp, vp, sz, vp, sz, PS, vp]
        L.cz_huff_encode.restype = i32
        L.cz_huff_decode.argtypes = [vp, vp, sz, vp, sz, vp]
        L.cz_huff_decode.restype = i32
        PU32 = ctypes.POINTER(u32)
        L.cz_decompress_blocks.argtypes = [vp, P, vp, sz, PU32, sz, vp, sz, vp]
        L.cz_decompress_blocks.restype = i32
        L.cz_cache_create.argtypes = [vp, P, sz, PP]
        L.cz_cache_create.restype = i32
        L.cz_cache_fetch.argtypes = [vp, vp, sz, PU32, sz, PP, vp]
        L.cz_cache_fetch.restype = i32
        L.cz_cache_region.argtypes = [vp, vp, sz, PU32, PU32, vp, sz, vp]
        L.cz_cache_region.restype = i32
        L.cz_cache_stats.argtypes = [vp, ctypes.POINTER(u64), ctypes.POINTER(u64)]
        L.cz_cache_stats.restype = i32
        L.cz_cache_destroy.argtypes = [vp]
        L.cz_cache_destroy.restype = None
        L.cz_server_start.argtypes = [vp, sz, i32, PP]
        L.cz_server_start.restype = i32
        L.cz_submit.argtypes = [vp, ctypes.POINTER(cz_request), ctypes.POINTER(u64)]
        L.cz_submit.restype = i32
        pd = ctypes.POINTER(ctypes.c_double)
        L.cz_poll.argtypes = [vp, u64, ctypes.POINTER(i32), ctypes.POINTER(i32), PS, pd, pd, pd]
        L.cz_poll.restype = i32
        L.cz_wait.argtypes = [vp, u64]
        L.cz_wait.restype = i32
        L.cz_server_time.argtypes = [vp]
        L.cz_server_time.restype = ctypes.c_double
        L.cz_server_stop.argtypes = [vp]
        L.cz_server_stop.restype = i32
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

    def compress_noalloc(self, p: cz_params, d_field: int, d_out: int, out_cap: int, stream: int = 0,
                         d_out_bytes: int | None = None, sync: bool = True) -> int | None:
        """cz_compress_noalloc; returns the stream size when sync."""
        nbytes = ctypes.c_size_t(0)
        rc = lib().cz_compress_noalloc(self.handle, ctypes.byref(p), d_field, d_out, out_cap, d_out_bytes,
                                       ctypes.byref(nbytes) if sync else None, stream)
        if rc != OK:
            raise CzError(rc, "cz_compress_noalloc", f"(required {nbytes.value} bytes)" if rc == ERR_CAPACITY else "")
        return nbytes.value if sync else None

    def compress_strided(self, p: cz_params, d_state: int, ncomp: int, comp: int, d_out: int, out_cap: int,
                         stream: int = 0, d_out_bytes: int | None = None, sync: bool = True) -> int | None:
        """cz_compress_strided; returns the stream size when sync."""
        nbytes = ctypes.c_size_t(0)
        rc = lib().cz_compress_strided(self.handle, ctypes.byref(p), d_state, ncomp, comp, d_out, out_cap,
                                       d_out_bytes, ctypes.byref(nbytes) if sync else None, stream)
        if rc != OK:
            raise CzError(rc, "cz_compress_strided")
        return nbytes.value if sync else None

    def decompress(self, d_in: int, in_bytes: int, d_field: int, field_cap: int, stream: int = 0,
                   expected: cz_params | None = None):
        rc = lib().cz_decompress(self.handle, ctypes.byref(expected) if expected is not None else None, d_in,
                                 in_bytes, d_field, field_cap, stream)
        _check(rc, "cz_decompress")

    def get_status(self, stream: int = 0) -> int:
        return lib().cz_get_status(self.handle, stream)

    def decompress_blocks(self, p: cz_params, d_in: int, in_bytes: int, blocks, d_out: int, out_cap: int,
                          stream: int = 0):
        ids = _u32s(blocks)
        _check(lib().cz_decompress_blocks(self.handle, ctypes.byref(p), d_in, in_bytes, ids, len(blocks), d_out,
                                          out_cap, stream), "cz_decompress_blocks")

    def huff_encode(self, d_in: int, nbytes: int, d_out: int, out_cap: int, stream: int = 0) -> int:
        n = ctypes.c_size_t(0)
        rc = lib().cz_huff_encode(self.handle, d_in, nbytes, d_out, out_cap, ctypes.byref(n), stream)
        if rc != OK:
            raise CzError(rc, "cz_huff_encode")
        return n.value

    def huff_decode(self, d_in: int, in_bytes: int, d_out: int, out_cap: int, stream: int = 0):
        _check(lib().cz_huff_decode(self.handle, d_in, in_bytes, d_out, out_cap, stream), "cz_huff_decode")

    def zero_details(self, p: cz_params, d_stream: int, nbytes: int, bits: int, stream: int = 0):
        _check(lib().cz_zero_details(self.handle, ctypes.byref(p), d_stream, nbytes, bits, stream), "cz_zero_details")

    def set_variant(self, block: int, elem_bytes: int, scheme, variant: int):
        s = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        _check(lib().cz_set_variant(self.handle, block, elem_bytes, s, variant), "cz_set_variant")

    def compress_batch(self, ps, d_fields, d_outs, caps, stream: int = 0, d_out_bytes: int | None = None,
                       sync: bool = True):
        """cz_compress_batch; returns the stream sizes when sync."""
        n = len(ps)
        sizes = _sizes(n)
        rc = lib().cz_compress_batch(self.handle, n, _params_array(ps), _ptrs(d_fields), _ptrs(d_outs),
                                     _sizes(n, caps), d_out_bytes, sizes if sync else None, stream)
        if rc != OK:
            raise CzError(rc, "cz_compress_batch", f"(required {list(sizes)} bytes)" if rc == ERR_CAPACITY else "")
        return list(sizes) if sync else None

    def decompress_batch(self, ps, d_ins, in_bytes, d_fields, caps, stream: int = 0):
        n = len(ps)
        _check(lib().cz_decompress_batch(self.handle, n, _params_array(ps), _ptrs(d_ins), _sizes(n, in_bytes),
                                         _ptrs(d_fields), _sizes(n, caps), stream), "cz_decompress_batch")


def _params_array(ps):
    arr = (cz_params * max(len(ps), 1))()
    for i, p in enumerate(ps):
        arr[i] = p
    return arr


def _ptrs(vals):
    arr = (ctypes.c_void_p * max(len(vals), 1))()
    for i, v in enumerate(vals):
        arr[i] = v
    return arr


def _sizes(n, vals=None):
    arr = (ctypes.c_size_t * max(n, 1))()
    if vals is not None:
        for i, v in enumerate(vals):
            arr[i] = int(v)
    return arr


def variant_count(block: int, elem_bytes: int) -> int:
    return int(lib().cz_variant_count(block, elem_bytes))


class Plan:
    """A captured batch (op "compress" or "decompress") with fixed parameters."""

    def __init__(self, ctx: Context, op: str, ps):
        self.ctx = ctx
        self.n = len(ps)
        self.forward = op == "compress"
        h = ctypes.c_void_p()
        _check(lib().cz_plan_create(ctx.handle, 0 if self.forward else 1, self.n, _params_array(ps),
                                    ctypes.byref(h)), "cz_plan_create")
        self.handle = h

    def run(self, srcs, dsts, caps, src_bytes=None, stream: int = 0):
        _check(lib().cz_plan_run(self.handle, _ptrs(srcs), _sizes(self.n, src_bytes) if src_bytes is not None
                                 else None, _ptrs(dsts), _sizes(self.n, caps), stream), "cz_plan_run")

    def result(self, stream: int = 0):
        sizes = _sizes(self.n)
        _check(lib().cz_plan_result(self.handle, stream, sizes), "cz_plan_result")
        return list(sizes) if self.forward else None

    def close(self):
        if self.handle:
            lib().cz_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def compress_bound(p: cz_params) -> int:
    return int(lib().cz_compress_bound(ctypes.byref(p)))


def read_header(hdr: bytes):
    """Parse a host copy of a stream header -> (params, nblocks, total bytes)."""
    buf = ctypes.create_string_buffer(bytes(hdr[:64]), 64)
    p = cz_params()
    nb, tot = ctypes.c_uint64(0), ctypes.c_uint64(0)
    _check(lib().cz_read_header(buf, 64, ctypes.byref(p), ctypes.byref(nb), ctypes.byref(tot)), "cz_read_header")
    return p, nb.value, tot.value


class Server:
    """A libcz serving scheduler (continuous batching under a memory budget)."""

    def __init__(self, ctx: Context, budget_bytes: int, max_inflight: int):
        h = ctypes.c_void_p()
        _check(lib().cz_server_start(ctx.handle, int(budget_bytes), int(max_inflight), ctypes.byref(h)),
               "cz_server_start")
        self.handle = h
        self.ctx = ctx

    def submit(self, op: int, p: cz_params, d_src: int, src_bytes: int, d_dst: int, dst_cap: int,
               tag: int = 0) -> int:
        r = cz_request(op, p, d_src, src_bytes, d_dst, dst_cap, tag)
        t = ctypes.c_uint64(0)
        _check(lib().cz_submit(self.handle, ctypes.byref(r), ctypes.byref(t)), "cz_submit")
        return t.value

    def poll(self, ticket: int) -> dict:
        done, st = ctypes.c_int(0), ctypes.c_int(0)
        nb = ctypes.c_size_t(0)
        ta, tb, tc = ctypes.c_double(0), ctypes.c_double(0), ctypes.c_double(0)
        _check(lib().cz_poll(self.handle, ticket, ctypes.byref(done), ctypes.byref(st), ctypes.byref(nb),
                             ctypes.byref(ta), ctypes.byref(tb), ctypes.byref(tc)), "cz_poll")
        return {"done": bool(done.value), "status": st.value, "out_bytes": nb.value, "t_arrive": ta.value,
                "t_admit": tb.value, "t_done": tc.value}

    def wait(self, ticket: int) -> int:
        return int(lib().cz_wait(self.handle, ticket))

    def time(self) -> float:
        return float(lib().cz_server_time(self.handle))

    def stop(self) -> int:
        rc = OK
        if self.handle:
            rc = int(lib().cz_server_stop(self.handle))
            self.handle = None
        return rc

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def shuffle(d_in: int, nbytes: int, elem: int, d_out: int, stream: int = 0):
    _check(lib().cz_shuffle(d_in, nbytes, elem, d_out, stream), "cz_shuffle")


def unshuffle(d_in: int, nbytes: int, elem: int, d_out: int, stream: int = 0):
    _check(lib().cz_unshuffle(d_in, nbytes, elem, d_out, stream), "cz_unshuffle")


def _u32s(vals):
    arr = (ctypes.c_uint32 * max(len(vals), 1))()
    for i, v in enumerate(vals):
        arr[i] = int(v)
    return arr


class Cache:
    """A device pool of decoded blocks of one stream (least recently used)."""

    def __init__(self, ctx: Context, p: cz_params, capacity_blocks: int):
        h = ctypes.c_void_p()
        _check(lib().cz_cache_create(ctx.handle, ctypes.byref(p), capacity_blocks, ctypes.byref(h)), "cz_cache_create")
        self.handle = h
        self.ctx = ctx

    def fetch(self, d_in: int, in_bytes: int, blocks, stream: int = 0):
        ptrs = (ctypes.c_void_p * max(len(blocks), 1))()
        _check(lib().cz_cache_fetch(self.handle, d_in, in_bytes, _u32s(blocks), len(blocks), ptrs, stream),
               "cz_cache_fetch")
        return [ptrs[i] for i in range(len(blocks))]

    def region(self, d_in: int, in_bytes: int, origin, extent, d_out: int, out_cap: int, stream: int = 0):
        _check(lib().cz_cache_region(self.handle, d_in, in_bytes, _u32s(origin), _u32s(extent), d_out, out_cap,
                                     stream), "cz_cache_region")

    def stats(self):
        h, m = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(lib().cz_cache_stats(self.handle, ctypes.byref(h), ctypes.byref(m)), "cz_cache_stats")
        return h.value, m.value

    def close(self):
        if self.handle:
            lib().cz_cache_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def huff_bound(nbytes: int) -> int:
    return int(lib().cz_huff_bound(nbytes))
