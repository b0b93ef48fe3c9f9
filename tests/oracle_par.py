"""The oracle over large fields, in threads, for tests.

Blocks are independent (arXiv 1903.07761, Sec. 2.1 and 2.3), so the
single-threaded oracle can be run on disjoint block ranges at once; the
ctypes calls release the interpreter lock, so threads run in parallel.  The
pieces are put together by the exclusive scan of their sizes (Sec. 2.2).
Used where a whole full-size stream or field is compared with libcz.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import streamfmt as S
from stitch import split_slabs, stream_from_records


def workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def compress(oracle, f: np.ndarray, N: int, scheme, eps: float) -> bytes:
    """The oracle's stream of the whole field, built from block ranges."""
    f = np.ascontiguousarray(f)
    nz, ny, nx = f.shape
    nb = (nz // N) * (ny // N) * (nx // N)
    template = oracle.compress(np.ascontiguousarray(f[:N]), N, scheme, eps)
    if nb == 0:
        return oracle.compress(f, N, scheme, eps)
    k = workers()
    step = max(1, -(-nb // (4 * k)))
    cuts = list(range(0, nb, step)) + [nb]

    def job(i):
        b0, b1 = cuts[i], cuts[i + 1]
        recs, sizes = oracle.compress_blocks(f, N, scheme, eps, b0, b1)
        return (b0, b1, recs, sizes)

    with ThreadPoolExecutor(k) as ex:
        ranges = list(ex.map(job, range(len(cuts) - 1)))
    return stream_from_records(template, ranges, nz=nz)


def decompress(oracle, stream: bytes) -> np.ndarray:
    """The oracle's reconstruction of a whole stream, slab by slab."""
    h = S.header(stream)
    layers = h.nz // h.block
    k = workers()
    per = max(1, -(-layers // k))
    parts = split_slabs(stream, per)
    with ThreadPoolExecutor(k) as ex:
        outs = list(ex.map(oracle.decompress, parts))
    return np.concatenate(outs, axis=0) if outs else np.zeros((0, h.ny, h.nx), h.dtype)
