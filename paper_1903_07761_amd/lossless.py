"""Host lossless back end (substage 2), off the GPU hot path.

The paper aggregates substage-1 output into per-thread buffers of 4 MB and
deflates each full buffer with zlib at its default level (Sec. 2.2, Sec. 4.1).
Here the packed stream is cut into consecutive 4 MiB chunks, each deflated
with zlib level 6 (zlib's default) on a thread pool (zlib releases the GIL).
The container adds an 8-byte length per chunk and a 64-byte header, so
CR after = raw / (sum of chunk sizes + 8 * chunks + 64).
"""
from __future__ import annotations

import os
import zlib
from concurrent.futures import ThreadPoolExecutor

CHUNK = 4 << 20
LEVEL = 6


def deflate_chunks(data, workers: int | None = None, chunk: int = CHUNK, level: int = LEVEL):
    """Deflate consecutive chunks of a bytes-like object; returns the list of
    compressed chunks."""
    mv = memoryview(data)
    pieces = [mv[i:i + chunk] for i in range(0, len(mv), chunk)]
    workers = workers or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda p: zlib.compress(p, level), pieces))


def container_bytes(chunks) -> int:
    return sum(len(c) for c in chunks) + 8 * len(chunks) + 64


def inflate_chunks(chunks) -> bytes:
    return b"".join(zlib.decompress(c) for c in chunks)
