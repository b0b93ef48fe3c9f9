"""Host lossless back end (zlib over 4 MiB chunks, off the GPU hot path):
round trip, chunking and the compressed-size accounting behind CR."""
import os
import zlib

import numpy as np

from paper_1903_07761_amd import lossless


def test_roundtrip_and_chunking():
    rng = np.random.default_rng(0)
    data = rng.integers(0, 4, size=(9 << 20) + 123, dtype=np.uint8).tobytes()  # three chunks, last ragged
    chunks = lossless.deflate_chunks(data, workers=4)
    assert len(chunks) == 3
    assert lossless.inflate_chunks(chunks) == data
    # each chunk is an independent zlib stream of one 4 MiB slice at level 6
    assert chunks[1] == zlib.compress(data[4 << 20:8 << 20], 6)
    assert lossless.container_bytes(chunks) == sum(map(len, chunks)) + 8 * 3 + 64


def test_empty_input():
    assert lossless.deflate_chunks(b"") == []
    assert lossless.container_bytes([]) == 64


def test_cr_after_zlib_on_oracle_stream(oracle):
    """CR after the lossless stage (raw / container bytes) is at least the
    stage-1 CR for a smooth field: zlib removes redundancy left in the stream."""
    from paper_1903_07761_amd import fields

    f = fields.gaussian_bumps(64, 1903).numpy()
    s = oracle.compress(f, 32, "W3_ai", 1e-3 * float(f.max() - f.min()))
    chunks = lossless.deflate_chunks(s)
    cr1 = f.nbytes / len(s)
    cr2 = f.nbytes / lossless.container_bytes(chunks)
    assert cr2 > cr1
    assert lossless.inflate_chunks(chunks) == s
