"""GPU lossless stage (canonical Huffman over bytes, independently decodable
chunks) against the oracle: containers byte-identical to the oracle's on the
same input, the oracle's containers decoded to the input, and corrupt
containers rejected."""
import struct

import numpy as np
import pytest
import torch

from gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu

CHUNK = 4096


@pytest.fixture(scope="module")
def codec():
    need_gpu()
    from paper_1903_07761_amd.codec import Codec

    return Codec(0)


def fib_bytes(seed):
    """Fibonacci counts over 20 symbols: an unlimited Huffman code would need
    19-bit codes, so the 12-bit limit is active."""
    a, b, counts = 1, 1, []
    for _ in range(20):
        counts.append(a)
        a, b = b, a + b
    data = np.repeat(np.arange(20, dtype=np.uint8) * 13, counts)
    return np.random.default_rng(seed).permutation(data)


def shuffled_stream(codec, seed):
    from paper_1903_07761_amd import fields

    f = fields.bubble_cloud(64, seed, nbubbles=12, dtype=torch.float32).cuda()
    eps = 1e-3 * float(f.max() - f.min())
    buf, nb = codec.compress(f, 16, "W3_ai", eps)
    sh = codec.shuffle(buf, nb, 4)
    torch.cuda.synchronize()
    return sh[:nb].cpu().numpy()


def inputs(codec):
    """Short codes (under 4 bits a byte: one symbol, two symbols, geometric,
    Fibonacci: a lane's words last many steps) and long ones (uniform,
    shuffled stream: a lane needs a new word every few steps)."""
    rng = np.random.default_rng(5)
    yield "empty", np.zeros(0, np.uint8)
    yield "one byte", np.array([200], np.uint8)
    yield "one symbol", np.full(40000, 7, np.uint8)
    yield "two symbols", rng.integers(0, 2, 3 * CHUNK + 1, dtype=np.uint8) * 255
    yield "uniform ragged", rng.integers(0, 256, 3 * CHUNK + 777, dtype=np.uint8)
    yield "geometric", np.minimum(rng.geometric(0.3, 2 * CHUNK + 5), 255).astype(np.uint8)
    yield "fibonacci", fib_bytes(6)
    yield "exact chunks", rng.integers(0, 64, 2 * CHUNK, dtype=np.uint8)
    yield "shuffled stream", shuffled_stream(codec, 7)[: 6 * CHUNK + 123]


def test_encode_matches_oracle(codec):
    from oracle import huffman

    for name, host in inputs(codec):
        dev = torch.from_numpy(host.copy()).cuda()
        out, n = codec.huff_encode(dev, host.size)
        ref = huffman.encode(host.tobytes())
        got = out[:n].cpu().numpy().tobytes()
        assert n == len(ref), (name, n, len(ref))
        assert got == ref, name
        say(f"[huff] encode {name}: {host.size} -> {n} bytes ok")


def test_encode_misaligned_inputs_match_oracle(codec):
    """Inputs that do not start on a 16-byte boundary take the encoder's
    byte-wise path: the containers are still the oracle's."""
    from oracle import huffman

    rng = np.random.default_rng(9)
    for shift in (1, 4, 8):
        for size in (1, 3 * CHUNK + 77, 9 * CHUNK):
            host = np.minimum(rng.geometric(0.2, size), 255).astype(np.uint8)
            buf = torch.zeros(size + 16, dtype=torch.uint8, device="cuda")
            buf[shift:shift + size] = torch.from_numpy(host).cuda()
            view = buf[shift:shift + size]
            assert view.data_ptr() % 16 != 0
            out, n = codec.huff_encode(view, size)
            assert out[:n].cpu().numpy().tobytes() == huffman.encode(host.tobytes()), (shift, size)
    say("[huff] misaligned encode inputs ok")


def test_decode_oracle_containers(codec):
    from oracle import huffman

    for name, host in inputs(codec):
        blob = huffman.encode(host.tobytes())
        dev = torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda()
        out = codec.huff_decode(dev, len(blob), host.size)
        torch.cuda.synchronize()
        assert codec.status() == 0, name
        assert out[: host.size].cpu().numpy().tobytes() == host.tobytes(), name
        say(f"[huff] decode {name} ok")


def test_large_round_trip_and_sampled_chunks(codec):
    """8 MiB + 5 of a shuffled compressed stream pattern: the code lengths are
    the oracle's for the histogram, sampled chunks are the oracle's encoding of
    those 4 KiB, and decoding gives back every byte."""
    from oracle import huffman

    base = shuffled_stream(codec, 8)
    reps = (8 * 2 ** 20 + 5 + base.size - 1) // base.size
    host = np.tile(base, reps)[: 8 * 2 ** 20 + 5]
    host[::4099] ^= 0x5A  # break the period
    dev = torch.from_numpy(host).cuda()
    out, n = codec.huff_encode(dev, host.size)
    blob = out[:n].cpu().numpy().tobytes()
    nchunks = (host.size + CHUNK - 1) // CHUNK
    lengths = huffman.package_merge(np.bincount(host, minlength=256))
    assert list(blob[32:288]) == lengths
    codes = huffman.canonical_codes(lengths)
    offs = struct.unpack_from(f"<{nchunks + 1}Q", blob, 288)
    p0 = (288 + 8 * (nchunks + 1) + 15) // 16 * 16
    assert p0 + offs[-1] == n
    for k in (0, 1, nchunks // 2, nchunks - 2, nchunks - 1):
        ref = huffman.encode_chunk(host[k * CHUNK:(k + 1) * CHUNK].tobytes(), codes)
        assert blob[p0 + offs[k]:p0 + offs[k + 1]] == ref, k
    back = codec.huff_decode(out, n, host.size)
    torch.cuda.synchronize()
    assert codec.status() == 0
    assert torch.equal(back[: host.size], dev)
    say(f"[huff] 8 MiB: ratio {host.size / n:.3f}")


def test_huffman_errors(codec):
    from oracle import huffman
    from paper_1903_07761_amd import _cz

    host = np.full(40000, 7, np.uint8)
    dev = torch.from_numpy(host).cuda()
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(_cz.CzError) as e:
        codec.ctx.huff_encode(dev.data_ptr(), host.size, small.data_ptr(), small.numel())
    assert e.value.code == _cz.ERR_CAPACITY
    blob = bytearray(huffman.encode(host.tobytes()))

    def decode(b, nbytes=None, raw=host.size):
        d = torch.frombuffer(bytearray(b), dtype=torch.uint8).cuda()
        return codec.huff_decode(d, len(b) if nbytes is None else nbytes, raw)

    bad = bytearray(blob)
    bad[0:4] = b"XZH1"
    with pytest.raises(_cz.CzError) as e:
        decode(bad)
    assert e.value.code == _cz.ERR_FORMAT
    bad = bytearray(blob)
    bad[32 + 3] = 1  # a second 1-bit code: Kraft sum 1.5 > 1
    bad[32 + 7] = 1
    bad[32 + 9] = 1
    with pytest.raises(_cz.CzError) as e:
        decode(bad)
    assert e.value.code == _cz.ERR_FORMAT
    with pytest.raises(_cz.CzError) as e:
        decode(blob, raw=host.size - 1)  # output too small for the raw size
    assert e.value.code == _cz.ERR_CAPACITY
    shifted = torch.zeros(len(blob) + 16, dtype=torch.uint8, device="cuda")
    shifted[8:8 + len(blob)] = torch.frombuffer(bytearray(blob), dtype=torch.uint8).cuda()
    outb = torch.empty(host.size, dtype=torch.uint8, device="cuda")
    with pytest.raises(_cz.CzError) as e:  # the container must start 16-byte aligned
        codec.ctx.huff_decode(shifted.data_ptr() + 8, len(blob), outb.data_ptr(), outb.numel())
    assert e.value.code == _cz.ERR_ARG
    # a payload bit pattern the single 1-bit code does not define
    bad = bytearray(blob)
    nchunks = (host.size + CHUNK - 1) // CHUNK
    p0 = len(blob) - struct.unpack_from("<Q", blob, 288 + 8 * nchunks)[0]
    bad[p0] = 1
    decode(bad)
    torch.cuda.synchronize()
    assert codec.status() == _cz.ERR_FORMAT
    # the container cut short: the last chunk's words lie past its end
    decode(blob, nbytes=len(blob) - 8)
    torch.cuda.synchronize()
    assert codec.status() == _cz.ERR_FORMAT
    assert codec.status() == 0
    # the same for long codes (8 bits a byte)
    wide = np.random.default_rng(3).integers(0, 256, 3 * CHUNK + 5, dtype=np.uint8)
    wblob = huffman.encode(wide.tobytes())
    d = torch.frombuffer(bytearray(wblob), dtype=torch.uint8).cuda()
    codec.huff_decode(d, len(wblob) - 8, wide.size)
    torch.cuda.synchronize()
    assert codec.status() == _cz.ERR_FORMAT
    # a valid container still decodes after the errors
    out = decode(blob)
    torch.cuda.synchronize()
    assert codec.status() == 0 and out[: host.size].cpu().numpy().tobytes() == host.tobytes()


def test_round_trip_past_4_gib(codec):
    """A container whose chunk offsets pass 2^31 and 2^32 bytes (4.4 GiB of
    uniform bytes, 8-bit codes): decoding gives back every byte, so the
    decoder's 64-bit payload positions hold past the 32-bit ranges."""
    n = 4400 * 2 ** 20 + 3
    gen = torch.Generator(device="cuda").manual_seed(11)
    dev = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda", generator=gen)
    out, nb = codec.huff_encode(dev, n)
    assert nb > 2 ** 32
    back = codec.huff_decode(out, nb, n)
    torch.cuda.synchronize()
    assert codec.status() == 0
    assert torch.equal(back[:n], dev)
    say(f"[huff] 4.4 GiB round trip: container {nb} bytes")
