"""The C-ABI library loads and exports every entry point include/cz.h
declares; host-only entry points (no GPU needed) behave as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cz.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cz_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def czlib():
    from paper_1903_07761_amd import _cz

    return _cz


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("cz_create", "cz_destroy", "cz_reserve", "cz_compress_bound", "cz_compress", "cz_decompress",
                 "cz_get_status", "cz_read_header", "cz_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol(czlib):
    L = czlib.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_compress_bound_matches_layout(czlib):
    p = czlib.params(64, 64, 64, 32, "W4", 4, 0.1)
    # 8 blocks: payload start roundup16(64 + 8 * 9) = 144; record roundup16(8 + 4096 + 32768 * 4)
    assert czlib.compress_bound(p) == 144 + 8 * 135184
    p = czlib.params(32, 16, 48, 16, "W3_ai", 8, 0.0)
    nb = 2 * 1 * 3
    assert czlib.compress_bound(p) == (64 + 8 * (nb + 1) + 15) // 16 * 16 + nb * ((8 + 512 + 4096 * 8 + 15) // 16 * 16)


def test_compress_bound_agrees_with_oracle(czlib, oracle):
    for shape, N, elem in [((32, 32, 32), 8, 4), ((64, 32, 96), 32, 8), ((16, 16, 16), 16, 4), ((0, 32, 32), 32, 4)]:
        nz, ny, nx = shape
        assert czlib.compress_bound(czlib.params(nx, ny, nz, N, 0, elem, 0.0)) == oracle.compress_bound(shape, N, elem)


def test_invalid_params_give_zero_bound(czlib):
    assert czlib.compress_bound(czlib.params(40, 32, 32, 32, 0, 4, 0.1)) == 0  # not a multiple
    assert czlib.compress_bound(czlib.params(32, 32, 32, 12, 0, 4, 0.1)) == 0  # not a power of two
    assert czlib.compress_bound(czlib.params(32, 32, 32, 32, 3, 4, 0.1)) == 0  # bad scheme
    assert czlib.compress_bound(czlib.params(32, 32, 32, 32, 0, 2, 0.1)) == 0  # bad element size
    assert czlib.compress_bound(czlib.params(32, 32, 32, 32, 0, 4, -1.0)) == 0  # eps < 0
    assert czlib.compress_bound(czlib.params(32, 32, 32, 32, 0, 4, float("nan"))) == 0


def test_read_header_parses_oracle_stream(czlib, oracle):
    import numpy as np

    f = np.ones((32, 16, 48), np.float64)
    s = oracle.compress(f, 16, "W4_li", 0.25)
    p, nb, total = czlib.read_header(s[:64])
    assert (p.nx, p.ny, p.nz, p.block, p.scheme, p.elem_bytes, p.epsilon) == (48, 16, 32, 16, 1, 8, 0.25)
    assert nb == 6 and total == len(s)
    bad = bytearray(s[:64])
    bad[0] = ord("X")
    with pytest.raises(czlib.CzError) as e:
        czlib.read_header(bytes(bad))
    assert e.value.code == czlib.ERR_FORMAT


def test_strerror(czlib):
    assert czlib.strerror(0) == "ok"
    assert "stream" in czlib.strerror(czlib.ERR_FORMAT)


def test_huff_bound_matches_container_layout(czlib):
    """Worst case of the lossless container: 32-byte header, 256 lengths,
    (chunks + 1) offsets padded to 16, and 12 bits a byte for every 4 KiB
    chunk (1536 words); the oracle's container of any input fits."""
    from oracle import huffman

    for n in (0, 1, 4095, 4096, 4097, 10 * 4096 + 3):
        chunks = (n + 4095) // 4096
        head = (288 + 8 * (chunks + 1) + 15) // 16 * 16
        assert czlib.huff_bound(n) == head + chunks * 1536 * 4, n
    import numpy as np

    data = np.random.default_rng(1).integers(0, 256, 3 * 4096 + 11, dtype=np.uint8).tobytes()
    assert len(huffman.encode(data)) <= czlib.huff_bound(len(data))


def test_variant_counts(czlib):
    """Tiling variants per block size (any precision): one for 8^3, two for
    16^3, three for 32^3 and for 64^3 (resident scratch slots)."""
    for elem in (4, 8):
        assert [czlib.variant_count(n, elem) for n in (8, 16, 32, 64)] == [1, 2, 3, 3]


def test_tuner_keeps_the_default_within_the_margin():
    from paper_1903_07761_amd.autotune import MARGIN, pick

    assert pick([1.0]) == 0
    assert pick([1.0, 0.99, 1.2]) == 0  # 1% faster: noise, the default stays
    assert pick([1.0, 1.1, 1.0 - 2 * MARGIN]) == 2
    assert pick([1.0, 1.0 - 2 * MARGIN, 1.0 - 3 * MARGIN]) == 2
    assert pick([0.5, 0.4, 0.45]) == 1


def test_tuner_ignores_the_forward_where_it_has_one_tiling():
    """8^3 and 16^3 blocks: the forward kernel takes no variant, so only the
    inverse times decide; other sizes compare forward + inverse."""
    from paper_1903_07761_amd.autotune import MARGIN, pick_entry

    fwd = [0.50, 0.55]  # noise in a kernel that does not change
    inv = [0.40, 0.40 * (1 - 2 * MARGIN)]
    assert pick_entry(16, fwd, inv) == 1
    assert pick_entry(8, [0.5], [0.4]) == 0
    assert pick_entry(32, fwd + [0.9], inv + [0.4]) == 0  # the totals: 0.90, 0.926, 1.3


def test_committed_table_follows_its_own_times(czlib):
    """Every entry of the committed table names a variant that exists and is
    the one the tuner's rule picks from the times recorded beside it."""
    import json

    from paper_1903_07761_amd.autotune import DEFAULT_TABLE, pick_entry

    with open(DEFAULT_TABLE) as fh:
        table = json.load(fh)
    assert table
    for arch, rec in table.items():
        for k, v in rec["variants"].items():
            nkey, tkey, _ = k.split("/")
            nv = czlib.variant_count(int(nkey[1:]), 4 if tkey == "f32" else 8)
            assert len(v["fwd_ms"]) == len(v["inv_ms"]) == nv, k
            assert v["variant"] == pick_entry(int(nkey[1:]), v["fwd_ms"], v["inv_ms"]), (arch, k)
