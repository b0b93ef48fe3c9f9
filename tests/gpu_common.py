"""Helpers shared by the GPU tests: device fixtures, the GPU <-> oracle
stream comparison rule, and block sampling."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import streamfmt as S


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def ordinal(a: np.ndarray) -> np.ndarray:
    """Map float bits to a monotone integer so |ord(a) - ord(b)| counts ulps
    across zero."""
    if a.dtype == np.float32:
        i = a.view(np.int32).astype(np.int64)
        return np.where(i < 0, -(i & 0x7FFFFFFF), i)
    i = a.view(np.int64)
    mag = (i & 0x7FFFFFFFFFFFFFFF).astype(object)
    return np.where(i < 0, -mag, mag)


def compare_records(g: bytes, o: bytes, bg: int, bo: int, eps: float, hg=None, ho=None):
    """The comparison rule for one block: masks equal except where the
    oracle's |c| lies within 1e-6 eps of eps; common values within 4 ulp.
    Returns (mask disagreements, max ulp)."""
    hg = hg or S.header(g)
    ho = ho or S.header(o)
    rg, ro = S.record(g, bg, hg), S.record(o, bo, ho)
    cg, co = S.coefficients(g, bg, hg).reshape(-1), S.coefficients(o, bo, ho).reshape(-1)
    dm = rg.mask != ro.mask
    ndis = int(dm.sum())
    if ndis:
        near = np.abs(np.abs(co[dm].astype(np.float64)) - eps) <= 1e-6 * eps
        # where the oracle dropped, its dense value is 0: recover |c| from the GPU side
        near |= np.abs(np.abs(cg[dm].astype(np.float64)) - eps) <= 1e-6 * eps
        assert near.all(), f"block {bg}: {int((~near).sum())} mask bits differ away from eps"
    common = rg.mask & ro.mask
    ulps = 0
    if common.any():
        d = np.abs(ordinal(cg[common]) - ordinal(co[common]))
        ulps = int(d.max())
        assert ulps <= 4, f"block {bg}: coefficient differs by {ulps} ulp"
    return ndis, ulps


def assert_stream_parity(g: bytes, o: bytes, eps: float) -> str:
    """Whole-stream rule: bit-identical, or (if some mask bits sit within
    1e-6 eps of eps) the per-block rule; with equal masks the layout (header,
    offsets, counts, masks, padding) must be byte-identical."""
    if g == o:
        return "bitexact"
    hg, ho = S.validate(g), S.validate(o)
    assert g[:64] == o[:64], "headers differ"
    total_dis, worst = 0, 0
    for b in range(hg.nblocks):
        nd, u = compare_records(g, o, b, b, eps, hg, ho)
        total_dis += nd
        worst = max(worst, u)
    if total_dis == 0:
        assert np.array_equal(S.offsets(g, hg), S.offsets(o, ho)), "offsets differ with equal masks"
    return f"rule: {total_dis} mask bits at eps, max {worst} ulp"


def block_of(field: np.ndarray, N: int, b: int) -> np.ndarray:
    nz, ny, nx = field.shape
    nbx, nby = nx // N, ny // N
    bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
    return np.ascontiguousarray(field[bz * N:(bz + 1) * N, by * N:(by + 1) * N, bx * N:(bx + 1) * N])


def sample_blocks(nblocks: int, k: int, seed: int):
    rng = np.random.default_rng(seed)
    pick = {0, nblocks - 1, nblocks // 2}
    pick.update(rng.choice(nblocks, size=min(k, nblocks), replace=False).tolist())
    return sorted(pick)
