"""Kernel-variant autotuner.

Block size is a tuning knob of the method (Sec. 2.3 discusses the trade-off
between block size, compression ratio and speed); on the GPU each (block
size, precision, scheme) additionally has one or more register/LDS tilings
of the same transform (workgroup size and slab depth), all producing
byte-identical output.  This module times every tiling on a synthetic field
of the paper's kind and keeps the fastest per (N, precision, scheme) in a
JSON table keyed by the device architecture; ``apply`` loads the table into
a libcz context.

    python -m paper_1903_07761_amd.autotune [--out FILE] [--edge 512] [--reps 5]
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys

import torch

from . import _cz
from . import fields as G

SCHEMES = ("W4", "W4_li", "W3_ai")
BLOCKS = (8, 16, 32, 64)
DTYPES = {4: torch.float32, 8: torch.float64}
DEFAULT_TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def arch_name(device: int = 0) -> str:
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def key(block: int, elem_bytes: int, scheme: str) -> str:
    return f"N{block}/{'f32' if elem_bytes == 4 else 'f64'}/{scheme}"


def _time_variant(codec, f, block, scheme, eps, reps):
    """Median forward and inverse milliseconds of one variant (HIP events on
    the launch stream), and the stream it produced."""
    st = torch.cuda.current_stream()
    buf = torch.empty(codec.bound(f.shape, f.dtype, block), dtype=torch.uint8, device=f.device)
    rec = torch.empty_like(f)
    size = torch.zeros(1, dtype=torch.int64, device=f.device)
    p = codec.params(f, block, scheme, eps)
    fwd, inv = [], []
    for r in range(reps + 1):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(st)
        codec.compress(f, block, scheme, eps, out=buf, sync=False, out_bytes=size)
        e[1].record(st)
        codec.decompress(buf, buf.numel(), out=rec, expected=p)
        e[2].record(st)
        torch.cuda.synchronize()
        if r:  # the first pass warms up
            fwd.append(e[0].elapsed_time(e[1]))
            inv.append(e[1].elapsed_time(e[2]))
    rc = codec.status()
    if rc != 0:
        raise _cz.CzError(rc, "autotune")
    n = int(size.item())
    return statistics.median(fwd), statistics.median(inv), buf[:n].cpu().numpy().tobytes()


# A variant replaces variant 0 only when its forward + inverse time is at
# least this much lower: differences within run-to-run noise on the tuning
# field do not carry over to other fields.
MARGIN = 0.03


def pick(totals) -> int:
    """Index of the variant to use given forward + inverse milliseconds per
    variant (index 0 the default)."""
    best = min(range(len(totals)), key=lambda v: totals[v])
    return best if totals[best] <= (1.0 - MARGIN) * totals[0] else 0


# Block sizes whose forward has a single tiling (the grouped small-block
# kernel): their variants differ in the inverse only, so they are compared on
# inverse times and the forward's run-to-run noise does not decide.
FWD_SINGLE = (8, 16)


def pick_entry(block: int, fwd_ms, inv_ms) -> int:
    """The variant for one (N, precision, scheme) entry from its timings."""
    if block in FWD_SINGLE:
        return pick(list(inv_ms))
    return pick([a + b for a, b in zip(fwd_ms, inv_ms)])


def tune(codec, edge: int = 512, reps: int = 5, blocks=BLOCKS, elems=(4, 8), schemes=SCHEMES, log=print):
    """Time every variant of every (N, precision, scheme); return the table
    entry for this device: {key: {"variant", "fwd_ms", "inv_ms"}}."""
    out = {}
    for elem in elems:
        for N in blocks:
            nv = _cz.variant_count(N, elem)
            if nv == 0:
                continue
            n = max(edge, 8 * N)  # at least 512 blocks: more than the chip holds at once
            f = G.bubble_cloud(n, 1906, dtype=DTYPES[elem], device=codec.device)
            eps = 1e-3 * G.value_range(f)
            for s in schemes:
                res = []
                ref = None
                for v in range(nv):
                    codec.ctx.set_variant(N, elem, s, v)
                    tf, ti, stream = _time_variant(codec, f, N, s, eps, reps)
                    if ref is None:
                        ref = stream
                    elif stream != ref:
                        raise RuntimeError(f"variant {v} of {key(N, elem, s)} changed the stream")
                    res.append((tf + ti, v, tf, ti))
                    log(f"{key(N, elem, s)} variant {v}: fwd {tf:.3f} ms inv {ti:.3f} ms")
                res.sort(key=lambda r: r[1])
                codec.ctx.set_variant(N, elem, s, 0)
                fwd_ms, inv_ms = [round(r[2], 4) for r in res], [round(r[3], 4) for r in res]
                out[key(N, elem, s)] = {"variant": pick_entry(N, fwd_ms, inv_ms), "fwd_ms": fwd_ms, "inv_ms": inv_ms}
            del f
    return out


def load(path: str = DEFAULT_TABLE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def apply(codec, table: dict | None = None, path: str = DEFAULT_TABLE) -> int:
    """Select the tuned variant of every entry for this device's architecture;
    returns how many were applied."""
    table = load(path) if table is None else table
    entries = table.get(arch_name(codec.device.index or 0), {}).get("variants", {})
    applied = 0
    for k, rec in entries.items():
        nkey, tkey, s = k.split("/")
        N, elem = int(nkey[1:]), 4 if tkey == "f32" else 8
        if 0 <= rec["variant"] < _cz.variant_count(N, elem):
            codec.ctx.set_variant(N, elem, s, rec["variant"])
            applied += 1
    return applied


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--edge", type=int, default=512)
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args(argv)
    from .codec import Codec

    codec = Codec(0)
    arch = arch_name(0)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    entries = tune(codec, edge=args.edge, reps=args.reps, log=log)
    table = load(args.out)
    table[arch] = {"field": f"bubble cloud of edge max({args.edge}, 8 N), eps 1e-3 of range", "reps": args.reps,
                   "margin": MARGIN, "variants": entries}
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    print(json.dumps({"arch": arch, "entries": len(entries)}))


if __name__ == "__main__":
    main()
