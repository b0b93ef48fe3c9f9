"""Benchmark of the wavelet stage on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c1]

One step = the whole hot path over one batch: every field of the workload is
compressed (3D forward transform, decimation, mask, compaction, offsets,
header) and then decompressed (unpack, inverse transform, store), all
device-resident.  The default workload is one GPU's share of the paper's
large in-situ runs: five 1024^3 float64 fields (density- and pressure-like
bubble clouds, three divergence-free velocity components), W3_ai, 32^3
blocks, eps = 1e-4 of each field's range.

Prints one JSON line: value = raw field bytes per step / step time (GB/s,
1e9 B), forward and inverse rates, per-field PSNR (Eq. 1), max error and
compression ratio, the roofline of the dominant kernel (algorithmic bytes =
raw field + stream per launch, timed with HIP events on the launch stream)
and the CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, AMD published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sources_sha() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1903_07761_amd", "csrc")
    for name in ("cz_kernels.hip", "cz_kernels.h", "cz_lines.h", "cz_lookback.h"):  # the block kernels' sources
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode() + fh.read())
    return h.hexdigest()


def workload(name: str, device):
    """[(label, field tensor, scheme, block, eps)] and a description."""
    import torch

    from paper_1903_07761_amd import fields as G

    out = []
    if name == "c3":
        n, dt = 1024, torch.float64
        log("generating 5 x 1024^3 float64 fields")
        rho = G.bubble_cloud(n, 1905, v_in=0.016, dtype=dt, device=device)
        out.append(("rho", rho))
        p = G.bubble_cloud(n, 1905, v_in=0.1, noise_seed=1906, dtype=dt, device=device)
        out.append(("p", p))
        for lab, comp in zip(("u", "v", "w"), G.div_free_velocity(n, 1907, dtype=dt, device=device)):
            out.append((lab, comp))
        desc = ("5 x 1024^3 float64 fields (rho, p: 200-bubble clouds with 1% noise; u, v, w: divergence-free "
                "sinusoid sums), W3_ai, block 32^3, eps 1e-4 of each field's range")
        scheme, block, frac = "W3_ai", 32, 1e-4
    elif name == "c2":
        log("generating 512^3 float32 bubble cloud")
        out.append(("p", G.bubble_cloud(512, 1904, dtype=torch.float32, device=device)))
        desc = "512^3 float32 bubble cloud (pressure-like), W4_li, block 32^3, eps 1e-3 of range"
        scheme, block, frac = "W4_li", 32, 1e-3
    else:
        out.append(("f", G.gaussian_bumps(128, 1903, dtype=torch.float32, device=device)))
        desc = "128^3 float32 Gaussian bumps, W4, block 32^3, eps 1e-3 of range"
        scheme, block, frac = "W4", 32, 1e-3
    items = [(lab, t, scheme, block, frac * G.value_range(t)) for lab, t in out]
    return items, desc


def copy_bandwidth(torch, nbytes: int = 4 << 30, reps: int = 5) -> float:
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 2 * nbytes / t / 1e9


def host_identity() -> dict:
    """The host the CPU baseline ran on: logical CPUs and the CPU model."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(items, blocks_per_field: int, threads: int = 1):
    """The oracle on blocks [0, k) of every field: one thread on k =
    blocks_per_field, or the OpenMP timing build (parallel-for over chunks of
    blocks, the paper's node layer) on `threads` threads and k =
    threads x blocks_per_field, so both legs take about the same time."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    t_fwd = t_inv = 0.0
    raw = 0
    want = blocks_per_field * max(threads, 1)
    used = want
    for lab, t, scheme, N, eps in items:
        nz, ny, nx = t.shape
        per_layer = (nx // N) * (ny // N)
        layers = min(-(-want // per_layer), nz // N)
        sub = t[:layers * N].cpu().numpy()
        k = min(want, per_layer * layers)
        back = np.zeros_like(sub)
        t0 = time.perf_counter()
        if threads > 1:
            recs, sizes = oracle.compress_blocks_par(sub, N, scheme, eps, 0, k, threads)
        else:
            recs, sizes = oracle.compress_blocks(sub, N, scheme, eps, 0, k)
        t1 = time.perf_counter()
        if threads > 1:
            oracle.decompress_blocks_par(recs, sizes, sub.shape, N, scheme, 0, k, back, threads)
        else:
            oracle.decompress_blocks(recs, sizes, sub.shape, N, scheme, 0, k, back)
        t2 = time.perf_counter()
        t_fwd += t1 - t0
        t_inv += t2 - t1
        raw += k * N ** 3 * sub.dtype.itemsize
        used = min(used, k)
        log(f"cpu oracle {lab} ({threads} thread{'s' if threads > 1 else ''}): {k} blocks "
            f"fwd {t1 - t0:.2f}s inv {t2 - t1:.2f}s")
        del sub, back, recs
    return raw, t_fwd, t_inv, used


def cpu_baseline_line(items, blocks_per_field: int) -> dict:
    """cpu_baseline of the bench line: all host cores (value) beside one
    thread, forward + inverse, with the host's identity."""
    import oracle

    threads = max(1, min(oracle.par_max_threads(), os.cpu_count() or 1))
    sraw, sf, si, sk = cpu_baseline(items, blocks_per_field, 1)
    praw, pf, pi, pk = cpu_baseline(items, blocks_per_field, threads)
    nf = len(items)
    return {"value": round(praw / (pf + pi) / 1e9, 5), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"blocks [0, {pk}) of each field ({nf * pk} blocks), forward + inverse, OpenMP "
                      f"parallel-for over chunks of 4 blocks on {threads} threads",
            "fwd_GBps": round(praw / pf / 1e9, 5), "inv_GBps": round(praw / pi / 1e9, 5),
            "single_thread": {"value": round(sraw / (sf + si) / 1e9, 5), "cores": 1,
                              "sample": f"blocks [0, {sk}) of each field ({nf * sk} blocks)",
                              "fwd_GBps": round(sraw / sf / 1e9, 5), "inv_GBps": round(sraw / si / 1e9, 5)},
            "host": host_identity()}


def zlib_ratio(stream_dev, nbytes: int, raw: int) -> float:
    """CR after the host lossless stage (zlib level 6 over 4 MiB chunks)."""
    from paper_1903_07761_amd import lossless

    host = stream_dev[:nbytes].cpu().numpy()
    return raw / lossless.container_bytes(lossless.deflate_chunks(memoryview(host)))


def c2_sweep(codec, torch):
    """512^3 float32 bubble cloud, W4_li, 32^3 blocks: CR before / after zlib
    (plain, byte-shuffled, and with Z4 / Z8 zeroing before the shuffle; and
    after the GPU Huffman stage over the shuffled stream), PSNR
    and max error for eps in {1e-2, 1e-3, 1e-4} of the range."""
    from paper_1903_07761_amd import fields as G
    from paper_1903_07761_amd import metrics

    f = G.bubble_cloud(512, 1904, dtype=torch.float32, device="cuda")
    rng = G.value_range(f)
    raw = f.numel() * 4
    out = []
    for frac in (1e-2, 1e-3, 1e-4):
        eps = frac * rng
        buf, n = codec.compress(f, 32, "W4_li", eps)
        rec = codec.decompress(buf, n)
        p, m = metrics.error_stats(f, rec)
        sh = codec.shuffle(buf, n, 4)
        row = {"eps_frac": frac, "cr_stage1": round(raw / n, 3), "cr_zlib": round(zlib_ratio(buf, n, raw), 3),
               "cr_shuffle_zlib": round(zlib_ratio(sh, n, raw), 3),
               "cr_shuffle_huff": round(raw / codec.huff_encode(sh, n)[1], 3),
               "psnr_db": round(p, 2), "max_err": float(f"{m:.4g}")}
        # Z4 / Z8: zero the low mantissa bits of the detail coefficients, then shuffle
        for bits in (4, 8):
            z = buf[:n].clone()
            codec.zero_details(z, n, codec.params(f, 32, "W4_li", eps), bits)
            pz, _ = metrics.error_stats(f, codec.decompress(z, n))
            row[f"z{bits}"] = {"cr_shuffle_zlib": round(zlib_ratio(codec.shuffle(z, n, 4), n, raw), 3),
                               "psnr_db": round(pz, 2)}
        out.append(row)
    return out


def gpu_lossless(codec, torch, streams, sizes, raw, elems, reps: int = 3, host_sample: int = 256 << 20):
    """The lossless substage on the GPU (byte shuffle, then canonical Huffman
    in 4 KiB chunks): CR after it and its rates in stream bytes per second
    (best of `reps`; encoding includes building the code on the host,
    decoding the header read).  Every container is decoded and checked
    against its input.  Beside it, host zlib (level 6, 4 MiB chunks, a thread
    pool) on the first `host_sample` bytes of each shuffled stream, with the
    GPU coder's container size on the same bytes."""
    from paper_1903_07761_amd import lossless

    out = {"cr_shuffle_huff": [], "huff_encode_GBps": [], "huff_decode_GBps": [],
           "host_sample_bytes": [], "zlib_host_GBps": [], "huff_over_zlib_bytes": [],
           "zlib_host_threads": min(16, os.cpu_count() or 1)}
    for buf, n, r, e in zip(streams, sizes, raw, elems):
        sh = codec.shuffle(buf, n, e)
        t_enc, t_dec = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            hb, hn = codec.huff_encode(sh, n)
            t_enc.append(time.perf_counter() - t0)
        back = torch.empty(max(n, 1), dtype=torch.uint8, device=sh.device)
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            codec.huff_decode(hb, hn, n, out=back)
            torch.cuda.synchronize()
            t_dec.append(time.perf_counter() - t0)
        if codec.status() != 0 or not torch.equal(back[:n], sh[:n]):
            raise SystemExit("GPU lossless stage: round trip failed")
        del back, hb
        k = min(n, host_sample)
        host = sh[:k].cpu().numpy()
        t0 = time.perf_counter()
        z = lossless.deflate_chunks(memoryview(host))
        t_zl = time.perf_counter() - t0
        out["cr_shuffle_huff"].append(round(r / hn, 3))
        out["huff_encode_GBps"].append(round(n / min(t_enc) / 1e9, 2))
        out["huff_decode_GBps"].append(round(n / min(t_dec) / 1e9, 2))
        out["host_sample_bytes"].append(k)
        out["zlib_host_GBps"].append(round(k / t_zl / 1e9, 3))
        out["huff_over_zlib_bytes"].append(round(codec.huff_encode(sh, k)[1] / lossless.container_bytes(z), 3))
        del sh
    return out


def traffic_record(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter runs
    (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size), or None when
    there is none or the kernel sources changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("sources_sha256") != sources_sha():
        return None
    return rec.get("kernels", {}).get(kernel)


def c4_fields(device):
    """24 fields of mixed edge, block size, precision and scheme: edge from
    {96, 160, 256, 384, 512, 768}, N from {16, 32, 64} redrawn until it divides
    the edge, float32/float64 at even odds, scheme uniform; bubble clouds for
    even i, Gaussian bumps for odd i; seed 1906000 + i; eps 1e-3 of range."""
    import numpy as np
    import torch

    from paper_1903_07761_amd import fields as G

    items = []
    for i in range(24):
        rng = np.random.Generator(np.random.PCG64(1906 * 1000 + i))
        edge = int(rng.choice([96, 160, 256, 384, 512, 768]))
        N = int(rng.choice([16, 32, 64]))
        while edge % N:
            N = int(rng.choice([16, 32, 64]))
        dt = torch.float32 if rng.random() < 0.5 else torch.float64
        scheme = ["W4", "W4_li", "W3_ai"][int(rng.integers(0, 3))]
        seed = 1906 * 1000 + i
        if i % 2 == 0:
            f = G.bubble_cloud(edge, seed, dtype=dt, device=device)
        else:
            f = G.gaussian_bumps(edge, seed, dtype=dt, device=device)
        items.append((f"f{i}", f, scheme, N, 1e-3 * G.value_range(f)))
        log(f"c4 field {i}: {edge}^3 {dt} N={N} {scheme}")
    return items


def main_c4(args):
    """Mixed batch: 24 single-field launches against one batched call (and its
    captured plan); streams and reconstructions must be identical."""
    import torch

    from paper_1903_07761_amd.codec import Codec

    dev = torch.device("cuda", 0)
    codec = Codec(0)
    items = c4_fields(dev)
    st = torch.cuda.current_stream(dev)
    n = len(items)
    ps = [codec.params(t, N, s, e) for _, t, s, N, e in items]
    caps = [codec.bound(t.shape, t.dtype, N) for _, t, _, N, _ in items]
    raw_total = sum(t.numel() * t.element_size() for _, t, _, _, _ in items)
    bufs = {k: [torch.empty(c, dtype=torch.uint8, device=dev) for c in caps] for k in ("plain", "batch", "plan")}
    recs = {k: [torch.empty_like(t) for _, t, _, _, _ in items] for k in ("plain", "batch", "plan")}
    sizes = {k: torch.zeros(n, dtype=torch.int64, device=dev) for k in ("plain", "batch")}
    codec.ctx.reserve(max(t.numel() // N ** 3 for _, t, _, N, _ in items))
    fields = [t for _, t, _, _, _ in items]
    plan_c = codec.plan("compress", ps)
    plan_d = codec.plan("decompress", ps)
    sh = st.cuda_stream

    def plain():
        for i, (_, t, s, N, e) in enumerate(items):
            codec.compress(t, N, s, e, out=bufs["plain"][i], sync=False, out_bytes=sizes["plain"][i:i + 1])
            codec.decompress(bufs["plain"][i], caps[i], out=recs["plain"][i], expected=ps[i])

    def batch():
        codec.compress_batch(fields, [N for _, _, _, N, _ in items], [s for _, _, s, _, _ in items],
                             [e for _, _, _, _, e in items], outs=bufs["batch"], sync=False,
                             out_bytes=sizes["batch"])
        codec.decompress_batch(bufs["batch"], caps, ps, outs=recs["batch"])

    def plan():
        plan_c.run([t.data_ptr() for t in fields], [b.data_ptr() for b in bufs["plan"]], caps, stream=sh)
        plan_d.run([b.data_ptr() for b in bufs["plan"]], [r.data_ptr() for r in recs["plan"]],
                   [r.numel() * r.element_size() for r in recs["plan"]], src_bytes=caps, stream=sh)

    res = {}
    for name, fn in (("plain", plain), ("batch", batch), ("plan", plan)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(args.steps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        rc = codec.status()
        if rc != 0:
            raise SystemExit(f"device status {rc} after {name}")
        ms = e0.elapsed_time(e1) / args.steps
        res[name] = {"ms_per_step": round(ms, 3), "GBps": round(raw_total / (ms / 1e3) / 1e9, 2)}
        log(f"c4 {name}: {ms:.3f} ms per step")
    plan_sizes = plan_c.result(stream=sh)

    # per-field single-launch timing (forward, inverse), for the breakdown
    per_field = []
    for i, (lab, t, s, N, e) in enumerate(items):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(st)
        codec.compress(t, N, s, e, out=bufs["plain"][i], sync=False, out_bytes=sizes["plain"][i:i + 1])
        ev[1].record(st)
        codec.decompress(bufs["plain"][i], caps[i], out=recs["plain"][i], expected=ps[i])
        ev[2].record(st)
        torch.cuda.synchronize()
        raw = t.numel() * t.element_size()
        tf, ti = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
        per_field.append({"edge": t.shape[0], "dtype": str(t.dtype).replace("torch.", ""), "N": N, "scheme": s,
                          "fwd_ms": round(tf, 3), "inv_ms": round(ti, 3),
                          "fwd_GBps": round(raw / tf / 1e6, 1), "inv_GBps": round(raw / ti / 1e6, 1)})
        log(f"c4 {lab}: {per_field[-1]}")

    log("c4 identity check")
    sp, sb = sizes["plain"].cpu().tolist(), sizes["batch"].cpu().tolist()
    identical = sp == sb == plan_sizes
    for i in range(n):
        k = sp[i]
        identical &= bool(torch.equal(bufs["plain"][i][:k], bufs["batch"][i][:k]))
        identical &= bool(torch.equal(bufs["plain"][i][:k], bufs["plan"][i][:k]))
        for other in ("batch", "plan"):
            identical &= bool(torch.equal(recs["plain"][i].view(torch.uint8), recs[other][i].view(torch.uint8)))
    classes = sorted({(N, str(t.dtype).replace("torch.", ""), s) for _, t, s, N, _ in items})
    line = {
        "metric": "GB/s raw field (FWT+threshold+pack, and inverse)",
        "value": res["plan"]["GBps"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["plan"]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "24 mixed fields (edges 96..768, N 16/32/64, float32/float64, W4/W4_li/W3_ai), "
                               "eps 1e-3 of range; captured batched plan",
                   "raw_bytes_per_step": raw_total, "classes": len(classes), "tuned_entries": codec.tuned},
        "single_field_launches": res["plain"],
        "batch_call": res["batch"],
        "captured_plan": res["plan"],
        "speedup_plan_vs_single": round(res["plain"]["ms_per_step"] / res["plan"]["ms_per_step"], 3),
        "identical_streams_and_fields": identical,
        "per_field_single_launch": per_field,
        "cr_stage1": [round(t.numel() * t.element_size() / sp[i], 3) for i, (_, t, _, _, _) in enumerate(items)],
    }
    print(json.dumps(line), flush=True)
    if not identical:
        raise SystemExit("batched output differs from the single-field calls")


def c5_requests(n_req: int = 2000):
    """Request mix of the serving workload: edge = clamp(exp(N(ln 181, 0.5)),
    64, 512) rounded to a multiple of 32, float32 with probability 0.7, scheme
    uniform, eps in {1e-2, 1e-3, 1e-4} of range, bubble cloud or Gaussian bumps
    at even odds, compress or decompress at even odds, N = 32; seed 1907."""
    import numpy as np

    rng = np.random.Generator(np.random.PCG64(1907))
    out = []
    for _ in range(n_req):
        edge = int(round(min(512.0, max(64.0, math.exp(rng.normal(math.log(181.0), 0.5)))) / 32.0)) * 32
        elem = 4 if rng.random() < 0.7 else 8
        scheme = ["W4", "W4_li", "W3_ai"][int(rng.integers(0, 3))]
        frac = [1e-2, 1e-3, 1e-4][int(rng.integers(0, 3))]
        gen = "bubbles" if rng.random() < 0.5 else "bumps"
        op = 0 if rng.random() < 0.5 else 1
        out.append((edge, elem, scheme, frac, gen, op))
    return out


def main_c5(args):
    """Serving: Poisson arrivals of the request mix at rates from 1/4 to 4x the
    plain path's capacity, served by the continuous-batching scheduler and by
    the plain FIFO (one request per launch, max_inflight 1); p50 / p99 latency
    (completion - scheduled arrival) and GB/s of raw field."""
    import numpy as np
    import torch

    from paper_1903_07761_amd import _cz
    from paper_1903_07761_amd import fields as G
    from paper_1903_07761_amd.codec import Codec

    dev = torch.device("cuda", 0)
    codec = Codec(0)
    reqs = c5_requests(args.requests)
    dt = {4: torch.float32, 8: torch.float64}
    pool = {}
    for edge, elem, _, _, gen, _ in reqs:
        k = (edge, elem, gen)
        if k not in pool:
            seed = 1907 * 1000 + len(pool)
            f = (G.bubble_cloud(edge, seed, dtype=dt[elem], device=dev) if gen == "bubbles"
                 else G.gaussian_bumps(edge, seed, dtype=dt[elem], device=dev))
            pool[k] = (f, G.value_range(f))
    log(f"c5: {len(reqs)} requests over {len(pool)} distinct fields")
    # decompress inputs, compressed once (untimed); every request writes its
    # own destination, so requests in flight together never share one and
    # the outputs of the last timed run can be checked afterwards
    streams, dsts, specs = {}, [], []
    raw_total = 0
    for edge, elem, scheme, frac, gen, op in reqs:
        f, rng = pool[(edge, elem, gen)]
        p = codec.params(f, 32, scheme, frac * rng)
        raw = f.numel() * elem
        raw_total += raw
        if op == 1:
            sk = (edge, elem, gen, scheme, frac)
            if sk not in streams:
                buf, n = codec.compress(f, 32, scheme, frac * rng)
                streams[sk] = (buf[:n].clone(), n)
                del buf
            src, sbytes = streams[sk]
            dsts.append(torch.empty(raw, dtype=torch.uint8, device=dev))
            specs.append((1, p, src.data_ptr(), sbytes, dsts[-1].data_ptr(), raw))
        else:
            dsts.append(torch.empty(_cz.compress_bound(p), dtype=torch.uint8, device=dev))
            specs.append((0, p, f.data_ptr(), 0, dsts[-1].data_ptr(), dsts[-1].numel()))
    torch.cuda.synchronize()
    src_bytes = sum(f.numel() * f.element_size() for f, _ in pool.values()) + sum(n for _, n in streams.values())
    dst_bytes = sum(d.numel() for d in dsts)
    log(f"c5: distinct bytes: sources {src_bytes / 1e9:.1f} GB, destinations {dst_bytes / 1e9:.1f} GB")
    budget = 200e9

    def serve(max_inflight, rate):
        """rate None: all requests arrive at t = 0 (saturation)."""
        srv = _cz.Server(codec.ctx, budget, max_inflight)
        n = len(specs)
        gaps = np.random.Generator(np.random.PCG64(1908)).exponential(1.0, n)
        arr = np.zeros(n) if rate is None else np.cumsum(gaps) / rate
        t0 = srv.time() + 0.01
        tickets, lag = [], 0.0
        for i, (op, p, src, sb, dst, cap) in enumerate(specs):
            due = t0 + arr[i]
            while srv.time() < due:
                pass
            lag = max(lag, srv.time() - due)
            tickets.append(srv.submit(op, p, src, sb, dst, cap, tag=i))
        for t in tickets:
            rc = srv.wait(t)
            if rc != 0:
                raise SystemExit(f"request {t} failed: {_cz.strerror(rc)}")
        info = [srv.poll(t) for t in tickets]
        if srv.stop() != 0:
            raise SystemExit("server reported a device failure")
        lat = np.array([d["t_done"] - (t0 + arr[i]) for i, d in enumerate(info)])
        span = max(d["t_done"] for d in info) - t0
        return {"p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
                "GBps": round(raw_total / span / 1e9, 1), "makespan_s": round(span, 4),
                "max_submit_lag_ms": round(float(lag) * 1e3, 3),
                "out_bytes": [d["out_bytes"] for d in info]}

    def check_sample(res, k_each: int = 4):
        """Served outputs of the last run against the oracle: the first
        k_each compress and k_each decompress requests of edge <= 128."""
        import oracle

        oracle.build(force=False)
        done = {0: 0, 1: 0}
        checked, identical, worst_ulp = 0, 0, 0
        for i, (edge, elem, scheme, frac, gen, op) in enumerate(reqs):
            if edge > 128 or done[op] >= k_each:
                continue
            done[op] += 1
            f, rng = pool[(edge, elem, gen)]
            host = f.cpu().numpy()
            if op == 0:
                n = res["out_bytes"][i]
                got = dsts[i][:n].cpu().numpy().tobytes()
                ok = got == oracle.compress(host, 32, scheme, frac * rng)
            else:
                src, n = streams[(edge, elem, gen, scheme, frac)]
                want = oracle.decompress(src[:n].cpu().numpy().tobytes())
                got = dsts[i].view(f.dtype).view(f.shape).cpu().numpy()
                ok = got.tobytes() == want.tobytes()
                if not ok:
                    iv = np.int32 if elem == 4 else np.int64
                    a, b = got.view(iv).astype(np.int64), want.view(iv).astype(np.int64)
                    worst_ulp = max(worst_ulp, int(np.abs(a - b).max()))
                    ok = worst_ulp <= 4
            checked += 1
            identical += int(ok)
        return {"requests": checked, "match": identical, "rule": "compress: stream bytes equal; "
                "decompress: field bit-identical or within 4 ulp", "max_ulp": worst_ulp}

    def strip(r):
        return {k: v for k, v in r.items() if k != "out_bytes"}

    log("c5: warm-up and plain-path capacity")
    for _ in range(max(args.warmup, 1)):
        serve(256, None)
    sat_plain = strip(serve(1, None))
    steps = max(args.steps, 3)
    sat_runs = [serve(256, None) for _ in range(steps)]
    checked = check_sample(sat_runs[-1])
    log(f"c5: served outputs against the oracle: {checked}")
    sat_runs = [strip(r) for r in sat_runs]
    span = float(np.mean([r["makespan_s"] for r in sat_runs]))
    cap = len(specs) / sat_plain["makespan_s"]
    sweep = []
    for mult in (0.25, 0.5, 1.0, 2.0, 4.0):
        rate = mult * cap
        b = strip(serve(256, rate))
        f = strip(serve(1, rate))
        sweep.append({"rate_x_plain_capacity": mult, "rate_per_s": round(rate, 1), "batched": b, "plain_fifo": f})
        log(f"c5 x{mult}: batched {b} plain {f}")
    line = {
        "metric": "GB/s raw field (FWT+threshold+pack, and inverse)",
        "value": round(raw_total / span / 1e9, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": round(span * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{len(specs)} serving requests (edges 64..512, block 32, 70% float32, "
                               "compress/decompress 50/50, eps 1e-2..1e-4 of range), budget 200e9 B",
                   "raw_bytes": raw_total, "distinct_fields": len(pool)},
        "distinct_bytes": {"sources": src_bytes, "destinations": dst_bytes, "last_level_cache": 256 << 20,
                           "note": "every request writes its own destination; sources are shared by requests "
                                   "of one (edge, precision, generator)"},
        "saturated": {"batched": sat_runs, "plain_fifo": sat_plain},
        "served_vs_oracle": checked,
        "plain_capacity_req_per_s": round(cap, 1),
        "poisson_sweep": sweep,
    }
    print(json.dumps(line), flush=True)
    if checked["match"] != checked["requests"]:
        raise SystemExit("served outputs differ from the oracle")


def main_small(args):
    """Small blocks (Sec. 3.2 compares 8^3, 16^3 and 32^3 blocks): 512^3
    bubble clouds (float32 and float64), W4_li and W3_ai, eps 1e-3 of range,
    blocks of 8^3 and 16^3; forward and inverse of each configuration timed
    with HIP events on the launch stream over `steps` repeats.  The streams
    are checked against the oracle on a 64^3 corner of each field."""
    import numpy as np
    import torch

    import oracle
    from paper_1903_07761_amd import fields as G
    from paper_1903_07761_amd.codec import Codec

    dev = torch.device("cuda", 0)
    codec = Codec(0)
    stream = torch.cuda.current_stream(dev)
    oracle.build(force=False)
    rows = []
    raw_total = 0.0
    t_total = 0.0
    for dt in (torch.float32, torch.float64):
        f = G.bubble_cloud(512, 1904, dtype=dt, device=dev)
        eps_frac = 1e-3
        eps = eps_frac * G.value_range(f)
        raw = f.numel() * f.element_size()
        corner = f[:64, :64, :64].contiguous()
        for N in (8, 16):
            for scheme in ("W4_li", "W3_ai"):
                buf, n = codec.compress(corner, N, scheme, eps)
                same = buf[:n].cpu().numpy().tobytes() == oracle.compress(corner.cpu().numpy(), N, scheme, eps)
                out = torch.empty(codec.bound(f.shape, f.dtype, N), dtype=torch.uint8, device=dev)
                back = torch.empty_like(f)
                nb = torch.zeros(1, dtype=torch.int64, device=dev)
                p = codec.params(f, N, scheme, eps)
                for _ in range(max(args.warmup, 1)):
                    codec.compress(f, N, scheme, eps, out=out, sync=False, out_bytes=nb)
                    codec.decompress(out, out.numel(), out=back, expected=p)
                torch.cuda.synchronize()
                ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
                for s in range(args.steps):
                    ev[s][0].record(stream)
                    codec.compress(f, N, scheme, eps, out=out, sync=False, out_bytes=nb)
                    ev[s][1].record(stream)
                    codec.decompress(out, out.numel(), out=back, expected=p)
                    ev[s][2].record(stream)
                torch.cuda.synchronize()
                if codec.status() != 0:
                    raise SystemExit("device status after the small-block runs")
                fwd = float(np.median([e[0].elapsed_time(e[1]) for e in ev]))
                inv = float(np.median([e[1].elapsed_time(e[2]) for e in ev]))
                sz = int(nb.item())
                rows.append({"dtype": str(dt).split(".")[-1], "block": N, "scheme": scheme, "fwd_ms": round(fwd, 4),
                             "inv_ms": round(inv, 4), "cr_stage1": round(raw / sz, 3),
                             "fwd_GBps_algo": round((raw + sz) / fwd / 1e6, 1),
                             "inv_GBps_algo": round((raw + sz) / inv / 1e6, 1),
                             "corner_stream_equals_oracle": same})
                log(f"small: {rows[-1]}")
                raw_total += 2 * raw
                t_total += (fwd + inv) / 1e3
                del out, back
        del f
        torch.cuda.empty_cache()
    line = {
        "metric": "GB/s raw field (FWT+threshold+pack, and inverse)",
        "value": round(raw_total / 2 / t_total / 1e9, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, 1),
        "ms_per_step": round(t_total * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "512^3 bubble clouds, float32 and float64, blocks 8^3 and 16^3, W4_li and W3_ai, "
                               "eps 1e-3 of range (median of the timed repeats)"},
        "runs": rows,
    }
    print(json.dumps(line), flush=True)
    if not all(r["corner_stream_equals_oracle"] for r in rows):
        raise SystemExit("a small-block stream differs from the oracle's")


def main_lossless(args):
    """The GPU lossless stage alone, on the streams of two of C3's fields:
    rho (noisy: the stream is mostly kept coefficients) and u (smooth: mostly
    masks and runs of zero bytes).  One JSON line: stream bytes through
    encode + decode per second, with the per-field detail of gpu_lossless."""
    import torch

    from paper_1903_07761_amd import fields as G
    from paper_1903_07761_amd.codec import Codec

    dev = torch.device("cuda", 0)
    codec = Codec(0)
    log("generating rho and u (1024^3 float64)")
    fields = [("rho", G.bubble_cloud(1024, 1905, v_in=0.016, dtype=torch.float64, device=dev)),
              ("u", G.div_free_velocity(1024, 1907, dtype=torch.float64, device=dev)[0])]
    streams, sizes, raw = [], [], []
    for lab, t in fields:
        buf, n = codec.compress(t, 32, "W3_ai", 1e-4 * G.value_range(t))
        streams.append(buf)
        sizes.append(n)
        raw.append(t.numel() * t.element_size())
    del fields
    torch.cuda.empty_cache()
    gl = gpu_lossless(codec, torch, streams, sizes, raw, [8, 8], reps=max(args.steps, 1))
    t_enc = sum(n / (r * 1e9) for n, r in zip(sizes, gl["huff_encode_GBps"]))
    t_dec = sum(n / (r * 1e9) for n, r in zip(sizes, gl["huff_decode_GBps"]))
    line = {"metric": "GB/s of stream through the GPU lossless stage (encode + decode)",
            "value": round(sum(sizes) / (t_enc + t_dec) / 1e9, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
            "warmup": 0, "higher_is_better": True, "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "byte shuffle + canonical Huffman (4 KiB chunks) of the W3_ai streams of two "
                                   "1024^3 float64 fields of C3 (rho, u)", "stream_bytes": sizes},
            "lossless_gpu": gl}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=["c3", "c2", "c1", "c4", "c5", "lossless", "small"])
    ap.add_argument("--requests", type=int, default=2000, help="c5: number of serving requests")
    ap.add_argument("--cpu-blocks", type=int, default=400, help="oracle sample: blocks per field")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-zlib", action="store_true", help="skip the host lossless stage and the C2 sweep")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU exchange is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(2)
    if args.workload == "c4":
        return main_c4(args)
    if args.workload == "c5":
        return main_c5(args)
    if args.workload == "lossless":
        return main_lossless(args)
    if args.workload == "small":
        return main_small(args)

    from paper_1903_07761_amd import metrics
    from paper_1903_07761_amd.codec import Codec

    dev = torch.device("cuda", 0)
    codec = Codec(0)
    items, desc = workload(args.workload, dev)
    stream = torch.cuda.current_stream(dev)

    # buffers: one stream per field, one reconstruction buffer per field
    streams, recons, exp_params = [], [], []
    for lab, t, scheme, N, eps in items:
        cap = codec.bound(t.shape, t.dtype, N)
        streams.append(torch.empty(cap, dtype=torch.uint8, device=dev))
        recons.append(torch.empty_like(t))
        exp_params.append(codec.params(t, N, scheme, eps))
    nbytes_dev = torch.zeros(len(items), dtype=torch.int64, device=dev)
    codec.ctx.reserve(max(t.numel() // N ** 3 for _, t, _, N, _ in items))

    def step(events=None):
        for i, (lab, t, scheme, N, eps) in enumerate(items):
            if events is not None:
                events[i][0].record(stream)
            codec.compress(t, N, scheme, eps, out=streams[i], sync=False, out_bytes=nbytes_dev[i:i + 1])
            if events is not None:
                events[i][1].record(stream)
            codec.decompress(streams[i], streams[i].numel(), out=recons[i], expected=exp_params[i])
            if events is not None:
                events[i][2].record(stream)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = codec.status()
    if st != 0:
        raise SystemExit(f"device status {st} after warmup")

    log(f"timing {args.steps} steps")
    ev = [[[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in items] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = codec.status()
    if st != 0:
        raise SystemExit(f"device status {st} after timing")

    sizes = [int(x) for x in nbytes_dev.cpu().tolist()]
    raw = [t.numel() * t.element_size() for _, t, _, _, _ in items]
    fwd_ms = [sum(ev[s][i][0].elapsed_time(ev[s][i][1]) for s in range(args.steps)) / args.steps
              for i in range(len(items))]
    inv_ms = [sum(ev[s][i][1].elapsed_time(ev[s][i][2]) for s in range(args.steps)) / args.steps
              for i in range(len(items))]
    ms_per_step = wall * 1e3 / args.steps
    raw_total = sum(raw)
    value = raw_total / (ms_per_step / 1e3) / 1e9
    fwd_gbps = raw_total / (sum(fwd_ms) / 1e3) / 1e9
    inv_gbps = raw_total / (sum(inv_ms) / 1e3) / 1e9

    # algorithmic bytes per launch = raw field + stream, both directions
    algo = [r + s for r, s in zip(raw, sizes)]
    fwd_rate = sum(algo) / (sum(fwd_ms) / 1e3) / 1e9
    inv_rate = sum(algo) / (sum(inv_ms) / 1e3) / 1e9
    dominant = "fwd" if sum(fwd_ms) >= sum(inv_ms) else "inv"
    achieved = fwd_rate if dominant == "fwd" else inv_rate
    kname = "fwd_kernel" if dominant == "fwd" else "inv_kernel"
    tr = traffic_record(kname)

    log("quality")
    psnr, maxerr, cr = [], [], []
    for i, (lab, t, scheme, N, eps) in enumerate(items):
        p, m = metrics.error_stats(t, recons[i])
        psnr.append(round(p, 2))
        maxerr.append(float(f"{m:.4g}"))
        cr.append(round(raw[i] / sizes[i], 3))

    crz = None
    if not args.no_zlib:
        log("host zlib (CR after the lossless stage)")
        crz = [round(zlib_ratio(streams[i], sizes[i], raw[i]), 3) for i in range(len(items))]

    gl = None
    if not args.no_zlib:
        log("GPU lossless stage beside host zlib")
        gl = gpu_lossless(codec, torch, streams, sizes, raw, [t.element_size() for _, t, _, _, _ in items])

    log("copy bandwidth")
    copy_gbps = copy_bandwidth(torch)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle: one thread, then all host cores)")
        cpu = cpu_baseline_line(items, args.cpu_blocks)

    sweep = None
    if not args.no_zlib and args.workload == "c3":
        log("C2 eps sweep")
        sweep = c2_sweep(codec, torch)

    dtype = {torch.float32: "f32", torch.float64: "f64"}[items[0][1].dtype]
    line = {
        "metric": "GB/s raw field (FWT+threshold+pack, and inverse)",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": desc, "fields": len(items), "grid": list(items[0][1].shape), "block": items[0][3],
                   "scheme": items[0][2], "raw_bytes_per_step": raw_total},
        "stream_bytes": sizes,
        "fwd_GBps": round(fwd_gbps, 2),
        "inv_GBps": round(inv_gbps, 2),
        "psnr_db": psnr,
        "max_err": maxerr,
        "cr_stage1": cr,
        "cr_zlib": crz,
        "lossless_gpu": gl,
        "copy_GBps": round(copy_gbps, 1),
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "frac_of_copy": round(achieved / copy_gbps, 4),
                     "traffic": round(tr["bytes_per_launch"]) if tr else None,
                     "traffic_detail": ({"fetch_bytes": round(tr["fetch_bytes_per_launch"]),
                                         "write_bytes": round(tr["write_bytes_per_launch"]),
                                         "algorithmic_bytes": round(tr["algorithmic_bytes_per_launch"]),
                                         "source": "profiles/hbm_traffic_c3_1024cubed_f64_w3ai.md"} if tr else None),
                     "algorithmic_bytes_per_launch": round(sum(algo) / len(algo)),
                     "fwd_GBps_algo": round(fwd_rate, 1), "inv_GBps_algo": round(inv_rate, 1)},
        "cpu_baseline": cpu,
        "c2_eps_sweep": sweep,
        "paper_reference": {"W3_ai_stage1_MBps": {"compress": 277, "decompress": 215},
                            "hardware": "1 core of an Intel Xeon E5-2690v3", "workload": "512^3 float32 pressure",
                            "source": "Table 3"},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
