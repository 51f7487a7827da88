#!/usr/bin/env python3
"""Benchmark of the dual-quantization + Huffman compression path on one MI355X.

A step is one pass of the whole hot path over one field already resident in
HBM: compress (range + eb, dual-quantization, histogram, codebook,
encode/deflate) and decompress (decoding tables, inflate + reconstruct) of
the 3D 100x500x500 fp32 workload at value-range-relative eb 1e-4 with 1024
quantization bins.  Both calls go through the C ABI of libdqz; each call ends
with its own small status readback, which is part of the measured time.

Cold cache (the headline): before every timed call a plain device copy
streams a 2 GiB scratch buffer (1 GiB read, 1 GiB written) so that neither
the 256 MB Infinity Cache nor the L2s hold any of the field or the archive;
the copy is outside the call's time.  Warm figures (no flush, the same field
again and again) are reported beside.

Printed: one JSON line.  `value` is the cold round-trip throughput, original
bytes (4 N) per mean step time (compress + decompress), in decimal GB/s.
Compress and decompress throughput, roofline fractions on the algorithmic
bytes, p50/p99 latency over at least 50 calls each, ratio, the per-stage
breakdown (HIP events on the library's stream), the dominant stage's roofline
and the CPU oracle's rate on the machine's host are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0   # MI355X HBM3E, published peak
FLUSH_BYTES = 1 << 30    # each of the flush copy's source and destination
LAT_SAMPLES = 60         # calls per latency percentile set (at least 50)

WORKLOADS = {
    "c1": "2D 1800x3600 fp32, 64 Fourier modes (|k|^-2) + N(0,1e-3) noise",
    "c2": "3D 100x500x500 fp32, Kolmogorov Gaussian random field + Lamb-Oseen vortex",
    "c3": "1D 280,953,867 fp32 particle coordinates, sorted U[0,256) + N(0,0.05), 4096-blocks shuffled",
    "c4": "64 uneven 3D fp32 fields (edges U[64,512], one 512^3 log-normal sigma=2), per-field valrel eb "
          "in {1e-2,1e-3,1e-4}: batched against plain per-field calls",
    "host": "host path: the 1D 280,953,867 and 3D 100x500x500 fields in pinned host memory, compressed slab by slab "
            "into a host container and back (copies overlapped with the kernels), and the device path plus the "
            "archive's copy to the host (overall)",
    "predictors": "the 1-layer (default) against the 2-layer Lorenzo predictor on the 2D 1800x3600, 3D 100x500x500 "
                  "and 1D 280,953,867 fields at valrel 1e-4 and 1e-3: ratio and device-path throughput",
    "c5": "serving: Poisson streams (50-2000 req/s) of mixed compress/decompress requests over 1D (1e5-1e8), "
          "2D (64..3600 edges) and 3D (32..256 edges) Kolmogorov GRF inputs, valrel eb log-uniform 1e-5..1e-2",
}

# What bounds each stage's kernel: "hbm" kernels stream the field or the
# codes; "latency" kernels are one-workgroup builds, small scans or the
# per-lane serial Huffman decode.
STAGE_BOUND = {"init": "latency", "range_eb": "hbm", "quantize": "hbm", "quantize_scan": "latency",
               "codebook": "latency", "encode": "hbm", "decode_tables": "latency", "inflate": "latency",
               "reconstruct": "hbm"}
KERNEL_OF_STAGE = {"range_eb": ("k_minmax", "kernels_quant.hip"), "quantize": ("k_quant", "kernels_quant.hip"),
                   "codebook": ("k_codebook", "kernels_huff.hip"),
                   "encode": ("k_enc_stream", "kernels_encode.hip"),
                   "decode_tables": ("k_decode_tables", "kernels_huff.hip"),
                   "inflate": ("k_inflate128", "kernels_decode.hip"), "reconstruct": ("k_recon", "kernels_decode.hip")}


def padded_positions(shape):
    """Positions of the zero-padded blocks (32, 16x16 or 8x8x8 points)."""
    b = {1: (32,), 2: (16, 16), 3: (8, 8, 8)}[len(shape)]
    p = 1
    for n, k in zip(shape, b):
        p *= (n + k - 1) // k * k
    return p


def counted_traffic(stage, workload):
    """HBM bytes per launch of the stage's main kernel from the committed
    FETCH_SIZE / WRITE_SIZE counter summary (profiles/traffic_<workload>.json),
    each counter scaled by what it reads for a plain device copy of known size.
    None when there is no summary for that kernel or when the kernel's source
    file has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if stage not in KERNEL_OF_STAGE or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    kernel, src = KERNEL_OF_STAGE[stage]
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    with open(os.path.join(ROOT, "paper_2007_09625_amd", "csrc", src), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != k["source_sha256"]:
            return None
    cal = rec["copy_calibration"]
    fetch_scale = cal["bytes"] / (cal["fetch_kib"] * 1024.0)
    write_scale = cal["bytes"] / (cal["write_kib"] * 1024.0)
    return k["fetch_kib"] * 1024.0 * fetch_scale + k["write_kib"] * 1024.0 * write_scale


def pct(v, q):
    s = sorted(v)
    if not s:
        return float("nan")
    k = (len(s) - 1) * q
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--eb", type=float, default=1e-4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stage-timing", action="store_true", help="time without per-stage HIP events")
    ap.add_argument("--latency-samples", type=int, default=LAT_SAMPLES)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="K",
                    help="after the timed steps, run K plain device copies of the field (4N bytes read, 4N "
                         "written) so hardware byte counters can be scaled against a copy of known size")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "this build has no multi-GPU path", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2007_09625_amd import dqz
    from synth import fields

    if args.workload == "c4":
        return bench_batch(args)
    if args.workload == "c5":
        return bench_serve(args)
    if args.workload == "host":
        return bench_host(args)
    if args.workload == "predictors":
        return bench_predictors(args)
    desc = WORKLOADS[args.workload]
    x_host = fields.workload(args.workload)
    n = x_host.size
    dev = torch.device("cuda:0")
    x = torch.from_numpy(x_host).to(dev)
    params = dqz.make_params(args.eb, dqz.DQZ_EB_VALREL)
    shape = tuple(x.shape)
    bound, ws_need = dqz.dqz_compress_bound(shape, params)
    ctx = dqz.Context(0, workspace=ws_need)
    arc = torch.empty(bound, dtype=torch.uint8, device=dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream(dev)
    fsrc = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device=dev).fill_(1.0)
    fdst = torch.empty_like(fsrc)

    def flush():
        fdst.copy_(fsrc)
        torch.cuda.synchronize()

    def compress():
        st, nbytes, hdr = ctx.dqz_compress(x.data_ptr(), shape, params, arc.data_ptr(), bound, stream)
        ctx._check(st, "dqz_compress")
        return nbytes, hdr

    def decompress(nbytes, hdr):
        st = ctx.dqz_decompress(arc.data_ptr(), nbytes, hdr, y.data_ptr(), y.numel(), stream)
        ctx._check(st, "dqz_decompress")

    def timed(fn, *a):
        t = time.perf_counter()
        r = fn(*a)
        return time.perf_counter() - t, r

    for _ in range(args.warmup):
        nbytes, hdr = compress()
        decompress(nbytes, hdr)

    # cold device-copy bandwidth of the flush itself (2 GiB moved per copy)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    cbw = []
    for _ in range(5):
        ev0.record(stream)
        fdst.copy_(fsrc)
        ev1.record(stream)
        torch.cuda.synchronize()
        cbw.append(2.0 * FLUSH_BYTES / (ev0.elapsed_time(ev1) * 1e-3) / 1e9)
    copy_gbps = sorted(cbw)[len(cbw) // 2]

    # per-stage breakdown (cold), outside the timed region: HIP events between
    # all kernels of a few calls
    stage_timing = not args.no_stage_timing
    st_c, st_d = {}, {}
    if stage_timing:
        ctx.dqz_ctx_set_timing(1)
        for _ in range(8):
            flush()
            nbytes, hdr = compress()
            flush()
            decompress(nbytes, hdr)
            for k, v in ctx.dqz_stage_times(0).items():
                st_c.setdefault(k, []).append(v)
            for k, v in ctx.dqz_stage_times(1).items():
                st_d.setdefault(k, []).append(v)
        ctx.dqz_ctx_set_timing(0)
    stages_us = {k: sum(v) / len(v) for k, v in list(st_c.items()) + list(st_d.items())}
    algo_stages = [k for k in stages_us if k in KERNEL_OF_STAGE]
    dom = max(algo_stages, key=lambda k: stages_us[k]) if algo_stages else None
    # the codebook, the encoder and quantization run within a few percent of
    # each other on the 3D workload, so event noise alone would pick any of
    # them: a latency-bound longest stage yields to an HBM-bound one within
    # 10% of it (the roofline means something for that one; the latency-bound
    # stage's time and share stay in `stages` and in the roofline block)
    latency_dom = None
    if dom and STAGE_BOUND.get(dom) == "latency":
        hbm = [k for k in algo_stages if STAGE_BOUND.get(k) == "hbm" and stages_us[k] >= 0.9 * stages_us[dom]]
        if hbm:
            latency_dom = dom
            dom = max(hbm, key=lambda k: stages_us[k])

    # timed region: K cold steps; each call is timed on its own (the flush
    # before it is not); only the dominant stage is bracketed by events (on
    # the library's stream), so its launch durations are measured live
    dom_which = 0 if dom in dqz.COMPRESS_STAGES else 1
    ctx.dqz_ctx_set_timing(dqz.timing_stage(dom_which, dom) if dom else 0)
    lat_c, lat_d, dom_us = [], [], []
    torch.cuda.synchronize()
    for _ in range(args.steps):
        flush()
        tc, (nbytes, hdr) = timed(compress)
        if dom and dom_which == 0:
            dom_us.append(ctx.dqz_stage_times(0)[dom])
        flush()
        td, _ = timed(decompress, nbytes, hdr)
        if dom and dom_which == 1:
            dom_us.append(ctx.dqz_stage_times(1)[dom])
        lat_c.append(tc)
        lat_d.append(td)
    torch.cuda.synchronize()
    ctx.dqz_ctx_set_timing(0)
    step_s = [a + b for a, b in zip(lat_c, lat_d)]
    sec_per_step = sum(step_s) / len(step_s)

    # latency percentiles: at least 50 calls of each kind, cold and warm
    ns = max(args.latency_samples, 50)
    cold_c, cold_d, warm_c, warm_d = list(lat_c), list(lat_d), [], []
    while len(cold_c) < ns:
        flush()
        tc, (nbytes, hdr) = timed(compress)
        flush()
        td, _ = timed(decompress, nbytes, hdr)
        cold_c.append(tc)
        cold_d.append(td)
    for _ in range(ns):
        tc, (nbytes, hdr) = timed(compress)
        td, _ = timed(decompress, nbytes, hdr)
        warm_c.append(tc)
        warm_d.append(td)

    for _ in range(args.copy_calibration):
        y.copy_(x)
    torch.cuda.synchronize()

    orig = 4.0 * n
    value = orig / sec_per_step / 1e9

    # correctness of the timed output (outside the timed region)
    decompress(nbytes, hdr)
    eb_abs = float(np.frombuffer(hdr[56:64], np.float64)[0])
    fin = torch.isfinite(x)
    err = (x.double() - y.double()).abs()[fin].max().item() if n else 0.0
    assert err <= eb_abs, f"error bound violated: {err} > {eb_abs}"
    n_out = int(np.frombuffer(hdr[88:92], np.uint32)[0])
    n_patch = int(np.frombuffer(hdr[92:96], np.uint32)[0])
    total_bits = int(np.frombuffer(hdr[96:104], np.uint64)[0])
    max_len = int(hdr[116])
    rmse = math.sqrt(float(((x.double() - y.double()) ** 2)[fin].mean().item())) if n else 0.0
    vrange = float(x[fin].max().item()) - float(x[fin].min().item())
    psnr = 20 * math.log10(vrange / rmse) if rmse > 0 else float("inf")
    A = float(nbytes)

    # algorithmic bytes per launch of each stage's kernel: what the method
    # itself must move (N elements; codes are 2 bytes per element; the
    # archive A = header + lengths + tables + exception records + stream is
    # written once, by the encoder; decode + reconstruct read A and write 4N)
    stream_bytes = 4.0 * ((total_bits + 31) // 32)
    exc_bytes = 8.0 * (n_out + n_patch)
    tables_bytes = A - stream_bytes - exc_bytes
    algo = {
        "range_eb": 4.0 * n,
        "quantize": 4.0 * n + 2.0 * n,
        "codebook": 4.0 * 1024,
        "encode": 2.0 * n + A,
        "decode_tables": 1024.0 + exc_bytes,
        "inflate": stream_bytes + tables_bytes,
        "reconstruct": exc_bytes + 4.0 * n,
    }
    roofline = None
    if dom and dom_us:
        dom_avg = sum(dom_us) / len(dom_us)
        ach = algo[dom] / (dom_avg * 1e-6) / 1e9
        traffic = counted_traffic(dom, args.workload)
        roofline = {"bound": "hbm", "kernel": KERNEL_OF_STAGE[dom][0], "stage": dom,
                    "limited_by": STAGE_BOUND[dom],
                    "achieved": round(ach, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBPS, 5),
                    "traffic": round(traffic) if traffic is not None else None,
                    "algorithmic_bytes": algo[dom], "avg_us": round(dom_avg, 2),
                    "timed_launches": len(dom_us), "cache": "cold"}
        if latency_dom:
            roofline["longest_stage"] = {"stage": latency_dom, "kernel": KERNEL_OF_STAGE[latency_dom][0],
                                         "limited_by": "latency", "us": round(stages_us[latency_dom], 2)}

    comp_algo = 12.0 * n + A
    dec_algo = 4.0 * n + A

    def summary(lc, ld):
        c50, d50 = pct(lc, 0.5), pct(ld, 0.5)
        return {"compress_p50_us": round(c50 * 1e6, 1), "compress_p99_us": round(pct(lc, 0.99) * 1e6, 1),
                "decompress_p50_us": round(d50 * 1e6, 1), "decompress_p99_us": round(pct(ld, 0.99) * 1e6, 1),
                "compress_GBps": round(orig / c50 / 1e9, 2), "decompress_GBps": round(orig / d50 / 1e9, 2),
                "compress_roofline_frac": round(comp_algo / c50 / 1e9 / HBM_PEAK_GBPS, 4),
                "decompress_roofline_frac": round(dec_algo / d50 / 1e9 / HBM_PEAK_GBPS, 4),
                "samples": len(lc)}

    cold = summary(cold_c, cold_d)
    warm = summary(warm_c, warm_d)
    comp_stages = [k for k in dqz.COMPRESS_STAGES if k in stages_us]
    dec_stages = [k for k in dqz.DECOMPRESS_STAGES if k in stages_us]
    tc_sum = sum(stages_us[k] for k in comp_stages) or 1.0
    td_sum = sum(stages_us[k] for k in dec_stages) or 1.0
    stage_info = {}
    for k, v in stages_us.items():
        tot = tc_sum if k in comp_stages else td_sum
        e = {"us": round(v, 2), "share": round(v / tot, 3), "bound": STAGE_BOUND.get(k, "latency")}
        if k in algo and v > 0:
            e["algorithmic_bytes"] = algo[k]
            e["hbm_frac"] = round(algo[k] / (v * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4)
        stage_info[k] = e
    result = {
        "metric": "compress/decompress GB/s and % of HBM roofline at eb=1e-4; ratio; p99 latency",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(sec_per_step * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "shape": list(shape), "eb_valrel": args.eb, "bins": 1024,
                   "value_definition": "4N bytes / mean cold step time (compress + decompress, each after a "
                                       "2 GiB cache-flushing copy that is not timed)",
                   "timed_region_events": f"around the {dom} stage only" if dom else "none"},
        "compress_GBps": cold["compress_GBps"],
        "decompress_GBps": cold["decompress_GBps"],
        "compress_roofline_frac": cold["compress_roofline_frac"],
        "decompress_roofline_frac": cold["decompress_roofline_frac"],
        "latency_us": {"compress_p50": cold["compress_p50_us"], "compress_p99": cold["compress_p99_us"],
                       "decompress_p50": cold["decompress_p50_us"], "decompress_p99": cold["decompress_p99_us"],
                       "samples": cold["samples"], "cache": "cold"},
        "cold": cold,
        "warm": warm,
        "algorithmic_bytes": {"compress": comp_algo, "decompress": dec_algo},
        "copy_kernel_GBps": round(copy_gbps, 1),
        "ratio": round(orig / A, 3),
        "bits_per_elem": round(8 * A / n, 4),
        "psnr_db": round(psnr, 3),
        "max_err_over_eb": round(err / eb_abs, 6),
        "outliers": n_out,
        "patches": n_patch,
        "max_code_len": max_len,
        "stages": stage_info,
        "roofline": roofline,
        "cpu_baseline": None,
    }

    if not args.no_cpu_baseline:
        import oracle
        tcs, tds = [], []
        same = True
        for _ in range(3):
            t = time.perf_counter()
            ref = oracle.compress(x_host, args.eb, oracle.EB_VALREL)
            tcs.append(time.perf_counter() - t)
            t = time.perf_counter()
            oracle.decompress(ref)
            tds.append(time.perf_counter() - t)
            same = same and bool(ref.size == nbytes and np.array_equal(ref, arc[:nbytes].cpu().numpy()))
        tc, td = sorted(tcs)[1], sorted(tds)[1]
        result["cpu_baseline"] = {"value": round(orig / (tc + td) / 1e9, 4), "unit": "GB/s", "cores": 1,
                                  "kind": "oracle", "cpu_model": cpu_model(),
                                  "sample": f"the full workload field, median of 3 runs of one compress "
                                            f"({tc:.2f} s) + one decompress ({td:.2f} s), single-threaded C",
                                  "archive_identical_to_gpu": same}
    print(json.dumps(result), flush=True)
    return 0


def bench_batch(args) -> int:
    """The batched workload: every field compressed and decompressed by plain
    single-field calls (one after another, each ending in its readback), then
    by dqz_compress_batch / dqz_decompress_batch over 1-4 lanes with the
    batch captured in a HIP graph; the archives and floats of both paths
    must be identical.  Parameters per shape class from dqz_tune (setup, not
    timed).  Prints one JSON line."""
    import numpy as np
    import torch

    from paper_2007_09625_amd import dqz
    from synth import fields

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    w = fields.BatchWorkload()
    xs = []
    for i in range(len(w)):
        xs.append(torch.from_numpy(w.field(i)).to(dev))
        print(f"field {i} {w.shapes[i]} eb {w.ebs[i]}", file=sys.stderr, flush=True)
    w._pool = None
    gen_s = time.perf_counter() - t0
    n_tot = sum(x.numel() for x in xs)
    orig = 4.0 * n_tot
    ctx = dqz.Context(0)
    t0 = time.perf_counter()
    tuned = [ctx.tune(x, eb) for x, eb in zip(xs, w.ebs)]
    tune_s = time.perf_counter() - t0
    kw = [dict(sub_size=p.sub_size, chunk_subs=p.chunk_subs) for p in tuned]
    params = [dqz.make_params(eb, dqz.DQZ_EB_VALREL, 0, p.sub_size, p.chunk_subs) for eb, p in zip(w.ebs, tuned)]
    bufs = None
    stream = torch.cuda.current_stream(dev)

    # plain path: the single-field calls, one after another, into the batch's
    # own archive buffers
    def plain_compress():
        out = []
        for i, x in enumerate(xs):
            a = bufs.archives[i]
            st, nb, hdr = ctx.dqz_compress(x.data_ptr(), tuple(x.shape), params[i], a.data_ptr(), a.numel(), stream)
            ctx._check(st, "dqz_compress")
            out.append((nb, hdr))
        return out

    def plain_decompress(meta, ys):
        for i, (nb, hdr) in enumerate(meta):
            st = ctx.dqz_decompress(bufs.archives[i].data_ptr(), nb, hdr, ys[i].data_ptr(), ys[i].numel(), stream)
            ctx._check(st, "dqz_decompress")

    ctx.dqz_ctx_set_lanes(1, 0)
    bufs = ctx.batch_buffers(xs, w.ebs, **{})
    bufs.params = params
    for i, x in enumerate(xs):
        ctx.dqz_ctx_reserve(dqz.dqz_compress_bound(tuple(x.shape), params[i])[1])
    meta = plain_compress()                                   # warm-up
    ys = [torch.empty_like(x) for x in xs]
    for nb, hdr in meta:
        ctx.dqz_ctx_reserve(dqz.dqz_decompress_bound(hdr))
    plain_decompress(meta, ys)
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 3))
    tpc, tpd = [], []
    for _ in range(reps):
        t = time.perf_counter()
        meta = plain_compress()
        tpc.append(time.perf_counter() - t)
        t = time.perf_counter()
        plain_decompress(meta, ys)
        torch.cuda.synchronize()
        tpd.append(time.perf_counter() - t)
    plain_arcs = [bufs.archives[i][:nb].clone() for i, (nb, _) in enumerate(meta)]
    plain_ys = [y.clone() for y in ys]
    arc_bytes = sum(nb for nb, _ in meta)
    torch.cuda.synchronize()

    per_lanes = {}
    best = None
    for lanes in (1, 2, 3, 4):
        ctx.dqz_ctx_set_lanes(lanes, dqz.DQZ_LANES_GRAPH)
        comps = ctx.compress_batch(xs, w.ebs, buffers=bufs)     # reserves, captures the graph
        outs = [torch.empty_like(x) for x in xs]
        ctx.decompress_batch(comps, outs=outs)
        tcs, tds = [], []
        for _ in range(reps):
            torch.cuda.synchronize()
            t = time.perf_counter()
            comps = ctx.compress_batch(xs, w.ebs, buffers=bufs)
            tcs.append(time.perf_counter() - t)
            t = time.perf_counter()
            ctx.decompress_batch(comps, outs=outs)
            torch.cuda.synchronize()
            tds.append(time.perf_counter() - t)
        same_a = all(c.archive.numel() == p.numel() and torch.equal(c.archive, p) for c, p in zip(comps, plain_arcs))
        same_y = all(torch.equal(a.view(torch.int32), b.view(torch.int32)) for a, b in zip(outs, plain_ys))
        tc, td = sorted(tcs)[len(tcs) // 2], sorted(tds)[len(tds) // 2]
        per_lanes[lanes] = {"compress_s": round(tc, 5), "decompress_s": round(td, 5),
                            "compress_GBps": round(orig / tc / 1e9, 2), "decompress_GBps": round(orig / td / 1e9, 2),
                            "identical_archives": same_a, "identical_floats": same_y}
        if not (same_a and same_y):
            raise SystemExit(f"batched output differs from the plain calls at {lanes} lanes")
        if best is None or tc + td < per_lanes[best]["compress_s"] + per_lanes[best]["decompress_s"]:
            best = lanes
        del outs
    tpc_m, tpd_m = sorted(tpc)[len(tpc) // 2], sorted(tpd)[len(tpd) // 2]
    b = per_lanes[best]
    # error bound on every element of every field (outside the timed region)
    worst = 0.0
    for i, (x, y) in enumerate(zip(xs, plain_ys)):
        eb_abs = float(np.frombuffer(meta[i][1][56:64], np.float64)[0])
        fin = torch.isfinite(x)
        err = (x.double() - y.double()).abs()[fin].max().item()
        assert err <= eb_abs, f"field {i}: error bound violated"
        worst = max(worst, err / eb_abs)
    classes = {}
    for sh, eb, p in zip(w.shapes, w.ebs, tuned):
        classes[f"S{p.sub_size}/C{p.chunk_subs}"] = classes.get(f"S{p.sub_size}/C{p.chunk_subs}", 0) + 1
    result = {
        "metric": "batched compress+decompress aggregate GB/s (original bytes) against plain per-field calls",
        "value": round(orig / (b["compress_s"] + b["decompress_s"]) / 1e9, 2),
        "unit": "GB/s", "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": round(1e3 * (b["compress_s"] + b["decompress_s"]), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOADS["c4"], "fields": len(xs), "elements": n_tot,
                   "value_definition": "4N bytes of all fields / (batched compress + batched decompress time, "
                                       "median of the timed repetitions)"},
        "batched": {"lanes": best, "graph": True, **b},
        "plain": {"compress_s": round(tpc_m, 5), "decompress_s": round(tpd_m, 5),
                  "compress_GBps": round(orig / tpc_m / 1e9, 2), "decompress_GBps": round(orig / tpd_m / 1e9, 2)},
        "speedup": {"compress": round(tpc_m / b["compress_s"], 3), "decompress": round(tpd_m / b["decompress_s"], 3)},
        "per_lanes": per_lanes,
        "ratio": round(orig / arc_bytes, 3),
        "max_err_over_eb": round(worst, 6),
        "tuner": {"choices": classes, "seconds": round(tune_s, 2)},
        "generation_s": round(gen_s, 1),
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        # the oracle over a bounded sample (in field order, the fields of at
        # most 2e7 values, up to 16 of them or about 1.6e8 values: some 20 s of
        # single-core work), fields spread over the host cores (the oracle's
        # C calls release the interpreter lock)
        from concurrent.futures import ThreadPoolExecutor

        import oracle
        sample, tot = [], 0
        for i in range(1, len(xs)):
            if tot >= 160_000_000 or len(sample) == 16:
                break
            if xs[i].numel() <= 20_000_000:
                sample.append(i)
                tot += xs[i].numel()
        hosts = {i: xs[i].cpu().numpy() for i in sample}
        workers = min(16, os.cpu_count() or 1, len(sample))

        def round_trip(i):
            ref = oracle.compress(hosts[i], w.ebs[i], oracle.EB_VALREL, 512, params[i].sub_size or 128,
                                  params[i].chunk_subs or 64)
            oracle.decompress(ref)
            nb = meta[i][0]
            return ref.size == nb and np.array_equal(ref, plain_arcs[i][:nb].cpu().numpy())

        t = time.perf_counter()
        with ThreadPoolExecutor(max_workers=workers) as pool:
            same = list(pool.map(round_trip, sample))
        tcpu = time.perf_counter() - t
        result["cpu_baseline"] = {
            "value": round(4.0 * tot / tcpu / 1e9, 4), "unit": "GB/s", "cores": workers, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{len(sample)} fields ({tot} values: fields {sample}), one compress + one decompress "
                      f"each, {workers} fields at a time on host threads ({tcpu:.1f} s)",
            "archives_identical_to_gpu": all(same)}
    print(json.dumps(result), flush=True)
    return 0


def bench_serve(args) -> int:
    """Serving: for each arrival rate, a seeded Poisson stream of requests
    (half compressions of pool fields at their own error bounds, half
    decompressions of pre-compressed pool archives) is submitted to a
    dqz server at its arrival times by one thread while another collects the
    completions.  Latency = completion seen by the server - scheduled arrival.
    Run with 4 slots (continuous batching) and with 1 slot (the same server
    as a plain queue).  Prints one JSON line."""
    import threading

    import torch

    from paper_2007_09625_amd import dqz
    from synth import fields

    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    w = fields.ServeWorkload()
    xs = []
    for i in range(len(w)):
        xs.append(torch.from_numpy(w.field(i)).to(dev))
        print(f"pool field {i} {w.shapes[i]}", file=sys.stderr, flush=True)
    w.release_sources()
    gen_s = time.perf_counter() - t0
    ctx = dqz.Context(0)
    pre = [ctx.compress(x, 1e-3) for x in xs]          # the decompression requests' archives
    bounds = {}
    torch.cuda.synchronize()
    del ctx

    def run(rate, slots, n):
        t_arr, kind, idx, eb = w.requests(rate, n, seed=0)
        sv = dqz.Server(0, slots=slots, workspace=4 << 30, budget=64 << 30)
        # warm-up: one request of each pool field and kind
        for i in range(len(xs)):
            sh = tuple(xs[i].shape)
            if sh not in bounds:
                bounds[sh] = dqz.dqz_compress_bound(sh, dqz.make_params(1e-3))[0]
        tickets = [None] * n
        lag = [0.0] * n
        done = [None] * n
        outs = [None] * n
        collected = [0]
        max_outstanding = 512   # back-pressure: the submitter waits (the wait counts as latency)

        def collector():
            for k in range(n):
                while tickets[k] is None:
                    time.sleep(0.0001)
                done[k] = sv.wait(tickets[k])
                outs[k] = None       # the request's output buffer may go now
                collected[0] = k + 1

        col = threading.Thread(target=collector)
        col.start()
        start = time.perf_counter()
        for k in range(n):
            target = start + t_arr[k]
            now = time.perf_counter()
            if target - now > 0.001:
                time.sleep(target - now - 0.0005)
            while time.perf_counter() < target:
                pass
            while k - collected[0] >= max_outstanding:
                time.sleep(0.0001)
            i = int(idx[k])
            if kind[k] == 0:
                out = torch.empty(bounds[tuple(xs[i].shape)], dtype=torch.uint8, device=dev)
                lag[k] = time.perf_counter() - target
                tickets[k] = sv.submit_compress(xs[i], float(eb[k]), out)
            else:
                out = torch.empty_like(xs[i])
                lag[k] = time.perf_counter() - target
                tickets[k] = sv.submit_decompress(pre[i].archive, pre[i].nbytes, pre[i].header, out)
            outs[k] = out
        col.join()
        wall = time.perf_counter() - start
        st = sv.stats()
        sv.close()
        lat = [float(lag[k] + (done[k].t_done_us - done[k].t_submit_us) * 1e-6) for k in range(n)]
        fails = sum(1 for c in done if c.status != 0)
        nbytes = sum(4.0 * xs[int(idx[k])].numel() for k in range(n))
        first = min(c.t_submit_us for c in done)
        last = max(c.t_done_us for c in done)
        return {"requests": n, "p50_ms": round(1e3 * pct(lat, 0.5), 3), "p99_ms": round(1e3 * pct(lat, 0.99), 3),
                "mean_ms": round(1e3 * sum(lat) / n, 3),
                "GBps": round(nbytes / ((last - first) * 1e-6) / 1e9, 2),
                "offered_GBps": round(float(nbytes / t_arr[-1]) / 1e9, 2), "achieved_req_per_s": round(n / wall, 1),
                "max_running": st["max_running"], "max_in_flight_GB": round(st["max_in_flight_bytes"] / 1e9, 3),
                "retried": st["retried"], "failed": fails}

    rates = [int(r) for r in fields.C5_RATES + fields.C5_RATES_SATURATION]
    sweep = {}
    for rate in rates:
        n = int(min(10000, max(200, 3 * rate)))
        r4 = run(rate, 4, n)
        r1 = run(rate, 1, n)
        sweep[rate] = {"slots4": r4, "slots1": r1}
        print(f"rate {rate}: {r4} | {r1}", file=sys.stderr, flush=True)
    top = sweep[int(fields.C5_RATES[-1])]["slots4"]
    result = {
        "metric": "served compress/decompress p50/p99 latency and aggregate GB/s under Poisson load",
        "value": top["GBps"], "unit": "GB/s", "n_gpus": 1, "steps": len(rates), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["c5"], "pool_fields": len(xs),
                   "pool_GB": round(sum(4.0 * x.numel() for x in xs) / 1e9, 3),
                   "requests_per_rate": "min(10000, max(200, 3 s x rate))",
                   "configured_rates": list(fields.C5_RATES),
                   "saturation_rates": list(fields.C5_RATES_SATURATION),
                   "value_definition": f"original bytes of the requests / (last completion - first submission) "
                                       f"at {fields.C5_RATES[-1]} req/s with 4 slots",
                   "hbm_budget_GB": 64, "workspace_arena_GB": 4, "decompress_archives_eb": 1e-3},
        "sweep": sweep,
        "generation_s": round(gen_s, 1),
    }
    print(json.dumps(result), flush=True)
    return 0


def bench_host(args) -> int:
    """Host path.  For each field: (a) overall, the device path plus the
    archive's trip over the host link (compress + archive to pinned host
    memory; archive from the host + decompress; also with the decompressed
    field copied to the host), warm, one call at a time,
    (b) streaming from pinned host memory to a host container and back with
    256 MB slabs (the field need not fit the device; here it does, for the
    comparison).  Original bytes / wall time, median of the repetitions.
    Prints one JSON line."""
    import numpy as np
    import torch

    from paper_2007_09625_amd import dqz
    from synth import fields

    dev = torch.device("cuda:0")
    reps = max(3, min(args.steps, 7))
    out = {}
    for name in ("c3", "c2"):
        x_host = fields.workload(name)
        n = x_host.size
        orig = 4.0 * n
        xp = torch.from_numpy(x_host).pin_memory()
        x = xp.to(dev)
        ctx = dqz.Context(0)
        params = dqz.make_params(args.eb, dqz.DQZ_EB_VALREL)
        bound, ws = dqz.dqz_compress_bound(tuple(x.shape), params)
        ctx.dqz_ctx_reserve(ws)
        arc = torch.empty(bound, dtype=torch.uint8, device=dev)
        harc = torch.empty(bound, dtype=torch.uint8).pin_memory()
        y = torch.empty_like(x)
        yh = torch.empty_like(xp).pin_memory()
        stream = torch.cuda.current_stream(dev)
        tc, tcd, td, tdd, tdh = [], [], [], [], []
        for r in range(reps + 1):
            torch.cuda.synchronize()
            t = time.perf_counter()
            st, nb, hdr = ctx.dqz_compress(x.data_ptr(), tuple(x.shape), params, arc.data_ptr(), bound, stream)
            ctx._check(st, "dqz_compress")
            t1 = time.perf_counter()
            harc[:nb].copy_(arc[:nb])
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            ctx.dqz_ctx_reserve(dqz.dqz_decompress_bound(hdr))
            t3 = time.perf_counter()
            arc[:nb].copy_(harc[:nb])
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            st = ctx.dqz_decompress(arc.data_ptr(), nb, hdr, y.data_ptr(), y.numel(), stream)
            ctx._check(st, "dqz_decompress")
            t5 = time.perf_counter()
            yh.copy_(y)
            torch.cuda.synchronize()
            t6 = time.perf_counter()
            if r:
                tcd.append(t1 - t)       # device path
                tc.append(t2 - t)        # + archive to the host
                td.append(t5 - t4)       # device path
                tdd.append(t5 - t3)      # archive from the host + device path
                tdh.append(t6 - t3)      # ... + field to the host
        slab = 256 << 20
        sws, cmax = dqz.dqz_stream_workspace(tuple(x.shape), params, slab)
        ctx.dqz_ctx_reserve(sws)
        cbuf = torch.empty(cmax, dtype=torch.uint8).pin_memory()
        ts, tsd = [], []
        c = None
        for r in range(reps + 1):
            t = time.perf_counter()
            c = ctx.stream_compress(xp, args.eb, "valrel", slab_bytes=slab, out=cbuf)
            t1 = time.perf_counter()
            ctx.dqz_ctx_reserve(dqz.dqz_stream_info(c)[3])
            t2 = time.perf_counter()
            ctx.stream_decompress(c, out=yh)
            t3 = time.perf_counter()
            if r:
                ts.append(t1 - t)
                tsd.append(t3 - t2)
        shape, n_slabs, eb_abs, _ = dqz.dqz_stream_info(c)
        err = float((xp.double() - yh.double()).abs().max())
        assert err <= eb_abs, f"{name}: error bound violated by the host path"
        med = lambda v: sorted(v)[len(v) // 2]
        out[name] = {
            "elements": n, "archive_bytes": nb, "container_bytes": int(c.numel()), "slabs": n_slabs,
            "device_compress_GBps": round(orig / med(tcd) / 1e9, 2),
            "overall_compress_GBps": round(orig / med(tc) / 1e9, 2),
            "device_decompress_GBps": round(orig / med(td) / 1e9, 2),
            "overall_decompress_GBps": round(orig / med(tdd) / 1e9, 2),
            "decompress_to_host_GBps": round(orig / med(tdh) / 1e9, 2),
            "stream_compress_GBps": round(orig / med(ts) / 1e9, 2),
            "stream_decompress_GBps": round(orig / med(tsd) / 1e9, 2),
            "max_err_over_eb": round(err / eb_abs, 6),
        }
        print(f"{name}: {out[name]}", file=sys.stderr, flush=True)
        del ctx, x, xp, arc, harc, y, yh, cbuf
        torch.cuda.empty_cache()
    # pinned host <-> device copy bandwidth for context
    a = torch.empty(1 << 28, dtype=torch.float32).pin_memory()
    d = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    bw = {}
    for direction in ("h2d", "d2h"):
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t = time.perf_counter()
            (d.copy_(a) if direction == "h2d" else a.copy_(d))
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t)
        bw[direction] = round(4.0 * a.numel() / sorted(ts)[1] / 1e9, 2)
    result = {
        "metric": "host path: overall (device path + archive copy) and streamed host-to-host compress/decompress GB/s",
        "value": out["c3"]["stream_compress_GBps"], "unit": "GB/s", "n_gpus": 1, "steps": reps, "warmup": 1,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS["host"], "eb_valrel": args.eb, "slab_bytes": 256 << 20,
                   "value_definition": "original bytes / wall time of the streamed compression of the 1D field "
                                       "from pinned host memory into a pinned host container (median)"},
        "fields": out, "pinned_copy_GBps": bw,
    }
    print(json.dumps(result), flush=True)
    return 0


def bench_predictors(args) -> int:
    """Ratio and throughput of the 2-layer Lorenzo predictor against the
    paper's 1-layer default (warm, median of the repetitions, device path).
    Prints one JSON line."""
    import numpy as np
    import torch

    from paper_2007_09625_amd import dqz
    from synth import fields

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    reps = max(5, args.steps)
    out = {}
    for name in ("c1", "c2", "c3"):
        x = torch.from_numpy(fields.workload(name)).to(dev)
        n = x.numel()
        ctx = dqz.Context(0)
        for eb in (1e-4, 1e-3):
            for layers in (1, 2):
                params = dqz.make_params(eb, dqz.DQZ_EB_VALREL, 0, 0, 0, layers)
                bound, ws = dqz.dqz_compress_bound(tuple(x.shape), params)
                ctx.dqz_ctx_reserve(ws)
                arc = torch.empty(bound, dtype=torch.uint8, device=dev)
                y = torch.empty_like(x)
                tc, td = [], []
                for r in range(reps + 1):
                    t = time.perf_counter()
                    st, nb, hdr = ctx.dqz_compress(x.data_ptr(), tuple(x.shape), params, arc.data_ptr(), bound,
                                                   stream)
                    ctx._check(st, "dqz_compress")
                    t1 = time.perf_counter()
                    ctx.dqz_ctx_reserve(dqz.dqz_decompress_bound(hdr))
                    t2 = time.perf_counter()
                    st = ctx.dqz_decompress(arc.data_ptr(), nb, hdr, y.data_ptr(), y.numel(), stream)
                    ctx._check(st, "dqz_decompress")
                    t3 = time.perf_counter()
                    if r:
                        tc.append(t1 - t)
                        td.append(t3 - t2)
                eb_abs = float(np.frombuffer(hdr[56:64], np.float64)[0])
                err = float((x.double() - y.double()).abs().max())
                assert err <= eb_abs
                med = lambda v: sorted(v)[len(v) // 2]
                out[f"{name}/eb{eb:g}/layers{layers}"] = {
                    "ratio": round(4.0 * n / nb, 4), "bits_per_elem": round(8.0 * nb / n, 4),
                    "outliers": int(np.frombuffer(hdr[88:92], np.uint32)[0]),
                    "compress_GBps": round(4.0 * n / med(tc) / 1e9, 2),
                    "decompress_GBps": round(4.0 * n / med(td) / 1e9, 2)}
                print(f"{name} eb {eb} layers {layers}: {out[f'{name}/eb{eb:g}/layers{layers}']}",
                      file=sys.stderr, flush=True)
                del arc, y
        del ctx, x
        torch.cuda.empty_cache()
    result = {"metric": "compression ratio and device-path GB/s, 1-layer against 2-layer Lorenzo",
              "value": out["c2/eb0.0001/layers2"]["ratio"], "unit": "ratio", "n_gpus": 1, "steps": reps,
              "warmup": 1, "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
              "dtype": "f32", "data": "synthetic",
              "config": {"workload": WORKLOADS["predictors"],
                         "value_definition": "ratio of the 3D field at valrel 1e-4 with the 2-layer predictor"},
              "cases": out}
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
