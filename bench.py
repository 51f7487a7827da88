#!/usr/bin/env python3
"""Benchmark of the dual-quantization + Huffman compression path on one MI355X.

A step is one pass of the whole hot path over one field already resident in
HBM: compress (range + eb, dual-quantization, histogram, codebook,
encode/deflate) and decompress (decoding tables, inflate + reconstruct) of
the 3D 100x500x500 fp32 workload at value-range-relative eb 1e-4 with 1024
quantization bins.  Both calls go through the C ABI of libdqz; each call ends
with its own small status readback, which is part of the measured time.

Printed: one JSON line.  `value` is the round-trip throughput, original bytes
(4 N) per step time, in decimal GB/s.  Compress and decompress throughput,
latency percentiles, ratio, the per-stage breakdown (HIP events on the
library's stream), the roofline of the dominant kernel and the CPU oracle's
rate on the machine's host are reported beside it.
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

WORKLOADS = {
    "c1": ("2D 1800x3600 fp32, 64 Fourier modes (|k|^-2) + N(0,1e-3) noise", "fourier2d"),
    "c2": ("3D 100x500x500 fp32, Kolmogorov Gaussian random field + Lamb-Oseen vortex", "hurricane3d"),
    "c3": ("1D 280,953,867 fp32 particle coordinates, sorted U[0,256) + N(0,0.05), 4096-blocks shuffled",
           "particles1d"),
}


KERNEL_OF_STAGE = {"range_eb": ("k_minmax", "kernels_quant.hip"), "quantize": ("k_quant", "kernels_quant.hip"),
                   "encode": ("k_enc_stream", "kernels_encode.hip"),
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


ALGO_STAGES = ("range_eb", "quantize", "encode", "inflate", "reconstruct")


def pct(v, q):
    s = sorted(v)
    if not s:
        return float("nan")
    k = (len(s) - 1) * q
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--eb", type=float, default=1e-4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-stage-timing", action="store_true", help="time without per-stage HIP events")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="K",
                    help="after the timed steps, run K plain device copies of the field (4N bytes read, 4N "
                         "written) so hardware byte counters can be scaled against a copy of known size")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU path is not built in this repository", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2007_09625_amd import dqz
    from synth import fields

    desc, gen = WORKLOADS[args.workload]
    x_host = fields.workload(args.workload)
    n = x_host.size
    dev = torch.device("cuda:0")
    x = torch.from_numpy(x_host).to(dev)
    ctx = dqz.Context(0)
    params = dqz.make_params(args.eb, dqz.DQZ_EB_VALREL)
    shape = tuple(x.shape)
    bound, _ = dqz.dqz_compress_bound(shape, params)
    arc = torch.empty(bound, dtype=torch.uint8, device=dev)
    y = torch.empty_like(x)
    stream = torch.cuda.current_stream(dev)

    def compress():
        st, nbytes, hdr = ctx.dqz_compress(x.data_ptr(), shape, params, arc.data_ptr(), bound, stream)
        ctx._check(st, "dqz_compress")
        return nbytes, hdr

    def decompress(nbytes, hdr):
        st = ctx.dqz_decompress(arc.data_ptr(), nbytes, hdr, y.data_ptr(), y.numel(), stream)
        ctx._check(st, "dqz_decompress")

    for _ in range(args.warmup):
        nbytes, hdr = compress()
        decompress(nbytes, hdr)
    stage_timing = not args.no_stage_timing

    # per-stage breakdown, outside the timed region: HIP events between all
    # kernels of a few steps
    st_c, st_d = {}, {}
    if stage_timing:
        ctx.dqz_ctx_set_timing(1)
        for _ in range(min(max(args.steps, 3), 10)):
            nbytes, hdr = compress()
            decompress(nbytes, hdr)
            for k, v in ctx.dqz_stage_times(0).items():
                st_c.setdefault(k, []).append(v)
            for k, v in ctx.dqz_stage_times(1).items():
                st_d.setdefault(k, []).append(v)
    stages_us = {k: sum(v) / len(v) for k, v in list(st_c.items()) + list(st_d.items())}
    dom = max((k for k in ALGO_STAGES if k in stages_us), key=lambda k: stages_us[k]) if stages_us else None

    # timed region: only the dominant stage's kernel is bracketed by events
    # (on the library's stream), so its launch durations are measured live
    dom_which = 0 if dom in dqz.COMPRESS_STAGES else 1
    ctx.dqz_ctx_set_timing(dqz.timing_stage(dom_which, dom) if dom else 0)
    lat_c, lat_d, dom_us = [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        nbytes, hdr = compress()
        b = time.perf_counter()
        decompress(nbytes, hdr)
        c = time.perf_counter()
        lat_c.append(b - a)
        lat_d.append(c - b)
        if dom:
            dom_us.append(ctx.dqz_stage_times(dom_which)[dom])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.dqz_ctx_set_timing(False)

    for _ in range(args.copy_calibration):
        y.copy_(x)
    torch.cuda.synchronize()

    sec_per_step = (t1 - t0) / args.steps
    orig = 4.0 * n
    value = orig / sec_per_step / 1e9

    # correctness of the timed output (outside the timed region)
    h = dqz.dqz_archive_info(hdr)
    eb_abs = float(np.frombuffer(hdr[56:64], np.float64)[0])
    fin = torch.isfinite(x)
    err = (x.double() - y.double()).abs()[fin].max().item() if n else 0.0
    assert err <= eb_abs, f"error bound violated: {err} > {eb_abs}"
    n_out = int(np.frombuffer(hdr[88:92], np.uint32)[0])
    n_patch = int(np.frombuffer(hdr[92:96], np.uint32)[0])
    total_bits = int(np.frombuffer(hdr[96:104], np.uint64)[0])
    rmse = math.sqrt(float(((x.double() - y.double()) ** 2)[fin].mean().item())) if n else 0.0
    vrange = float(x[fin].max().item()) - float(x[fin].min().item())
    psnr = 20 * math.log10(vrange / rmse) if rmse > 0 else float("inf")
    A = float(nbytes)

    # algorithmic bytes per launch of each stage's kernel (u16 codes per
    # padded position, 128-position subchunks, 64-subchunk chunks, 512-position
    # reconstruction units)
    stream_bytes = 4.0 * ((total_bits + 31) // 32)
    exc_bytes = 8.0 * (n_out + n_patch)
    padded = padded_positions(shape)
    n_sub = (padded + 127) // 128
    n_chunks = (n_sub + 63) // 64
    n_units = (padded + 511) // 512
    algo = {
        "range_eb": 4.0 * n,
        "quantize": 4.0 * n + 2.0 * padded + exc_bytes,
        "encode": 2.0 * padded + stream_bytes + 2.0 * n_sub + 8.0 * n_chunks,
        "inflate": stream_bytes + 2.0 * n_sub + 8.0 * n_chunks + 2.0 * padded,
        "reconstruct": 2.0 * padded + exc_bytes + 4.0 * n + 4.0 * (n_units + 1),
    }
    assert set(algo) == set(ALGO_STAGES)
    roofline = None
    if dom:
        dom_avg = sum(dom_us) / len(dom_us)
        ach = algo[dom] / (dom_avg * 1e-6) / 1e9
        traffic = counted_traffic(dom, args.workload)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBPS, 4),
                    "traffic": round(traffic) if traffic is not None else None,
                    "algorithmic_bytes": algo[dom], "avg_us": round(dom_avg, 2),
                    "timed_launches": len(dom_us)}

    comp_p50, dec_p50 = pct(lat_c, 0.5), pct(lat_d, 0.5)
    comp_algo = 12.0 * n + A
    dec_algo = 4.0 * n + A
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
                   "value_definition": "4N bytes / (compress + decompress) step time",
                   "timed_region_events": f"around the {dom} stage only" if dom else "none"},
        "compress_GBps": round(orig / comp_p50 / 1e9, 2),
        "decompress_GBps": round(orig / dec_p50 / 1e9, 2),
        "compress_roofline_frac": round(comp_algo / comp_p50 / 1e9 / HBM_PEAK_GBPS, 4),
        "decompress_roofline_frac": round(dec_algo / dec_p50 / 1e9 / HBM_PEAK_GBPS, 4),
        "latency_us": {"compress_p50": round(comp_p50 * 1e6, 1), "compress_p99": round(pct(lat_c, 0.99) * 1e6, 1),
                       "decompress_p50": round(dec_p50 * 1e6, 1),
                       "decompress_p99": round(pct(lat_d, 0.99) * 1e6, 1)},
        "ratio": round(orig / A, 3),
        "bits_per_elem": round(8 * A / n, 4),
        "psnr_db": round(psnr, 3),
        "max_err_over_eb": round(err / eb_abs, 6),
        "outliers": n_out,
        "patches": n_patch,
        "stages_us": {k: round(v, 2) for k, v in stages_us.items()},
        "roofline": roofline,
        "cpu_baseline": None,
    }

    if not args.no_cpu_baseline:
        import oracle
        t = time.perf_counter()
        ref = oracle.compress(x_host, args.eb, oracle.EB_VALREL)
        tc = time.perf_counter() - t
        t = time.perf_counter()
        oracle.decompress(ref)
        td = time.perf_counter() - t
        same = bool(ref.size == nbytes and np.array_equal(ref, arc[:nbytes].cpu().numpy()))
        result["cpu_baseline"] = {"value": round(orig / (tc + td) / 1e9, 4), "unit": "GB/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"the full workload field, one compress ({tc:.2f} s) + one "
                                            f"decompress ({td:.2f} s), single-threaded C",
                                  "archive_identical_to_gpu": same}
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
