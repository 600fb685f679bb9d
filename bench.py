#!/usr/bin/env python3
"""Benchmark of the G-Interp compressor on one MI355X.

A step is one pass of the whole hot path over the workload: compression
(range, profiling, plan, interpolation predictor-quantiser with fused
histogram, host codebook, Huffman encode with outlier compaction) and
decompression (Huffman decode, outlier scatter, interpolation replay) of a
field already resident in HBM.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--workload large|small]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "compress/decompress GB/s and % HBM roofline at rel eb 1e-3; ratio; p99 latency"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "large": dict(shape=(512, 512, 512), desc="512x512x512 FP32 spectral field k^-5/3 + offset 10"),
    "small": dict(shape=(64, 64, 64), desc="64x64x64 FP32 bumps + sinusoids + N(0,1e-4)"),
}


def algorithmic_bytes(stage, n, n_anchors, n_out, n_words, n_chunks):
    """Bytes each kernel stage must move per launch (no halo re-reads, no
    scratch): the per-point figures times the points of the launch."""
    return {
        "range": 4 * n,
        "interp": 4 * n + 2 * n + 4 * n_anchors,
        "huff_stats": 2 * n + 2 * n_chunks,
        "encode": 2 * n + 4 * n_words + 8 * n_out + 4 * n_out,
        "decode": 4 * n_words + 2 * n_chunks + 2 * n,
        "scatter": 8 * n_out + 4 * n_out,
        "replay": 2 * n + 4 * n_anchors + 4 * n + 4 * n_out,
    }.get(stage)


def pct(a, q):
    a = sorted(a)
    if not a:
        return None
    k = min(len(a) - 1, max(0, int(round(q / 100.0 * (len(a) - 1)))))
    return a[k]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--eb", type=float, default=1e-3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain device copy of the input (4n bytes read, 4n written) "
                         "before the steps, to scale HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU; the compressor's path is single-GPU "
              "(see the sharding note in DESIGN.md). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2312_05492_amd as szi
    from paper_2312_05492_amd import synth

    wl = WORKLOADS[args.workload]
    x = synth.workload_large(shape=wl["shape"]) if args.workload == "large" else synth.workload_small()
    n = x.size
    in_bytes = 4 * n
    dev = torch.device("cuda:0")
    d_x = torch.from_numpy(x).to(dev)
    out = torch.empty_like(d_x)
    ctx = szi.Context(0)
    kw = dict(eb=args.eb)

    if args.calibrate_copy:
        out.copy_(d_x)
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        r = ctx.compress(d_x, **kw)
        ctx.decompress(r, out)
        r.free()
    torch.cuda.synchronize()

    ctx.set_timing(True)
    comp_stages, decomp_stages = {}, {}
    t_c, t_d = [], []
    last = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    def collect(tgt):
        # host bookkeeping only: totals accumulated by the library's events
        for k, (ms, cnt) in ctx.read_timing(reset=True).items():
            if cnt:
                acc = tgt.setdefault(k, [0.0, 0])
                acc[0] += ms
                acc[1] += cnt

    for i in range(args.steps):
        a = time.perf_counter()
        r = ctx.compress(d_x, **kw)
        b = time.perf_counter()
        collect(comp_stages)
        b2 = time.perf_counter()
        ctx.decompress(r, out)
        c = time.perf_counter()
        collect(decomp_stages)
        t_c.append(b - a)
        t_d.append(c - b2)
        if i == args.steps - 1:
            last = r
        else:
            r.free()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / args.steps

    # quality metrics of the last step (untimed)
    cr = 4.0 * n / last.compressed_bytes
    xd = d_x.double()
    diff = out.double() - xd
    max_err = float(diff.abs().max())
    mse = float((diff * diff).mean())
    rng = float(xd.max() - xd.min())
    psnr = 20 * np.log10(rng) - 10 * np.log10(mse) if mse > 0 else float("inf")
    n_out, n_words, n_chunks, n_anch = (last.raw.n_outliers, last.raw.n_words, last.raw.n_chunks,
                                        last.raw.n_anchors)
    eb_abs = args.eb * rng
    del xd, diff

    def kernel_report(stages):
        rep = {}
        for k, (ms, cnt) in stages.items():
            if k == "codebook":
                rep[k] = {"avg_ms": ms / cnt}
                continue
            avg = ms / cnt
            ab = algorithmic_bytes(k, n, n_anch, n_out, n_words, n_chunks)
            rep[k] = {"avg_ms": round(avg, 5)}
            if ab is not None and avg > 0:
                rep[k]["GBps"] = round(ab / (avg * 1e-3) / 1e9, 1)
        return rep

    comp_rep = kernel_report(comp_stages)
    decomp_rep = kernel_report(decomp_stages)
    comp_kernel_ms = sum(v["avg_ms"] for k, v in comp_rep.items() if k != "codebook")
    decomp_kernel_ms = sum(v["avg_ms"] for v in decomp_rep.values())
    # dominant kernel: the longest device stage of the step
    allk = [(v["avg_ms"], k) for k, v in list(comp_rep.items()) + list(decomp_rep.items())
            if k != "codebook"]
    dom_ms, dom = max(allk)
    dom_bytes = algorithmic_bytes(dom, n, n_anch, n_out, n_words, n_chunks)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9

    line = {
        "metric": METRIC,
        "value": round(in_bytes / step_s / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "shape": list(wl["shape"]), "eb_rel": args.eb,
                   "interp": "cubic auto (profiled)", "anchor_stride": 8, "radius": 512,
                   "huffman_chunk": 1024},
        "compress_GBps": round(in_bytes / float(np.median(t_c)) / 1e9, 2),
        "decompress_GBps": round(in_bytes / float(np.median(t_d)) / 1e9, 2),
        "compress_kernel_GBps": round(in_bytes / (comp_kernel_ms * 1e-3) / 1e9, 2),
        "decompress_kernel_GBps": round(in_bytes / (decomp_kernel_ms * 1e-3) / 1e9, 2),
        "latency_ms": {"compress_p50": round(pct(t_c, 50) * 1e3, 3),
                       "compress_p99": round(pct(t_c, 99) * 1e3, 3),
                       "decompress_p50": round(pct(t_d, 50) * 1e3, 3),
                       "decompress_p99": round(pct(t_d, 99) * 1e3, 3)},
        "kernels": {"compress": comp_rep, "decompress": decomp_rep},
        "ratio": round(cr, 3),
        "bitrate": round(32.0 / cr, 4),
        "psnr_db": round(psnr, 2),
        "max_abs_err": max_err,
        "eb_abs": eb_abs,
        "outlier_fraction": n_out / n,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": None},
    }
    last.free()
    ctx.close()
    del d_x, out

    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        p = oracle.Params(shape=x.shape, eb=args.eb)
        a = time.perf_counter()
        ref = oracle.compress(x, p)
        blob = ref.blob()
        b = time.perf_counter()
        oracle.decompress_blob(blob)
        c = time.perf_counter()
        line["cpu_baseline"] = {"value": round(in_bytes / (c - a) / 1e9, 4), "unit": "GB/s",
                                "cores": 1, "kind": "oracle",
                                "sample": "the full workload field, one compress + one decompress, "
                                          "single-threaded C oracle (%.1f s + %.1f s)" % (b - a, c - b)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
