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
    "line": dict(shape=(1 << 27,), desc="2^27-point 1D FP32 spectral field k^-5/3 + offset 10 "
                                        "(anchors every 512, windows of 2048)"),
}


def algorithmic_bytes(stage, n, n_anchors, n_out, n_words, n_chunks):
    """Bytes each kernel stage must move per launch (no halo re-reads, no
    scratch): the per-point figures times the points of the launch.  The
    pass over the codes that counts each chunk's bits (huff_stats) moves
    nothing the pipeline needs beyond what the encode reads, so it has none:
    its time counts, its bytes do not."""
    return {
        "range": 4 * n,
        "interp": 4 * n + 2 * n + 4 * n_anchors,
        "huff_stats": 0,
        "encode": 2 * n + 4 * n_words + 2 * n_chunks + 8 * n_out,
        "decode": 4 * n_words + 2 * n_chunks + 16 * n_chunks + 2 * n,   # + the part offsets
        "replay": 2 * n + 4 * n_anchors + 4 * n + 8 * n_out,
    }.get(stage)


def pipeline_bytes(n, n_anchors, n_out, n_words, n_chunks):
    """Algorithmic bytes of a whole compression and decompression: read the
    field twice (range, interpolation), write and read the quant-codes once,
    the anchors, the outlier lists (index and value) and the bitstream with
    its chunk sizes; decompression reads the bitstream, writes and reads the
    codes, reads anchors and outliers and writes the field (about 12 + b/8
    and 8 + b/8 bytes per point for b bits per symbol)."""
    meta = 4 * n_anchors + 8 * n_out + 4 * n_words + 2 * n_chunks
    return {"compress": 4 * n + 4 * n + 2 * n + 2 * n + meta,
            "decompress": 2 * n + 2 * n + 4 * n + meta}


INTERP = {   # per numpy axis, slowest first (0 linear, 1 not-a-knot, 2 natural, 3 profiled)
    "auto": (3, 3, 3), "linear": (0, 0, 0), "mixed": (0, 3, 3), "nak": (1, 1, 1), "natural": (2, 2, 2),
}
INTERP_DESC = {"auto": "cubic per dimension by profiling (Sec. V-C.1)", "linear": "linear in every dimension",
               "mixed": "linear along z, cubic by profiling along y and x", "nak": "not-a-knot cubic",
               "natural": "natural cubic"}


def host_cpu():
    """Model name and usable logical CPUs of the host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return model, ncpu


# per-launch HBM traffic from rocprofv3 read-request and WRITE_SIZE runs
# (python bench.py --pmc-summary), kept with a hash of the kernel sources
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_512cube_rel1e-3.md")
STAGE_KERNELS = {"range": "k_range", "interp": "k_compress<3>", "huff_stats": "k_huff_stats",
                 "encode": "k_huff_encode", "decode": "k_huff_decode",
                 "replay": "k_decompress<3>"}


def kernel_source_hash():
    """A hash of the device sources (the kernels and the headers they
    include): host-only code does not change what the counters measured."""
    import hashlib
    h = hashlib.sha256()
    for sub in ("paper_2312_05492_amd/csrc", "include"):
        d = os.path.join(ROOT, sub)
        for f in sorted(os.listdir(d)):
            if f.endswith((".hip", ".h")):
                h.update(f.encode())
                h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


def read_traffic():
    """{kernel: bytes per launch} if the profile matches the current sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return {}
    txt = open(TRAFFIC_FILE).read()
    if "kernel-source-sha256: " + kernel_source_hash() not in txt:
        return {}
    out = {}
    for line in txt.split("\n"):
        if line.startswith("bytes-per-launch "):
            _, k, v = line.split()
            out[k] = int(v)
    return out


def pmc_summary(read_csv, write_csv, n, cmd, out_path):
    """HBM bytes per launch of every stage kernel from two rocprofv3 counter
    runs: reads from the L2's requests to memory by size (32, 64 and 128
    bytes: TCC_EA0_RDREQ_32B/64B/128B), writes from WRITE_SIZE (KiB, which
    counts 32- and 64-byte write requests).  The calibration copy of the
    input (4n bytes read, 4n written) is reported as a check of both."""
    import csv
    import collections

    def load(path):
        acc = collections.defaultdict(lambda: collections.defaultdict(list))
        for r in csv.DictReader(open(path)):
            acc[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
        return {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}, \
            {k: max(len(v) for v in cs.values()) for k, cs in acc.items()}

    def short(k):
        k = k.replace("void ", "").replace("szi::", "")
        k = k[:k.index("(")] if "(" in k else k
        # the window kernels keep their dimensionality (not the register
        # variant), the rest their base name
        base = k.split("<")[0]
        if k.startswith(("k_compress", "k_decompress")) and "<" in k:
            return base + "<" + k.split("<")[1].split(",")[0].split(">")[0].strip() + ">"
        return base

    rd, nrd = load(read_csv)
    wr, _ = load(write_csv)
    need = ("TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum")
    if not any(all(c in cs for c in need) for cs in rd.values()):
        raise SystemExit("%s holds no %s counters" % (read_csv, ", ".join(need)))
    if not any("WRITE_SIZE" in cs for cs in wr.values()):
        raise SystemExit("%s holds no WRITE_SIZE counter" % write_csv)

    def read_bytes(c):
        return (32.0 * c.get("TCC_EA0_RDREQ_32B_sum", 0.0) + 64.0 * c.get("TCC_EA0_RDREQ_64B_sum", 0.0)
                + 128.0 * c.get("TCC_EA0_RDREQ_128B_sum", 0.0))

    def largest_copy(path, value):
        """(bytes, microseconds) of the device copy dispatch with the most
        bytes (the calibration copy), its duration from the dispatch's
        timestamps."""
        per = collections.defaultdict(dict)
        for r in csv.DictReader(open(path)):
            if "copyBuffer" in r["Kernel_Name"]:
                per[r["Dispatch_Id"]][r["Counter_Name"]] = float(r["Counter_Value"])
                per[r["Dispatch_Id"]]["_us"] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        return max(((value(c), c["_us"]) for c in per.values()), default=(float("nan"), float("nan")))

    copy_r, copy_us = largest_copy(read_csv, read_bytes)
    copy_w, _ = largest_copy(write_csv, lambda c: c.get("WRITE_SIZE", 0.0) * 1024.0)
    rows = []
    for k in rd:
        sk = short(k)
        if sk not in STAGE_KERNELS.values() or k not in wr:
            continue
        rows.append((sk, nrd[k], read_bytes(rd[k]), wr[k]["WRITE_SIZE"] * 1024.0))
    with open(out_path, "w") as o:
        o.write("# HBM traffic per launch, 512^3 FP32 field, rel eb 1e-3\n\n")
        o.write("From two rocprofv3 counter runs of the same command:\n\n")
        o.write("```\n" + cmd + "\n```\n\n")
        o.write("Reads are 32, 64 and 128 bytes times the L2's read requests to memory of each size "
                "(TCC_EA0_RDREQ_32B, _64B, _128B, summed over the L2 channels of all XCDs), writes "
                "WRITE_SIZE (KiB, 32- and 64-byte write requests), each averaged over the kernel's "
                "dispatches.  Check: the calibration copy of the input (`--calibrate-copy`, %d bytes "
                "read once and written once) reads %.1f MB and writes %.1f MB by these counters "
                "(%.1f MB each expected), in %.1f us: %.2f TB/s read and written together (the "
                "streaming rate the chip reaches).\n\n" % (4 * n, copy_r / 1e6, copy_w / 1e6, 4 * n / 1e6,
                                                          copy_us, (copy_r + copy_w) / (copy_us * 1e-6) / 1e12))
        o.write("| kernel | dispatches | HBM read MB | HBM write MB | total MB |\n|---|---|---|---|---|\n")
        for sk, c, f, w in rows:
            o.write("| %s | %d | %.1f | %.1f | %.1f |\n" % (sk, c, f / 1e6, w / 1e6, (f + w) / 1e6))
        o.write("\nThe numbers hold for the kernel sources with this hash (bench.py reports "
                "them as roofline.traffic only while it matches):\n\n")
        o.write("kernel-source-sha256: %s\n\n```\n" % kernel_source_hash())
        for sk, c, f, w in rows:
            o.write("bytes-per-launch %s %d\n" % (sk, int(round(f + w))))
        o.write("```\n")


def short_kernel(k):
    """A kernel's name without its namespace, return type and arguments
    (library kernels of torch cut to their first template argument)."""
    k = k.replace("void ", "").replace("szi::", "")
    k = k[:k.index("(")] if "(" in k else k
    if k.startswith("at::native::"):
        k = "torch: " + k[len("at::native::"):].split(",")[0] + (">" if "<" in k else "")
    return k


def trace_summary(stats_csv, cmd, out_path, title):
    """rocprofv3 --kernel-trace --stats kernel table as a short markdown file."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    with open(out_path, "w") as o:
        o.write("# %s\n\nCommand (from the repository root on an MI355X host, $REPO being that "
                "root):\n\n```\n%s\n```\n\n" % (title, cmd))
        o.write("| kernel | calls | total us | average us | min us | max us | % |\n"
                "|---|---|---|---|---|---|---|\n")
        for r in rows:
            o.write("| %s | %s | %.1f | %.1f | %.1f | %.1f | %.1f |\n" % (
                short_kernel(r["Name"]), r["Calls"], float(r["TotalDurationNs"]) / 1e3,
                float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
                float(r["Percentage"])))


COUNTER_KERNELS = ("k_range", "k_compress", "k_huff_stats", "k_huff_encode", "k_elide_count",
                   "k_huff_decode", "k_decompress")


def counter_summary(csvs, cmd, out_path, title):
    """Per-dispatch averages of SQ/GRBM counters over one or more rocprofv3
    --pmc runs (one pass each), per kernel, with per-wave instruction counts
    and the derived ratios the kernels are tuned on."""
    import csv
    import collections
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    res = {}
    for path in csvs:
        for r in csv.DictReader(open(path)):
            k = short_kernel(r["Kernel_Name"])
            if not k.startswith(COUNTER_KERNELS):
                continue
            acc[k][r["Counter_Name"]].append(float(r["Counter_Value"]))
            res[k] = (r["Workgroup_Size"], r["LDS_Block_Size"], r["VGPR_Count"],
                      r["Accum_VGPR_Count"], r["SGPR_Count"])
    avg = {k: {c: sum(v) / len(v) for c, v in cs.items()} for k, cs in acc.items()}
    names = sorted({c for cs in avg.values() for c in cs})
    with open(out_path, "w") as o:
        o.write("# %s\n\nOne rocprofv3 counter pass per line (the SQ block collects at most 8 "
                "counters a pass), from the repository root on an MI355X host, $REPO being that "
                "root:\n\n```\n%s\n```\n\n" % (title, cmd))
        o.write("## Resources per kernel\n\n| kernel | workgroup | LDS bytes | VGPR | AGPR | SGPR |\n"
                "|---|---|---|---|---|---|\n")
        for k in sorted(res):
            o.write("| %s | %s | %s | %s | %s | %s |\n" % ((k,) + res[k]))
        o.write("\n## Counters, average per dispatch\n\n| counter | " + " | ".join(sorted(avg)) +
                " |\n|---|" + "---|" * len(avg) + "\n")
        for c in names:
            o.write("| %s | " % c + " | ".join(
                "%.0f" % avg[k][c] if c in avg[k] else "" for k in sorted(avg)) + " |\n")
        o.write("\n## Derived\n\n"
                "* per wave: instructions of each kind over SQ_WAVES;\n"
                "* kernel cycles: GRBM_GUI_ACTIVE / 8 (the counter sums the 8 XCDs);\n"
                "* resident waves per CU: 4 SQ_WAVE_CYCLES / (256 x kernel cycles) (wave "
                "cycles count in units of 4 cycles);\n"
                "* VALU busy: 4 SQ_ACTIVE_INST_VALU / (1024 SIMDs x kernel cycles);\n"
                "* LDS bank conflicts: SQ_LDS_BANK_CONFLICT over SQ_ACTIVE_INST_LDS (cycles);\n"
                "* issue stall: SQ_WAIT_INST_ANY over SQ_WAVE_CYCLES.\n\n")
        o.write("| kernel | waves | VALU/wave | SALU/wave | LDS/wave | VMEM rd/wave | VMEM wr/wave | "
                "kernel cycles | waves/CU | VALU busy | LDS conflict/active | issue stall |\n"
                "|---|---|---|---|---|---|---|---|---|---|---|---|\n")

        def g(d, c):
            return d.get(c)

        def ratio(a, b, scale=1.0, fmt="%.0f"):
            return fmt % (scale * a / b) if a is not None and b else ""

        for k in sorted(avg):
            d = avg[k]
            w = g(d, "SQ_WAVES")
            cyc = g(d, "GRBM_GUI_ACTIVE")
            cyc = cyc / 8.0 if cyc else None
            o.write("| %s | %s | %s | %s | %s | %s | %s | %s | %s | %s | %s | %s |\n" % (
                k, "%.0f" % w if w else "",
                ratio(g(d, "SQ_INSTS_VALU"), w), ratio(g(d, "SQ_INSTS_SALU"), w),
                ratio(g(d, "SQ_INSTS_LDS"), w), ratio(g(d, "SQ_INSTS_VMEM_RD"), w),
                ratio(g(d, "SQ_INSTS_VMEM_WR"), w), "%.0f" % cyc if cyc else "",
                ratio(g(d, "SQ_WAVE_CYCLES"), (256 * cyc) if cyc else None, 4.0, "%.1f"),
                ratio(g(d, "SQ_ACTIVE_INST_VALU"), (1024 * cyc) if cyc else None, 4.0, "%.2f"),
                ratio(g(d, "SQ_LDS_BANK_CONFLICT"), g(d, "SQ_ACTIVE_INST_LDS"), 1.0, "%.2f"),
                ratio(g(d, "SQ_WAIT_INST_ANY"), g(d, "SQ_WAVE_CYCLES"), 1.0, "%.2f")))


def pct(a, q):
    a = sorted(a)
    if not a:
        return None
    k = min(len(a) - 1, max(0, int(round(q / 100.0 * (len(a) - 1)))))
    return a[k]


BATCHES = {
    "c3": "24 x 1800x3600 FP32 climate-like 2D fields (zonal + k^-3, 5 % fill), rel eb 1e-3",
    "c4": "13 x 100x500x500 + 6 x 256x384x384 FP32 fields (k^-5/3, k^-3, one tanh front), "
          "rel eb cycling 1e-2, 1e-3, 1e-4",
}


def run_batch(args):
    """Many fields: one batched compress and decompress call over all of them
    versus one call per field, on the same GPU and inputs.  Prints one JSON
    line; every batched blob and reconstruction must equal the per-field one."""
    import numpy as np
    import torch

    import paper_2312_05492_amd as szi
    from paper_2312_05492_amd import synth

    if args.batch == "c3":
        fields = synth.climate_batch()
        params = [dict(eb=1e-3) for _ in fields]
    else:
        fields, ebs = synth.uneven_batch()
        params = [dict(eb=e) for e in ebs]
    dev = torch.device("cuda:0")
    xs = [torch.from_numpy(f).to(dev) for f in fields]
    host_fields = fields
    outs = [torch.empty_like(x) for x in xs]
    in_bytes = sum(4 * x.numel() for x in xs)
    ctx = szi.Context(0)

    def per_field():
        rs = []
        for x, kw, o in zip(xs, params, outs):
            r = ctx.compress(x, **kw)
            ctx.decompress(r, o)
            rs.append(r)
        return rs

    def batched():
        rs = ctx.compress_batch(xs, params)
        ctx.decompress_batch(rs, outs)
        return rs

    def timed(fn):
        for r in fn():   # warm-up
            r.free()
        ts = []
        for _ in range(args.steps):
            torch.cuda.synchronize()
            a = time.perf_counter()
            rs = fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - a)
            for r in rs:
                r.free()
        return float(np.median(ts))

    t_single = timed(per_field)
    t_batch_untuned = timed(batched)
    # the launch-shape tuner: the first call per (kind, ndim, radius) times
    # the candidate shapes and keeps the fastest (results unchanged)
    ctx.set_tuning(True)
    t_batch = timed(batched)
    # the same batches through the library's captured graphs
    ctx.set_graphs(True)
    t_batch_graph = timed(batched)
    ctx.set_graphs(False)
    # given code books (each field's own histogram, every count plus one,
    # as a time series would reuse them): no host round trip in the batch
    rs = batched()
    books = [szi.code_lengths(r.read(szi.SEC_HIST)) for r in rs]
    for r in rs:
        r.free()

    def batched_books():
        rs = ctx.compress_batch_with_code(xs, books, params)
        ctx.decompress_batch(rs, outs)
        return rs

    t_books = timed(batched_books)
    ctx.set_graphs(True)
    t_books_graph = timed(batched_books)
    ctx.set_graphs(False)
    rs = batched_books()
    comp_books = sum(r.compressed_bytes for r in rs)
    for r in rs:
        r.free()
    nd = xs[0].dim()
    shapes = {k: ctx.shape(i, nd)[:2] for i, k in enumerate(("interp", "replay"))}
    # identity: the batched results equal the per-field ones, bit for bit
    rs1 = per_field()
    y1 = [o.clone() for o in outs]
    rs2 = batched()
    same = all(a.blob() == b.blob() for a, b in zip(rs1, rs2)) and all(
        torch.equal(a.view(torch.int32), b.view(torch.int32)) for a, b in zip(y1, outs))
    comp = sum(r.compressed_bytes for r in rs2)
    for r in rs1 + rs2:
        r.free()
    ctx.close()
    print(json.dumps({
        "metric": "batched compress+decompress GB/s vs one field per call",
        "value": round(in_bytes / t_batch / 1e9, 2), "unit": "GB/s",
        "per_field_call_GBps": round(in_bytes / t_single / 1e9, 2),
        "speedup": round(t_single / t_batch, 3),
        "ms_batched": round(t_batch * 1e3, 3), "ms_per_field_calls": round(t_single * 1e3, 3),
        "ms_batched_default_shape": round(t_batch_untuned * 1e3, 3),
        "ms_batched_graphs": round(t_batch_graph * 1e3, 3),
        "ms_batched_given_books": round(t_books * 1e3, 3),
        "ms_batched_given_books_graphs": round(t_books_graph * 1e3, 3),
        "ratio_given_books": round(in_bytes / comp_books, 3),
        "tuned_shapes": {k: {"variant": v[0], "workgroups_per_cu": v[1]} for k, v in shapes.items()},
        "steps": args.steps, "fields": len(xs), "input_bytes": in_bytes,
        "ratio": round(in_bytes / comp, 3), "identical": bool(same),
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": BATCHES[args.batch]},
        "cpu_baseline": None if args.no_cpu_baseline else threaded_oracle(host_fields, params)}),
        flush=True)


def threaded_oracle(fields, params):
    """The CPU oracle over a batch: every field compressed and decompressed
    once, one host thread per field (up to the usable logical CPUs; the C
    oracle runs without the interpreter lock)."""
    import concurrent.futures as cf

    import oracle
    oracle.build(force=False)
    model, ncpu = host_cpu()
    workers = max(1, min(len(fields), ncpu))

    def one(k):
        x, kw = fields[k], params[k]
        p = oracle.Params(shape=x.shape, eb=kw.get("eb", 1e-3))
        oracle.decompress_blob(oracle.compress(x, p).blob())

    a = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(one, range(len(fields))))
    t = time.perf_counter() - a
    nbytes = sum(4 * f.size for f in fields)
    return {"value": round(nbytes / t / 1e9, 4), "unit": "GB/s", "cores": workers, "kind": "oracle",
            "sample": "every field of the batch compressed and decompressed once, one thread per "
                      "field on %d threads, %.1f s" % (workers, t),
            "cpu_model": model, "host_logical_cpus": ncpu}


SERVE_DESC = ("Poisson stream of 2000 requests, half compress, half decompress; sizes log-uniform "
              "64^3..512^3 (3D, k^-5/3 + offset) and 512^2..3600^2 (2D climate-like), drawn from a "
              "pool of 10 + 8 pre-generated fields; rel eb from {1e-2, 1e-3, 1e-4}; 200 GB budget; "
              "server_books: compressions name a resident code book per field and bound")


def run_serve(args):
    """Serving: the same request trace through the request server (slots
    overlapping on the device, HBM admission) and through sequential plain
    calls, at 0.8 of the sequential capacity (latency) and saturated (all
    requests queued at once: throughput).  Prints one JSON line."""
    import gc
    import threading

    import numpy as np
    import torch

    import paper_2312_05492_amd as szi
    from paper_2312_05492_amd import synth

    rng = np.random.default_rng(5)
    dev = torch.device("cuda:0")
    sides3 = np.unique(np.round(np.exp(np.linspace(np.log(64), np.log(512), 10))).astype(int))
    sides2 = np.unique(np.round(np.exp(np.linspace(np.log(512), np.log(3600), 8))).astype(int))
    pool = []   # (tensor, bytes)
    for k, a in enumerate(sides3):
        pool.append(torch.from_numpy(synth.spectral_field((a, a, a), seed=700 + k, mean=10.0)).to(dev))
    for k, a in enumerate(sides2):
        pool.append(torch.from_numpy(synth.climate_field(800 + k, shape=(a, a))).to(dev))
    logn = np.log([x.numel() for x in pool])
    n3 = len(sides3)
    ebs = [1e-2, 1e-3, 1e-4]
    ctx = szi.Context(0)
    src = {}   # (field, eb) -> compressed result for decompression requests
    for i, x in enumerate(pool):
        for e in ebs:
            src[(i, e)] = ctx.compress(x, eb=e)
    nreq = args.requests
    reqs = []
    for _ in range(nreq):
        three = rng.random() < 0.5
        lo, hi = (np.log(64 ** 3), np.log(512 ** 3)) if three else (np.log(512 ** 2), np.log(3600 ** 2))
        want = rng.uniform(lo, hi)
        cand = range(n3) if three else range(n3, len(pool))
        f = min(cand, key=lambda i: abs(logn[i] - want))
        reqs.append(("c" if rng.random() < 0.5 else "d", f, ebs[rng.integers(3)]))
    slots = args.slots
    nout = slots + 2
    outs = {}
    for _, f, _ in reqs:
        if f not in outs:
            outs[f] = [torch.empty_like(pool[f]) for _ in range(nout)]
    req_bytes = [4 * pool[f].numel() for _, f, _ in reqs]
    total = float(sum(req_bytes))

    def plain(i, k):
        kind, f, e = reqs[i]
        if kind == "c":
            ctx.compress(pool[f], eb=e).free()
        else:
            ctx.decompress(src[(f, e)], outs[f][k % nout])

    # warm-up, and the mean service time of plain calls
    for i in range(min(50, nreq)):
        plain(i, i)
    torch.cuda.synchronize()
    a = time.perf_counter()
    for i in range(min(200, nreq)):
        plain(i, i)
    torch.cuda.synchronize()
    svc = (time.perf_counter() - a) / min(200, nreq)
    rate = 0.8 / svc
    gaps = rng.exponential(1.0 / rate, nreq)
    arrive = np.cumsum(gaps) - gaps[0]

    def sequential(at):
        lat = []
        t0 = time.perf_counter()
        for i in range(nreq):
            now = time.perf_counter() - t0
            if at[i] > now:
                time.sleep(at[i] - now)
            plain(i, i)
            lat.append(time.perf_counter() - t0 - at[i])
        return time.perf_counter() - t0, lat

    def book_of(f, e):   # a resident code book per pool field and bound
        return 1 + 3 * f + ebs.index(e)

    def served(at, books=False):
        srv = szi.Server(0, slots=slots, hbm_budget=200 * 10 ** 9)
        # warm-up like the plain calls': the slots' pools and caches fill
        for i in range(min(250, nreq)):
            kind, f, e = reqs[i]
            if kind == "c":
                srv.submit_compress(pool[f], tag=i, eb=e, book=book_of(f, e) if books else 0)
            else:
                srv.submit_decompress(src[(f, e)], outs[f][i % nout], tag=i)
        left = min(250, nreq)
        while left:
            for c in srv.poll(wait=True):
                assert c["status"] == 0, c
                if c["result"] is not None:
                    c["result"].free()
                left -= 1
        lat = [None] * nreq
        t_first = [None]

        def submit():
            t0 = time.perf_counter()
            for i in range(nreq):
                now = time.perf_counter() - t0
                if at[i] > now:
                    time.sleep(at[i] - now)
                kind, f, e = reqs[i]
                if kind == "c":
                    srv.submit_compress(pool[f], tag=i, eb=e, book=book_of(f, e) if books else 0)
                else:
                    srv.submit_decompress(src[(f, e)], outs[f][i % nout], tag=i)

        th = threading.Thread(target=submit)
        th.start()
        got = 0
        t_sub, t_done = [], []
        while got < nreq:
            for c in srv.poll(wait=True):
                assert c["status"] == 0, c
                lat[c["tag"]] = c["t_done"] - c["t_submit"]
                t_sub.append(c["t_submit"])
                t_done.append(c["t_done"])
                if c["result"] is not None:
                    c["result"].free()
                got += 1
        th.join()
        srv.close()
        return max(t_done) - min(t_sub), lat

    out = {"metric": "served compress/decompress GB/s and p50/p99 latency vs sequential plain calls",
           "unit": "GB/s", "higher_is_better": True, "requests": nreq, "slots": slots,
           "data": "synthetic", "dtype": "f32", "config": {"workload": SERVE_DESC},
           "plain_call_mean_ms": round(svc * 1e3, 3), "offered_rate_per_s": round(rate, 1)}
    for name, at in (("load0.8", arrive), ("saturated", np.zeros(nreq))):
        for mode, fn in (("server", served), ("server_books", lambda at: served(at, True)),
                         ("sequential", sequential)):
            # no cyclic garbage collection inside a timed run: its pauses
            # (tens of ms) would hold up the submitting thread
            gc.collect()
            gc.disable()
            try:
                span, lat = fn(at)
            finally:
                gc.enable()
            lat = sorted(lat)
            out["%s_%s" % (mode, name)] = {
                "GBps": round(total / span / 1e9, 2),
                "p50_ms": round(pct(lat, 50) * 1e3, 3), "p99_ms": round(pct(lat, 99) * 1e3, 3),
                "makespan_s": round(span, 3)}
    out["value"] = out["server_load0.8"]["GBps"]
    for r in src.values():
        r.free()
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=sorted(WORKLOADS))
    ap.add_argument("--eb", type=float, default=1e-3)
    ap.add_argument("--interp", default="auto", choices=sorted(INTERP),
                    help="spline per dimension: " + "; ".join("%s = %s" % kv for kv in sorted(INTERP_DESC.items())))
    ap.add_argument("--chunk", type=int, default=1024, choices=(256, 512, 1024, 2048),
                    help="Huffman chunk length in symbols")
    ap.add_argument("--stride", type=int, default=0,
                    help="anchor stride (0: 8 in 3D, 16 in 2D, 512 in 1D)")
    ap.add_argument("--window", default="",
                    help="window per numpy axis, e.g. 8,16,16 (default: four chunks along x, one "
                         "along the others); other strides and windows run the generic window kernels")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain device copy of the input (4n bytes read, 4n written) "
                         "before the steps, to scale HBM byte counters")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("READ_CSV", "WRITE_CSV"),
                    help="write the HBM traffic summary from two rocprofv3 counter runs and exit")
    ap.add_argument("--pmc-command", default="", help="the profiled command, for the summary")
    ap.add_argument("--trace-summary", nargs=2, metavar=("STATS_CSV", "OUT_MD"),
                    help="write a kernel time summary from a rocprofv3 --kernel-trace --stats "
                         "run and exit")
    ap.add_argument("--counter-summary", nargs="+", metavar="CSV",
                    help="OUT_MD then the counter_collection.csv of each rocprofv3 --pmc pass: "
                         "write a counter summary and exit")
    ap.add_argument("--title", default="", help="the summary's title")
    ap.add_argument("--serve", action="store_true",
                    help="request server vs sequential plain calls on a Poisson trace (own JSON line)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--batch", choices=sorted(BATCHES),
                    help="batched vs per-field calls on a many-field workload (own JSON line)")
    args = ap.parse_args()
    if args.batch:
        run_batch(args)
        return
    if args.serve:
        run_serve(args)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary[0], args.pmc_command, args.trace_summary[1], args.title)
        return
    if args.counter_summary:
        counter_summary(args.counter_summary[1:], args.pmc_command, args.counter_summary[0], args.title)
        return
    if args.pmc_summary:
        shape = WORKLOADS[args.workload]["shape"]
        n = 1
        for d in shape:
            n *= d
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], n, args.pmc_command, TRAFFIC_FILE)
        return
    if args.gpus != 1:
        print("bench.py: measures one GPU only (windows are independent, so a field would "
              "shard into slabs with one borrowed plane each, which is not built); "
              "run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2312_05492_amd as szi
    from paper_2312_05492_amd import synth

    wl = WORKLOADS[args.workload]
    x = synth.workload_small() if args.workload == "small" else synth.workload_large(shape=wl["shape"])
    n = x.size
    in_bytes = 4 * n
    dev = torch.device("cuda:0")
    d_x = torch.from_numpy(x).to(dev)
    out = torch.empty_like(d_x)
    ctx = szi.Context(0)
    kw = dict(eb=args.eb, chunk=args.chunk, interp=INTERP[args.interp][-x.ndim:])
    if args.stride:
        kw["S"] = args.stride
    if args.window:
        kw["window"] = tuple(int(v) for v in args.window.split(","))

    if args.calibrate_copy:
        out.copy_(d_x)
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        r = ctx.compress(d_x, **kw)
        ctx.decompress(r, out)
        r.free()
    torch.cuda.synchronize()

    def run_steps(k, keep_last, collect=None):
        tc, td, r_last = [], [], None
        for i in range(k):
            a = time.perf_counter()
            r = ctx.compress(d_x, **kw)
            b = time.perf_counter()
            if collect:
                collect[0]()
            b2 = time.perf_counter()
            ctx.decompress(r, out)
            c = time.perf_counter()
            if collect:
                collect[1]()
            tc.append(b - a)
            td.append(c - b2)
            if keep_last and i == k - 1:
                r_last = r
            else:
                r.free()
        return tc, td, r_last

    # the timed steps: the plain one-field-per-call path, no instrumentation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_c, t_d, last = run_steps(args.steps, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_s = (t1 - t0) / args.steps

    # untimed: per-stage device time from the library's events
    comp_stages, decomp_stages = {}, {}

    def collector(tgt):
        def f():
            for k, (ms, cnt) in ctx.read_timing(reset=True).items():
                if cnt:
                    acc = tgt.setdefault(k, [0.0, 0])
                    acc[0] += ms
                    acc[1] += cnt
        return f

    ctx.set_timing(True)
    ctx.read_timing(reset=True)
    run_steps(max(1, min(args.steps, 5)), False, (collector(comp_stages), collector(decomp_stages)))
    ctx.set_timing(False)
    # untimed: the same calls through the library's captured graphs
    ctx.set_graphs(True)
    run_steps(2, False)
    g_c, g_d, _ = run_steps(max(1, min(args.steps, 5)), False)
    ctx.set_graphs(False)
    torch.cuda.synchronize()
    # untimed: compression with a reused code book (the last step's
    # histogram, every count plus one), which skips the host round trip
    book = szi.code_lengths(last.read(szi.SEC_HIST))
    for _ in range(2):
        ctx.compress_with_code(d_x, book, **kw).free()
    b_c = []
    for _ in range(max(3, min(args.steps, 10))):
        torch.cuda.synchronize()
        a = time.perf_counter()
        r = ctx.compress_with_code(d_x, book, **kw)
        b_c.append(time.perf_counter() - a)
        r.free()
    torch.cuda.synchronize()
    # the same through the captured graphs (both run back to back)
    ctx.set_graphs(True)
    for _ in range(2):
        ctx.compress_with_code(d_x, book, **kw).free()
    bg_c = []
    for _ in range(max(3, min(args.steps, 10))):
        torch.cuda.synchronize()
        a = time.perf_counter()
        r = ctx.compress_with_code(d_x, book, **kw)
        bg_c.append(time.perf_counter() - a)
        r.free()
    ctx.set_graphs(False)
    torch.cuda.synchronize()

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
                rep[k] = {"avg_ms": round(ms / cnt, 5)}
                continue
            avg = ms / cnt
            ab = algorithmic_bytes(k, n, n_anch, n_out, n_words, n_chunks)
            rep[k] = {"avg_ms": round(avg, 5)}
            if ab and avg > 0:
                rep[k]["GBps"] = round(ab / (avg * 1e-3) / 1e9, 1)
        return rep

    comp_rep = kernel_report(comp_stages)
    decomp_rep = kernel_report(decomp_stages)
    comp_kernel_ms = sum(v["avg_ms"] for k, v in comp_rep.items() if k != "codebook")
    decomp_kernel_ms = sum(v["avg_ms"] for v in decomp_rep.values())
    # dominant kernel: the longest device stage of the step that moves the
    # field's data (on small fields a fixed-cost stage can take longer)
    allk = [(v["avg_ms"], k) for k, v in list(comp_rep.items()) + list(decomp_rep.items())
            if k != "codebook" and algorithmic_bytes(k, n, n_anch, n_out, n_words, n_chunks)]
    dom_ms, dom = max(allk)
    dom_bytes = algorithmic_bytes(dom, n, n_anch, n_out, n_words, n_chunks)
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    pb = pipeline_bytes(n, n_anch, n_out, n_words, n_chunks)
    pipe = {}
    for k, ms in (("compress", comp_kernel_ms), ("decompress", decomp_kernel_ms)):
        gbs = pb[k] / (ms * 1e-3) / 1e9
        pipe[k] = {"kernel_ms": round(ms, 4), "algorithmic_bytes": int(pb[k]),
                   "bytes_per_point": round(pb[k] / n, 3), "GBps": round(gbs, 1),
                   "frac": round(gbs / HBM_PEAK_GBS, 4)}
    default_geometry = not args.stride and not args.window
    traffic = read_traffic().get(STAGE_KERNELS.get(dom)) if args.workload == "large" and default_geometry else None

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
                   "interp": INTERP_DESC[args.interp],
                   "anchor_stride": args.stride or {3: 8, 2: 16, 1: 512}[x.ndim],
                   "window": list(kw["window"]) if "window" in kw else "default", "radius": 512,
                   "huffman_chunk": args.chunk},
        "compress_GBps": round(in_bytes / float(np.median(t_c)) / 1e9, 2),
        "decompress_GBps": round(in_bytes / float(np.median(t_d)) / 1e9, 2),
        "compress_kernel_GBps": round(in_bytes / (comp_kernel_ms * 1e-3) / 1e9, 2),
        "decompress_kernel_GBps": round(in_bytes / (decomp_kernel_ms * 1e-3) / 1e9, 2),
        "latency_ms": {"compress_p50": round(pct(t_c, 50) * 1e3, 3),
                       "compress_p99": round(pct(t_c, 99) * 1e3, 3),
                       "decompress_p50": round(pct(t_d, 50) * 1e3, 3),
                       "decompress_p99": round(pct(t_d, 99) * 1e3, 3)},
        "graph_latency_ms": {"compress_p50": round(pct(g_c, 50) * 1e3, 3),
                             "decompress_p50": round(pct(g_d, 50) * 1e3, 3)},
        "reused_code_book_compress_p50_ms": round(pct(b_c, 50) * 1e3, 3),
        "reused_code_book_graph_compress_p50_ms": round(pct(bg_c, 50) * 1e3, 3),
        "kernels": {"compress": comp_rep, "decompress": decomp_rep},
        "pipeline_roofline": pipe,
        "ratio": round(cr, 3),
        "bitrate": round(32.0 / cr, 4),
        "psnr_db": round(psnr, 2),
        "max_abs_err": max_err,
        "eb_abs": eb_abs,
        "outlier_fraction": n_out / n,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "algorithmic_bytes": int(dom_bytes)},
    }
    last.free()
    ctx.close()
    del d_x, out

    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        p = oracle.Params(shape=x.shape, eb=args.eb, chunk=args.chunk, interp=INTERP[args.interp][-x.ndim:],
                          S=args.stride or None, window=kw.get("window"))
        # whole-field round trips until about 10 s of CPU work
        reps, tc, td = 0, 0.0, 0.0
        while reps < 1 or (tc + td < 10.0 and reps < 8):
            a = time.perf_counter()
            ref = oracle.compress(x, p)
            blob = ref.blob()
            b = time.perf_counter()
            oracle.decompress_blob(blob)
            c = time.perf_counter()
            tc, td, reps = tc + (b - a), td + (c - b), reps + 1
            del ref, blob
        model, ncpu = host_cpu()
        line["cpu_baseline"] = {"value": round(reps * in_bytes / (tc + td) / 1e9, 4), "unit": "GB/s",
                                "cores": 1, "kind": "oracle",
                                "sample": "%d round trips (compress + decompress) of the full workload "
                                          "field, single-threaded C oracle, %.1f s compress + %.1f s "
                                          "decompress in total" % (reps, tc, td),
                                "cpu_model": model, "host_logical_cpus": ncpu}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
