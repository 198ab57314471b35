"""Benchmark of the offload path on one MI355X.

A step is one run of the large application (16 loop nests, 3 of them --
two loop-carried recurrences and a sequential generator -- on the CPU; FP32
product 8192 x 8192, element-wise nests on 8192 x 8192, a BF16 product
8192 x 8192, the 19-point sweep on 513 x 513 x 1025 for 50 sweeps with the
FP64 residual) under the pattern that puts all 13 parallelisable nests on
the GPU, through ofl_run_pattern: verdicts, plan, kernels, the three host
nests and the copies they need.  Inputs are resident in HBM when the timed
region starts (set-up content restored device-side, untimed) and outputs stay
there; the rate with set-up content copied in and outputs copied out over
PCIe is reported beside it.

Prints one JSON line; `value` is application runs per second.  `roofline` is
that of the kernel with the largest total time in a pass where every launch
is timed; its live figure comes from HIP events in the dispatch packets of a
sample of its launches on the run's stream during the timed steps.
`cpu_baseline` is the oracle's serial run of the same application (the
all-CPU gene) timed on one pinned host core on a bounded sample: every nest
once at full size (the sweep and the interior copy once each, counted 50
times), the two products at N = 1024 and 2048 extrapolated as N^3.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "app time & speedup vs 1-core oracle; stencil GB/s, GEMM MFMA % of peak"
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0}
LIVE_STRIDE = 10
# product sizes the CPU baseline times (leading blocks of the real operands);
# the largest is extrapolated to the full size as n^3
SAMPLE_N = (1024, 2048, 2896)
CSRC = os.path.join(ROOT, "paper_1806_01430_amd", "csrc")
# sources each kernel kind is compiled from: a profile's byte counts hold only
# while these are unchanged
KERNEL_SOURCES = {
    "stencil19": ["k_stencil.hip", "stencil_item.hpp", "dev_common.hpp", "launch.hpp"],
    "copy_interior": ["k_stencil.hip", "stencil_item.hpp", "dev_common.hpp", "launch.hpp"],
    "gemm": ["k_gemm.hip", "gemm_tile.hpp", "launch.hpp"],
}
# every kernel kind of the large application
LARGE_OPS = ["init_uniform", "gemm", "add_scaled", "transpose", "avg2", "sumsq", "stencil19", "copy_interior",
             "copy", "scale", "cast_bf16", "gemm_bf16"]


_T_START = time.perf_counter()


def log(*a):
    print("[%6.1f s]" % (time.perf_counter() - _T_START), *a, file=sys.stderr, flush=True)


def nan_none(x, nd=3):
    return None if x != x else round(x, nd)


def stencil_bytes(I, J, K):
    # read every element of p once, write every interior element of q once
    return 4 * I * J * K + 4 * (I - 2) * (J - 2) * (K - 2)


def copy_interior_bytes(I, J, K):
    # read and write every interior element once
    return 8 * (I - 2) * (J - 2) * (K - 2)


def sources_sha(kind):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kind, []):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kind, workload):
    """HBM bytes per launch of `kind` on `workload` from the byte-counter
    summary under profiles/ (a line `traffic: KIND WORKLOAD BYTES sources SHA`),
    or None when there is none or the kernel's sources changed since."""
    pat = re.compile(r"^traffic: (\S+) (\S+) (\d+) sources ([0-9a-f]{16})\s*$")
    pdir = os.path.join(ROOT, "profiles")
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(pdir, name)) as f:
            for line in f:
                m = pat.match(line.strip())
                if m and m.group(1) == kind and m.group(2) == workload:
                    return int(m.group(3)) if m.group(4) == sources_sha(kind) else None
    return None


def kernel_table(app, ops):
    out = {}
    for op in ops:
        n, ms = app.kernel_stats(op)
        if n:
            out[op] = {"launches": n, "total_ms": ms, "avg_us": 1e3 * ms / n}
    return out


def large_work(P):
    """Algorithmic work per launch of the large application's dominant
    kernels: (bytes or flops, unit, bound, peak)."""
    I, J, K, N = P["I"], P["J"], P["K"], P["N"]
    return {"stencil19": (stencil_bytes(I, J, K), "GB/s", "hbm", HBM_PEAK_GBS),
            "copy_interior": (copy_interior_bytes(I, J, K), "GB/s", "hbm", HBM_PEAK_GBS),
            "gemm": (2.0 * N ** 3, "TFLOP/s", "mfma", MFMA_PEAK_TFLOPS["f32"]),
            # the nest's span: B transposed to k-contiguous bf16, then the product
            "gemm_bf16": (2.0 * N ** 3, "TFLOP/s", "mfma", MFMA_PEAK_TFLOPS["bf16"],
                          "nest: B transpose pass + product kernel")}


def roof_entry(kind, work, live, workload):
    amount, unit, bound, peak = work[:4]
    secs = live["avg_us"] * 1e-6
    achieved = amount / secs / (1e9 if unit == "GB/s" else 1e12)
    traffic = measured_traffic(kind, workload) if unit == "GB/s" else None
    out = {"kernel": kind, "bound": bound, "achieved": round(achieved, 1), "peak": peak, "unit": unit,
           "frac": round(achieved / peak, 4), "traffic": traffic,
           ("bytes_per_launch" if unit == "GB/s" else "flops_per_launch"): amount,
           "avg_launch_us": round(live["avg_us"], 3), "launches_timed": live["launches"],
           "total_ms_timed": round(live["total_ms"], 3)}
    if len(work) > 4:
        out["span"] = work[4]
    return out


def run_large(args):
    """The headline: the large application, all parallelisable nests on the
    GPU, inputs resident in HBM."""
    import torch

    import paper_1806_01430_amd as ofl
    import workloads

    doc = workloads.app_doc("large")
    P = doc["params"]
    app = ofl.App(json.dumps(doc), seed=1)
    gene = [1] * app.gene_len
    bufs = app.alloc_device_buffers("cuda:0")
    flags = ofl.PRESTAGED | ofl.KEEP_OUTPUTS
    policy = ofl.SECTIONS
    for _ in range(max(1, args.warmup)):
        app.run_pattern(gene, bufs, policy=policy, flags=flags)
    # every kernel's time in an instrumented pass (events around every
    # launch): which kernel dominates the step
    app.set_kernel_timing_sample(1, 0)
    app.set_kernel_timing_op(None)
    app.set_kernel_timing(True)
    for _ in range(2):
        app.run_pattern(gene, bufs, policy=policy, flags=flags)
    app.set_kernel_timing(False)
    ktab = kernel_table(app, LARGE_OPS)
    work = large_work(P)
    dom = max(work, key=lambda k: ktab.get(k, {"total_ms": 0.0})["total_ms"])
    # the timed region: eager runs, events in the dispatch packets of every
    # LIVE_STRIDE-th sweep and interior copy and of each product (a launch
    # carrying events starts on a drained queue, ~10 us idle once per
    # sampled launch)
    app.set_kernel_timing_sample(LIVE_STRIDE, 0)
    app.set_kernel_timing_op(",".join(work))
    app.set_kernel_timing(True)
    torch.cuda.synchronize()
    internal = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = app.run_pattern(gene, bufs, policy=policy, flags=flags)
        internal.append(st["t_total_s"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    app.set_kernel_timing(False)
    live = kernel_table(app, list(work))
    # the paper's protocol (context): set-up content copied in over PCIe and
    # outputs copied out, inside the timed region; then both protocols with
    # the application's independent parts (the matrix nests, the grid nests,
    # the generator) on streams of their own.  Left out under --large-only,
    # so that a profile of it holds the resident steps alone.
    pcie = conc = pcie_conc = [float("nan")] * 3
    if not args.large_only:
        pcie = sorted(app.run_pattern(gene, bufs, policy=policy, flags=0)["t_total_s"] for _ in range(3))
        conc = sorted(app.run_pattern(gene, bufs, policy=policy, flags=flags | ofl.CONCURRENT)["t_total_s"]
                      for _ in range(3))
        pcie_conc = sorted(app.run_pattern(gene, bufs, policy=policy, flags=ofl.CONCURRENT)["t_total_s"]
                           for _ in range(3))
    internal.sort()
    return {"params": P, "wall": wall, "internal_median_s": internal[len(internal) // 2], "pcie_median_s": pcie[1],
            "concurrent_median_s": conc[1], "pcie_concurrent_median_s": pcie_conc[1],
            "kernels": ktab, "live": live, "dominant": dom, "work": work, "last": st,
            "plan_pcie": app.plan_transfers(gene, policy, 0), "plan_resident": app.plan_transfers(gene, policy, flags)}


def run_medium(args):
    """The medium application (GEMM 1024, 129 x 129 x 257 x 100 sweeps, 12
    nests), all 10 parallelisable nests on the GPU, inputs resident (context:
    its grids sit in the 256 MB last-level cache)."""
    import torch

    import paper_1806_01430_amd as ofl
    import workloads

    doc = workloads.app_doc("medium")
    P = doc["params"]
    app = ofl.App(json.dumps(doc), seed=1)
    gene = [1] * app.gene_len
    bufs = app.alloc_device_buffers("cuda:0")
    flags = ofl.PRESTAGED | ofl.KEEP_OUTPUTS
    for _ in range(3):
        app.run_pattern(gene, bufs, policy=ofl.SECTIONS, flags=flags)
    app.set_kernel_timing_sample(25, 12)
    app.set_kernel_timing_op("stencil19,copy_interior")
    app.set_kernel_timing(True)
    torch.cuda.synchronize()
    steps = 20
    t0 = time.perf_counter()
    ts = [app.run_pattern(gene, bufs, policy=ofl.SECTIONS, flags=flags)["t_total_s"] for _ in range(steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    app.set_kernel_timing(False)
    live = kernel_table(app, ["stencil19", "copy_interior"])
    I, J, K = P["I"], P["J"], P["K"]
    ts.sort()
    out = {"runs_per_s": round(steps / wall, 2), "app_time_ms": round(1e3 * ts[steps // 2], 4),
           "app_time_pcie_ms": round(1e3 * sorted(app.run_pattern(gene, bufs, policy=ofl.SECTIONS)["t_total_s"]
                                                  for _ in range(3))[1], 4)}
    for kind, nbytes in (("stencil19", stencil_bytes(I, J, K)), ("copy_interior", copy_interior_bytes(I, J, K))):
        if kind in live:
            gbs = nbytes / (live[kind]["avg_us"] * 1e-6) / 1e9
            out[kind] = {"avg_us": round(live[kind]["avg_us"], 3), "GBps": round(gbs, 1),
                         "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def run_kernels_large(args):
    """Element-wise nests on 8192 x 8192 (HBM-bound) and the FFT call: one
    line per kernel kind."""
    import numpy as np

    import paper_1806_01430_amd as ofl
    from workloads import appgen

    out = {}
    R = C = 8192
    app = ofl.App(json.dumps(appgen.ewise_app(R, C)), seed=1)
    bufs = app.alloc_device_buffers("cuda:0")
    gene = [1] * app.gene_len
    app.run_pattern(gene, bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
    app.set_kernel_timing(True)
    runs = 3
    for _ in range(runs):
        app.run_pattern(gene, bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
    per_elem = {"init_uniform": 8, "add_scaled": 12, "transpose": 8, "avg2": 12, "copy": 8, "scale": 8,
                "cast_bf16": 6, "sumsq": 4}
    for op, b in per_elem.items():
        n, ms = app.kernel_stats(op)
        if n:
            gbs = b * R * C * runs / (ms * 1e-3) / 1e9
            out["ewise_8192_" + op] = {"launches_per_run": n // runs, "ms_per_run": round(ms / runs, 4),
                                       "GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    Rf, n = 8192, 1024
    for inverse in (False, True):
        del bufs, app
        app = ofl.App(json.dumps(appgen.fft_app(Rf, n, inverse=inverse)), seed=1)
        app.set_input("X", np.random.default_rng(5).standard_normal((Rf, 2 * n)).astype(np.float32))
        bufs = app.alloc_device_buffers("cuda:0")
        app.run_pattern([1], bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
        app.set_kernel_timing(True)
        for _ in range(5):
            app.run_pattern([1], bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
        nl, ms = app.kernel_stats("fft_rows")
        avg = ms / nl * 1e-3
        gbs = 16.0 * Rf * n / avg / 1e9
        out[("ifft" if inverse else "fft") + "_rows_8192x1024"] = {
            "avg_us": round(avg * 1e6, 3), "GBps": round(gbs, 1), "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    # the real call on 8192 rows of 2048 values (the same 64 MB): the
    # 1024-point complex kernel and the unpacking pass, each reading and
    # writing the array once
    del bufs, app
    app = ofl.App(json.dumps(appgen.fft_app(Rf, 2 * n, real=True)), seed=1)
    app.set_input("X", np.random.default_rng(5).standard_normal((Rf, 2 * n)).astype(np.float32))
    bufs = app.alloc_device_buffers("cuda:0")
    app.run_pattern([1], bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
    app.set_kernel_timing(True)
    for _ in range(5):
        app.run_pattern([1], bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
    nl, ms = app.kernel_stats("fft_rows")
    out["rfft_rows_8192x2048"] = {"avg_us_per_call": round(ms / nl * 1e3, 3), "calls": nl}
    return out


def run_precision(args):
    """The precision workload (GEMM 4096, sweep 257 x 257 x 513 x 200, FP64
    residual) under each GEMM form, all nests on the GPU: application time and
    the product nest's kernel time per form."""
    import paper_1806_01430_amd as ofl
    import workloads

    out = {}
    for prec in ("f32", "bf16x3", "fp8x2"):
        doc = workloads.app_doc("precision")
        doc["program"][1]["args"]["prec"] = prec
        N = doc["params"]["N"]
        app = ofl.App(json.dumps(doc), seed=1)
        bufs = app.alloc_device_buffers("cuda:0")
        gene = [1] * app.gene_len
        flags = ofl.PRESTAGED | ofl.KEEP_OUTPUTS
        app.run_pattern(gene, bufs, flags=flags)
        app.set_kernel_timing(True)
        ts = sorted(app.run_pattern(gene, bufs, flags=flags)["t_total_s"] for _ in range(3))
        n, ms = app.kernel_stats("gemm")
        gemm_ms = ms / 3                 # per execution of the product nest (all its launches)
        out[prec] = {"app_time_ms": round(1e3 * ts[1], 3), "gemm_ms": round(gemm_ms, 4),
                     "gemm_TFLOPs_fp32_equiv": round(2.0 * N ** 3 / (gemm_ms * 1e-3) / 1e12, 1)}
        del app, bufs
    return out


def run_batch(args):
    """The batching workload: 256 instances (product order log-uniform in
    [32, 512), grids 17..65 x same x 2I-1, 10 sweeps), all nests on the GPU,
    as per-instance launches, as grouped launches, and as one graph; then the
    tuner's choice."""
    import paper_1806_01430_amd as ofl
    import workloads

    params, seeds = workloads.batch_instances(256, seed=1)
    for p in params:
        p["SWEEPS"] = 10
    b = ofl.Batch(workloads.app_doc("batch"), params, seeds)
    bufs = b.alloc_device_buffers("cuda:0")
    b.setup(bufs)

    def timed(mode, reps=5):
        b.run(bufs, mode)
        ts = sorted(b.run(bufs, mode)["t_total_s"] for _ in range(reps))
        return ts[reps // 2]

    out = {"instances": 256, "per_instance_launches_ms": round(1e3 * timed(ofl.BATCH_LOOP), 3),
           "grouped_ms": round(1e3 * timed(ofl.BATCH_GROUPED), 3),
           "graph_ms": round(1e3 * timed(ofl.BATCH_GROUPED_GRAPH), 3)}
    t0 = time.perf_counter()
    ents = b.tune(bufs, reps=3)
    out["tune_s"] = round(time.perf_counter() - t0, 3)
    # rooflines of the grouped launches: the tuner's fastest candidate of each
    # phase (median of 3 event-timed launches) against the work of all 256
    # instances (2 N^3 flops per product; read p once, write q's interior
    # once per sweep)
    flops = sum(2.0 * pp["N"] ** 3 for pp in params)
    sweep_b = sum(stencil_bytes(pp["I"], pp["J"], pp["K"]) for pp in params)
    best = {ph: min(e["ms"] for e in ents if e["phase"] == ph) for ph in ("gemm", "stencil")}
    tf = flops / (best["gemm"] * 1e-3) / 1e12
    gbs = sweep_b / (best["stencil"] * 1e-3) / 1e9
    out["roofline_grouped"] = {
        "gemm": {"bound": "mfma", "achieved": round(tf, 1), "peak": MFMA_PEAK_TFLOPS["f32"], "unit": "TFLOP/s",
                 "frac": round(tf / MFMA_PEAK_TFLOPS["f32"], 4), "ms": round(best["gemm"], 4), "flops": flops},
        "sweep": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(gbs / HBM_PEAK_GBS, 4), "ms": round(best["stencil"], 4), "bytes": sweep_b}}
    out["tuned_config"] = b.config
    b.setup(bufs)
    out["graph_tuned_ms"] = round(1e3 * timed(ofl.BATCH_GROUPED_GRAPH), 3)
    out["speedup_vs_per_instance"] = round(out["per_instance_launches_ms"] / out["graph_tuned_ms"], 2)
    return out


def run_population(args):
    """Population evaluation on the tiny application: all 64 genes, measured
    gene by gene as graph replays vs in one submission (graph chain)."""
    import torch

    import paper_1806_01430_amd as ofl
    import workloads

    app = ofl.App(json.dumps(workloads.app_doc("tiny")), seed=1)
    bufs = app.alloc_device_buffers("cuda:0")
    genes = [[(i >> k) & 1 for k in range(6)] for i in range(64)]
    out = {"genes": 64, "reps": 3, "warmup": 1}
    for name, flags in (("per_gene_graph", ofl.GRAPH), ("one_submission", ofl.BATCHED)):
        app.eval_population(genes, bufs, reps=1, warmup=0, flags=flags)   # capture the graphs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        app.eval_population(genes, bufs, reps=3, warmup=1, flags=flags)
        out[name + "_s"] = round(time.perf_counter() - t0, 4)
    return out


def calibration_copy():
    """A plain copy nest of known size (1 GiB read, 1 GiB written), run once:
    the reference against which rocprofv3's FETCH_SIZE / WRITE_SIZE readings
    of the other kernels are scaled."""
    import paper_1806_01430_amd as ofl
    from workloads import appgen

    n = 1 << 14
    doc = {"name": "copy1GiB", "params": {"N": n},
           "buffers": [{"name": "C", "dims": ["N", "N"]}, {"name": "D", "dims": ["N", "N"], "output": True}],
           "program": [appgen.copy_nest("D", "C")]}
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers("cuda:0")
    app.run_pattern([1], bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
    del app, bufs


def host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def cpu_baseline_large():
    """The oracle's serial run of the large application (all 16 nests on the
    CPU: the all-zero gene), on one pinned host core, from a bounded sample:
    every nest once at full size in program order (the sweep and the interior
    copy once each, counted SWEEPS times); the two products at n = 1024, 2048
    and 2896 (about N / 2.83) on leading blocks of their real operands,
    extrapolated as t(2896) (N / 2896)^3."""
    import numpy as np

    import workloads
    from oracle import cnests as C
    from oracle import ir
    from oracle import run as orun

    core = max(os.sched_getaffinity(0))
    os.sched_setaffinity(0, {core})
    doc = workloads.app_doc("large")
    P = doc["params"]
    app = ir.load(doc)
    # set-up content (untimed): zeros, and the sine field for the grid; every
    # page touched once here so that no timed nest pays first-touch faults
    bufs = {}
    for b in app.buffers:
        if b.setup == "sin":
            bufs[b.name] = C.sin_field(*b.dims, b.mode)
        else:
            bufs[b.name] = np.zeros(b.dims, {"f32": np.float32, "f64": np.float64, "bf16": np.uint16}[b.dtype])
            bufs[b.name].fill(0)
    per = []
    gemm_fit = {}

    def timed_nest(nest, env):
        t0 = time.perf_counter()
        orun.run_nest(app, nest, bufs, 1, env)
        return time.perf_counter() - t0

    def sample_product(nest):
        a = nest.args
        A, B = bufs[a["A"]], bufs[a["B"]]
        fn = C.gemm_f32 if nest.op == "gemm" else C.gemm_bf16
        ts = {}
        for n in SAMPLE_N:
            As, Bs = np.ascontiguousarray(A[:n, :n]), np.ascontiguousarray(B[:n, :n])
            t0 = time.perf_counter()
            fn(As, Bs)
            ts[n] = time.perf_counter() - t0
        big = SAMPLE_N[-1]
        est = ts[big] * (A.shape[0] / float(big)) ** 3
        gemm_fit[nest.name] = {"t_s": {str(n): round(ts[n], 3) for n in SAMPLE_N},
                               # t(n) / n^3 relative to the largest sample: 1.0 where the cost is cubic
                               "per_n3": {str(n): round((ts[n] / n ** 3) / (ts[big] / big ** 3), 3)
                                          for n in SAMPLE_N},
                               "extrapolated_s": round(est, 1)}
        return est

    def walk(items, env, mult):
        for it in items:
            if it[0] == "nest":
                nest = app.nests[it[1]]
                if nest.op in ("gemm", "gemm_bf16"):
                    per.append((nest.name, mult * sample_product(nest)))
                else:
                    per.append((nest.name, mult * timed_nest(nest, env)))
            else:
                _, var, count, body = it
                e2 = dict(env)
                e2[var] = 0
                walk(body, e2, mult * count)
    t_all = time.perf_counter()
    walk(app.program, {}, 1)
    sample_s = time.perf_counter() - t_all
    total = sum(t for _, t in per)
    model, n_cpu, n_aff = host_cpu()
    return {"total_s": total, "per_nest_s": {n: round(t, 3) for n, t in per}, "gemm_fit": gemm_fit,
            "sample_s": sample_s, "core": core, "model": model, "n_cpu": n_cpu, "n_affinity": n_aff,
            "params": P}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the medium, element-wise, precision, batching and population lines")
    ap.add_argument("--large-only", action="store_true",
                    help="only the large application's resident steps (for profiling): no PCIe or "
                         "concurrent runs, no extra lines, no CPU baseline")
    ap.add_argument("--extras-only", action="store_true", help="only the extra lines (for profiling)")
    ap.add_argument("--only", choices=["medium", "kernels", "precision", "batch", "population"], default=None,
                    help="only one extra line (for profiling)")
    ap.add_argument("--calibration-copy", action="store_true",
                    help="first run a plain 1 GiB copy kernel (reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)

    if args.calibration_copy:
        log("bench: calibration copy (1 GiB)")
        calibration_copy()
        torch.cuda.empty_cache()
    if args.only:
        fn = {"medium": run_medium, "kernels": run_kernels_large, "precision": run_precision, "batch": run_batch,
              "population": run_population}[args.only]
        print(json.dumps({args.only: fn(args)}), flush=True)
        return
    if args.extras_only:
        out = {"medium": run_medium(args), "kernels_large": run_kernels_large(args)}
        torch.cuda.empty_cache()
        out["precision"] = run_precision(args)
        torch.cuda.empty_cache()
        out["batch"] = run_batch(args)
        torch.cuda.empty_cache()
        out["population_eval"] = run_population(args)
        print(json.dumps(out), flush=True)
        return
    log("bench: large app, %d warmup + %d timed steps" % (args.warmup, args.steps))
    r = run_large(args)
    P = r["params"]
    workload = "large_%dx%dx%d_N%d" % (P["I"], P["J"], P["K"], P["N"])
    ms_per_step = 1e3 * r["wall"] / args.steps
    value = args.steps / r["wall"]
    roofs = {k: roof_entry(k, r["work"][k], r["live"][k], workload) for k in r["work"] if k in r["live"]}
    roofline = dict(roofs[r["dominant"]])
    line = {"metric": METRIC, "value": round(value, 4), "unit": "large-app runs/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16",
            "data": "synthetic (seeded SplitMix64 matrices, sine-mode grid)",
            "config": {"workload": "large app: 16 loop nests (2 loop-carried recurrences and a sequential "
                                   "generator on the CPU), FP32 GEMM 8192x8192, element-wise nests on "
                                   "8192x8192, BF16 GEMM 8192x8192, 19-point sweep 513x513x1025 x 50 + FP64 "
                                   "residual",
                       "gene": "all 13 parallelisable nests on the GPU",
                       "policy": "sections (CPU nests copy out only the column / row they read)",
                       "execution": "each step one eager ofl_run_pattern (kernel by kernel on one stream); "
                                    "HIP events in the dispatch packets of every %d-th sweep and interior "
                                    "copy and of each product" % LIVE_STRIDE,
                       "inputs": "resident in HBM at the start of the timed region; outputs left in HBM"},
            "app_time_ms": round(1e3 * r["internal_median_s"], 3),
            "app_time_pcie_ms": nan_none(1e3 * r["pcie_median_s"]),
            "pcie_runs_per_s": nan_none(1.0 / r["pcie_median_s"]),
            "app_time_concurrent_ms": nan_none(1e3 * r["concurrent_median_s"]),
            "app_time_pcie_concurrent_ms": nan_none(1e3 * r["pcie_concurrent_median_s"]),
            "plan_bytes": {"pcie_h2d_d2h_copies": r["plan_pcie"], "resident_h2d_d2h_copies": r["plan_resident"]},
            "roofline": roofline,
            "roofline_kernels": roofs,
            "kernels_large_app": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in r["kernels"].items()}}
    if args.large_only:
        print(json.dumps(line), flush=True)
        return
    torch.cuda.empty_cache()
    if not args.no_extras:
        log("bench: medium app")
        line["medium"] = run_medium(args)
        torch.cuda.empty_cache()
        log("bench: element-wise kernels and FFT call")
        line["kernels_large"] = run_kernels_large(args)
        torch.cuda.empty_cache()
        log("bench: precision workload under each GEMM form")
        line["precision"] = run_precision(args)
        torch.cuda.empty_cache()
        log("bench: batching workload (256 instances)")
        line["batch"] = run_batch(args)
        torch.cuda.empty_cache()
        log("bench: population evaluation (tiny, 64 genes)")
        line["population_eval"] = run_population(args)
    if not args.no_cpu_baseline:
        log("bench: oracle on one pinned host core (large application, bounded sample)")
        cb = cpu_baseline_large()
        fit = "; ".join("%s %s -> %.0f s at %d" % (
            n, ", ".join("%.2f s at %s" % (t, k) for k, t in f["t_s"].items()), f["extrapolated_s"], P["N"])
            for n, f in cb["gemm_fit"].items())
        line["cpu_baseline"] = {
            "value": round(1.0 / cb["total_s"], 6), "unit": "large-app runs/s", "cores": 1, "kind": "oracle",
            "sample": "serial oracle of the large application on host core %d: every non-product nest once at "
                      "full size (the sweep and interior copy once each, x%d), the two %d products "
                      "extrapolated as t(n) (N/n)^3 from n = %d [%s]; estimated all-CPU run %.1f s from %.1f s "
                      "of CPU work" % (cb["core"], P["SWEEPS"], P["N"], SAMPLE_N[-1], fit, cb["total_s"],
                                       cb["sample_s"]),
            "host_cpu": cb["model"], "host_logical_cpus": cb["n_cpu"], "cpus_available": cb["n_affinity"],
            "per_nest_s": cb["per_nest_s"], "product_fit": cb["gemm_fit"]}
        line["speedup_vs_1core_oracle"] = round(cb["total_s"] / r["internal_median_s"], 1)
        line["speedup_vs_1core_oracle_pcie"] = round(cb["total_s"] / r["pcie_median_s"], 1)
    log("bench: done")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
