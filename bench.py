"""Benchmark of the offload path on one MI355X.

A step is one run of the medium application (12 loop nests, 2 of them
loop-carried recurrences that stay on the CPU; GEMM 1024 x 1024, 19-point
sweep on 129 x 129 x 257 for 100 sweeps with the FP64 residual) under the
pattern that puts every parallelisable nest on the GPU, through
ofl_run_pattern: verdicts, plan, kernels, the two host nests and the copies
they require.  Inputs are resident in HBM when the timed region starts (set-up
content restored device-side, untimed) and outputs stay there.

Prints one JSON line; `value` is application runs per second.  The rooflines
of the two grid kernels (the sweep and the interior copy) come from HIP events
in the dispatch packets of a sample of their launches on the run's stream
during the timed steps (each kernel in every second step, every 25th launch);
`roofline` is that of the one with the larger total time in a pass where
every kernel is timed.  `cpu_baseline` times the oracle's serial run of the
same application on one host core.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "app time & speedup vs 1-core oracle; stencil GB/s, GEMM MFMA % of peak"
# HBM bytes per launch measured with rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled
# by the readings of a plain 1 GiB copy (reads x2.000, writes x1.000); see
# profiles/stencil19_medium_129x129x257.md.  Must be re-measured (or dropped)
# whenever the kernel changes.
MEASURED_TRAFFIC = {("stencil19", 129, 129, 257): (2.000 * 9356.3 + 19094.7) * 1024,
                    ("copy_interior", 129, 129, 257): (2.000 * 8207.3 + 16288.3) * 1024}
LIVE_KERNELS = ("stencil19", "copy_interior")
TIMING_STRIDE = 25
HBM_PEAK_GBS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stencil_bytes(I, J, K):
    # read every element of p once, write every interior element of q once
    return 4 * I * J * K + 4 * (I - 2) * (J - 2) * (K - 2)


def copy_interior_bytes(I, J, K):
    # read and write every interior element once
    return 8 * (I - 2) * (J - 2) * (K - 2)


def kernel_table(app, ops):
    out = {}
    for op in ops:
        n, ms = app.kernel_stats(op)
        if n:
            out[op] = {"launches": n, "total_ms": ms, "avg_us": 1e3 * ms / n}
    return out


def run_medium(args):
    import torch

    import paper_1806_01430_amd as ofl
    import workloads

    doc = workloads.app_doc("medium")
    P = doc["params"]
    app = ofl.App(json.dumps(doc), seed=1)
    gene = [1] * app.gene_len
    bufs = app.alloc_device_buffers("cuda:0")
    flags = ofl.PRESTAGED | ofl.KEEP_OUTPUTS
    policy = ofl.SECTIONS
    # the timed region: eager runs (one launch per kernel) with HIP events in
    # the dispatch packets of a sample of the launches of the two grid
    # kernels, the sweep and the interior copy (together nearly all of the
    # kernel time): the kernels take turns step by step, and in a step every
    # TIMING_STRIDE-th execution of the kernel is timed.  A launch carrying
    # events leaves the queue idle for a few microseconds around it (the
    # launches are no longer back to back), so timing every launch would slow
    # the step by ~0.3 ms per kernel kind
    app.set_kernel_timing_sample(TIMING_STRIDE, TIMING_STRIDE // 2)
    app.set_kernel_timing_op(LIVE_KERNELS[0])
    for _ in range(args.warmup):
        app.run_pattern(gene, bufs, policy=policy, flags=flags)
    torch.cuda.synchronize()
    app.set_kernel_timing(True)
    internal = []
    t0 = time.perf_counter()
    for step in range(args.steps):
        app.set_kernel_timing_op(LIVE_KERNELS[step % len(LIVE_KERNELS)])
        st = app.run_pattern(gene, bufs, policy=policy, flags=flags)
        internal.append(st["t_total_s"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    app.set_kernel_timing(False)
    dom = kernel_table(app, LIVE_KERNELS)
    # every kernel's time, in a separate instrumented pass (context)
    app.set_kernel_timing_sample(1, 0)
    app.set_kernel_timing_op(None)
    app.set_kernel_timing(True)
    for _ in range(10):
        app.run_pattern(gene, bufs, policy=policy, flags=flags)
    app.set_kernel_timing(False)
    ktab = kernel_table(app, ["stencil19", "copy_interior", "gemm", "init_uniform", "add_scaled", "transpose",
                              "avg2", "sumsq", "copy", "scale"])
    # uninstrumented graph replays (context)
    gflags = flags | ofl.GRAPH
    for _ in range(3):
        app.run_pattern(gene, bufs, policy=policy, flags=gflags)
    torch.cuda.synchronize()
    tg0 = time.perf_counter()
    ginternal = []
    for _ in range(args.steps):
        ginternal.append(app.run_pattern(gene, bufs, policy=policy, flags=gflags)["t_total_s"])
    torch.cuda.synchronize()
    gwall = time.perf_counter() - tg0
    ginternal.sort()
    # paper protocol for context: set-up content copied in, outputs copied out
    pcie = []
    for _ in range(3):
        pcie.append(app.run_pattern(gene, bufs, policy=policy, flags=0)["t_total_s"])
    # the whole-buffer transfer policy for comparison
    res_t = []
    for _ in range(3):
        app.run_pattern(gene, bufs, policy=ofl.RESIDENT, flags=flags)
    for _ in range(10):
        res_t.append(app.run_pattern(gene, bufs, policy=ofl.RESIDENT, flags=flags)["t_total_s"])
    res_t.sort()
    internal.sort()
    pcie.sort()
    return {"app": app, "params": P, "wall": wall, "internal_median_s": internal[len(internal) // 2],
            "pcie_median_s": pcie[1], "kernels": ktab, "live": dom, "last": st, "graph_wall": gwall,
            "resident_median_s": res_t[len(res_t) // 2],
            "graph_internal_median_s": ginternal[len(ginternal) // 2]}


def run_kernels_large(args):
    """Stencil on the largest grid and the FP32 GEMM at 8192 (the sizes where
    the HBM and MFMA rooflines are meaningful)."""
    import paper_1806_01430_amd as ofl
    from workloads import appgen

    out = {}
    I, J, K = 513, 513, 1025
    app = ofl.App(json.dumps(appgen.stencil_app(I, J, K, 10)), seed=1)
    bufs = app.alloc_device_buffers("cuda:0")
    app.run_pattern([1, 1], bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
    app.set_kernel_timing(True)
    for _ in range(2):
        app.run_pattern([1, 1], bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
    n, ms = app.kernel_stats("stencil19")
    avg = ms / n * 1e-3
    gbs = stencil_bytes(I, J, K) / avg / 1e9
    nc, msc = app.kernel_stats("copy_interior")
    out["stencil19_513x513x1025"] = {"avg_us": avg * 1e6, "GBps": gbs, "frac_hbm": gbs / HBM_PEAK_GBS,
                                     "copy_interior_GBps": 8 * (I - 2) * (J - 2) * (K - 2) / (msc / nc * 1e-3) / 1e9}
    del bufs, app
    N = 8192
    doc = {"name": "gemm8192", "params": {"N": N},
           "buffers": [{"name": b, "dims": ["N", "N"], "output": b == "C"} for b in ("A", "B", "C")],
           "program": [appgen.init_nest(["A", "B"], [0, 1]), appgen.gemm_nest("A", "B", "C")]}
    app = ofl.App(json.dumps(doc), seed=1)
    bufs = app.alloc_device_buffers("cuda:0")
    app.run_pattern([1, 1], bufs, flags=ofl.KEEP_OUTPUTS)
    app.set_kernel_timing(True)
    for _ in range(3):
        app.run_pattern([1, 1], bufs, flags=ofl.KEEP_OUTPUTS)
    n, ms = app.kernel_stats("gemm")
    avg = ms / n * 1e-3
    tf = 2.0 * N ** 3 / avg / 1e12
    out["gemm_f32_8192"] = {"avg_ms": avg * 1e3, "TFLOPs": tf, "frac_mfma": tf / FP32_MFMA_PEAK_TFLOPS}
    del bufs, app
    # element-wise nests, transpose, cast and sum of squares on 8192 x 8192
    # (256 MB per FP32 matrix: HBM-bound); algorithmic bytes per element
    R = C = 8192
    app = ofl.App(json.dumps(appgen.ewise_app(R, C)), seed=1)
    bufs = app.alloc_device_buffers("cuda:0")
    gene = [1] * app.gene_len
    app.run_pattern(gene, bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
    app.set_kernel_timing(True)
    for _ in range(3):
        app.run_pattern(gene, bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
    per_elem = {"init_uniform": 8, "add_scaled": 12, "transpose": 8, "avg2": 12, "copy": 8, "scale": 8,
                "cast_bf16": 6, "sumsq": 4}
    for op, b in per_elem.items():
        n, ms = app.kernel_stats(op)
        runs = 3
        if n:
            gbs = b * R * C * runs / (ms * 1e-3) / 1e9
            out["ewise_8192_" + op] = {"launches_per_run": n // runs, "ms_per_run": ms / runs, "GBps": gbs,
                                       "frac_hbm": gbs / HBM_PEAK_GBS}
    del bufs, app
    out.update(run_fft_kernel(args))
    return out


def run_fft_kernel(args):
    """The FFT call on 8192 rows of 1024 complex points (64 MB): each row read
    and written once, 16 algorithmic bytes per point; 5 n log2 n flops a row."""
    import numpy as np
    import paper_1806_01430_amd as ofl
    from workloads import appgen

    out = {}
    R, n = 8192, 1024
    app = ofl.App(json.dumps(appgen.fft_app(R, n)), seed=1)
    app.set_input("X", np.random.default_rng(5).standard_normal((R, 2 * n)).astype(np.float32))
    bufs = app.alloc_device_buffers("cuda:0")
    app.run_pattern([1], bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
    app.set_kernel_timing(True)
    for _ in range(5):
        app.run_pattern([1], bufs, flags=ofl.PRESTAGED | ofl.KEEP_OUTPUTS)
    nl, ms = app.kernel_stats("fft_rows")
    avg = ms / nl * 1e-3
    gbs = 16.0 * R * n / avg / 1e9
    out["fft_rows_8192x1024"] = {"avg_us": avg * 1e6, "GBps": gbs, "frac_hbm": gbs / HBM_PEAK_GBS,
                                 "GFLOPs": 5.0 * n * 10 * R / avg / 1e9}
    return out


def run_precision(args):
    """The precision workload (GEMM 4096, sweep 257 x 257 x 513 x 200, FP64
    residual) under each GEMM form, all nests on the GPU: application time and
    the product nest's kernel time per form."""
    import paper_1806_01430_amd as ofl
    import workloads

    out = {}
    N = None
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
    b.tune(bufs, reps=3)
    out["tune_s"] = round(time.perf_counter() - t0, 3)
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


def cpu_baseline():
    """The oracle's serial run of the medium application (the all-CPU gene),
    one host core."""
    import workloads
    from oracle import ir
    from oracle import run as orun

    app_o = ir.load(workloads.app_doc("medium"))
    ts = []
    for _ in range(3):
        bufs = orun.setup_buffers(app_o)
        t0 = time.perf_counter()
        orun.run_app(app_o, 1, bufs=bufs)
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[1]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 513^3-class stencil / 8192 GEMM lines")
    ap.add_argument("--large-only", action="store_true",
                    help="only the 513x513x1025 stencil and 8192 GEMM kernel lines (for profiling)")
    ap.add_argument("--fft-only", action="store_true", help="only the FFT kernel line (for profiling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision, batching and population-evaluation lines")
    ap.add_argument("--extras-only", action="store_true",
                    help="only the precision, batching and population-evaluation lines (for profiling)")
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
    if args.fft_only:
        print(json.dumps({"kernels_large": run_fft_kernel(args)}), flush=True)
        return
    if args.large_only:
        print(json.dumps({"kernels_large": run_kernels_large(args)}), flush=True)
        return
    if args.extras_only:
        out = {"precision": run_precision(args)}
        torch.cuda.empty_cache()
        out["batch"] = run_batch(args)
        torch.cuda.empty_cache()
        out["population_eval"] = run_population(args)
        print(json.dumps(out), flush=True)
        return
    log("bench: medium app, %d warmup + %d timed steps" % (args.warmup, args.steps))
    r = run_medium(args)
    P = r["params"]
    ms_per_step = 1e3 * r["wall"] / args.steps
    value = args.steps / r["wall"]
    ks = r["kernels"]
    # the dominant kernel is the one of the two with the larger total time in
    # the instrumented pass where every launch carries events (the live
    # figure of a kernel depends a little on which neighbouring launches
    # carry events); "roofline" is its roofline from the live timing of the
    # timed steps, "roofline_kernels" has both
    I, J, K = P["I"], P["J"], P["K"]
    algo = {"stencil19": stencil_bytes(I, J, K), "copy_interior": copy_interior_bytes(I, J, K)}
    for name, nbytes in algo.items():
        if name in ks:
            ks[name]["GBps"] = nbytes / (ks[name]["avg_us"] * 1e-6) / 1e9

    def roof(rk):
        live = r["live"][rk]
        achieved = algo[rk] / (live["avg_us"] * 1e-6) / 1e9
        traffic = MEASURED_TRAFFIC.get((rk, I, J, K))
        return {"kernel": rk, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(traffic) if traffic else None,
                "bytes_per_launch": algo[rk], "avg_launch_us": round(live["avg_us"], 3),
                "launches_timed": live["launches"], "total_ms_timed": round(live["total_ms"], 3)}

    roofs = {rk: roof(rk) for rk in LIVE_KERNELS}
    dom = max(LIVE_KERNELS, key=lambda rk: ks[rk]["total_ms"])
    roofline = dict(roofs[dom])
    g = ks.get("gemm")
    gemm_tf = 2.0 * 1024 ** 3 / (g["avg_us"] * 1e-6) / 1e12 if g else None

    line = {"metric": METRIC, "value": round(value, 3), "unit": "medium-app runs/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic (seeded SplitMix64 inputs, sine-mode grid)",
            "config": {"workload": "medium app: 12 loop nests (2 loop-carried recurrences on the CPU), "
                                   "GEMM 1024x1024, 19-point sweep 129x129x257 x 100 sweeps + FP64 residual",
                       "gene": "all 10 parallelisable nests on the GPU",
                       "policy": "sections (CPU recurrences copy out only the column / row they read)",
                       "execution": "each step one eager ofl_run_pattern (kernel by kernel on one stream); "
                                    "HIP events in the dispatch packets of every 25th stencil19 sweep "
                                    "launch (even steps) or copy_interior launch (odd steps)",
                       "inputs": "resident in HBM at the start of the timed region; outputs left in HBM"},
            "app_time_ms": round(1e3 * r["internal_median_s"], 4),
            "app_time_pcie_ms": round(1e3 * r["pcie_median_s"], 4),
            "graph_runs_per_s": round(args.steps / r["graph_wall"], 3),
            "graph_app_time_ms": round(1e3 * r["graph_internal_median_s"], 4),
            "app_time_resident_policy_ms": round(1e3 * r["resident_median_s"], 4),
            "gemm1024_TFLOPs": round(gemm_tf, 2) if gemm_tf else None,
            "roofline": roofline,
            "roofline_kernels": roofs,
            "kernels_medium": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in ks.items()}}
    if not args.no_large:
        log("bench: large-grid stencil and 8192 GEMM")
        line["kernels_large"] = {k: {kk: round(vv, 4) for kk, vv in v.items()}
                                 for k, v in run_kernels_large(args).items()}
    if not args.no_extras:
        log("bench: precision workload under each GEMM form")
        line["precision"] = run_precision(args)
        torch.cuda.empty_cache()
        log("bench: batching workload (256 instances)")
        line["batch"] = run_batch(args)
        torch.cuda.empty_cache()
        log("bench: population evaluation (tiny, 64 genes)")
        line["population_eval"] = run_population(args)
    if not args.no_cpu_baseline:
        log("bench: oracle on one host core (full medium application)")
        dt = cpu_baseline()
        line["cpu_baseline"] = {"value": round(1.0 / dt, 5), "unit": "medium-app runs/s", "cores": 1,
                                "kind": "oracle", "sample": "median of 3 full serial runs of the medium "
                                                            "application (all 12 nests; %.2f s each)" % dt}
        line["speedup_vs_1core_oracle"] = round(dt / r["internal_median_s"], 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
