"""GA parameter study over a measured landscape (the search-cost and
convergence questions the paper leaves open, Sec. 5.2 and Sec. 6).

    python -m paper_1806_01430_amd.ga_study --app medium --set N=256 --set I=33 \\
        --set J=33 --set K=65 --set SWEEPS=10 --seeds 200

Measures every gene of the application once (median of `--reps` timed runs
after `--warmup`), then runs the library's GA (ofl_ga_run_table, the same GA
as ofl_ga_run with the measured times in place of new measurements) for many
GA seeds under each parameter setting, and reports per setting: how often the
GA ends on the landscape's best gene, the rank of the gene it ends on, how
many distinct genes it measures, and the search time those measurements
would have taken (each measured gene costs warmup + reps runs; with a
deadline, a gene cut off at the limit costs the limit once).  Prints one JSON
line and a markdown table.

Large applications (``--cap S --prune``): every run is cut at S seconds (the
timeout of the paper's trials, Sec. 5.2) and the landscape is measured only
where it can hold a time under S.  First, for each gene bit i, the gene with
every parallelisable nest on the GPU except nest i is measured with the cap
4 S: if it still runs out, nest i's CPU form alone takes more than 4 S minus
the rest of that run (a few tenths of a second at most here), so every gene
that keeps nest i on the CPU runs past S and is recorded as a TIMEOUT at S
without being run.  The other genes are measured with the cap S.

    python -m paper_1806_01430_amd.ga_study --app large --cap 0.5 --prune --seeds 200
"""
import argparse
import json
import sys
import time

import numpy as np

from . import App, app_doc, ga_params, ga_run_table, RESIDENT, PER_REGION, SECTIONS, BATCHED

# (M, T, Pc, Pm, p, deadline_factor): the paper's setting first (Sec. 5.1.2)
SETTINGS = [
    (12, 12, 0.9, 0.05, 0.5, 0.0),
    (12, 12, 0.9, 0.05, 0.5, 3.0),
    (12, 12, 0.9, 0.05, 1.0, 0.0),
    (12, 12, 0.9, 0.10, 0.5, 0.0),
    (12, 12, 0.6, 0.05, 0.5, 0.0),
    (4, 4, 0.9, 0.05, 0.5, 0.0),
    (8, 8, 0.9, 0.05, 0.5, 0.0),
    (20, 20, 0.9, 0.05, 0.5, 0.0),
    (30, 10, 0.9, 0.05, 0.5, 0.0),
    (10, 30, 0.9, 0.05, 0.5, 0.0),
    (30, 20, 0.9, 0.05, 0.5, 3.0),
]


def study(a, times, status, settings, seeds, runs_per_gene, timeout=0.0):
    """GA outcome statistics over a measured table of 2^a times / statuses."""
    times = np.asarray(times, np.float64)
    status = np.asarray(status, np.int32)
    ok = np.where(status == 0, times, np.inf)
    order = np.argsort(ok, kind="stable")
    best = int(order[0])
    rank_of = np.empty(1 << a, np.int64)
    rank_of[order] = np.arange(1 << a)
    out = []
    for (M, T, Pc, Pm, p, dl) in settings:
        hits, ranks, measured, cost = 0, [], [], []
        for s in range(1, seeds + 1):
            r = ga_run_table(a, ga_params(M=M, T=T, Pc=Pc, Pm=Pm, p=p, seed=s, deadline_factor=dl,
                                          timeout_s=timeout), times, status)
            g = sum(int(b) << i for i, b in enumerate(r["best_gene"]))
            hits += int(g == best)
            ranks.append(int(rank_of[g]))
            measured.append(int(r["n_measured"]))
            # search time: every distinct measured gene once, at what its
            # measurement cost (a run cut off at the limit ends the gene)
            seen = {}
            if dl > 0:   # the all-zero baseline, measured first (limited by the timeout only)
                t0_, s0_ = float(times[0]), int(status[0])
                if timeout > 0 and s0_ == 0 and t0_ > timeout:
                    t0_, s0_ = timeout, 1
                seen[0] = (t0_, s0_)
            for gen in range(r["n_generations"]):
                for gene, t, st in zip(r["pops"][gen], r["times"][gen], r["status"][gen]):
                    key = sum(int(b) << i for i, b in enumerate(gene))
                    if key not in seen:
                        seen[key] = (float(t), int(st))
            c = 0.0
            for t, st in seen.values():
                c += t if st == 1 else t * runs_per_gene   # a timed-out gene ends at its first run
            cost.append(c)
        out.append({"M": M, "T": T, "Pc": Pc, "Pm": Pm, "p": p, "deadline_factor": dl, "seeds": seeds,
                    "p_best": hits / seeds, "median_rank": float(np.median(ranks)),
                    "p_top1pct": float(np.mean(np.asarray(ranks) < max(1, (1 << a) // 100))),
                    "mean_measured": float(np.mean(measured)), "mean_search_s": float(np.mean(cost))})
    return {"best_gene": [(best >> i) & 1 for i in range(a)], "best_time_s": float(ok[best]),
            "all_cpu_time_s": float(ok[0]) if np.isfinite(ok[0]) else None,
            "exhaustive_search_s": float(np.sum(np.where(np.isfinite(ok), ok, 0.0)) * runs_per_gene),
            "settings": out}


def table(res):
    lines = ["| M | T | Pc | Pm | p | deadline | P(best) | P(top 1%) | median rank | genes measured | search s |",
             "|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in res["settings"]:
        lines.append("| %d | %d | %.1f | %.2f | %.1f | %s | %.2f | %.2f | %g | %.1f | %.2f |" % (
            r["M"], r["T"], r["Pc"], r["Pm"], r["p"], ("%gx" % r["deadline_factor"]) if r["deadline_factor"] else "-",
            r["p_best"], r["p_top1pct"], r["median_rank"], r["mean_measured"], r["mean_search_s"]))
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--app", default="medium", help="application name, JSON description or C source")
    ap.add_argument("--seed", type=int, default=1, help="application seed")
    ap.add_argument("--set", action="append", default=[], metavar="NAME=VALUE")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--policy", choices=["resident", "per_region", "sections"], default="sections")
    ap.add_argument("--seeds", type=int, default=200)
    ap.add_argument("--chunk", type=int, default=64, help="genes per batched submission while measuring")
    ap.add_argument("--cap", type=float, default=0.0, help="seconds; cut off every run at this time (0 = none)")
    ap.add_argument("--prune", action="store_true",
                    help="with --cap: record genes that keep a nest too slow for the cap on the CPU as "
                         "timeouts without running them")
    ap.add_argument("--out", default=None, help="also write the measured table (JSON) here")
    args = ap.parse_args(argv)

    import torch
    if not torch.cuda.is_available():
        print("ga_study needs a GPU to measure the landscape", file=sys.stderr)
        return 2
    src = app_doc(args.app, args.set)
    app = App(src, seed=args.seed)
    bufs = app.alloc_device_buffers("cuda:0")
    policy = {"resident": RESIDENT, "per_region": PER_REGION, "sections": SECTIONS}[args.policy]
    a = app.gene_len
    genes = [[(idx >> i) & 1 for i in range(a)] for idx in range(1 << a)]
    t0 = time.perf_counter()
    times = np.full(1 << a, args.cap)
    status = np.ones(1 << a, np.int32)   # TIMEOUT until measured
    heavy = []
    if args.prune:
        if not args.cap > 0:
            print("--prune needs --cap", file=sys.stderr)
            return 2
        probes = [[0 if k == i else 1 for k in range(a)] for i in range(a)]
        t, s = app.eval_population(probes, bufs, reps=1, warmup=0, policy=policy, flags=BATCHED,
                                   deadline_s=4 * args.cap)
        heavy = [i for i in range(a) if s[i] == 1]
        print("nests too slow on the CPU for the cap (gene bits): %s, %.1f s" % (heavy, time.perf_counter() - t0),
              file=sys.stderr, flush=True)
    todo = [idx for idx in range(1 << a) if all((idx >> i) & 1 for i in heavy)]
    for c0 in range(0, len(todo), args.chunk):
        part = todo[c0:c0 + args.chunk]
        t, s = app.eval_population([genes[i] for i in part], bufs, reps=args.reps, warmup=args.warmup,
                                   policy=policy, flags=BATCHED, deadline_s=args.cap)
        times[part] = t
        status[part] = s
        print("measured %d / %d genes, %.1f s" % (min(c0 + args.chunk, len(todo)), len(todo),
                                                  time.perf_counter() - t0), file=sys.stderr, flush=True)
    res = study(a, times, status, SETTINGS, args.seeds, args.reps + args.warmup, timeout=args.cap)
    res["cap_s"] = args.cap
    res["heavy_bits"] = heavy
    res["genes_measured"] = len(todo) + (a if args.prune else 0)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"gene_len": a, "times": times.tolist(), "status": status.tolist(), "cap_s": args.cap,
                       "heavy_bits": heavy}, f)
    res.update({"app": args.app, "params": src["params"], "gene_len": a, "reps": args.reps,
                "warmup": args.warmup, "policy": args.policy, "measure_wall_s": time.perf_counter() - t0,
                "times_quantiles_s": [float(np.quantile(times, q)) for q in (0.0, 0.25, 0.5, 0.75, 1.0)],
                "n_ok": int(np.sum(status == 0))})
    print(json.dumps(res), flush=True)
    print(table(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
