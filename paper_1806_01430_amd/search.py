"""GA search for the fastest offload pattern of an application (the method of
Sec. 3.3 / Sec. 4: parallelisable nests -> gene, Simple GA over measured run
times, same-pattern skip).

    python -m paper_1806_01430_amd.search --app medium --M 20 --T 20 --p 1.0

Prints one JSON line: the nests and their verdicts, the best gene, its time,
the all-CPU time when measured, the speedup, search wall time, time to the
final best, measurements made, and per-generation best times.  Given a C
source (``--app paper_1806_01430_amd/apps/medium.c``), ``--emit PATH`` writes
the program with ``#pragma acc kernels`` before each nest the best gene
offloads.
"""
import argparse
import json
import sys
import time

import numpy as np

from . import App, app_doc, ga_params, RESIDENT, PER_REGION, SECTIONS, PRESTAGED, KEEP_OUTPUTS, GRAPH, BATCHED, PROGRESS, \
    CONCURRENT


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--app", default="tiny", help="application name, JSON description or C source")
    ap.add_argument("--seed", type=int, default=1, help="application seed")
    ap.add_argument("--set", action="append", default=[], metavar="NAME=VALUE",
                    help="override an application parameter (repeatable)")
    ap.add_argument("--M", type=int, default=12)
    ap.add_argument("--T", type=int, default=12)
    ap.add_argument("--Pc", type=float, default=0.9)
    ap.add_argument("--Pm", type=float, default=0.05)
    ap.add_argument("--p", type=float, default=0.5, help="fitness = time^-p")
    ap.add_argument("--ga-seed", type=int, default=1)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--policy", choices=["resident", "per_region", "sections"], default="resident")
    ap.add_argument("--graph", action="store_true", help="measure graph replays")
    ap.add_argument("--batched", action="store_true",
                    help="measure each generation's new genes in one submission (graph chain)")
    ap.add_argument("--concurrent", action="store_true",
                    help="run the application's independent parts at once (eager runs, OFL_RUN_CONCURRENT)")
    ap.add_argument("--deadline-factor", type=float, default=0.0)
    ap.add_argument("--timeout", type=float, default=0.0, help="seconds; cut off any run longer than this (0 = none)")
    ap.add_argument("--progress", action="store_true", help="one line per generation on stderr")
    ap.add_argument("--log", metavar="PATH", default=None,
                    help="measurement log of the search: resume from it, append to it (JSON lines)")
    ap.add_argument("--baseline", action="store_true", help="also measure the all-CPU gene")
    ap.add_argument("--emit", metavar="PATH", default=None,
                    help="with a C source as --app: write the program with the best gene's directives to PATH")
    ap.add_argument("--exhaustive", action="store_true",
                    help="also measure every gene (gene length <= 12) and rank the GA's answer")
    args = ap.parse_args(argv)

    import torch
    if not torch.cuda.is_available():
        print("search needs a GPU", file=sys.stderr)
        return 2
    src = app_doc(args.app, args.set)
    app = App(src, seed=args.seed)
    bufs = app.alloc_device_buffers("cuda:0")
    policy = {"resident": RESIDENT, "per_region": PER_REGION, "sections": SECTIONS}[args.policy]
    flags = (GRAPH if args.graph else 0) | (BATCHED if args.batched else 0) | (PROGRESS if args.progress else 0) | \
        (CONCURRENT if args.concurrent else 0)
    params = ga_params(M=args.M, T=args.T, Pc=args.Pc, Pm=args.Pm, p=args.p, seed=args.ga_seed, reps=args.reps,
                       warmup=args.warmup, policy=policy, flags=flags, deadline_factor=args.deadline_factor,
                       timeout_s=args.timeout, cache_path=args.log)
    t0 = time.perf_counter()
    res = app.ga_run(params, bufs)
    wall = time.perf_counter() - t0
    out = {"app": args.app, "nests": [{"name": app.nest_name(i), "verdict": v, "reason": r, "gene_pos": g}
                                      for i, (v, r, g) in enumerate(app.verdicts())],
           "gene_len": app.gene_len, "M": args.M, "T": args.T, "Pc": args.Pc, "Pm": args.Pm, "p": args.p,
           "reps": args.reps, "policy": args.policy, "graph": args.graph, "batched": args.batched,
           "best_gene": res["best_gene"], "best_time_s": res["best_time"], "n_measured": res["n_measured"],
           "search_wall_s": res["search_wall_s"], "time_to_best_s": res["time_to_best_s"],
           "per_generation_best_s": [float(np.min(np.where(res["status"][g] == 0, res["times"][g], np.inf)))
                                     for g in range(res["n_generations"])],
           "wall_s": wall}
    t_all0 = res["t_all0"] if res["t_all0"] > 0 else None
    if args.baseline and t_all0 is None:
        t, s = app.eval_population([[0] * app.gene_len], bufs, reps=args.reps, warmup=args.warmup, policy=policy)
        t_all0 = float(t[0]) if s[0] == 0 else None
    if args.exhaustive:
        a = app.gene_len
        if a > 12:
            print("exhaustive enumeration needs gene length <= 12", file=sys.stderr)
            return 2
        genes = [[(idx >> i) & 1 for i in range(a)] for idx in range(1 << a)]
        te0 = time.perf_counter()
        t, s = app.eval_population(genes, bufs, reps=args.reps, warmup=args.warmup, policy=policy, flags=flags)
        ok = np.where(s == 0, t, np.inf)
        order = np.argsort(ok, kind="stable")
        gi = sum(b << i for i, b in enumerate(res["best_gene"]))
        out["exhaustive"] = {"n_genes": 1 << a, "wall_s": time.perf_counter() - te0,
                             "best_gene": genes[int(order[0])], "best_time_s": float(ok[order[0]]),
                             "ga_gene_rank": int(np.sum(ok < ok[gi])), "ga_gene_time_s": float(ok[gi]),
                             "all_cpu_time_s": float(ok[0]),
                             "worst_time_s": float(np.max(ok[np.isfinite(ok)]))}
        if t_all0 is None and s[0] == 0:
            t_all0 = float(t[0])
    out["all_cpu_time_s"] = t_all0
    out["speedup_vs_all_cpu"] = (t_all0 / res["best_time"]) if t_all0 else None
    if args.emit:
        if not args.app.endswith(".c"):
            print("--emit needs a C source as --app", file=sys.stderr)
            return 2
        from .cfront import offloaded_source
        with open(args.app) as f:
            text = offloaded_source(f.read(), app.verdicts(), res["best_gene"])
        with open(args.emit, "w") as f:
            f.write(text)
        out["emitted"] = args.emit
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
