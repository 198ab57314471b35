"""Condenses rocprofv3 CSV output into the short summaries kept here.

    python profiles/summarize.py stats <kernel_stats.csv>
    python profiles/summarize.py pmc <counter_collection.csv> [<counter_collection.csv> ...]
    python profiles/summarize.py sampled <kernel_trace.csv> FIRST LAST STEP STRIDE PHASE KERNEL...

`stats` prints calls / average / total per kernel; `pmc` prints the per-kernel
average of every counter (per dispatch), so FETCH_SIZE and WRITE_SIZE of a
kernel can be set against those of the 1 GiB calibration copy.  `sampled`
splits a kernel trace into application runs (one GEMM dispatch opens a run)
and, for each named kernel, compares over runs FIRST, FIRST + STEP, ... up
to LAST (0-based, inclusive) the average duration of its executions i with
i % STRIDE == PHASE (the launches a sampled kernel timing gives events) with
that of the others, and reports the median idle time before each.
"""
import collections
import csv
import sys


def short(name):
    name = name.replace("ofl::k::(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0]


def stats(path):
    rows = list(csv.DictReader(open(path)))
    print("| kernel | calls | avg us | total ms |")
    print("|---|---|---|---|")
    for r in rows:
        print("| %s | %s | %.3f | %.3f |" % (short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3,
                                           float(r["TotalDurationNs"]) / 1e6))


def pmc(paths):
    acc = collections.OrderedDict()
    for path in paths:
        per_dispatch = collections.OrderedDict()
        for r in csv.DictReader(open(path)):
            key = (r["Dispatch_Id"], short(r["Kernel_Name"]), r["Grid_Size"])
            d = per_dispatch.setdefault(key, {})
            d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        for (_, kern, grid), d in per_dispatch.items():
            for c, v in d.items():
                acc.setdefault((kern, grid, c), []).append(v)
    print("| kernel | grid size | counter | dispatches | mean per dispatch |")
    print("|---|---|---|---|---|")
    for (kern, grid, c), vs in acc.items():
        print("| %s | %s | %s | %d | %.1f |" % (kern, grid, c, len(vs), sum(vs) / len(vs)))


def sampled(path, first, last, step, stride, phase, kernels):
    rows = sorted(csv.DictReader(open(path)), key=lambda r: int(r["Start_Timestamp"]))
    runs = []
    prev_end = None
    for r in rows:
        name = short(r["Kernel_Name"])
        start, end = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        if name.startswith("k_gemm"):
            runs.append(collections.defaultdict(list))
        if runs:
            gap = (start - prev_end) if prev_end is not None else 0
            runs[-1][name].append((end - start, max(gap, 0)))
        prev_end = end
    print("| kernel | runs | sampled: n, avg us, median idle before us | others: n, avg us, median idle before us |")
    print("|---|---|---|---|")
    for k in kernels:
        samp, rest = [], []
        for run in runs[first:last + 1:step]:
            for name, ds in run.items():
                if not name.startswith(k):
                    continue
                for i, d in enumerate(ds):
                    (samp if i % stride == phase else rest).append(d)

        def fmt(v):
            if not v:
                return "0, -, -"
            gaps = sorted(g for _, g in v)
            return "%d, %.3f, %.2f" % (len(v), sum(d for d, _ in v) / len(v) / 1e3, gaps[len(gaps) // 2] / 1e3)
        print("| %s | %d..%d step %d | %s | %s |" % (k, first, last, step, fmt(samp), fmt(rest)))


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    elif sys.argv[1] == "sampled":
        a = sys.argv
        sampled(a[2], int(a[3]), int(a[4]), int(a[5]), int(a[6]), int(a[7]), a[8:])
    else:
        pmc(sys.argv[2:])
