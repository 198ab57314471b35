"""Condenses rocprofv3 CSV output into the short summaries kept here.

    python profiles/summarize.py stats <kernel_stats.csv>
    python profiles/summarize.py pmc <counter_collection.csv> [<counter_collection.csv> ...]

`stats` prints calls / average / total per kernel; `pmc` prints the per-kernel
average of every counter (per dispatch), so FETCH_SIZE and WRITE_SIZE of a
kernel can be set against those of the 1 GiB calibration copy.
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


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(sys.argv[2])
    else:
        pmc(sys.argv[2:])
