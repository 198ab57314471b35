"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

Holds none of the offload method's arithmetic: it only loads application
descriptions with chosen sizes and draws seeded random fixtures (small loop
nests for the dependence check, time tables standing in for measured run
times, sizes of uneven application instances).
"""
import json
import math
import os
import random

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
APPS_DIR = os.path.join(ROOT, "paper_1806_01430_amd", "apps")


def app_path(name):
    return os.path.join(APPS_DIR, name + ".json")


def app_doc(name, **params):
    """The named application description with some params overridden."""
    with open(app_path(name)) as f:
        doc = json.load(f)
    doc["params"].update({k: int(v) for k, v in params.items()})
    return doc


# Reduced sizes that keep every structural feature (several GEMM / transpose
# tiles plus a ragged tail, grids whose extents are not multiples of any tile)
# while the serial oracle finishes in about a second.
SMALL_MEDIUM = dict(N=200, I=19, J=23, K=71, SWEEPS=4)
SMALL_LARGE = dict(N=136, I=13, J=17, K=131, SWEEPS=3)


def random_nest_doc(rng, max_loops=3, max_dims=3, max_extent=6, n_access=3):
    """A random nest over one or two small buffers with affine subscripts
    (var + c or a constant), for brute-force checks of the dependence test."""
    nl = rng.randint(1, max_loops)
    names = ["i", "j", "k"][:nl]
    loops = []
    for v in names:
        lo = rng.randint(0, 2)
        hi = lo + rng.randint(1, max_extent - 2)
        loops.append([v, str(lo), str(hi)])
    nd = rng.randint(1, max_dims)
    ext = max_extent + 4
    bufs = [{"name": "X", "dtype": "f32", "dims": [str(ext)] * nd},
            {"name": "Y", "dtype": "f32", "dims": [str(ext)] * nd}]
    acc = []
    for t in range(n_access):
        buf = "X" if (t == 0 or rng.random() < 0.7) else "Y"
        mode = "w" if t == 0 else rng.choice(["r", "r", "w", "rw"])
        subs = []
        for _ in range(nd):
            if rng.random() < 0.2:
                subs.append(str(rng.randint(0, 3)))
            else:
                v = rng.choice(names)
                c = rng.randint(-1, 2)
                subs.append(v if c == 0 else "%s%+d" % (v, c))
                # keep in bounds: subscripts only shift by -1..2, bounds start >= 0
        acc.append([buf, mode] + subs)
    # shift loops so that var-1 stays >= 0
    for L in loops:
        L[1] = str(int(L[1]) + 1)
        L[2] = str(int(L[2]) + 1)
    return {"name": "rand", "params": {}, "buffers": bufs,
            "program": [{"nest": "rand", "op": "none", "loops": loops, "access": acc}]}


def batch_instances(n=256, seed=1, n_lo=32, n_hi=512, g_lo=17, g_hi=65):
    """Per-instance sizes of the batching configuration: product order
    N = floor(exp(U[ln n_lo, ln n_hi])) (not rounded to any tile), grid
    I = J ~ U{g_lo..g_hi}, K = 2I - 1; instance seeds seed*1000 + i."""
    rng = random.Random(seed)
    out = []
    for _ in range(n):
        N = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        I = rng.randint(g_lo, g_hi)
        out.append({"N": min(N, n_hi - 1), "I": I, "J": I, "K": 2 * I - 1})
    seeds = [seed * 1000 + i for i in range(n)]
    return out, seeds


def time_table(a, seed, lo=0.001, hi=1.0):
    """A seeded table of 2^a positive 'run times' (log-uniform in [lo, hi])."""
    rng = random.Random(seed)
    return [math.exp(rng.uniform(math.log(lo), math.log(hi))) for _ in range(1 << a)]
