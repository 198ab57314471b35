"""Oracle Simple GA over offload genes (test infrastructure only).

Sec. 3.3 and Sec. 4 of the paper: genes are 0/1 strings, one bit per
parallelisable loop (1 = offload).  M individuals start with random bits.
Each is evaluated by running the pattern and measuring the benchmark time; a
faster pattern gets a higher fitness.  Selection is roulette by fitness plus
elite preservation of the best gene of the generation (kept without crossover
or mutation).  Crossover swaps genes between selected individuals at one
point with rate Pc; mutation flips each gene value with rate Pm.  After T
generations the best gene is the answer.  A pattern that was already measured
is not measured again: its earlier value is reused.  Sec. 5.1.2 settings:
fitness = (time)^(-1/2), roulette + elite, Pc = 0.9, Pm = 0.05.

Readings where the paper is silent (all are parameters or fixed here):
T counts evaluated generations including the first; the elite is one of the M;
M-1 roulette draws with replacement, paired in draw order (0,1), (2,3), ...;
the crossover point is uniform in [1, a-1] and both children are kept; an
unpaired last parent is copied; mutation is per bit and skips the elite;
a failed or timed-out run has fitness 0; the answer is the best fitness over
every evaluation (ties: the earliest).

Random numbers: one SplitMix64 stream (Steele, Lea & Flood 2014) seeded with
the GA seed; u() = (next >> 11) * 2^-53; draws in this order: initial bits
(next >> 63), then per generation the M-1 roulette draws, per pair one u()
for the crossover test and, if it passes, next() % (a-1) for the point, then
per child and bit one u() for mutation.
"""
import math

MASK64 = 0xFFFFFFFFFFFFFFFF
GAMMA = 0x9E3779B97F4A7C15

ST_OK, ST_TIMEOUT, ST_FAILED = 0, 1, 2


class SplitMix64:
    def __init__(self, seed):
        self.s = seed & MASK64

    def next(self):
        self.s = (self.s + GAMMA) & MASK64
        z = self.s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def u(self):
        return (self.next() >> 11) * (1.0 / 9007199254740992.0)


def gene_index(g):
    """idx = sum g_i 2^i (bit i = gene position i)."""
    return sum(int(b) << i for i, b in enumerate(g))


def fitness(t, status, p):
    if status != ST_OK or not (t > 0.0):
        return 0.0
    return t ** (-p)


def run_ga(a, M, T, evaluate, Pc=0.9, Pm=0.05, p=0.5, seed=1,
           deadline_factor=0.0, batched=False, timeout=None):
    """Run the GA.  ``evaluate(gene_tuple, deadline) -> (time, status)``
    measures an uncached pattern; ``deadline`` is None or a time limit.
    When deadline_factor > 0 the all-zero gene is measured first (baseline,
    also entered in the cache and the best-so-far), and every later
    measurement gets the limit min(t_all0, deadline_factor * t_best).
    ``timeout`` (seconds, None = none) caps every measurement, the baseline
    included: the paper's trials that ran too long were cut off (Sec. 5.2);
    the limit is the smaller of the two.

    ``batched``: all uncached genes of a generation are measured together (in
    order of first appearance), so they share the limit taken at the start
    of the generation; everything else is unchanged.

    Returns a dict with the per-generation populations, times, statuses,
    fitness values, the evaluation log and the best gene."""
    if a < 1 or M < 1 or T < 1:
        raise ValueError("need a >= 1, M >= 1, T >= 1")
    rng = SplitMix64(seed)
    cache = {}
    log = []          # (gene, time, status) per fresh measurement, in order
    best = {"f": -1.0, "gene": None, "t": None}

    def consider(g, t, st):
        f = fitness(t, st, p)
        if f > best["f"]:
            best.update(f=f, gene=g, t=t)

    t_all0 = None
    if deadline_factor > 0:
        g0 = tuple([0] * a)
        t0, s0 = evaluate(g0, timeout)
        cache[g0] = (t0, s0)
        log.append((g0, t0, s0))
        consider(g0, t0, s0)
        t_all0 = t0 if s0 == ST_OK else None

    def current_limit():
        cands = []
        if deadline_factor > 0 and best["t"] is not None:
            cands.append(deadline_factor * best["t"])
            if t_all0 is not None:
                cands.append(t_all0)
        if timeout is not None:
            cands.append(timeout)
        return min(cands) if cands else None

    pop = [tuple(rng.next() >> 63 for _ in range(a)) for _ in range(M)]
    gens = []
    for gen in range(1, T + 1):
        if batched:
            limit = current_limit()
            for g in pop:
                if g not in cache:
                    t, st = evaluate(g, limit)
                    cache[g] = (t, st)
                    log.append((g, t, st))
                    consider(g, t, st)
        times, stats, fits = [], [], []
        for g in pop:
            if g in cache:
                t, st = cache[g]
            else:
                limit = current_limit()
                t, st = evaluate(g, limit)
                cache[g] = (t, st)
                log.append((g, t, st))
                consider(g, t, st)
            times.append(t)
            stats.append(st)
            fits.append(fitness(t, st, p))
        gens.append({"pop": list(pop), "time": times, "status": stats, "fitness": fits})
        if gen == T:
            break
        # elite: highest fitness, ties -> lowest index
        e = 0
        for m in range(1, M):
            if fits[m] > fits[e]:
                e = m
        total = 0.0
        for f in fits:
            total += f
        parents = []
        for _ in range(M - 1):
            if total > 0.0:
                r = rng.u() * total
                acc, pick = 0.0, M - 1
                for m in range(M):
                    acc += fits[m]
                    if acc > r:
                        pick = m
                        break
            else:
                pick = rng.next() % M
            parents.append(list(pop[pick]))
        children = []
        k = 0
        while k + 1 < len(parents):
            c1, c2 = parents[k][:], parents[k + 1][:]
            if rng.u() < Pc and a >= 2:
                c = 1 + rng.next() % (a - 1)
                c1[c:], c2[c:] = parents[k + 1][c:], parents[k][c:]
            children += [c1, c2]
            k += 2
        if k < len(parents):
            children.append(parents[k][:])
        for ch in children:
            for i in range(a):
                if rng.u() < Pm:
                    ch[i] ^= 1
        pop = [pop[e]] + [tuple(ch) for ch in children]
    return {"generations": gens, "log": log, "best_gene": best["gene"],
            "best_time": best["t"], "best_fitness": best["f"], "t_all0": t_all0,
            "n_measured": len(log)}


def table_evaluator(t_table, status_table=None):
    """Evaluator over a table indexed by gene_index (an injected fitness
    landscape in place of timing).  With a deadline, a time above it is a
    TIMEOUT reported at the deadline."""
    def ev(g, limit):
        idx = gene_index(g)
        t = float(t_table[idx])
        st = ST_OK if status_table is None else int(status_table[idx])
        if st == ST_OK and limit is not None and t > limit:
            return limit, ST_TIMEOUT
        return t, st
    return ev


def exhaustive_best(a, t_table, status_table=None, p=0.5):
    """Brute force over all 2^a genes: index of the best fitness (ties ->
    lowest index).  The GA can never beat this."""
    best_i, best_f = None, -1.0
    for idx in range(1 << a):
        st = ST_OK if status_table is None else int(status_table[idx])
        f = fitness(float(t_table[idx]), st, p)
        if f > best_f:
            best_i, best_f = idx, f
    return best_i, best_f


def median(xs):
    ys = sorted(xs)
    n = len(ys)
    if n % 2:
        return ys[n // 2]
    return 0.5 * (ys[n // 2 - 1] + ys[n // 2])


def is_finite(x):
    return not (math.isinf(x) or math.isnan(x))
