"""Pins of the oracle's dependence check, transfer planner, GA and whole-app
run: brute force on tiny inputs, hand-computed plans, invariants of the GA
definition, and closed forms of the application's outputs."""
import random

import numpy as np
import pytest

import workloads
from oracle import depcheck as D
from oracle import enum as E
from oracle import ga as G
from oracle import ir, run, xfer


def _nest_app(loops, access, flags=(), bufs=None, repeat=None):
    nest = {"nest": "t", "op": "none", "loops": loops, "access": access, "flags": list(flags)}
    prog = [nest] if repeat is None else [{"repeat": str(repeat), "var": "n", "body": [nest]}]
    return ir.load({"name": "t", "params": {},
                    "buffers": bufs or [{"name": "X", "dims": ["10", "10"]},
                                        {"name": "Y", "dims": ["10", "10"]},
                                        {"name": "s", "dims": ["4"]}],
                    "program": prog})


L2 = [["i", "1", "8"], ["j", "1", "8"]]


@pytest.mark.parametrize("access,flags,want", [
    ([["X", "w", "i", "j"], ["Y", "r", "i", "j"]], (), (D.PARALLEL, D.R_NONE)),
    ([["X", "w", "i", "j"], ["X", "r", "i-1", "j"]], (), (D.REJECT, D.R_DATA_DEP)),   # flow
    ([["X", "w", "i", "j"], ["X", "r", "i+1", "j"]], (), (D.REJECT, D.R_DATA_DEP)),   # anti
    ([["X", "w", "i", "j"], ["X", "r", "i", "j-1"]], (), (D.PARALLEL, D.R_NONE)),     # inner only
    ([["X", "w", "i", "j"], ["X", "r", "j", "i"]], (), (D.REJECT, D.R_DATA_DEP)),     # in-place T
    ([["X", "w", "0", "j"]], (), (D.REJECT, D.R_DATA_DEP)),                           # output dep
    ([["s", "sum", "0"], ["X", "r", "i", "j"]], (), (D.PARALLEL_REDUCTION, D.R_NONE)),
    ([["s", "sum", "0"], ["s", "r", "1"], ["X", "r", "i", "j"]], (), (D.REJECT, D.R_DATA_DEP)),
    ([["X", "w", "i", "j"]], ("opaque_call",), (D.REJECT, D.R_EXTERNAL_CALL)),
    ([["X", "w", "i", "j"]], ("early_exit",), (D.REJECT, D.R_BREAK)),
    ([["X", "rw", "i", "j"]], (), (D.PARALLEL, D.R_NONE)),
    ([["X", "w", "i", "5"], ["X", "r", "i", "6"]], (), (D.PARALLEL, D.R_NONE)),
    ([["X", "w", "5", "j"], ["X", "r", "6", "j"]], (), (D.REJECT, D.R_DATA_DEP)),     # row 5 rewritten by every i
])
def test_reason_fixtures(access, flags, want):
    app = _nest_app(L2, access, flags)
    assert D.check_nest(app.nests[0]) == want


def test_inplace_transpose_single_row_is_parallel():
    # with one outer iteration there is nothing to carry
    app = _nest_app([["i", "2", "3"], ["j", "0", "9"]], [["X", "w", "i", "j"], ["X", "r", "j", "i"]])
    assert D.check_nest(app.nests[0]) == (D.PARALLEL, D.R_NONE)


def test_repeat_variable_subscript():
    bufs = [{"name": "r", "dims": ["5"]}, {"name": "X", "dims": ["9"]}]
    # r[n] written at every i -> output dependence across outer iterations
    app = _nest_app([["i", "0", "9"]], [["r", "w", "n"], ["X", "r", "i"]], bufs=bufs, repeat=5)
    assert D.check_nest(app.nests[0])[0] == D.REJECT
    app = _nest_app([["i", "0", "9"]], [["r", "sum", "n"], ["X", "r", "i"]], bufs=bufs, repeat=5)
    assert D.check_nest(app.nests[0]) == (D.PARALLEL_REDUCTION, D.R_NONE)


def test_affine_test_equals_brute_force():
    rng = random.Random(2024)
    n_dep = 0
    for trial in range(400):
        app = ir.load(workloads.random_nest_doc(rng))
        nest = app.nests[0]
        writes = [a for a in nest.access if a.mode in ("w", "rw")]
        for w in writes:
            for x in nest.access:
                if x.buf != w.buf:
                    continue
                got = D.carried(nest, w, x)
                want = D.brute_force_carried(nest, w, x)
                assert got == want, (trial, w.subs, x.subs, nest.loops)
                n_dep += want
    assert n_dep > 50       # the fixtures exercise both answers


def test_app_verdicts():
    want = {"tiny": (6, 6, []), "medium": (12, 10, ["rec_prefix_v", "rec_decay_w"]),
            "large": (16, 13, ["rec_prefix_v", "rec_decay_w", "lcg_fill_L"]),
            "precision": (4, 4, [])}
    for name, (n, a, rejected) in want.items():
        app = ir.load(workloads.app_path(name))
        v = D.check_app(app)
        assert len(app.nests) == n
        assert D.gene_length(app) == a
        assert [app.nests[i].name for i, x in enumerate(v) if x[0] == D.REJECT] == rejected
        assert [x[2] for x in v if x[2] >= 0] == list(range(a))
    app = ir.load(workloads.app_path("large"))
    reasons = {app.nests[i].name: x[1] for i, x in enumerate(D.check_app(app))}
    assert reasons["lcg_fill_L"] == D.R_EXTERNAL_CALL
    assert reasons["rec_prefix_v"] == D.R_DATA_DEP


# ------------------------------------------------------------ transfer plan
def test_plan_tiny_all_gpu_by_hand():
    app = ir.load(workloads.app_path("tiny"))
    grid = 33 * 33 * 65 * 4
    mat = 64 * 64 * 4
    pl = [1] * 6
    # H2D: p (read by the sweep), q (partially written -> its boundary is read),
    # res (sum target).  D2H at the end: outputs C, T, p, res.
    assert xfer.totals(app, pl, xfer.RESIDENT) == (2 * grid + 80, 2 * mat + grid + 80, 7)
    assert xfer.totals(app, pl, xfer.RESIDENT, xfer.FLAG_PRESTAGED | xfer.FLAG_KEEP_OUTPUTS) == (0, 0, 0)


def test_plan_tiny_mixed_by_hand():
    app = ir.load(workloads.app_path("tiny"))
    grid = 33 * 33 * 65 * 4
    mat = 64 * 64 * 4
    # nests: init, gemm, axpy, stencil, copy_interior, transpose
    pl = [0, 1, 0, 1, 0, 0]
    # gemm on GPU: H2D A, B; C -> device.  axpy on CPU: D2H C.
    # per sweep (10x): stencil GPU reads p, q(partial), res -> H2D each time p is
    # host-newer: sweep 1 H2D p, q, res; stencil writes q, res on device.
    # copy on CPU reads q (D2H), p (host valid) -> writes p on host.
    # sweep n>1: H2D p again (host-newer), q and res still device valid.
    # end: res D2H (output, device-newer).  C, T, p host valid.
    h2d = 2 * mat + (grid + grid + 80) + 9 * grid
    d2h = mat + 10 * grid + 80
    copies = 2 + 3 + 9 + 1 + 10 + 1
    assert xfer.totals(app, pl, xfer.RESIDENT) == (h2d, d2h, copies)


@pytest.mark.parametrize("name", ["tiny", "medium", "large"])
def test_plan_invariants(name):
    app = ir.load(workloads.app_path(name))
    v = D.check_app(app)
    a = D.gene_length(app)
    rng = random.Random(5)
    genes = [tuple([0] * a), tuple([1] * a)] + [tuple(rng.randint(0, 1) for _ in range(a))
                                                  for _ in range(60)]
    for g in genes:
        pl = xfer.placement_of_gene(app, v, g)
        r = xfer.totals(app, pl, xfer.RESIDENT)
        pr = xfer.totals(app, pl, xfer.PER_REGION)
        assert pr[0] + pr[1] >= r[0] + r[1]
        if not any(g):
            assert r == (0, 0, 0) and pr == (0, 0, 0)
    # rejected nests never move to the GPU
    pl = xfer.placement_of_gene(app, v, [1] * a)
    for i, x in enumerate(v):
        assert pl[i] == (0 if x[0] == D.REJECT else 1)


def test_enumeration_tiny():
    app = ir.load(workloads.app_path("tiny"))
    plans = E.enumerate_plans(app)
    assert len(plans) == 64
    assert plans[0][1] == (0, 0, 0)
    assert len({p[0] for p in plans}) == 64


# ------------------------------------------------------------ GA
def test_ga_invariants_random_tables():
    for seed in range(12):
        a = 6
        table = workloads.time_table(a, seed)
        out = G.run_ga(a, 6, 5, G.table_evaluator(table), seed=seed + 1)
        gens = out["generations"]
        best = -1.0
        for gi, gen in enumerate(gens):
            cur = max(gen["fitness"])
            # elite survives into the next generation at position 0
            if gi + 1 < len(gens):
                e = gen["fitness"].index(cur)
                assert gens[gi + 1]["pop"][0] == gen["pop"][e]
                assert max(gens[gi + 1]["fitness"]) >= cur
            best = max(best, cur)
            for g, t in zip(gen["pop"], gen["time"]):
                assert t == table[G.gene_index(g)]
        assert out["best_fitness"] == best
        bi, bf = G.exhaustive_best(a, table)
        assert out["best_fitness"] <= bf
        # each distinct pattern measured exactly once
        measured = [g for g, _, _ in out["log"]]
        assert len(measured) == len(set(measured))
        assert set(measured) == {g for gen in gens for g in gen["pop"]}


def test_ga_no_variation_only_copies():
    a, table = 8, workloads.time_table(8, 3)
    out = G.run_ga(a, 10, 6, G.table_evaluator(table), Pc=0.0, Pm=0.0, seed=9)
    gens = out["generations"]
    for g0, g1 in zip(gens, gens[1:]):
        assert set(g1["pop"]) <= set(g0["pop"])


def test_ga_full_mutation_complements():
    a, table = 5, workloads.time_table(5, 4)
    out = G.run_ga(a, 7, 2, G.table_evaluator(table), Pc=0.0, Pm=1.0, seed=11)
    g0, g1 = out["generations"]
    comp = {tuple(1 - b for b in g) for g in g0["pop"]}
    assert g1["pop"][0] in g0["pop"]
    assert set(g1["pop"][1:]) <= comp


def test_ga_fitness_exponent():
    assert G.fitness(4.0, G.ST_OK, 0.5) == 0.5
    assert G.fitness(4.0, G.ST_OK, 1.0) == 0.25
    assert G.fitness(4.0, G.ST_TIMEOUT, 0.5) == 0.0


def test_ga_finds_optimum_with_enough_budget():
    # a 4-bit landscape, 16 individuals x 8 generations: the optimum is found
    a = 4
    table = workloads.time_table(a, 77)
    bi, _ = G.exhaustive_best(a, table)
    out = G.run_ga(a, 16, 8, G.table_evaluator(table), seed=3)
    assert G.gene_index(out["best_gene"]) == bi


def test_ga_deadline_marks_slow_genes():
    a = 6
    table = workloads.time_table(a, 8, lo=0.01, hi=10.0)
    out = G.run_ga(a, 8, 4, G.table_evaluator(table), seed=2, deadline_factor=2.0)
    assert out["log"][0][0] == tuple([0] * a)
    for g, t, st in out["log"][1:]:
        if st == G.ST_TIMEOUT:
            assert table[G.gene_index(g)] > t


def test_ga_timeout_caps_every_run():
    # a fixed timeout cuts off every run above it, the all-zero baseline included
    a = 6
    table = workloads.time_table(a, 8, lo=0.01, hi=10.0)
    table[0] = 9.0
    out = G.run_ga(a, 8, 4, G.table_evaluator(table), seed=2, deadline_factor=2.0, timeout=3.0)
    assert out["log"][0] == (tuple([0] * a), 3.0, G.ST_TIMEOUT)
    assert out["t_all0"] is None
    for g, t, st in out["log"]:
        assert t <= 3.0
        assert (st == G.ST_TIMEOUT) == (table[G.gene_index(g)] > t)


def test_ga_all_failed_uniform_selection():
    a = 4
    out = G.run_ga(a, 5, 3, G.table_evaluator([1.0] * 16, [G.ST_FAILED] * 16), seed=1)
    assert out["best_fitness"] == 0.0
    assert len(out["generations"]) == 3


# ------------------------------------------------------------ whole-app run
def test_run_tiny_closed_forms():
    app = ir.load(workloads.app_path("tiny"))
    out = run.run_app(app, seed=1)
    A, B = out["A"].astype(np.float64), out["B"].astype(np.float64)
    want_C = A @ B + 0.5 * A
    assert np.max(np.abs(out["C"] - want_C) / want_C) < 1e-5
    assert np.array_equal(out["T"], out["C"].T)
    # stencil part: the sine mode decays by mu per sweep (closed form)
    mu = 9.959411894901419e-01
    p0 = run.setup_buffers(app)["p"].astype(np.float64)
    inner = (slice(1, -1),) * 3
    err = np.max(np.abs(out["p"][inner] - mu ** 10 * p0[inner]))
    assert err < 100 * 2.0 ** -24
    assert abs(out["res"][0] - 1.349545390484256e-01) / 1.349545390484256e-01 < 1e-3
    twin = run.run_app(app, seed=1, twin=True)
    assert np.max(np.abs(twin["res"] - out["res"]) / twin["res"]) < 1e-3


def test_run_medium_small_closed_forms():
    app = ir.load(workloads.app_doc("medium", **workloads.SMALL_MEDIUM))
    out = run.run_app(app, seed=4)
    S = out["S"].astype(np.float64)
    Cm = out["C"].astype(np.float64)
    assert np.array_equal(out["T"], out["C"].T)
    assert np.array_equal(out["S"], (np.float32(0.5) * (out["C"] + out["T"])))
    assert np.array_equal(out["D"], out["C"] * np.float32(2))
    v_ref = np.concatenate([[0.0], np.cumsum(S[1:, 0])])
    assert np.max(np.abs(out["v"] - v_ref) / np.maximum(v_ref, 1)) < 1e-5
    assert abs(out["s"][0] - np.sum(S * S)) / np.sum(S * S) < 1e-12
    w_ref = np.zeros(app.params["K"])
    prow = out["p"][1, 1, :].astype(np.float64)
    for k in range(1, len(w_ref)):
        w_ref[k] = 0.5 * w_ref[k - 1] + prow[k]
    assert np.max(np.abs(out["w"] - w_ref)) < 1e-6
    A, B = out["A"].astype(np.float64), out["B"].astype(np.float64)
    assert np.max(np.abs(Cm - (A @ B + 0.5 * A)) / Cm) < 1e-5


def test_sections_plan_medium_by_hand():
    # all parallel nests on the GPU: the two CPU recurrences read one column
    # of S (rows 1..N-1 of column 0) and one row of p (p[1][1][1..K-1]); with
    # sections only those boxes cross PCIe instead of the whole arrays
    o = ir.load(workloads.app_doc("medium"))
    v = D.check_app(o)
    pl = xfer.placement_of_gene(o, v, [1] * 10)
    N, K = o.params["N"], o.params["K"]
    cs = xfer.plan(o, pl, xfer.SECTIONS, xfer.FLAG_PRESTAGED | xfer.FLAG_KEEP_OUTPUTS)
    assert [(c[0], o.buffers[c[1]].name, c[2]) for c in cs] == [("D2H", "S", 4 * (N - 1)), ("D2H", "p", 4 * (K - 1))]
    rs = xfer.plan(o, pl, xfer.RESIDENT, xfer.FLAG_PRESTAGED | xfer.FLAG_KEEP_OUTPUTS)
    assert [c[2] for c in rs] == [4 * N * N, 4 * o.params["I"] * o.params["J"] * K]


def test_sections_boxes_reused_and_dropped():
    # two CPU readers of the same stale buffer: the second reads inside the
    # first one's box (no copy); a GPU write in between drops the box
    doc = {"name": "t", "params": {"N": 16},
           "buffers": [{"name": "X", "dims": ["N", "N"]}, {"name": "Y", "dims": ["N"]}],
           "program": [
               {"nest": "w", "op": "none", "loops": [["i", "0", "N"], ["j", "0", "N"]], "access": [["X", "w", "i", "j"]]},
               {"nest": "r1", "op": "none", "loops": [["i", "2", "10"]], "access": [["Y", "w", "i"], ["X", "r", "i", "3"], ["X", "r", "i", "5"]]},
               {"nest": "r2", "op": "none", "loops": [["i", "4", "6"]], "access": [["Y", "w", "i"], ["X", "r", "i", "4"]]},
               {"nest": "w2", "op": "none", "loops": [["i", "0", "N"], ["j", "0", "N"]], "access": [["X", "w", "i", "j"]]},
               {"nest": "r3", "op": "none", "loops": [["i", "4", "6"]], "access": [["Y", "w", "i"], ["X", "r", "i", "4"]]},
               {"nest": "r4", "op": "none", "loops": [["i", "0", "N"], ["j", "0", "N"]], "access": [["Y", "w", "i"], ["X", "r", "i", "j"]]}]}
    o = ir.load(doc)
    cs = xfer.plan(o, [1, 0, 0, 1, 0, 0], xfer.SECTIONS, xfer.FLAG_KEEP_OUTPUTS)
    got = [(c[0], o.buffers[c[1]].name, c[2]) for c in cs]
    # r1: rows 2..9, columns 3..5 -> 8 x 3 floats; r2 inside it; w2 drops the
    # box; r3 copies rows 4..5 column 4; r4 reads the whole array: whole copy
    assert got == [("D2H", "X", 4 * 8 * 3), ("D2H", "X", 4 * 2 * 1), ("D2H", "X", 4 * 16 * 16)]


# ------------------------------------------------------------ GA operators
# Pins of the GA's operators against the paper's definitions (Sec. 3.3,
# Sec. 5.1.2: roulette selection in proportion to fitness, one elite kept
# unchanged, one-point crossover, per-value mutation), independent of the
# library's GA (which is compared with this oracle elsewhere).

# SplitMix64 with state 29 (the generator is pinned to the published outputs
# from state 0 above); the draws the worked generation below consumes
_STREAM29 = [0xbb7b49ab8801cf70, 0xba57b7db607f9d1a, 0xe1b9ae67265f7887, 0x5330404c13ee7598,
             0x14527c80ce1ad689, 0x868c79fa78c0d7ff, 0xc6b9305886e78606, 0x52042190b08a9d24,
             0xea18a3744e5c0d78, 0x330743f27ac6ddee, 0xd8dc1ac9a40cbb0c, 0xc087f4e359a1e03c,
             0xc18278c01db3075a, 0x950e8017dc3ab596, 0x2885f7c664c239ff, 0x15d19423ee5387c5,
             0x9493fee70e8c82bc, 0xffe028b40f65d177, 0x69ef7462eed1a5a8, 0x8892364d1ec21082,
             0xe9f707722d38e5e1, 0x10a553fb9e99492d, 0x4a101b61e826fb26, 0x845cb7606cf7929c]


def worked_generation_table():
    """Time table of the worked generation (a = 4): genes 7, 6, 13 take
    0.25, 16 and 1 time units (fitness t^-1/2 = 2, 1/4, 1); every other gene 100."""
    t = [100.0] * 16
    t[7], t[6], t[13] = 0.25, 16.0, 1.0
    return t


# One generation of a = 4, M = 3, Pc = 0.9, Pm = 0.3, p = 1/2, seed 29,
# worked by hand from the draws above:
#  initial bits (draw >> 63): draws 0-3 -> (1,1,1,0), gene 7; draws 4-7 ->
#    (0,1,1,0), gene 6; draws 8-11 -> (1,0,1,1), gene 13
#  fitness (2, 1/4, 1), total 13/4; elite = individual 0 (1,1,1,0)
#  roulette draw 1: u(draw 12) = 0.7559, u * total = 2.457; running sums
#    2, 2.25, 3.25 -> the first above it is individual 2 (1,0,1,1)
#  roulette draw 2: u(draw 13) = 0.5823, u * total = 1.892 < 2 -> individual 0
#  pair (individual 2, individual 0): u(draw 14) = 0.1583 < Pc -> crossover
#    at 1 + draw 15 mod 3 = 2; the tails from position 2 on are exchanged:
#    (1,0 | 1,1) x (1,1 | 1,0) -> (1,0,1,0) and (1,1,1,1)
#  mutation, one u per bit of each child: child 1 draws 16-19 (0.580, 0.9995,
#    0.414, 0.533) none below 0.3; child 2 draws 20-23 (0.914, 0.065, 0.289,
#    0.517): bits 1 and 2 flip -> (1,0,0,1)
WORKED_NEXT = [(1, 1, 1, 0), (1, 0, 1, 0), (1, 0, 0, 1)]


def test_ga_worked_generation_by_hand():
    rng = G.SplitMix64(29)
    assert [rng.next() for _ in range(len(_STREAM29))] == _STREAM29
    out = G.run_ga(4, 3, 2, G.table_evaluator(worked_generation_table()), Pc=0.9, Pm=0.3, p=0.5, seed=29)
    g0, g1 = out["generations"]
    assert g0["pop"] == [(1, 1, 1, 0), (0, 1, 1, 0), (1, 0, 1, 1)]
    assert g0["fitness"] == [2.0, 0.25, 1.0]
    assert g1["pop"] == WORKED_NEXT


def test_ga_roulette_follows_fitness_shares():
    # Pc = Pm = 0: the M-1 children are the roulette's picks in draw order;
    # over 10^5 draws each gene's count is within 4 sigma of the binomial
    # mean sum over runs of (M-1) * n_g f_g / sum_h n_h f_h (n_g its copies in
    # the population, f_g = t_g^-1/2 = 1 + g here)
    a, M, runs = 4, 201, 500
    table = [1.0 / (1.0 + g) ** 2 for g in range(16)]
    obs = np.zeros(16)
    mean = np.zeros(16)
    var = np.zeros(16)
    for seed in range(runs):
        out = G.run_ga(a, M, 2, G.table_evaluator(table), Pc=0.0, Pm=0.0, p=0.5, seed=seed)
        g0, g1 = out["generations"]
        w = np.zeros(16)
        for g in g0["pop"]:
            w[G.gene_index(g)] += 1.0 + G.gene_index(g)
        share = w / w.sum()
        mean += (M - 1) * share
        var += (M - 1) * share * (1.0 - share)
        for g in g1["pop"][1:]:
            obs[G.gene_index(g)] += 1
    assert obs.sum() == runs * (M - 1)
    assert np.all(np.abs(obs - mean) <= 4.0 * np.sqrt(var) + 1e-9), (obs, mean)


def test_ga_one_point_crossover_cuts():
    # only the all-zero gene Z and the all-one gene O run (every other gene
    # fails, fitness 0), so every parent is Z or O; with Pc = 1 and Pm = 0 a
    # pair of one Z and one O must give the two complementary step genes
    # 0^c 1^(a-c) and 1^c 0^(a-c) with the cut c in [1, a-1] -- never the
    # parents themselves -- and the cuts are uniform over [1, a-1]
    a, M = 6, 257
    Z, O = (0,) * a, (1,) * a
    table = [1.0] * (1 << a)
    status = [G.ST_FAILED] * (1 << a)
    status[0] = status[(1 << a) - 1] = G.ST_OK
    cuts = np.zeros(a + 1)
    runs = 0
    for seed in range(120):
        out = G.run_ga(a, M, 2, G.table_evaluator(table, status), Pc=1.0, Pm=0.0, p=0.5, seed=seed)
        g0, g1 = out["generations"]
        if Z not in g0["pop"] or O not in g0["pop"]:
            continue
        runs += 1
        kids = g1["pop"][1:]
        for c1, c2 in zip(kids[0::2], kids[1::2]):
            if (c1, c2) in ((Z, Z), (O, O)):
                continue
            assert (c1, c2) not in ((Z, O), (O, Z))
            c = next(i for i in range(1, a) if c1[i] != c1[0])
            step = tuple([c1[0]] * c + [1 - c1[0]] * (a - c))
            assert c1 == step and c2 == tuple(1 - b for b in step), (c1, c2)
            cuts[c] += 1
    assert runs >= 40
    n = cuts.sum()
    assert cuts[0] == 0 and cuts[a] == 0 and n > 2000
    p = 1.0 / (a - 1)
    assert np.all(np.abs(cuts[1:a] - n * p) <= 4.0 * np.sqrt(n * p * (1 - p))), cuts
