"""The C-ABI library's host logic against the oracle, on the CPU (no GPU call):
parallelisability verdicts, transfer plans, the GA under an injected time
table, and the error paths of the boundary."""
import json
import os
import random
import re

import numpy as np
import pytest

import paper_1806_01430_amd as ofl
import workloads
from oracle import depcheck as D
from oracle import enum as E
from oracle import ga as G
from oracle import ir, xfer

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    with open(os.path.join(ROOT, "include", "ofl.h")) as f:
        text = f.read()
    declared = set(re.findall(r"\b(ofl_[a-z0-9_]+)\s*\(", text))
    assert declared == set(ofl.EXPORTS)
    L = ofl.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_status_strings():
    L = ofl.lib()
    assert L.ofl_status_str(0) == b"ok"
    for code in ofl.E:
        assert L.ofl_status_str(code) != b"unknown status"


@pytest.mark.parametrize("name", ["tiny", "medium", "precision", "large", "spectral"])
def test_verdicts_match_oracle(name):
    app = ofl.App(workloads.app_path(name))
    o = ir.load(workloads.app_path(name))
    assert app.n_nests == len(o.nests)
    assert app.gene_len == D.gene_length(o)
    assert app.verdicts() == [tuple(v) for v in D.check_app(o)]
    assert [app.nest_name(i) for i in range(app.n_nests)] == [n.name for n in o.nests]
    for b, buf in enumerate(o.buffers):
        assert app.buf_name(b) == buf.name
        assert app.buf_dims(b) == tuple(buf.dims)
        assert app.buf_info(b)[0] == buf.nbytes
        assert app.buf_info(b)[2] == buf.output


def test_random_nests_match_oracle():
    rng = random.Random(99)
    seen = set()
    for _ in range(300):
        doc = workloads.random_nest_doc(rng)
        o = ir.load(doc)
        app = ofl.App(json.dumps(doc))
        want = tuple(D.check_app(o)[0])
        assert app.nest_info(0) == want, doc
        seen.add(want[0])
    assert seen == {D.PARALLEL, D.REJECT}


def test_random_nests_with_flags_and_reductions():
    rng = random.Random(7)
    for t in range(100):
        doc = workloads.random_nest_doc(rng)
        nest = doc["program"][0]
        if t % 3 == 0:
            nest["access"].append(["Y", "sum"] + ["0"] * len(doc["buffers"][1]["dims"]))
        if t % 5 == 0:
            nest["flags"] = [rng.choice(["opaque_call", "early_exit"])]
        if t % 7 == 0:
            doc["program"] = [{"repeat": "3", "var": "n", "body": [nest]}]
        o = ir.load(doc)
        app = ofl.App(json.dumps(doc))
        assert app.nest_info(0) == tuple(D.check_app(o)[0]), doc


def test_plans_tiny_all_genes_match_oracle():
    app = ofl.App(workloads.app_path("tiny"))
    o = ir.load(workloads.app_path("tiny"))
    for flags in (0, ofl.PRESTAGED, ofl.KEEP_OUTPUTS, ofl.PRESTAGED | ofl.KEEP_OUTPUTS):
        for g, res, per in E.enumerate_plans(o, flags):
            assert app.plan_transfers(g, ofl.RESIDENT, flags) == res
            assert app.plan_transfers(g, ofl.PER_REGION, flags) == per


@pytest.mark.parametrize("name", ["medium", "large"])
def test_plans_random_genes_match_oracle(name):
    app = ofl.App(workloads.app_path(name))
    o = ir.load(workloads.app_path(name))
    v = D.check_app(o)
    rng = random.Random(3)
    for _ in range(80):
        g = tuple(rng.randint(0, 1) for _ in range(app.gene_len))
        pl = xfer.placement_of_gene(o, v, g)
        for pol in (xfer.RESIDENT, xfer.PER_REGION):
            for flags in (0, 3):
                assert app.plan_transfers(g, pol, flags) == xfer.totals(o, pl, pol, flags)


@pytest.mark.parametrize("name", ["tiny", "medium", "large", "spectral"])
def test_sections_plans_match_oracle(name):
    app = ofl.App(workloads.app_path(name))
    o = ir.load(workloads.app_path(name))
    v = D.check_app(o)
    rng = random.Random(5)
    genes = [tuple([1] * app.gene_len), tuple([0] * app.gene_len)]
    genes += [tuple(rng.randint(0, 1) for _ in range(app.gene_len)) for _ in range(60)]
    for g in genes:
        pl = xfer.placement_of_gene(o, v, g)
        for flags in (0, 1, 2, 3):
            want = xfer.totals(o, pl, xfer.SECTIONS, flags)
            assert app.plan_transfers(g, ofl.SECTIONS, flags) == want, (g, flags)
            # device-side copies do not depend on how much the host copies out
            assert want[0] == xfer.totals(o, pl, xfer.RESIDENT, flags)[0]


def test_mask_to_gene():
    app = ofl.App(workloads.app_path("medium"))
    v = app.verdicts()
    mask = [1 if x[0] != ofl.REJECT else 0 for x in v]
    assert app.mask_to_gene(mask) == tuple([1] * app.gene_len)
    bad = [1] * app.n_nests
    with pytest.raises(ofl.OflError) as ei:
        app.mask_to_gene(bad)
    assert ei.value.code == -7


def test_gene_errors():
    app = ofl.App(workloads.app_path("tiny"))
    with pytest.raises(ofl.OflError) as ei:
        app.plan_transfers([1] * 5)
    assert ei.value.code == -5
    with pytest.raises(ofl.OflError) as ei:
        app.plan_transfers([1, 0, 2, 0, 0, 0])
    assert ei.value.code == -6


def test_kernel_timing_kind_lists():
    app = ofl.App(workloads.app_path("tiny"))
    for ok in (None, "", "stencil19", "stencil19,copy_interior", "gemm,stencil19,copy_interior"):
        app.set_kernel_timing_op(ok)
    for bad in ("fft", "stencil19,", "stencil19,,gemm", ",gemm", "stencil19 ,gemm"):
        with pytest.raises(ofl.OflError) as ei:
            app.set_kernel_timing_op(bad)
        assert ei.value.code == -1
    for stride, phase in ((1, 0), (25, 12), (100, 99)):
        app.set_kernel_timing_sample(stride, phase)
    for stride, phase in ((0, 0), (-1, 0), (10, 10), (10, -1)):
        with pytest.raises(ofl.OflError) as ei:
            app.set_kernel_timing_sample(stride, phase)
        assert ei.value.code == -1


@pytest.mark.parametrize("mutate,code", [
    (lambda d: d.update(program="x"), -3),
    (lambda d: d["program"][1].update(op="fft"), -4),
    (lambda d: d["program"][1]["access"].append(["A", "r", "i+70", "k"]), -4),
    (lambda d: d["program"][1]["access"].append(["A", "r", "i*2", "k"]), -3),
    (lambda d: d["buffers"][0].update(dims=["N", "N", "N"]), -4),
    (lambda d: d["program"][2]["args"].update(A="nope"), -4),
    (lambda d: d["program"][1]["args"].update(prec="fp4"), -4),
])
def test_invalid_applications(mutate, code):
    doc = workloads.app_doc("tiny")
    mutate(doc)
    with pytest.raises(ofl.OflError) as ei:
        ofl.App(json.dumps(doc))
    assert ei.value.code == code


def test_malformed_json_and_missing_file():
    with pytest.raises(ofl.OflError) as ei:
        ofl.App('{"name": "x", "buffers": [ }')
    assert ei.value.code == -3
    with pytest.raises(ofl.OflError) as ei:
        ofl.App("/nonexistent/app.json")
    assert ei.value.code == -2


def test_accepted_host_only_op_is_invalid():
    # a recurrence body declared with parallel-looking accesses has no kernel
    doc = workloads.app_doc("medium")
    for nest in doc["program"]:
        if nest.get("op") == "rec_prefix":
            nest["access"] = [["v", "w", "i"], ["S", "r", "i", "0"]]
    with pytest.raises(ofl.OflError) as ei:
        ofl.App(json.dumps(doc))
    assert ei.value.code == -4


# ------------------------------------------------------------ GA parity
def _oracle_ga(a, params, table, status=None):
    return G.run_ga(a, params.M, params.T, G.table_evaluator(table, status), Pc=params.Pc, Pm=params.Pm,
                    p=params.p, seed=params.seed, deadline_factor=params.deadline_factor,
                    batched=bool(params.flags & ofl.BATCHED),
                    timeout=params.timeout_s if params.timeout_s > 0 else None)


@pytest.mark.parametrize("a,M,T,Pc,Pm,p,seed,dl,tmo", [
    (6, 4, 3, 0.9, 0.05, 0.5, 1, 0.0, 0.0),
    (6, 12, 12, 0.9, 0.05, 0.5, 7, 0.0, 0.0),
    (10, 20, 20, 0.9, 0.05, 1.0, 3, 0.0, 0.0),
    (13, 30, 20, 0.9, 0.05, 0.5, 11, 3.0, 0.0),
    (1, 3, 4, 0.9, 0.5, 0.5, 2, 0.0, 0.0),
    (5, 7, 6, 0.0, 0.0, 0.5, 5, 0.0, 0.0),
    (5, 8, 6, 1.0, 1.0, 0.5, 6, 2.0, 0.0),
    (12, 12, 12, 0.9, 0.05, 0.5, 2018, 0.0, 0.0),
    (8, 10, 8, 0.9, 0.05, 0.5, 4, 0.0, 2.5),
    (10, 12, 10, 0.9, 0.05, 0.5, 9, 3.0, 1.0),
])
@pytest.mark.parametrize("batched", [False, True])
def test_ga_trajectory_matches_oracle(a, M, T, Pc, Pm, p, seed, dl, tmo, batched):
    table = workloads.time_table(a, seed * 31 + a, lo=0.01, hi=5.0)
    params = ofl.ga_params(M=M, T=T, Pc=Pc, Pm=Pm, p=p, seed=seed, deadline_factor=dl, timeout_s=tmo,
                           flags=ofl.BATCHED if batched else 0)
    got = ofl.ga_run_table(a, params, table)
    want = _oracle_ga(a, params, table)
    assert got["n_generations"] == len(want["generations"])
    for gi, gen in enumerate(want["generations"]):
        assert [tuple(int(x) for x in g) for g in got["pops"][gi]] == list(gen["pop"])
        assert list(got["times"][gi]) == gen["time"]
        assert list(got["status"][gi]) == gen["status"]
    assert got["best_gene"] == want["best_gene"]
    assert got["best_time"] == want["best_time"]
    assert got["n_measured"] == want["n_measured"]
    if dl > 0:
        # the library reports a baseline that did not finish as -1
        assert got["t_all0"] == (want["t_all0"] if want["t_all0"] is not None else -1.0)


def test_ga_worked_generation_by_hand():
    # the generation worked out by hand from the SplitMix64 draws of state 29
    # (tests/test_oracle_logic.py): the library's GA takes the same steps
    from test_oracle_logic import WORKED_NEXT, worked_generation_table
    params = ofl.ga_params(M=3, T=2, Pc=0.9, Pm=0.3, p=0.5, seed=29)
    got = ofl.ga_run_table(4, params, worked_generation_table())
    assert [tuple(int(x) for x in g) for g in got["pops"][0]] == [(1, 1, 1, 0), (0, 1, 1, 0), (1, 0, 1, 1)]
    assert [tuple(int(x) for x in g) for g in got["pops"][1]] == WORKED_NEXT


def test_batched_generations_change_only_the_deadline():
    # without deadlines, measuring a generation's genes together leaves the
    # trajectory unchanged; with deadlines the limits differ, and the batched
    # run gives every fresh gene of a generation the limit at its start
    for seed in range(1, 6):
        table = workloads.time_table(8, seed, lo=0.01, hi=5.0)
        ev = G.table_evaluator(table)
        seq = G.run_ga(8, 10, 8, ev, seed=seed)
        bat = G.run_ga(8, 10, 8, ev, seed=seed, batched=True)
        assert [g["pop"] for g in seq["generations"]] == [g["pop"] for g in bat["generations"]]
        assert seq["best_gene"] == bat["best_gene"]
    limits = []

    def spy(g, limit):
        limits.append(limit)
        return ev(g, limit)
    G.run_ga(8, 10, 3, spy, seed=3, deadline_factor=2.0, batched=True)
    assert len(set(limits[1:11])) == 1 and limits[0] is None


def test_ga_with_failed_statuses_matches_oracle():
    a = 6
    rng = random.Random(4)
    table = workloads.time_table(a, 5)
    status = [G.ST_FAILED if rng.random() < 0.3 else G.ST_OK for _ in range(1 << a)]
    params = ofl.ga_params(M=8, T=6, seed=9)
    got = ofl.ga_run_table(a, params, table, status)
    want = _oracle_ga(a, params, table, status)
    for gi, gen in enumerate(want["generations"]):
        assert [tuple(int(x) for x in g) for g in got["pops"][gi]] == list(gen["pop"])
        assert list(got["status"][gi]) == gen["status"]
    assert got["best_gene"] == want["best_gene"]


def test_ga_table_argument_errors():
    params = ofl.ga_params(M=0)
    with pytest.raises(ofl.OflError):
        ofl.ga_run_table(3, params, np.ones(8))
    with pytest.raises(ofl.OflError):
        ofl.ga_run_table(3, ofl.ga_params(Pc=1.5), np.ones(8))


# ---------------------------------------------------------------- instance batches (host side)
def _batch_doc():
    return workloads.app_doc("batch")


def test_batch_create_and_buffer_shapes():
    params, seeds = workloads.batch_instances(7, seed=3)
    for p in params:
        p["SWEEPS"] = 4
    b = ofl.Batch(_batch_doc(), params, seeds)
    assert (b.n_inst, b.n_bufs, b.n_nests) == (7, 6, 4)
    assert b.buf_names == ["A", "B", "C", "p", "q", "res"]
    for i, p in enumerate(params):
        assert b.buf_info(i, 0)[2] == (p["N"], p["N"])
        assert b.buf_info(i, 3)[2] == (p["I"], p["J"], p["K"])
        assert b.buf_info(i, 3)[0] == 4 * p["I"] * p["J"] * p["K"]
        assert b.buf_info(i, 5)[1] == np.float64 and b.buf_info(i, 5)[2] == (4,)


def test_batch_instance_generator_matches_recipe():
    params, seeds = workloads.batch_instances(256, seed=1)
    Ns = np.array([p["N"] for p in params])
    assert Ns.min() >= 32 and Ns.max() <= 511 and len(set(seeds)) == 256
    assert all(p["I"] == p["J"] and p["K"] == 2 * p["I"] - 1 and 17 <= p["I"] <= 65 for p in params)
    # log-uniform: about half the orders below the geometric midpoint 128
    assert 0.35 < np.mean(Ns < 128) < 0.65


def test_batch_errors():
    doc = _batch_doc()
    with pytest.raises(ofl.OflError) as e:
        ofl.Batch(doc, [{"NOPE": 3}], [1])
    assert e.value.code == -1                                    # unknown parameter
    with pytest.raises(ofl.OflError) as e:
        ofl.Batch(doc, [{"SWEEPS": 3}, {"SWEEPS": 4}], [1, 2])
    assert e.value.code == -15                                   # repeat counts differ
    with pytest.raises(ofl.OflError) as e:
        ofl.Batch(workloads.app_doc("medium"), [{"N": 64}], [1])
    assert e.value.code == -7                                    # rejected recurrences
    with pytest.raises(ofl.OflError) as e:
        ofl.Batch(workloads.app_doc("tiny"), [{"N": 64}], [1])
    assert e.value.code == -15                                   # element-wise nests have no grouped form
    d = _batch_doc()
    d["program"][1]["args"]["prec"] = "bf16x3"
    with pytest.raises(ofl.OflError) as e:
        ofl.Batch(d, [{"N": 64}], [1])
    assert e.value.code == -15
    with pytest.raises(ValueError):
        ofl.Batch(doc, [{"N": 64}, {"I": 20}], [1, 2])


def test_batch_config_roundtrip_and_range():
    b = ofl.Batch(_batch_doc(), [{"N": 40}, {"N": 50}], [1, 2])
    c = b.config
    assert c["stencil_rows"] in (2, 4, 8) and 0 <= c["gemm_cfg"] < 8
    b.set_config(gemm_cfg=5, gemm_blocks_per_cu=1, stencil_rows=8, stencil_planes=16, stencil_blocks_per_cu=4)
    assert b.config == {"gemm_cfg": 5, "gemm_blocks_per_cu": 1, "stencil_rows": 8, "stencil_planes": 16,
                        "stencil_blocks_per_cu": 4}
    for bad in [dict(gemm_cfg=8), dict(gemm_blocks_per_cu=0), dict(stencil_rows=3), dict(stencil_blocks_per_cu=9),
                dict(stencil_planes=-1)]:
        with pytest.raises(ofl.OflError) as e:
            b.set_config(**bad)
        assert e.value.code == -1


def test_batch_run_checks_pointer_table():
    import ctypes
    b = ofl.Batch(_batch_doc(), [{"N": 40}, {"N": 50}], [1, 2])
    st = ofl.BatchStats()
    ptrs = (ctypes.c_void_p * 3)()
    assert ofl.lib().ofl_batch_run(b._h, ptrs, 3, None, ofl.BATCH_GROUPED, ctypes.byref(st)) == -8
    ptrs = (ctypes.c_void_p * 12)()
    assert ofl.lib().ofl_batch_run(b._h, ptrs, 12, None, ofl.BATCH_GROUPED, ctypes.byref(st)) == -8
    assert ofl.lib().ofl_batch_run(b._h, ptrs, 12, None, 7, ctypes.byref(st)) == -1


def test_ga_study_statistics_on_a_table():
    # the study's statistics on an injected landscape equal those recomputed
    # from the oracle GA's trajectories (same seeds, same table)
    from paper_1806_01430_amd import ga_study
    a, seeds, runs = 5, 12, 4
    table = workloads.time_table(a, 91, lo=0.01, hi=1.0)
    status = [G.ST_OK] * (1 << a)
    settings = [(16, 8, 0.9, 0.05, 0.5, 0.0), (4, 3, 0.9, 0.1, 1.0, 3.0)]
    res = ga_study.study(a, table, status, settings, seeds, runs)
    order = sorted(range(1 << a), key=lambda i: (table[i], i))
    assert res["best_gene"] == [(order[0] >> i) & 1 for i in range(a)]
    assert abs(res["exhaustive_search_s"] - runs * sum(table)) < 1e-9
    for (M, T, Pc, Pm, p, dl), got in zip(settings, res["settings"]):
        hits, ranks, measured, cost = 0, [], [], []
        for seed in range(1, seeds + 1):
            o = G.run_ga(a, M, T, G.table_evaluator(table), Pc=Pc, Pm=Pm, p=p, seed=seed, deadline_factor=dl)
            g = G.gene_index(o["best_gene"])
            hits += g == order[0]
            ranks.append(order.index(g))
            measured.append(o["n_measured"])
            cost.append(sum(t if st == G.ST_TIMEOUT else runs * t for _, t, st in o["log"]))
        assert got["p_best"] == hits / seeds
        assert got["median_rank"] == float(np.median(ranks))
        assert got["mean_measured"] == float(np.mean(measured))
        assert abs(got["mean_search_s"] - float(np.mean(cost))) < 1e-9
    assert "| 16 | 8 |" in ga_study.table(res)
    # every run cut at a timeout (the large application's study): the GA and
    # the cost of its measurements as the oracle GA gives them
    tmo = float(np.median(table))
    res = ga_study.study(a, table, status, settings, seeds, runs, timeout=tmo)
    for (M, T, Pc, Pm, p, dl), got in zip(settings, res["settings"]):
        measured, cost = [], []
        for seed in range(1, seeds + 1):
            o = G.run_ga(a, M, T, G.table_evaluator(table), Pc=Pc, Pm=Pm, p=p, seed=seed, deadline_factor=dl,
                         timeout=tmo)
            measured.append(o["n_measured"])
            cost.append(sum(t if st == G.ST_TIMEOUT else runs * t for _, t, st in o["log"]))
        assert got["mean_measured"] == float(np.mean(measured))
        assert abs(got["mean_search_s"] - float(np.mean(cost))) < 1e-9


@pytest.mark.parametrize("R,n,ok", [(4, 1, True), (4, 4096, True), (3, 3, False), (2, 8192, False), (2, 12, False)])
def test_fft_call_shapes(R, n, ok):
    # the FFT function block takes rows of n complex values, n a power of two
    # up to 4096; anything else is an invalid application
    from workloads import appgen
    doc = appgen.fft_app(R, n)
    if ok:
        app = ofl.App(json.dumps(doc))
        assert app.verdicts() == [(D.PARALLEL, D.R_NONE, 0)]
    else:
        with pytest.raises(ofl.OflError):
            ofl.App(json.dumps(doc))


@pytest.mark.parametrize("flag,ok", [(1, True), (0, True), (True, True), (2, False), ("yes", False)])
def test_inverse_fft_flag(flag, ok):
    # the inverse call is the FFT op with "inverse": true / 1 (0 / false is
    # the forward one); any other value is an invalid application
    from workloads import appgen
    doc = appgen.fft_app(4, 64)
    doc["program"][0]["args"]["inverse"] = flag
    if ok:
        assert ofl.App(json.dumps(doc)).verdicts() == [(D.PARALLEL, D.R_NONE, 0)]
    else:
        with pytest.raises(ofl.OflError):
            ofl.App(json.dumps(doc))


@pytest.mark.parametrize("n,extra,ok", [(2, {}, True), (4096, {}, True), (6, {}, False), (8192, {}, False),
                                         (64, {"inverse": 1}, True), (4096, {"inverse": 1}, True),
                                         (12, {"inverse": 1}, False), (64, {"real": 0}, True),
                                         (64, {"real": 3}, False)])
def test_real_fft_call_shapes(n, extra, ok):
    # the real call and its inverse: rows of n real values (or packed
    # spectra), n a power of two from 2 to 4096
    from workloads import appgen
    doc = appgen.fft_app(3, n, real=True)
    doc["program"][0]["args"].update(extra)
    if ok:
        assert ofl.App(json.dumps(doc)).verdicts() == [(D.PARALLEL, D.R_NONE, 0)]
    else:
        with pytest.raises(ofl.OflError):
            ofl.App(json.dumps(doc))


def test_irregular_program_verdicts_and_plans_match_oracle():
    # a C program with loops the library does not implement: those nests run
    # on the CPU from their own compiled text; verdicts (with the reason of
    # each rejection) and every gene's transfers agree with the oracle
    from paper_1806_01430_amd import cfront
    doc = cfront.load(os.path.join(ROOT, "paper_1806_01430_amd", "apps", "irregular.c"))
    app = ofl.App(doc)
    o = ir.load(doc)
    v = D.check_app(o)
    assert app.verdicts() == [tuple(x) for x in v]
    reasons = {app.nest_name(i): v[i][1] for i in range(app.n_nests) if v[i][0] == D.REJECT}
    assert sorted(reasons.values()) == [D.R_EXTERNAL_CALL, D.R_BREAK] + [D.R_NO_KERNEL] * 5
    assert app.gene_len == 5
    for idx in range(1 << app.gene_len):
        g = tuple((idx >> k) & 1 for k in range(app.gene_len))
        pl = xfer.placement_of_gene(o, v, g)
        for pol in (xfer.RESIDENT, xfer.PER_REGION, xfer.SECTIONS):
            for flags in (0, 3):
                assert app.plan_transfers(g, pol, flags) == xfer.totals(o, pl, pol, flags), (g, pol, flags)


def test_grids_of_2_gib_or_more_are_rejected():
    # the sweep and the interior copy address a grid with 32-bit byte
    # offsets: a grid of 2^31 bytes or more is an invalid application
    from workloads import appgen
    # (the sweep's offsets reach up to five planes past the grid: I + 6 planes)
    ok = appgen.stencil_app(1000, 1024, 511, 1)          # 1006 planes: 2.106e9 bytes < 2^31
    ofl.App(json.dumps(ok))
    big = appgen.stencil_app(1024, 1024, 511, 1)         # 1030 planes: 2.156e9 bytes
    with pytest.raises(ofl.OflError) as e:
        ofl.App(json.dumps(big))
    assert e.value.code == -4 and "2 GiB" in str(e.value)
    only_copy = {"name": "c", "params": {"I": 1024, "J": 1024, "K": 513},
                 "buffers": [{"name": "p", "dims": ["I", "J", "K"]}, {"name": "q", "dims": ["I", "J", "K"]}],
                 "program": [appgen.copy_interior_nest("p", "q")]}
    with pytest.raises(ofl.OflError) as e:
        ofl.App(json.dumps(only_copy))
    assert e.value.code == -4


@pytest.mark.parametrize("batched", [False, True])
def test_ga_log_resume_retraces_the_search(tmp_path, batched):
    # a search interrupted after generation g (or in the middle of one) and
    # resumed from its log has the trajectory of an uninterrupted one, and
    # measures none of the logged genes again
    a, M, T = 10, 12, 12
    table = workloads.time_table(a, 21, lo=0.01, hi=5.0)
    kw = dict(M=M, Pc=0.9, Pm=0.05, p=0.5, seed=7, deadline_factor=3.0, flags=ofl.BATCHED if batched else 0)
    full = ofl.ga_run_table(a, ofl.ga_params(T=T, **kw), table)
    log = str(tmp_path / "ga.jsonl")
    part = ofl.ga_run_table(a, ofl.ga_params(T=5, cache_path=log, **kw), table)
    assert part["n_generations"] == 5
    lines = open(log).read().splitlines()
    assert json.loads(lines[0])["search"].startswith("a=10;M=12;")
    recs = [json.loads(x) for x in lines[1:]]
    assert sum(1 for r in recs if "gene" in r) == part["n_measured"]
    assert [r["gen"] for r in recs if "gen" in r] == [1, 2, 3, 4, 5]
    for cut in (len(lines), len(lines) - 4, 9):
        with open(log, "w") as f:
            f.write("\n".join(lines[:cut]) + "\n")
        got = ofl.ga_run_table(a, ofl.ga_params(T=T, cache_path=log, **kw), table)
        for gi in range(T):
            assert np.array_equal(got["pops"][gi], full["pops"][gi]), (cut, gi)
            assert np.array_equal(got["times"][gi], full["times"][gi])
        assert got["best_gene"] == full["best_gene"] and got["n_measured"] == full["n_measured"]
        # every measurement is in the log once, in the order taken
        genes = [json.loads(x)["gene"] for x in open(log).read().splitlines()[1:] if '"gene"' in x]
        assert len(genes) == len(set(genes)) == full["n_measured"]
    # a line cut short by an interrupted write ends the log there
    with open(log, "w") as f:
        f.write("\n".join(lines[:6]) + "\n" + lines[6][:12])
    got = ofl.ga_run_table(a, ofl.ga_params(T=T, cache_path=log, **kw), table)
    assert got["best_gene"] == full["best_gene"]


def test_ga_log_of_another_search_is_refused(tmp_path):
    a = 8
    table = workloads.time_table(a, 2, lo=0.01, hi=5.0)
    log = str(tmp_path / "ga.jsonl")
    ofl.ga_run_table(a, ofl.ga_params(M=8, T=3, seed=1, cache_path=log), table)
    with pytest.raises(ofl.OflError) as e:
        ofl.ga_run_table(a, ofl.ga_params(M=8, T=3, seed=2, cache_path=log), table)
    assert e.value.code == -12
    other = list(table)
    other[5] *= 2.0
    with pytest.raises(ofl.OflError):
        ofl.ga_run_table(a, ofl.ga_params(M=8, T=3, seed=1, cache_path=log), other)
    # a log whose measurements are out of order disagrees with the search
    lines = open(log).read().splitlines()
    body = [x for x in lines[1:] if '"gene"' in x]
    with open(log, "w") as f:
        f.write("\n".join([lines[0]] + body[1:2] + body[0:1]) + "\n")
    with pytest.raises(ofl.OflError) as e:
        ofl.ga_run_table(a, ofl.ga_params(M=8, T=3, seed=1, cache_path=log), table)
    assert e.value.code == -12
