"""GPU path vs the oracle, through the C ABI (needs an MI355X).

Every case runs the application under a gene with ofl_run_pattern, reads the
buffers back and compares them with the oracle's serial run (bits) or its
FP64 twin (GEMM-dependent values), see tests/parity.py for the bar."""
import json
import random
import sys

import numpy as np
import pytest

import paper_1806_01430_amd as ofl
import workloads
from workloads import appgen
from oracle import cnests as OC
from oracle import ir

import parity

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield


def _run_and_compare(doc, genes, seed=1, inputs=None, policies=(ofl.RESIDENT,), flags_list=(0,), names=None):
    app = ofl.App(json.dumps(doc), seed=seed)
    o = ir.load(doc)
    for name, arr in (inputs or {}).items():
        app.set_input(name, arr)
    cache = {}
    bufs = app.alloc_device_buffers()
    for g in genes:
        key = parity.offloaded_split(o, g)
        if key not in cache:
            cache[key] = parity.oracle_outputs(o, seed, inputs, offloaded=key)
        o32, o64 = cache[key]
        for pol in policies:
            for fl in flags_list:
                say("case", doc["name"], doc["params"], "gene", list(g), "policy", pol, "flags", fl)
                st = app.run_pattern(g, bufs, policy=pol, flags=fl)
                assert st["status"] == ofl.ST_OK
                assert (st["bytes_h2d"], st["bytes_d2h"], st["n_copies"]) == app.plan_transfers(g, pol, fl)
                bad = parity.compare(o, app.read_all(), o32, o64, names=names,
                                     rel_gemm=parity.rel_gemm_for(o, key))
                assert not bad, (list(g), pol, fl, bad)
    return app, bufs


# ---------------------------------------------------------------- applications
def test_tiny_all_64_genes():
    doc = workloads.app_doc("tiny")
    genes = [[(idx >> i) & 1 for i in range(6)] for idx in range(64)]
    _run_and_compare(doc, genes)


def test_tiny_policies_and_flags():
    doc = workloads.app_doc("tiny")
    genes = [[1] * 6, [0, 1, 0, 1, 0, 1], [1, 0, 1, 0, 1, 0]]
    _run_and_compare(doc, genes, policies=(ofl.RESIDENT, ofl.PER_REGION),
                     flags_list=(0, ofl.PRESTAGED, ofl.KEEP_OUTPUTS, ofl.PRESTAGED | ofl.KEEP_OUTPUTS))


def test_medium_reduced_random_genes():
    doc = workloads.app_doc("medium", **workloads.SMALL_MEDIUM)
    rng = random.Random(1)
    genes = [[1] * 10, [0] * 10] + [[rng.randint(0, 1) for _ in range(10)] for _ in range(10)]
    _run_and_compare(doc, genes, seed=3, policies=(ofl.RESIDENT, ofl.PER_REGION))


def test_large_reduced_random_genes():
    doc = workloads.app_doc("large", **workloads.SMALL_LARGE)
    rng = random.Random(2)
    genes = [[1] * 13] + [[rng.randint(0, 1) for _ in range(13)] for _ in range(5)]
    _run_and_compare(doc, genes, seed=5, flags_list=(0, ofl.PRESTAGED | ofl.KEEP_OUTPUTS))


def test_repeated_runs_restore_inputs():
    # consecutive runs with different genes must each start from the set-up
    doc = workloads.app_doc("medium", **workloads.SMALL_MEDIUM)
    genes = [[1] * 10, [0] * 10, [1] * 10, [1, 0] * 5, [1] * 10]
    _run_and_compare(doc, genes, seed=2, flags_list=(ofl.PRESTAGED | ofl.KEEP_OUTPUTS, 0))


def test_medium_full_size_all_gpu():
    doc = workloads.app_doc("medium")
    _run_and_compare(doc, [[1] * 10], seed=1, flags_list=(ofl.PRESTAGED | ofl.KEEP_OUTPUTS,))


# ---------------------------------------------------------------- GEMM
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (17, 33, 5), (64, 64, 64), (130, 70, 37), (257, 129, 300),
                                   (1000, 1000, 1000), (1024, 1024, 1024), (2048, 2048, 128)])
def test_gemm_f32_shapes(M, N, K):
    doc = appgen.gemm_app(M, N, K)
    A = OC.init_uniform(M * K, 11, 0).reshape(M, K)
    B = OC.init_uniform(K * N, 11, 1).reshape(K, N)
    _run_and_compare(doc, [[1]], inputs={"A": A, "B": B})


def test_gemm_f32_large_sampled():
    # 4096^3 in the launch configuration of the large products: sampled rows
    # against the FP64 twin (the full serial oracle would take minutes)
    import torch
    M = N = K = 4096
    doc = appgen.gemm_app(M, N, K)
    app = ofl.App(json.dumps(doc))
    A = OC.init_uniform(M * K, 12, 0).reshape(M, K)
    B = OC.init_uniform(K * N, 12, 1).reshape(K, N)
    app.set_input("A", A)
    app.set_input("B", B)
    bufs = app.alloc_device_buffers()
    say("case gemm 4096 sampled")
    app.run_pattern([1], bufs, flags=ofl.KEEP_OUTPUTS)
    C = app.read_buffer("C")
    rows = np.random.default_rng(0).choice(M, 24, replace=False)
    ref = OC.gemm_f64(np.ascontiguousarray(A[rows]), B)
    err = np.max(np.abs(C[rows] - ref) / ref)
    assert err < 1e-5, err
    del torch


@pytest.mark.parametrize("M,N,K", [(2048, 4096, 160), (2048, 4096, 32), (2049, 4096, 160), (2048, 4100, 96)])
def test_gemm_f32_lds_direct_form(M, N, K, monkeypatch):
    # products of 512 tiles of 128 x 128 and more take the LDS-direct form
    # when the shape is whole tiles and 32-deep slabs (the first case), else
    # the register-staged one; both sum each output in the same order, so
    # the forms must agree bit for bit; sampled rows (and the ragged last
    # rows) against the FP64 twin
    A = OC.init_uniform(M * K, 13, 0).reshape(M, K)
    B = OC.init_uniform(K * N, 13, 1).reshape(K, N)
    out = {}
    for form in (None, "reg"):
        if form:
            monkeypatch.setenv("OFL_GEMM_F32_FORM", form)
        app = ofl.App(json.dumps(appgen.gemm_app(M, N, K)))
        app.set_input("A", A)
        app.set_input("B", B)
        bufs = app.alloc_device_buffers()
        say("case gemm f32 form", form, M, N, K)
        app.run_pattern([1], bufs, flags=ofl.KEEP_OUTPUTS)
        out[form] = app.read_buffer("C")
        del app, bufs
    assert np.array_equal(out[None].view(np.uint32), out["reg"].view(np.uint32))
    rows = np.array(sorted(set(list(np.random.default_rng(3).choice(M, 8, replace=False)) + [0, M - 1])))
    ref = OC.gemm_f64(np.ascontiguousarray(A[rows]), B)
    err = np.max(np.abs(out[None][rows] - ref) / ref)
    assert err < parity.REL_GEMM, err


def test_gemm_identity_and_rank1_exact():
    for N in (64, 200, 1024):
        doc = appgen.gemm_app(N, N, N)
        B = OC.init_uniform(N * N, 3, 1).reshape(N, N)
        app = ofl.App(json.dumps(doc))
        app.set_input("A", np.eye(N, dtype=np.float32))
        app.set_input("B", B)
        bufs = app.alloc_device_buffers()
        say("case gemm identity", N)
        app.run_pattern([1], bufs)
        assert np.array_equal(app.read_buffer("C"), B)
        u = (np.arange(N) % 7 + 1).astype(np.float32)
        v = (np.arange(N) % 5 + 1).astype(np.float32)
        app.set_input("A", np.repeat(u[:, None], N, axis=1))
        app.set_input("B", np.repeat(v[None, :], N, axis=0))
        say("case gemm rank-1", N)
        app.run_pattern([1], bufs)
        assert np.array_equal(app.read_buffer("C"), (N * np.outer(u, v)).astype(np.float32))


# tile "256": the 8-wave 256 x 256 form forced (chosen by size from 256 tiles
# up; operands loaded straight into LDS), "256reg": that tile with
# register-staged loads
@pytest.mark.parametrize("M,N,K,tile", [(16, 16, 32, None), (100, 70, 45, None), (512, 512, 512, None),
                                        (100, 70, 45, "256"), (512, 512, 512, "256"), (300, 600, 130, "256"),
                                        (300, 600, 130, "256reg"), (520, 260, 700, "256"),
                                        (256, 256, 64, "256")])
def test_gemm_bf16_shapes(M, N, K, tile, monkeypatch):
    if tile:
        monkeypatch.setenv("OFL_GEMM_NT_TILE", "256")
        if tile.endswith("reg"):
            monkeypatch.setenv("OFL_GEMM_NT_FORM", "reg")
    doc = appgen.gemm_app(M, N, K, op="gemm_bf16")
    A = OC.cast_bf16(OC.init_uniform(M * K, 4, 0).reshape(M, K))
    B = OC.cast_bf16(OC.init_uniform(K * N, 4, 1).reshape(K, N))
    _run_and_compare(doc, [[1]], inputs={"A": A, "B": B})


# ---------------------------------------------------------------- split-precision GEMM
SPLIT = ["bf16x3", "fp8x2"]


def _wide(shape, seed):
    """Signed values over ~10 decades: many land on e4m3 subnormals after scaling."""
    r = np.random.default_rng(seed)
    return (r.standard_normal(shape) * np.exp(r.uniform(-11, 11, shape))).astype(np.float32)


@pytest.mark.parametrize("prec", SPLIT)
# K a multiple of 4: A split 4 elements per lane; K and N whole 64-element
# tiles: B split through 16-byte accesses
@pytest.mark.parametrize("M,N,K,tile", [(1, 1, 1, None), (17, 33, 5, None), (130, 70, 37, None),
                                        (257, 129, 300, None), (384, 256, 200, None), (128, 192, 64, None),
                                        (1, 1, 1, "256"), (257, 129, 300, "256"), (520, 300, 70, "256"),
                                        (300, 320, 128, "256")])
def test_gemm_split_shapes(prec, M, N, K, tile, monkeypatch):
    # gene 1: the split product (oracle: its definition summed in FP64);
    # gene 0: the nest as written, plain FP32 on the CPU
    if tile:
        monkeypatch.setenv("OFL_GEMM_NT_TILE", tile)
    doc = appgen.gemm_app(M, N, K, prec=prec)
    A = OC.init_uniform(M * K, 21, 0).reshape(M, K)
    B = OC.init_uniform(K * N, 21, 1).reshape(K, N)
    _run_and_compare(doc, [[1], [0]], inputs={"A": A, "B": B})


@pytest.mark.parametrize("tile", ["128", "256"])
def test_gemm_nt_padded_row_layout(tile, monkeypatch):
    # the products with their slabs staged in padded rows (the alternative LDS
    # layout, a knob) on ragged shapes, each form against the oracle
    monkeypatch.setenv("OFL_GEMM_NT_LAYOUT", "0")
    monkeypatch.setenv("OFL_GEMM_NT_TILE", tile)
    monkeypatch.setenv("OFL_GEMM_NT_FORM", "reg")
    M, N, K = 300, 270, 140
    A = OC.init_uniform(M * K, 23, 0).reshape(M, K)
    B = OC.init_uniform(K * N, 23, 1).reshape(K, N)
    for prec in SPLIT:
        say("case nt padded layout", tile, prec)
        _run_and_compare(appgen.gemm_app(M, N, K, prec=prec), [[1]], inputs={"A": A, "B": B})
    say("case nt padded layout", tile, "bf16")
    _run_and_compare(appgen.gemm_app(M, N, K, op="gemm_bf16"), [[1]],
                     inputs={"A": OC.cast_bf16(A), "B": OC.cast_bf16(B)})


@pytest.mark.parametrize("prec", SPLIT)
def test_gemm_split_signed_wide_range(prec):
    M, N, K = 200, 150, 333
    A, B = _wide((M, K), 1), _wide((K, N), 2)
    app = ofl.App(json.dumps(appgen.gemm_app(M, N, K, prec=prec)))
    app.set_input("A", A)
    app.set_input("B", B)
    bufs = app.alloc_device_buffers()
    say("case split wide", prec)
    app.run_pattern([1], bufs)
    got = app.read_buffer("C").astype(np.float64)
    emu = OC.gemm_split_f64(A, B, prec)
    mag = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
    err = np.max(np.abs(got - emu) / mag)
    say("split wide", prec, "max err / sum|a||b|", err)
    assert err < (parity.REL_GEMM if prec == "bf16x3" else parity.REL_FP8_MFMA), err


@pytest.mark.parametrize("prec", SPLIT)
@pytest.mark.parametrize("tile", [None, "256"])
def test_gemm_split_identity_and_rank1_exact(prec, tile, monkeypatch):
    # A = I: every output is hi + lo of one element of B, exact in FP32, so the
    # GPU must equal the oracle's split bit for bit -- including e4m3
    # subnormals, as B spans many decades within each column
    if tile:
        monkeypatch.setenv("OFL_GEMM_NT_TILE", tile)
    for N in (64, 200):
        app = ofl.App(json.dumps(appgen.gemm_app(N, N, N, prec=prec)))
        B = _wide((N, N), N)
        app.set_input("A", np.eye(N, dtype=np.float32))
        app.set_input("B", B)
        bufs = app.alloc_device_buffers()
        say("case split identity", prec, N)
        app.run_pattern([1], bufs)
        want = OC.gemm_split_f64(np.eye(N, dtype=np.float32), B, prec).astype(np.float32)
        assert np.array_equal(app.read_buffer("C"), want)
        u = (np.arange(N) % 7 + 1).astype(np.float32)
        v = (np.arange(N) % 5 + 1).astype(np.float32)
        app.set_input("A", np.repeat(u[:, None], N, axis=1))
        app.set_input("B", np.repeat(v[None, :], N, axis=0))
        say("case split rank-1", prec, N)
        app.run_pattern([1], bufs)
        assert np.array_equal(app.read_buffer("C"), (N * np.outer(u, v)).astype(np.float32))


@pytest.mark.parametrize("prec", SPLIT)
def test_gemm_split_4096_sampled(prec):
    # the GEMM of the precision workload at full size, sampled rows against
    # the split definition (1e-5) and against the exact product (reported)
    M = N = K = 4096
    app = ofl.App(json.dumps(appgen.gemm_app(M, N, K, prec=prec)))
    A = OC.init_uniform(M * K, 12, 0).reshape(M, K)
    B = OC.init_uniform(K * N, 12, 1).reshape(K, N)
    app.set_input("A", A)
    app.set_input("B", B)
    bufs = app.alloc_device_buffers()
    say("case split 4096 sampled", prec)
    app.run_pattern([1], bufs, flags=ofl.KEEP_OUTPUTS)
    C = app.read_buffer("C").astype(np.float64)
    rows = np.random.default_rng(1).choice(M, 8, replace=False)
    emu = OC.gemm_split_f64(np.ascontiguousarray(A[rows]), B, prec)
    exact = OC.gemm_f64(np.ascontiguousarray(A[rows]), B)
    err_emu = np.max(np.abs(C[rows] - emu) / emu)
    err_exact = np.max(np.abs(C[rows] - exact) / exact)
    say("split 4096", prec, "max rel err vs split definition", err_emu, "vs exact product", err_exact)
    assert err_emu < (parity.REL_GEMM if prec == "bf16x3" else parity.REL_FP8_MFMA), err_emu
    assert err_exact < (1e-5 if prec == "bf16x3" else 1e-3), err_exact


def test_gemm_fp8_run_truncation():
    # the premise of the fp8 tolerance, through the product path: one row
    # A = [416, 3 * 2^-8], B = [1; 1].  Scales 1/2 and 128 make every split
    # exact (lo parts 0); the products 26624 and 0.75 share one run of 8, and
    # 0.75 lies below 2^-14 of 2^14, so the MFMA drops it: C = 416 exactly,
    # where the split definition gives 416 + 3 * 2^-8.
    app = ofl.App(json.dumps(appgen.gemm_app(1, 1, 2, prec="fp8x2")))
    app.set_input("A", np.array([[416.0, 3 * 2.0 ** -8]], np.float32))
    app.set_input("B", np.ones((2, 1), np.float32))
    bufs = app.alloc_device_buffers()
    say("case fp8 run truncation")
    app.run_pattern([1], bufs)
    emu = OC.gemm_split_f64(np.array([[416.0, 3 * 2.0 ** -8]], np.float32), np.ones((2, 1), np.float32), "fp8x2")
    assert emu[0, 0] == 416.0 + 3 * 2.0 ** -8
    assert app.read_buffer("C")[0, 0] == 416.0


def test_precision_app_reduced_all_forms():
    # the precision workload at reduced size under each GEMM form, all-GPU and
    # all-CPU genes
    for prec in ["f32"] + SPLIT:
        doc = workloads.app_doc("precision", N=160, I=13, J=17, K=67, SWEEPS=3)
        doc["program"][1]["args"]["prec"] = prec
        _run_and_compare(doc, [[1] * 4, [0] * 4, [1, 1, 0, 1]])


# ---------------------------------------------------------------- stencil
@pytest.mark.parametrize("I,J,K,S", [(3, 3, 3, 2), (4, 5, 6, 3), (33, 33, 65, 10), (19, 23, 71, 4),
                                     (5, 130, 300, 2), (70, 9, 64, 2), (10, 11, 127, 3), (129, 129, 257, 3)])
def test_stencil_shapes(I, J, K, S):
    _run_and_compare(appgen.stencil_app(I, J, K, S), [[1, 1], [1, 0], [0, 1]])


# every sweep kernel form (rows per item, planes per item; one or two columns
# per lane; store policy), forced through the library's tuning knobs, on
# ragged shapes: k-tiles with a partial last tile, j-runs past the last row,
# i-runs shorter than the item; the band form (a block per band of rows
# across the whole row, planes staged in LDS) with every row length it takes,
# whole and partial bands, and its automatic plane runs (IC = 0); the band
# form with its planes loaded straight into LDS (d), runs of 1 to 32 planes
@pytest.mark.parametrize("cfg,form,nt", [("2,1", "1", "0"), ("4,3", "1", "1"), ("8,5", "1", "0"), ("2,2", "w", "1"),
                                         ("4,6", "w", "0"), ("8,4", "w", "1"), ("8,16", "w", "0"),
                                         ("8,2", "b", "0"), ("8,7", "b", "1"), ("8,32", "b", "0"), ("8,0", "b", "0"),
                                         ("8,1", "d", "0"), ("8,2", "d", "1"), ("8,4", "d", "0"), ("8,7", "d", "1"),
                                         ("8,32", "d", "0"), ("8,0", "d", "0"), ("8,0", "bl", "0"),
                                         ("8,5", "bl", "1")])
def test_stencil_kernel_forms(cfg, form, nt, monkeypatch):
    monkeypatch.setenv("OFL_STENCIL_CFG", cfg)
    if form == "bl":   # band form, planes read with the streaming policy
        form = "b"
        monkeypatch.setenv("OFL_STENCIL_LNT", "1")
    monkeypatch.setenv("OFL_STENCIL_FORM", form)
    monkeypatch.setenv("OFL_STENCIL_NT", nt)
    shapes = [(4, 5, 6), (19, 23, 71), (5, 130, 300), (10, 11, 129), (6, 9, 254), (7, 6, 128)]
    if form in ("b", "d"):   # band form: 1, 2, 4 and 8 waves across a row, whole and partial bands;
        # rows longer than 8 tiles fall back to the two-columns form
        shapes += [(9, 26, 258), (6, 70, 131), (5, 40, 520), (4, 20, 1025), (9, 150, 130), (12, 66, 514),
                   (5, 9, 1100)]
    for I, J, K in shapes:
        say("case stencil form %s %s nt=%s grid %dx%dx%d" % (cfg, form, nt, I, J, K))
        _run_and_compare(appgen.stencil_app(I, J, K, 2), [[1, 1]])


@pytest.mark.parametrize("nt,flat", [("0", None), ("1", None), ("0", "1,0,0"), ("0", "1,1,1"), ("0", "2,1,0"),
                                     ("0", "4,0,1")])
def test_copy_interior_plane_range_form(nt, flat, monkeypatch):
    # the interior copy in its plane-range form (16-byte pieces of each
    # plane's contiguous interior range, the row-boundary columns left alone):
    # rows of every alignment, ranges shorter than one piece, one-row planes;
    # 1, 2 or 4 pieces per lane, streaming loads and / or stores
    monkeypatch.setenv("OFL_COPY_FORM", "flat")
    monkeypatch.setenv("OFL_COPY_CFG", "2,32,%s" % nt)
    if flat:
        monkeypatch.setenv("OFL_COPY_FLAT", flat)
    for I, J, K in [(3, 3, 3), (4, 5, 6), (3, 4, 7), (19, 23, 71), (5, 130, 300), (10, 11, 129), (6, 9, 254),
                    (7, 6, 128), (4, 20, 1025), (33, 33, 65), (5, 3, 1030)]:
        say("case copy plane-range nt=%s grid %dx%dx%d" % (nt, I, J, K))
        _run_and_compare(appgen.stencil_app(I, J, K, 2), [[1, 1], [0, 1]])


def _two_sweep_app(I, J, K, S):
    # two sweeps back to back (the second reads the first one's output), then
    # the interior copy; a single sweep as the program's last nest
    doc = appgen.stencil_app(I, J, K, S)
    doc["name"] = "two_sweeps"
    doc["buffers"] += [appgen.grid("r", "zero", True), {"name": "res2", "dtype": "f64", "dims": ["SWEEPS"],
                                                        "output": True},
                       {"name": "res3", "dtype": "f64", "dims": ["LAST"], "output": True}]
    doc["params"]["LAST"] = 2
    second = appgen.stencil_nest("q", "r", "res2", "n")
    second["nest"] = "stencil19_b"
    doc["program"] = [{"repeat": "SWEEPS", "var": "n",
                       "body": [appgen.stencil_nest("p", "q", "res", "n"), second,
                                appgen.copy_interior_nest("p", "r")]},
                      {"repeat": "LAST", "var": "m",
                       "body": [dict(appgen.stencil_nest("p", "q", "res3", "m"), nest="stencil19_last")]}]
    return doc


def test_stencil_residual_finish_placement():
    # the residual finish a sweep owes runs in the next interior copy's extra
    # block, or by itself before any other step / at the end of the run: every
    # placement of the four nests (the last sweep repeated twice: a sweep
    # directly after a sweep), eager and as graph replays
    doc = _two_sweep_app(9, 12, 131, 3)
    genes = [[(g >> b) & 1 for b in range(4)] for g in range(16)]
    _run_and_compare(doc, genes, flags_list=(0, ofl.GRAPH | ofl.PRESTAGED | ofl.KEEP_OUTPUTS))


def test_stencil_fixed_point_exact():
    I, J, K = 21, 34, 133
    ii, jj, kk = np.meshgrid(np.arange(I), np.arange(J), np.arange(K), indexing="ij")
    field = (ii + 2 * jj + 3 * kk).astype(np.float32)
    doc = appgen.stencil_app(I, J, K, 3)
    app = ofl.App(json.dumps(doc))
    app.set_input("p", field)
    bufs = app.alloc_device_buffers()
    say("case stencil fixed point")
    app.run_pattern([1, 1], bufs)
    inner = (slice(1, -1),) * 3
    assert np.array_equal(app.read_buffer("p"), field)
    assert np.array_equal(app.read_buffer("q")[inner], field[inner])
    assert np.all(app.read_buffer("res") == 0.0)


def test_stencil_eigenmode_decay():
    I, J, K = 33, 33, 65
    rows = [line.split() for line in open(workloads.ROOT + "/tests/golden/stencil_eigen.txt")
            if not line.startswith("#")]
    mu = [float(r[4]) for r in rows if r[:4] == ["33", "33", "65", "1"]][0]
    doc = appgen.stencil_app(I, J, K, 10)
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers()
    app.run_pattern([1, 1], bufs)
    _, p0 = OC.sin_field(I, J, K, 1, want64=True)
    inner = (slice(1, -1),) * 3
    err = np.max(np.abs(app.read_buffer("p")[inner] - mu ** 10 * p0[inner]))
    assert err < 100 * 2.0 ** -24


# the default forms at full size (a grid of 512 MB or more copies in the
# plane-range form with streaming accesses, 64-512 MB cached with two pieces
# per lane), the band sweep loading straight into LDS, the row-form copy
@pytest.mark.parametrize("I,J,K,form", [(257, 257, 513, None), (513, 513, 1025, None), (257, 257, 513, "d"),
                                         (513, 513, 1025, "d"), (257, 257, 513, "rows"), (513, 513, 1025, "rows")])
def test_stencil_full_size_one_sweep(I, J, K, form, monkeypatch):
    if form == "rows":
        monkeypatch.setenv("OFL_COPY_FORM", "rows")
    elif form:
        monkeypatch.setenv("OFL_STENCIL_FORM", form)
    _run_and_compare(appgen.stencil_app(I, J, K, 1), [[1, 1]], flags_list=(ofl.PRESTAGED | ofl.KEEP_OUTPUTS,))


# ---------------------------------------------------------------- element-wise
# (the transpose takes 16-byte accesses when both sides are multiples of 4)
@pytest.mark.parametrize("R,C", [(1, 1), (3, 5), (4, 8), (64, 64), (65, 127), (68, 132), (1000, 333), (1000, 332),
                                 (2048, 2048)])
def test_ewise_transpose_cast_sumsq(R, C):
    _run_and_compare(appgen.ewise_app(R, C), [[1] * 8, [1, 0] * 4, [0, 1] * 4])


# ---------------------------------------------------------------- runtime
def test_deadline_abandons_run():
    doc = workloads.app_doc("medium", **workloads.SMALL_MEDIUM)
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers()
    say("case deadline")
    st = app.run_pattern([0] * 10, bufs, deadline_s=1e-6, check=False)
    assert st["rc"] == -10 and st["status"] == ofl.ST_TIMEOUT
    with pytest.raises(ofl.OflError):
        app.read_buffer("C")
    st = app.run_pattern([1] * 10, bufs)
    assert st["status"] == ofl.ST_OK


def test_kernel_timing_and_bad_buffers():
    doc = workloads.app_doc("tiny")
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers()
    app.set_kernel_timing(True)
    app.run_pattern([1] * 6, bufs)
    n, ms = app.kernel_stats("stencil19")
    assert n == 10 and ms > 0
    n, ms = app.kernel_stats("gemm")
    assert n == 1 and ms > 0
    # sampled timing of two kinds: executions 1, 5, 9 of the 10 sweeps and
    # copies, eager and in a graph replay
    app.set_kernel_timing_op("stencil19,copy_interior")
    app.set_kernel_timing_sample(4, 1)
    for flags in (0, ofl.GRAPH):
        app.set_kernel_timing(True)
        app.run_pattern([1] * 6, bufs, flags=flags)
        assert [app.kernel_stats(k)[0] for k in ("stencil19", "copy_interior", "gemm")] == [3, 3, 0]
        assert min(app.kernel_stats(k)[1] for k in ("stencil19", "copy_interior")) > 0
    app.set_kernel_timing(False)
    app.set_kernel_timing_sample(1, 0)
    app.set_kernel_timing_op(None)
    with pytest.raises(ofl.OflError) as ei:
        app.run_pattern([1] * 6, bufs[:-1])
    assert ei.value.code == -8


def test_eval_population_and_ga_tiny():
    doc = workloads.app_doc("tiny")
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers()
    genes = [[(idx >> i) & 1 for i in range(6)] for idx in range(64)]
    say("case eval population 64")
    t, s = app.eval_population(genes, bufs, reps=3, warmup=1)
    assert np.all(s == ofl.ST_OK) and np.all(t > 0)
    best_idx = int(np.argmin(t))
    say("case GA tiny 4x3")
    res = app.ga_run(ofl.ga_params(M=4, T=3, seed=1, reps=3, warmup=1), bufs)
    assert res["n_generations"] == 3
    assert len(res["best_gene"]) == 6
    assert res["best_time"] > 0
    rank = int(np.sum(t < t[sum(b << i for i, b in enumerate(res["best_gene"]))]))
    say("GA best gene", res["best_gene"], "exhaustive best", genes[best_idx], "rank", rank)


# ---------------------------------------------------------------- FFT call
@pytest.mark.parametrize("inverse", [False, True])
@pytest.mark.parametrize("R,n", [(1, 1), (3, 2), (5, 4), (7, 8), (37, 64), (16, 128), (9, 256), (33, 512),
                                 (64, 1024), (7, 1024), (1, 1024), (20, 2048), (3, 2048), (6, 4096), (3, 4096)])
def test_fft_rows_shapes(R, n, inverse):
    # the function block (forward or inverse) on the GPU (gene 1) and its CPU
    # form (gene 0), each row within the FFT error bound of the exact
    # transform (the inverse's conjugations and 1/n scale are exact)
    from oracle.dft import dft_rows, idft_rows
    X = np.random.default_rng(R * 4099 + n).standard_normal((R, 2 * n)).astype(np.float32)
    doc = appgen.fft_app(R, n, inverse=inverse)
    app, bufs = _run_and_compare(doc, [[0], [1]], inputs={"X": X})
    ref = idft_rows(X) if inverse else dft_rows(X)
    outs = {}
    for g in (0, 1):
        app.run_pattern([g], bufs, flags=ofl.KEEP_OUTPUTS)
        outs[g] = app.read_buffer("X").copy()
        err = np.max(np.linalg.norm(outs[g] - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300))
        assert err <= parity.rel_fft(n) + 2.0 ** -23, (g, err)
    # beyond the bound: the GPU kernel and the CPU form run the same
    # butterflies on the same twiddle values, so they give the same bits
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32)), (R, n)


def test_fft_rows_full_size_sampled():
    # 8192 rows of 1024 points (64 MB), the launch the kernel benchmark times:
    # sampled rows against the exact transform
    from oracle.dft import dft_rows
    R, n = 8192, 1024
    X = np.random.default_rng(5).standard_normal((R, 2 * n)).astype(np.float32)
    app = ofl.App(json.dumps(appgen.fft_app(R, n)))
    app.set_input("X", X)
    bufs = app.alloc_device_buffers()
    say("case fft 8192 x 1024 sampled")
    assert app.run_pattern([1], bufs, flags=ofl.KEEP_OUTPUTS)["status"] == ofl.ST_OK
    Y = app.read_buffer("X")
    rows = np.concatenate([[0, R - 1], np.random.default_rng(1).choice(R, 30, replace=False)])
    ref = dft_rows(X[rows])
    err = np.max(np.linalg.norm(Y[rows] - ref, axis=1) / np.linalg.norm(ref, axis=1))
    assert err <= parity.rel_fft(n) + 2.0 ** -23, err


@pytest.mark.parametrize("inverse", [False, True])
@pytest.mark.parametrize("R,n", [(1, 2), (3, 4), (5, 8), (7, 16), (37, 128), (16, 256), (9, 512), (33, 1024),
                                 (64, 2048), (7, 2048), (6, 4096), (3, 4096)])
def test_fft_real_rows_shapes(R, n, inverse):
    # the real call or its inverse on the GPU (gene 1; the half-length
    # complex kernels and the (un)packing pass) and its CPU form (gene 0):
    # the oracle within the call's bound, and the same bits on both sides
    from oracle.dft import irdft_packed_rows, rdft_packed_rows
    X = np.random.default_rng(R * 31 + n).standard_normal((R, n)).astype(np.float32)
    doc = appgen.fft_app(R, n, inverse=inverse, real=True)
    app, bufs = _run_and_compare(doc, [[0], [1]], inputs={"X": X})
    ref = irdft_packed_rows(X) if inverse else rdft_packed_rows(X)
    bound = parity.rel_irfft(n) if inverse else parity.rel_rfft(n)
    outs = {}
    for g in (0, 1):
        app.run_pattern([g], bufs, flags=ofl.KEEP_OUTPUTS)
        outs[g] = app.read_buffer("X").copy()
        err = np.max(np.linalg.norm(outs[g] - ref, axis=1) / np.linalg.norm(ref, axis=1))
        assert err <= bound + 2.0 ** -23, (g, err)
    assert np.array_equal(outs[0].view(np.uint32), outs[1].view(np.uint32)), (R, n)


@pytest.mark.parametrize("R,n", [(5, 64), (9, 512), (3, 4096)])
def test_fft_real_round_trip(R, n):
    # the real call then its inverse under every gene: the rows come back
    # within sqrt 2 rel_rfft + rel_irfft, the same bits whichever side runs
    # each call
    X = np.random.default_rng(R * 7 + n).standard_normal((R, n)).astype(np.float32)
    app = ofl.App(json.dumps(appgen.rfft_roundtrip_app(R, n)))
    app.set_input("X", X)
    bufs = app.alloc_device_buffers()
    outs = {}
    bound = np.sqrt(2.0) * parity.rel_rfft(n) + parity.rel_irfft(n) + 2.0 ** -22
    for g in ([0, 0], [1, 1], [1, 0], [0, 1]):
        say("case rfft round trip", R, n, g)
        assert app.run_pattern(g, bufs)["status"] == ofl.ST_OK
        outs[tuple(g)] = app.read_buffer("X").copy()
        err = np.max(np.linalg.norm(outs[tuple(g)] - X, axis=1) / np.linalg.norm(X, axis=1))
        assert err <= bound, (g, err)
    for g in ((1, 1), (1, 0), (0, 1)):
        assert np.array_equal(outs[g].view(np.uint32), outs[(0, 0)].view(np.uint32)), g


@pytest.mark.parametrize("R,n", [(5, 64), (9, 256), (6, 1024), (3, 4096)])
def test_fft_round_trip(R, n):
    # the forward call then the inverse one: every gene gives the row back
    # within twice the FFT bound, and the genes that place both calls alike
    # agree bit for bit (the GPU and CPU forms run the same butterflies)
    X = np.random.default_rng(R + n).standard_normal((R, 2 * n)).astype(np.float32)
    app = ofl.App(json.dumps(appgen.fft_roundtrip_app(R, n)))
    app.set_input("X", X)
    bufs = app.alloc_device_buffers()
    outs = {}
    for g in ([0, 0], [1, 1], [1, 0], [0, 1]):
        say("case fft round trip", R, n, g)
        assert app.run_pattern(g, bufs)["status"] == ofl.ST_OK
        outs[tuple(g)] = app.read_buffer("X").copy()
        err = np.max(np.linalg.norm(outs[tuple(g)] - X, axis=1) / np.linalg.norm(X, axis=1))
        assert err <= 2 * (parity.rel_fft(n) + 2.0 ** -23), (g, err)
    for g in ((1, 1), (1, 0), (0, 1)):
        assert np.array_equal(outs[g].view(np.uint32), outs[(0, 0)].view(np.uint32)), g


def test_spectral_all_genes():
    # every gene under both transfer policies, eager and as graph replays
    doc = workloads.app_doc("spectral", R=37, M=512)
    genes = [[(idx >> i) & 1 for i in range(4)] for idx in range(16)]
    _run_and_compare(doc, genes, policies=(ofl.RESIDENT, ofl.SECTIONS), flags_list=(0, ofl.GRAPH))


def test_spectral_population_batched():
    # the FFT call inside one batched submission of a whole population
    doc = workloads.app_doc("spectral", R=64, M=2048)
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers()
    genes = [[(idx >> i) & 1 for i in range(4)] for idx in range(16)]
    say("case spectral population batched")
    t, s = app.eval_population(genes, bufs, reps=2, warmup=1, flags=ofl.BATCHED)
    assert np.all(s == ofl.ST_OK) and np.all(t > 0)
    o = ir.load(doc)
    o32, o64 = parity.oracle_outputs(o, 1)
    assert app.run_pattern([1, 1, 1, 1], bufs, flags=ofl.GRAPH)["status"] == ofl.ST_OK
    assert not parity.compare(o, app.read_all(), o32, o64)


def test_level1_blas_calls_every_gene():
    # saxpy / scopy / sscal function blocks from C source: every gene of the
    # program (init, three calls, one loop-form axpy) against the oracle
    import os
    from paper_1806_01430_amd import cfront
    doc = cfront.load(os.path.join(os.path.dirname(ofl.__file__), "apps", "blas1.c"))
    genes = [[(idx >> i) & 1 for i in range(5)] for idx in range(32)]
    _run_and_compare(doc, genes, policies=(ofl.RESIDENT, ofl.SECTIONS))


def test_search_from_c_source(tmp_path, capsys):
    # the whole flow from C source: parse, check, GA over measured runs,
    # the program written back with the best gene's directives; the parsed
    # application's all-GPU run matches the oracle
    import os
    from paper_1806_01430_amd import cfront, search
    src = os.path.join(os.path.dirname(ofl.__file__), "apps", "tiny.c")
    out = str(tmp_path / "tiny_offloaded.c")
    say("case search from tiny.c with --emit")
    assert search.main(["--app", src, "--M", "4", "--T", "3", "--emit", out]) == 0
    res = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    with open(out) as f:
        text = f.read()
    assert text.count("#pragma acc kernels") == sum(res["best_gene"])
    doc = cfront.load(src)
    assert cfront.parse(text, "tiny") == doc
    app = ofl.App(src)
    bufs = app.alloc_device_buffers()
    assert app.run_pattern([1] * app.gene_len, bufs)["status"] == ofl.ST_OK
    o = ir.load(doc)
    o32, o64 = parity.oracle_outputs(o, 1)
    assert not parity.compare(o, app.read_all(), o32, o64, rel_gemm=parity.rel_gemm_for(o, ()))


def test_batched_deadline_cuts_host_nests():
    # with a limit, batched measurement stops host work at the limit: the
    # product left on the CPU (gene bit 1; ~1 s of serial work) is cut inside
    # the submitted graph; the all-CPU gene of the medium application, whose
    # sweeps sit in the repeated block, takes its warm-up eagerly and ends
    # there -- both TIMEOUTs after about the limit, not after their full run
    import time
    doc = workloads.app_doc("medium")
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers()
    say("case batched deadline, medium all-CPU, all-GPU and CPU-product genes")
    cpu_gemm = [1] * 10
    cpu_gemm[1] = 0
    app.eval_population([[1] * 10], bufs, reps=1, warmup=0, flags=ofl.BATCHED)   # capture, warm
    t0 = time.perf_counter()
    t, s = app.eval_population([[0] * 10, [1] * 10, cpu_gemm], bufs, reps=3, warmup=1, flags=ofl.BATCHED,
                               deadline_s=0.05)
    wall = time.perf_counter() - t0
    assert list(s) == [ofl.ST_TIMEOUT, ofl.ST_OK, ofl.ST_TIMEOUT]
    assert t[0] == 0.05 and 0 < t[1] < 0.05 and t[2] == 0.05
    assert wall < 2.0, wall   # eight runs of ~1-1.5 s each without the cut
    # later runs are not limited: the all-CPU gene completes and matches the oracle
    o = ir.load(doc)
    o32, o64 = parity.oracle_outputs(o, 1)
    st = app.run_pattern([0] * 10, bufs, flags=ofl.GRAPH)
    assert st["status"] == ofl.ST_OK
    assert not parity.compare(o, app.read_all(), o32, o64, rel_gemm=parity.rel_gemm_for(o, ()))


def test_ga_timeout_and_progress_lines(capfd):
    # an absolute timeout below the all-CPU gene's time cuts that run off
    # (TIMEOUT, fitness 0); the progress flag prints one line per generation
    doc = workloads.app_doc("tiny")
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers()
    t0, s0 = app.eval_population([[0] * 6], bufs, reps=3, warmup=1)
    assert s0[0] == ofl.ST_OK
    tmo = float(t0[0]) / 4
    say("case GA tiny with timeout %.6f s and progress" % tmo)
    res = app.ga_run(ofl.ga_params(M=4, T=3, seed=1, reps=3, warmup=1, deadline_factor=2.0, timeout_s=tmo,
                                   flags=ofl.PROGRESS), bufs)
    err = capfd.readouterr().err
    lines = [ln for ln in err.splitlines() if ln.startswith("ga generation ")]
    assert [ln.split()[2].rstrip(":") for ln in lines] == ["1/3", "2/3", "3/3"]
    assert res["t_all0"] == -1.0            # the all-CPU baseline was cut off
    for g in range(res["n_generations"]):
        for t, st in zip(res["times"][g], res["status"][g]):
            assert st == ofl.ST_TIMEOUT or (st == ofl.ST_OK and t <= tmo)


# ---------------------------------------------------------------- graph runs
@pytest.mark.parametrize("name,params,genes", [
    ("tiny", {}, [[1] * 6, [0, 1, 0, 1, 1, 0], [1, 0, 1, 1, 0, 1]]),
    ("medium", workloads.SMALL_MEDIUM, [[1] * 10, [1, 0, 1, 1, 0, 1, 0, 1, 1, 0]]),
])
def test_graph_replays_match_oracle(name, params, genes):
    # every replay of a captured run is checked, with eager runs of other
    # genes and host synchronisation in between
    doc = workloads.app_doc(name, **params)
    app = ofl.App(json.dumps(doc), seed=2)
    o = ir.load(doc)
    o32, o64 = parity.oracle_outputs(o, 2)
    bufs = app.alloc_device_buffers()
    for g in genes:
        for flags in (ofl.GRAPH, ofl.GRAPH | ofl.PRESTAGED | ofl.KEEP_OUTPUTS):
            for rep in range(3):
                say("case graph", name, list(g), flags, rep)
                st = app.run_pattern(g, bufs, flags=flags)
                assert st["status"] == ofl.ST_OK
                assert (st["bytes_h2d"], st["bytes_d2h"], st["n_copies"]) == app.plan_transfers(g, 0, flags)
                bad = parity.compare(o, app.read_all(), o32, o64)
                assert not bad, (list(g), flags, rep, bad)
                other = [1 - b for b in g]
                app.run_pattern(other, bufs)                     # eager work in between
                bad = parity.compare(o, app.read_all(), o32, o64)
                assert not bad, ("eager", other, bad)


def test_eval_population_graph_mode():
    doc = workloads.app_doc("tiny")
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers()
    genes = [[1] * 6, [1] * 6, [0] * 6, [1, 1, 1, 0, 0, 0]]
    t, s = app.eval_population(genes, bufs, reps=3, warmup=1, flags=ofl.GRAPH)
    assert np.all(s == ofl.ST_OK) and np.all(t > 0)
    assert t[0] == t[1]          # duplicates measured once


def test_eval_population_batched_one_submission():
    # all 64 genes of the tiny application in one submission: every gene
    # measured, duplicates once, and afterwards the device / host state is
    # that of the last gene's run (its outputs match the oracle)
    doc = workloads.app_doc("tiny")
    app = ofl.App(json.dumps(doc))
    o = ir.load(doc)
    o32, o64 = parity.oracle_outputs(o, 1)
    bufs = app.alloc_device_buffers()
    genes = [[(idx >> i) & 1 for i in range(6)] for idx in range(64)] + [[1] * 6]
    say("case eval batched tiny 64")
    t, s = app.eval_population(genes, bufs, reps=3, warmup=1, flags=ofl.BATCHED)
    assert np.all(s == ofl.ST_OK) and np.all(t > 0)
    assert t[63] == t[64]
    assert t[0] > t[63]                       # the all-CPU gene is the slowest kind here
    bad = parity.compare(o, app.read_all(), o32, o64)
    assert not bad, bad
    # with a limit below the slowest genes: those become timeouts at the limit
    lim = float(np.median(t))
    t2, s2 = app.eval_population(genes[:64], bufs, reps=1, warmup=0, flags=ofl.BATCHED, deadline_s=lim)
    assert np.all((s2 == ofl.ST_OK) | (s2 == ofl.ST_TIMEOUT)) and np.any(s2 == ofl.ST_TIMEOUT)
    assert np.all(t2[s2 == ofl.ST_TIMEOUT] == lim)
    # a following eager run is unaffected
    st = app.run_pattern([1, 0, 1, 1, 0, 1], bufs)
    assert st["status"] == ofl.ST_OK
    assert not parity.compare(o, app.read_all(), o32, o64)


def test_ga_batched_generations_medium_reduced():
    doc = workloads.app_doc("medium", **workloads.SMALL_MEDIUM)
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers()
    params = ofl.ga_params(M=8, T=4, p=1.0, seed=5, reps=2, warmup=1, flags=ofl.BATCHED)
    say("case GA batched medium reduced")
    res = app.ga_run(params, bufs)
    assert res["n_generations"] == 4
    uniq = {tuple(int(x) for x in g) for gen in res["pops"] for g in gen}
    assert res["n_measured"] == len(uniq)
    assert np.all(res["status"] == ofl.ST_OK)
    assert res["best_time"] == float(np.min(res["times"]))


def test_ga_batched_generations_gene_by_gene_for_long_runs(monkeypatch):
    # the batched GA measures a generation gene by gene while no run measured
    # so far was faster than the threshold (here forced to 0 s: every
    # generation); the search keeps its batched semantics (one limit per
    # generation) and its results stay consistent
    monkeypatch.setenv("OFL_BATCH_EAGER_S", "0")
    doc = workloads.app_doc("medium", **workloads.SMALL_MEDIUM)
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers()
    params = ofl.ga_params(M=8, T=4, p=1.0, seed=5, reps=2, warmup=1, flags=ofl.BATCHED, deadline_factor=3.0)
    say("case GA batched medium reduced, gene by gene")
    res = app.ga_run(params, bufs)
    assert res["n_generations"] == 4
    # with a deadline the all-CPU gene is measured first, as the reference
    uniq = {tuple(int(x) for x in g) for gen in res["pops"] for g in gen} | {(0,) * app.gene_len}
    assert res["n_measured"] == len(uniq) and res["t_all0"] > 0
    ok = res["status"] == ofl.ST_OK
    assert np.any(ok) and np.all((res["status"] == ofl.ST_OK) | (res["status"] == ofl.ST_TIMEOUT))
    assert res["best_time"] == float(np.min(res["times"][ok]))
    o = ir.load(doc)
    o32, o64 = parity.oracle_outputs(o, 1)
    st = app.run_pattern([int(x) for x in res["best_gene"]], bufs)
    assert st["status"] == ofl.ST_OK
    assert not parity.compare(o, app.read_all(), o32, o64)


def test_kernel_timing_in_graph_replays():
    doc = workloads.app_doc("medium", **workloads.SMALL_MEDIUM)
    app = ofl.App(json.dumps(doc))
    o = ir.load(doc)
    o32, o64 = parity.oracle_outputs(o, 1)
    bufs = app.alloc_device_buffers()
    gene = [1] * app.gene_len
    app.set_kernel_timing(True)
    say("case graph replays with timing nodes")
    for _ in range(3):
        st = app.run_pattern(gene, bufs, flags=ofl.GRAPH | ofl.PRESTAGED)
        assert st["status"] == ofl.ST_OK
        assert not parity.compare(o, app.read_all(), o32, o64)
    n, ms = app.kernel_stats("stencil19")
    assert n == 3 * doc["params"]["SWEEPS"] and ms > 0
    n, ms = app.kernel_stats("gemm")
    assert n == 3 and ms > 0
    app.set_kernel_timing(False)
    app.run_pattern(gene, bufs, flags=ofl.GRAPH | ofl.PRESTAGED)
    assert not parity.compare(o, app.read_all(), o32, o64)


@pytest.mark.parametrize("name,params", [("medium", workloads.SMALL_MEDIUM), ("large", workloads.SMALL_LARGE)])
def test_sections_policy_random_genes(name, params):
    # the SECTIONS policy copies boxes (columns, rows, sub-blocks) out for the
    # CPU nests; every gene must still give the oracle's values, eager and as
    # graph replays
    doc = workloads.app_doc(name, **params)
    rng = random.Random(17)
    a = ofl.App(json.dumps(doc)).gene_len
    genes = [[1] * a] + [[rng.randint(0, 1) for _ in range(a)] for _ in range(5)]
    _run_and_compare(doc, genes, policies=(ofl.SECTIONS,),
                     flags_list=(0, ofl.PRESTAGED | ofl.KEEP_OUTPUTS, ofl.GRAPH | ofl.PRESTAGED))


@pytest.mark.parametrize("op,prec,form", [("gemm", "bf16x3", None), ("gemm", "bf16x3", "reg"), ("gemm", "fp8x2", None),
                                          ("gemm", "fp8x2", "reg"), ("gemm_bf16", None, None),
                                          ("gemm_bf16", None, "reg")])
def test_gemm_nt_256_tiles_ragged_sampled(op, prec, form, monkeypatch):
    # the 256 x 256 tiles (8 waves; chosen by size from 256 tiles up, forced
    # here; operands loaded straight into LDS unless form "reg");
    # ragged edges exercise the zero padding; sampled rows (and the ragged
    # last rows) against the oracle
    monkeypatch.setenv("OFL_GEMM_NT_TILE", "256")
    if form:
        monkeypatch.setenv("OFL_GEMM_NT_FORM", form)
    M, N, K = 2100, 2060, 300
    app = ofl.App(json.dumps(appgen.gemm_app(M, N, K, op=op, prec=prec)))
    A = OC.init_uniform(M * K, 31, 0).reshape(M, K)
    B = OC.init_uniform(K * N, 31, 1).reshape(K, N)
    if op == "gemm_bf16":
        A, B = OC.cast_bf16(A), OC.cast_bf16(B)
    app.set_input("A", A)
    app.set_input("B", B)
    bufs = app.alloc_device_buffers()
    say("case nt 256 tiles", op, prec)
    app.run_pattern([1], bufs, flags=ofl.KEEP_OUTPUTS)
    C = app.read_buffer("C").astype(np.float64)
    rows = np.array(sorted(set(list(np.random.default_rng(2).choice(M, 6, replace=False)) + [M - 1, M - 2, 0])))
    Ar = np.ascontiguousarray(A[rows])
    if op == "gemm_bf16":
        want = OC.gemm_bf16_f64(Ar, B)
        tol = parity.REL_GEMM
    else:
        want = OC.gemm_split_f64(Ar, B, prec)
        tol = parity.REL_GEMM if prec == "bf16x3" else parity.REL_FP8_MFMA
    err = np.max(np.abs(C[rows] - want) / want)
    assert err < tol, err


def test_precision_workload_error_report():
    # the precision configuration at full size under each GEMM form: max
    # relative error of each output against FP64 references -- C against the
    # exact product on sampled rows; the sweep field p and the residuals r_S
    # against the closed form of the sine mode (p_n = mu^n p_0,
    # r_n = (mu - 1)^2 mu^(2n-2) (I-1)(J-1)(K-1) / 8), which the sweep follows
    # exactly in exact arithmetic
    import torch
    doc0 = workloads.app_doc("precision")
    P = doc0["params"]
    N, I, J, K, S = P["N"], P["I"], P["J"], P["K"], P["SWEEPS"]
    rows = [line.split() for line in open(workloads.ROOT + "/tests/golden/stencil_eigen.txt")
            if not line.startswith("#")]
    mu = [float(r[4]) for r in rows if r[:4] == [str(I), str(J), str(K), "1"]][0]
    _, p0 = OC.sin_field(I, J, K, 1, want64=True)
    inner = (slice(1, -1),) * 3
    p_exact = mu ** S * p0[inner]
    n = np.arange(1, S + 1)
    r_exact = (mu - 1) ** 2 * mu ** (2 * n - 2) * (I - 1) * (J - 1) * (K - 1) / 8
    A = OC.init_uniform(N * N, 1, 0).reshape(N, N)
    B = OC.init_uniform(N * N, 1, 1).reshape(N, N)
    sample = np.random.default_rng(4).choice(N, 6, replace=False)
    exact_C = OC.gemm_f64(np.ascontiguousarray(A[sample]), B)
    report = {}
    for prec in ("f32", "bf16x3", "fp8x2"):
        doc = workloads.app_doc("precision")
        doc["program"][1]["args"]["prec"] = prec
        app = ofl.App(json.dumps(doc), seed=1)
        bufs = app.alloc_device_buffers()
        say("case precision workload", prec)
        app.run_pattern([1] * app.gene_len, bufs, policy=ofl.SECTIONS, flags=ofl.KEEP_OUTPUTS)
        C = app.read_buffer("C")[sample].astype(np.float64)
        p = app.read_buffer("p")[inner].astype(np.float64)
        r = app.read_buffer("res")
        report[prec] = {"C": float(np.max(np.abs(C - exact_C) / exact_C)),
                        "p": float(np.max(np.abs(p - p_exact)) / np.max(np.abs(p_exact))),
                        "r_S": float(np.max(np.abs(r - r_exact) / r_exact))}
        say("precision errors", prec, report[prec])
        del app, bufs
        torch.cuda.empty_cache()
    assert report["f32"]["C"] < 1e-5 and report["bf16x3"]["C"] < 1e-5 and report["fp8x2"]["C"] < 1e-3
    for prec in report:
        # the sweep does not depend on the product: the same field in every form
        assert report[prec]["p"] == report["f32"]["p"] and report[prec]["p"] < S * 8 * 2.0 ** -24
        assert report[prec]["r_S"] < 1e-2   # FP32 field: ~2^-24 / |mu - 1| relative (reported, not tight)


# ---------------------------------------------------------------- general C programs
def test_irregular_program_all_genes():
    # a C program with loops the library does not implement (index
    # arithmetic, a partial update, a math routine, double arithmetic, a
    # branch, an early exit): they run on the CPU from their own compiled
    # text, and every one of the 32 patterns of the other five nests must
    # give the serial run of the unmodified program (compiled by the oracle)
    import os
    from oracle import cprog
    from paper_1806_01430_amd import cfront
    path = os.path.join(workloads.ROOT, "paper_1806_01430_amd", "apps", "irregular.c")
    with open(path) as f:
        want = cprog.run_program(f.read())
    app = ofl.App(cfront.load(path))
    assert app.gene_len == 5
    bufs = app.alloc_device_buffers()
    Cw, Ew = want["C"].astype(np.float64), want["E"].astype(np.float64)
    # values downstream of the product: the GPU product is within 1e-5 of the
    # exact one and the serial FP32 product within N u = 1.2e-5 (positive
    # terms), so C, and what depends on it smoothly (E, G, T), differ by
    # < 3e-5 relative; F = |C - 8 E| by < 3e-5 (C + 8 E) absolute
    tol_f = 3e-5 * (Cw + 8.0 * Ew) + 1e-6
    for idx in range(32):
        g = [(idx >> k) & 1 for k in range(5)]
        for pol in (ofl.RESIDENT, ofl.SECTIONS):
            say("case irregular gene", g, "policy", pol)
            st = app.run_pattern(g, bufs, policy=pol)
            assert st["status"] == ofl.ST_OK
            assert (st["bytes_h2d"], st["bytes_d2h"], st["n_copies"]) == app.plan_transfers(g, pol, 0)
            got = app.read_all()
            for name in ("A", "r", "p", "q"):
                assert np.array_equal(got[name], want[name]), (g, name)
            assert np.max(np.abs(got["res"] - want["res"]) / want["res"]) <= 1e-12 + 17 * 19 * 65 * 2.0 ** -52
            for name in ("C", "E", "G", "T"):
                w = want[name].astype(np.float64)
                assert np.max(np.abs(got[name].astype(np.float64) - w) / w) < 3e-5, (g, name)
            if g[0] == 0:
                # the product on the CPU: the same serial code as the program
                # (the sum of squares too, unless the GPU adds it up in
                # another order)
                for name in ("C", "E", "G", "T", "F", "B") + (("s",) if g[4] == 0 else ()):
                    assert np.array_equal(got[name], want[name]), (g, name)
            assert np.all(np.abs(got["F"].astype(np.float64) - want["F"]) <= tol_f), g
            assert np.all(np.abs(got["B"].astype(np.float64) - want["B"]) <= tol_f.T), g
            assert abs(got["s"][0] - want["s"][0]) / want["s"][0] < 1e-4, g


# ---------------------------------------------------------------- output check
def test_output_check_against_the_all_cpu_run():
    # every pattern of the tiny application reproduces the all-CPU run's
    # outputs at the probes (the product within 1e-4 of each output's scale)
    doc = workloads.app_doc("tiny")
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers()
    genes = [[(idx >> i) & 1 for i in range(6)] for idx in range(64)]
    say("case output check, 64 genes eagerly")
    t, s = app.eval_population(genes, bufs, reps=1, warmup=1, verify_rtol=1e-4)
    assert np.all(s == ofl.ST_OK) and np.all(t > 0)
    say("case output check, 64 genes in one submission")
    t, s = app.eval_population(genes, bufs, reps=1, warmup=0, flags=ofl.BATCHED, verify_rtol=1e-4)
    assert np.all(s == ofl.ST_OK)
    say("case output check in the GA")
    res = app.ga_run(ofl.ga_params(M=6, T=3, seed=3, reps=1, warmup=0, verify_rtol=1e-4), bufs)
    assert np.all(res["status"] == ofl.ST_OK)
    # new inputs: the reference is taken again from them
    p0 = app.read_buffer("p")
    app.set_input("p", np.zeros_like(p0) + np.float32(0.5))
    st = app.run_pattern([1] * 6, bufs, verify_rtol=1e-4)
    assert st["status"] == ofl.ST_OK
    assert np.all(app.read_buffer("p") == np.float32(0.5))


def test_output_check_flags_a_less_accurate_product():
    # the FP8x2 product differs from the FP32 loop run on the CPU by ~1e-4 of
    # its scale: within a tolerance of 1e-3, beyond one of 1e-6 (a MISMATCH,
    # fitness 0); the all-CPU pattern always agrees with itself, and so does
    # every pattern that keeps the product (gene bit 1) on the CPU
    doc = workloads.app_doc("precision", N=160, I=13, J=17, K=67, SWEEPS=3)
    doc["program"][1]["args"]["prec"] = "fp8x2"
    app = ofl.App(json.dumps(doc))
    bufs = app.alloc_device_buffers()
    say("case output check fp8x2")
    assert app.run_pattern([1] * 4, bufs, verify_rtol=1e-3)["status"] == ofl.ST_OK
    st = app.run_pattern([1] * 4, bufs, verify_rtol=1e-6, check=False)
    assert st["rc"] == -11 and st["status"] == ofl.ST_MISMATCH
    assert "differs from the all-CPU run" in ofl.last_error()
    assert app.run_pattern([0] * 4, bufs, verify_rtol=1e-12)["status"] == ofl.ST_OK
    assert app.run_pattern([1, 0, 1, 1], bufs, verify_rtol=1e-9)["status"] == ofl.ST_OK
    t, s = app.eval_population([[1] * 4, [0] * 4, [1, 0, 1, 1]], bufs, reps=1, warmup=0, verify_rtol=1e-6)
    assert list(s) == [ofl.ST_MISMATCH, ofl.ST_OK, ofl.ST_OK]
    res = app.ga_run(ofl.ga_params(M=4, T=2, seed=5, reps=1, warmup=0, verify_rtol=1e-6), bufs)
    for gen_pop, gen_st in zip(res["pops"], res["status"]):
        for g, st_ in zip(gen_pop, gen_st):
            assert st_ == (ofl.ST_MISMATCH if g[1] == 1 else ofl.ST_OK), (list(g), st_)


# ---------------------------------------------------------------- concurrent components
@pytest.mark.parametrize("name,params", [("large", workloads.SMALL_LARGE), ("medium", workloads.SMALL_MEDIUM)])
def test_components_concurrent_match_oracle(name, params):
    # OFL_RUN_CONCURRENT: the matrix nests and the grid nests share no buffer
    # and run at once, each part on its own stream and host thread; results,
    # copies and byte counts are those of the sequential run, for genes that
    # leave nests of either part (and both parts' host nests) on the CPU
    doc = workloads.app_doc(name, **params)
    app = ofl.App(json.dumps(doc), seed=1)
    a = app.gene_len
    rng = random.Random(11)
    genes = [[1] * a, [0] * a] + [[rng.randint(0, 1) for _ in range(a)] for _ in range(4)]
    o = ir.load(doc)
    o32, o64 = parity.oracle_outputs(o, 1)
    bufs = app.alloc_device_buffers()
    for pol in (ofl.SECTIONS, ofl.RESIDENT):
        for fl in (ofl.CONCURRENT, ofl.CONCURRENT | ofl.PRESTAGED | ofl.KEEP_OUTPUTS):
            for g in genes:
                say("case concurrent", name, "gene", g, "policy", pol, "flags", fl)
                st = app.run_pattern(g, bufs, policy=pol, flags=fl)
                assert st["status"] == ofl.ST_OK
                assert (st["bytes_h2d"], st["bytes_d2h"], st["n_copies"]) == app.plan_transfers(g, pol, fl)
                bad = parity.compare(o, app.read_all(), o32, o64)
                assert not bad, (g, pol, fl, bad)
    # kernel timing across both streams: every sweep and product timed
    app.set_kernel_timing(True)
    app.run_pattern([1] * a, bufs, policy=ofl.SECTIONS, flags=ofl.CONCURRENT)
    app.set_kernel_timing(False)
    assert app.kernel_stats("stencil19")[0] == doc["params"]["SWEEPS"]
    assert app.kernel_stats("gemm")[0] >= 1
    # a deadline cuts the concurrent run (the all-CPU gene takes far longer)
    st = app.run_pattern([0] * a, bufs, flags=ofl.CONCURRENT, deadline_s=1e-6, check=False)
    assert st["status"] == ofl.ST_TIMEOUT


# ---------------------------------------------------------------- the sweep as a call
@pytest.mark.parametrize("I,J,K", [(3, 3, 3), (5, 7, 9), (33, 33, 65), (19, 23, 71), (130, 40, 260)])
def test_sweep19_call_matches_oracle(I, J, K):
    import torch
    say("case sweep19 call", I, J, K)
    rng = np.random.default_rng(I * 1000 + K)
    p0 = rng.random((I, J, K), dtype=np.float32)
    q0 = rng.random((I, J, K), dtype=np.float32)
    p = torch.from_numpy(p0).cuda()
    q = torch.from_numpy(q0).cuda()
    res = torch.zeros(3, dtype=torch.float64, device="cuda")
    res[1] = 0.25
    for _ in range(2):
        ofl.sweep19(p, q, res, slot=1)
    torch.cuda.synchronize()
    want_q = q0.copy()
    cell = np.array([0.25])
    for _ in range(2):
        OC.stencil19(p0, want_q, cell)
    assert np.array_equal(q.cpu().numpy(), want_q)
    assert np.array_equal(p.cpu().numpy(), p0)
    got = res.cpu().numpy()
    assert got[0] == 0.0 and got[2] == 0.0
    n = max(1, (I - 2) * (J - 2) * (K - 2))
    assert abs(got[1] - cell[0]) <= (1e-12 + 2 * n * 2.0 ** -52) * cell[0]
    with pytest.raises(ofl.OflError):
        ofl.sweep19(p, p, res)
