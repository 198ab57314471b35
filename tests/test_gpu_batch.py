"""Instance batches on the GPU vs the oracle, through the C ABI (needs an
MI355X): every instance of a batch, run by grouped launches (eager and as a
captured graph) or by per-instance launches, must give what the oracle gives
for that instance alone under the all-GPU gene (tests/parity.py bar)."""
import sys

import numpy as np
import pytest

import paper_1806_01430_amd as ofl
import workloads
from oracle import ir

import parity

pytestmark = pytest.mark.gpu

MODES = {"loop": ofl.BATCH_LOOP, "grouped": ofl.BATCH_GROUPED, "graph": ofl.BATCH_GROUPED_GRAPH}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    yield


def _small_batch():
    # uneven, ragged sizes: orders off every tile multiple, grids from the
    # smallest of the recipe up, one instance with N % 4 == 0 (vector loads)
    params = [{"N": n, "I": i, "J": j, "K": k, "SWEEPS": 3}
              for n, i, j, k in [(33, 17, 17, 33), (64, 20, 18, 39), (100, 17, 21, 65), (17, 25, 25, 49),
                                 (130, 19, 17, 127), (47, 30, 22, 45), (200, 18, 18, 35), (5, 17, 19, 130)]]
    seeds = [11 + 7 * t for t in range(len(params))]
    return params, seeds


_ORACLE = {}


def _oracle(params, seed):
    key = (tuple(sorted(params.items())), seed)
    if key not in _ORACLE:
        doc = workloads.app_doc("batch", **params)
        o = ir.load(doc)
        _ORACLE[key] = (o, parity.oracle_outputs(o, seed))
    return _ORACLE[key]


def _check_instances(b, bufs, params, seeds, which=None):
    for i in (range(len(params)) if which is None else which):
        o, (o32, o64) = _oracle(params[i], seeds[i])
        got = {name: b.read(bufs, i, name) for name in b.buf_names}
        bad = parity.compare(o, got, o32, o64)
        assert not bad, (i, params[i], bad)


@pytest.mark.parametrize("mode", ["loop", "grouped", "graph"])
def test_batch_small_matches_oracle(mode):
    params, seeds = _small_batch()
    b = ofl.Batch(workloads.app_doc("batch"), params, seeds)
    bufs = b.alloc_device_buffers()
    for rep in range(2):
        say("case batch small", mode, "rep", rep)
        b.setup(bufs)
        st = b.run(bufs, MODES[mode])
        assert st["status"] == ofl.ST_OK
        if mode == "graph":
            assert st["n_submissions"] == 1
        _check_instances(b, bufs, params, seeds)


@pytest.mark.parametrize("cfg", [dict(gemm_cfg=0, stencil_rows=2, stencil_planes=8),
                                 dict(gemm_cfg=2, gemm_blocks_per_cu=1, stencil_rows=8, stencil_planes=5),
                                 dict(gemm_cfg=3, stencil_rows=4, stencil_planes=32, stencil_blocks_per_cu=1),
                                 dict(gemm_cfg=4, gemm_blocks_per_cu=8, stencil_rows=8, stencil_planes=1),
                                 dict(gemm_cfg=5, gemm_blocks_per_cu=1, stencil_rows=2, stencil_planes=16),
                                 dict(gemm_cfg=6, gemm_blocks_per_cu=1, stencil_rows=4, stencil_planes=8),
                                 dict(gemm_cfg=7, gemm_blocks_per_cu=1, stencil_rows=4, stencil_planes=8)])
def test_batch_configs_match_oracle(cfg):
    params, seeds = _small_batch()
    b = ofl.Batch(workloads.app_doc("batch"), params, seeds)
    b.set_config(**cfg)
    bufs = b.alloc_device_buffers()
    say("case batch config", cfg)
    b.setup(bufs)
    b.run(bufs, ofl.BATCH_GROUPED_GRAPH)
    _check_instances(b, bufs, params, seeds)


def test_batch_graph_replays_with_eager_work_between():
    import torch
    params, seeds = _small_batch()
    b = ofl.Batch(workloads.app_doc("batch"), params, seeds)
    bufs = b.alloc_device_buffers()
    for rep in range(3):
        say("case batch graph replay", rep)
        b.setup(bufs)
        x = torch.ones(1 << 20, device="cuda")
        (x * 3.0).sum().item()                     # unrelated eager work on the stream
        b.run(bufs, ofl.BATCH_GROUPED_GRAPH)
        _check_instances(b, bufs, params, seeds, which=[0, 3, 6])


def test_batch_tune_then_match_oracle():
    params, seeds = _small_batch()
    b = ofl.Batch(workloads.app_doc("batch"), params, seeds)
    bufs = b.alloc_device_buffers()
    say("case batch tune")
    entries = b.tune(bufs, reps=2)
    assert any(e["phase"] == "gemm" for e in entries) and any(e["phase"] == "stencil" for e in entries)
    best_g = min((e for e in entries if e["phase"] == "gemm"), key=lambda e: e["ms"])
    c = b.config
    assert (c["gemm_cfg"], c["gemm_blocks_per_cu"]) == (best_g["gemm_cfg"], best_g["gemm_blocks_per_cu"])
    b.setup(bufs)
    b.run(bufs, ofl.BATCH_GROUPED_GRAPH)
    _check_instances(b, bufs, params, seeds)


def test_batch_full_recipe_sampled():
    # the batching configuration at full size (256 instances): grouped graph
    # vs per-instance launches for every instance (sweep field bit-identical,
    # products within the FP32 product tolerance of each other through the
    # oracle's FP64 twin on sampled instances), and sampled instances vs the
    # oracle
    params, seeds = workloads.batch_instances(256, seed=1)
    for p in params:
        p["SWEEPS"] = 10
    b = ofl.Batch(workloads.app_doc("batch"), params, seeds)
    bufs = b.alloc_device_buffers()
    say("case batch 256 grouped graph")
    b.setup(bufs)
    b.run(bufs, ofl.BATCH_GROUPED_GRAPH)
    fields = [b.read(bufs, i, "p") for i in range(256)]
    res = [b.read(bufs, i, "res") for i in range(256)]
    say("case batch 256 loop")
    b.setup(bufs)
    b.run(bufs, ofl.BATCH_LOOP)
    for i in range(256):
        assert np.array_equal(fields[i], b.read(bufs, i, "p")), i
        r2 = b.read(bufs, i, "res")
        n = (params[i]["I"] - 2) * (params[i]["J"] - 2) * (params[i]["K"] - 2)
        assert np.all(np.abs(res[i] - r2) <= 2 * (parity.REL_SUM + n * 2.0 ** -52) * np.abs(r2)), i
    b.setup(bufs)
    b.run(bufs, ofl.BATCH_GROUPED_GRAPH)
    pick = sorted(set([0, 255] + list(np.random.default_rng(0).choice(256, 4, replace=False))))
    say("case batch 256 oracle sample", pick)
    _check_instances(b, bufs, params, seeds, which=pick)
