"""The no-allocation sweep call (ofl_sweep19_noalloc) against ofl_sweep19
(needs an MI355X): identical grids and residual bits on two calls in a row,
the second on a smaller grid, so that the second call runs over the first
one's partials left in the library's fixed scratch."""
import sys

import numpy as np
import pytest

import paper_1806_01430_amd as ofl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pair(shape, seed):
    import torch
    rng = np.random.default_rng(seed)
    p0 = rng.random(shape, dtype=np.float32)
    q0 = rng.random(shape, dtype=np.float32)
    return [(torch.from_numpy(p0).cuda(), torch.from_numpy(q0).cuda()) for _ in range(2)]


def test_sweep19_noalloc_matches_sweep19():
    import torch
    assert torch.cuda.is_available()
    res = torch.zeros((2, 4), dtype=torch.float64, device="cuda")
    # the second grid is smaller than the first (fewer waves, fewer partials)
    for call, (shape, sweeps) in enumerate((((130, 40, 260), 2), ((19, 23, 71), 3))):
        say("case sweep19_noalloc call", call, shape)
        (p_a, q_a), (p_b, q_b) = _pair(shape, 100 + call)
        for _ in range(sweeps):
            ofl.sweep19(p_a, q_a, res[0], slot=call)
            ofl.sweep19(p_b, q_b, res[1], slot=call, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(q_a.view(torch.int32), q_b.view(torch.int32))
        assert torch.equal(p_a.view(torch.int32), p_b.view(torch.int32))
        r = res.cpu().numpy()
        assert r[0, call] > 0 and r[0, call].tobytes() == r[1, call].tobytes(), (r[0, call], r[1, call])


def test_sweep19_noalloc_full_size_grid():
    # the large application's grid (513 x 513 x 1025), the size the sweep is
    # benchmarked at: one sweep each way, same bits
    import torch
    shape = (513, 513, 1025)
    say("case sweep19_noalloc", shape)
    (p_a, q_a), (p_b, q_b) = _pair(shape, 7)
    res = torch.zeros(2, dtype=torch.float64, device="cuda")
    ofl.sweep19(p_a, q_a, res, slot=0)
    ofl.sweep19(p_b, q_b, res, slot=1, noalloc=True)
    torch.cuda.synchronize()
    assert torch.equal(q_a.view(torch.int32), q_b.view(torch.int32))
    r = res.cpu().numpy()
    assert r[0] > 0 and r[0].tobytes() == r[1].tobytes()
    del p_a, q_a, p_b, q_b
    torch.cuda.empty_cache()


def test_sweep19_noalloc_rejects_bad_arguments():
    import torch
    p = torch.zeros((5, 6, 7), dtype=torch.float32, device="cuda")
    res = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(ofl.OflError):
        ofl.sweep19(p, p, res, noalloc=True)
