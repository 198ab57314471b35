"""Pins of the compiled-program oracle (oracle/cprog.py): the serial run of
a whole C program, the reference for applications with loops the library
does not implement.  Each result is checked against what the C semantics
fix independently: closed forms evaluated with numpy in the same IEEE
precision (bit for bit), the exact product within the serial FP32 bound, the
sweep against the oracle's own C nest and the sine mode's closed form, and
the bf16 rounding against torch."""
import os

import numpy as np
import torch

from oracle import cnests, cprog

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
IRREGULAR = os.path.join(ROOT, "paper_1806_01430_amd", "apps", "irregular.c")


def _irregular():
    with open(IRREGULAR) as f:
        return f.read()


def test_index_arithmetic_math_routine_double_and_branch_closed_forms():
    out = cprog.run_program(_irregular())
    N, H = 200, 72
    i, j = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    f32 = np.float32
    A = ((i * 37 + j * 11) % 101).astype(f32) * f32(0.01) + f32(0.05)
    B0 = ((i * 13 + j * 29) % 97).astype(f32) * f32(0.01)
    assert np.array_equal(out["A"], A)
    # the product: within the serial FP32 bound of the exact one (all terms
    # are positive, so N u relative)
    exact = A.astype(np.float64) @ B0.astype(np.float64)
    C = out["C"].astype(np.float64)
    Cp = exact.copy()
    Cp[:H] += 0.5 * A[:H].astype(np.float64)
    assert np.max(np.abs(C - Cp) / Cp) <= (N + 2) * 2.0 ** -24
    # the partial update touched only the first H rows: the others are the
    # plain product
    Cf = out["C"]
    E = np.sqrt(Cf) + f32(1.0)
    assert np.array_equal(out["E"], E)
    G = 0.1 * E.astype(np.float64) + Cf.astype(np.float64)
    assert np.array_equal(out["G"], G)
    assert np.array_equal(out["T"], G.T)
    x = Cf - f32(8.0) * E
    F = np.where(x < 0, -x, x)
    assert np.array_equal(out["F"], F)
    assert np.array_equal(out["B"], F.T)
    s = 0.0
    for v in out["B"].reshape(-1).astype(np.float64):
        s += v * v
    assert out["s"][0] == s
    # the loop that leaves early: r[i] written up to the first diagonal
    # value above 0.95, zero after
    d = np.diagonal(A)
    stop = int(np.argmax(d > f32(0.95)))
    assert 0 < stop < N
    want = np.zeros(N, f32)
    want[:stop] = f32(2.0) * d[:stop] + f32(1.0)
    assert np.array_equal(out["r"], want)


def test_sweep_equals_the_oracle_nest_and_the_closed_form():
    out = cprog.run_program(_irregular())
    I, J, K, S = 21, 19, 67, 4
    p = cnests.sin_field(I, J, K, 1)
    q = np.zeros_like(p)
    res = np.zeros(S)
    for n in range(S):
        cell = res[n:n + 1]
        cnests.stencil19(p, q, cell)
        res[n] = cell[0]
        cnests.copy_interior(p, q)
    assert np.array_equal(out["p"], p) and np.array_equal(out["q"], q)
    assert np.array_equal(out["res"], res)
    # the sine mode decays by mu per sweep (the 19-point weights 1/4, 1/16,
    # 1/32): r_1 = (mu - 1)^2 (I-1)(J-1)(K-1) / 8 up to FP32 rounding
    c = [np.cos(np.pi / (d - 1)) for d in (I, J, K)]
    mu = 0.25 + sum(c) / 8 + (c[0] * c[1] + c[1] * c[2] + c[2] * c[0]) / 8
    r1 = (mu - 1) ** 2 * (I - 1) * (J - 1) * (K - 1) / 8
    assert abs(out["res"][0] - r1) / r1 < 1e-2


def test_bf16_rounding_matches_torch():
    src = """#define N 4096
float X[N];
bf16 Y[N];
float Z[N];
for (int e = 0; e < N; e++) X[e] = (float)(e * 7919 % 4096) * 0.000977f - 2.0f + (float)e * 0.0001f;
for (int e = 0; e < N; e++) Y[e] = bf16(X[e]);
for (int e = 0; e < N; e++) Z[e] = Y[e] * 3.0f;
"""
    out = cprog.run_program(src)
    want = torch.from_numpy(out["X"]).to(torch.bfloat16)
    assert np.array_equal(out["Y"], want.view(torch.int16).numpy().view(np.uint16))
    assert np.array_equal(out["Z"], want.float().numpy() * np.float32(3.0))
