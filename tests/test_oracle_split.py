"""Pins of the oracle's split-precision GEMM (hi/lo split with one refinement
pass, bf16 and OCP e4m3 with power-of-two scales) against facts that come
from the number formats' definitions and from error analysis, not from the
oracle itself."""
import numpy as np
import pytest

from oracle import cnests as C

U_BF16 = 2.0 ** -8     # unit roundoff of an 8-bit significand
U_E4M3 = 2.0 ** -4     # unit roundoff of a 4-bit significand
SUB_E4M3 = 2.0 ** -9   # spacing of e4m3 subnormals


# ------------------------------------------------------------ e4m3 format
def test_e4m3_published_code_points():
    # OCP 8-bit floating point specification, E4M3: max 448, min normal 2^-6,
    # min subnormal 2^-9, 1.0 = 0 0111 000, NaN = S 1111 111
    assert C.e4m3_value(0x7E) == 448.0
    assert C.e4m3_value(0x08) == 2.0 ** -6
    assert C.e4m3_value(0x01) == 2.0 ** -9
    assert C.e4m3_value(0x38) == 1.0
    assert C.e4m3_value(0xB8) == -1.0
    assert np.isnan(C.e4m3_value(0x7F)) and np.isnan(C.e4m3_value(0xFF))
    assert C.e4m3_value(0x00) == 0.0


def _table():
    return np.array([C.e4m3_value(c) for c in range(127)])


def test_e4m3_code_table_structure():
    v = _table()
    assert np.all(np.diff(v) > 0)                      # monotone in the code
    d = np.diff(v)
    assert np.all(d[:8] == SUB_E4M3)                   # subnormals and the first normal binade
    for e in range(1, 15):                             # constant spacing per binade, doubling
        assert np.all(d[8 * e:8 * e + 7] == 2.0 ** (e - 10)), e


def test_e4m3_round_to_nearest_even_brute_force():
    v = _table()
    rng = np.random.default_rng(5)
    xs = list(rng.uniform(0, 448, 3000)) + list(np.exp(rng.uniform(np.log(1e-5), np.log(448), 3000)))
    xs += list((v[1:] + v[:-1]) / 2)                   # every tie
    xs += list(v) + [2.0 ** -10, 3 * 2.0 ** -11]
    for x in xs:
        dist = np.abs(v - x)
        best = np.flatnonzero(dist == dist.min())
        want = best[0] if len(best) == 1 else [c for c in best if c % 2 == 0][0]
        got = C.e4m3_rne(x)
        assert got == want, (x, got, want)
        assert C.e4m3_rne(-x) == (want | 0x80 if want else (0x80 if -x == 0 or np.signbit(-x) else 0)), x


def test_e4m3_scale_is_largest_power_of_two_within_224():
    rng = np.random.default_rng(6)
    amaxes = list(np.exp(rng.uniform(np.log(1e-20), np.log(1e20), 500))) + [7.0, 224.0, 1.75, 1.76, 1.0, 448.0]
    for a in amaxes:
        cands = [2.0 ** e for e in range(-126, 127) if a * 2.0 ** e <= 224.0]
        assert C.e4m3_scale(a) == max(cands), a
    assert C.e4m3_scale(0.0) == 1.0 and C.e4m3_scale(float("inf")) == 1.0


# ------------------------------------------------------------ split product
@pytest.mark.parametrize("prec", ["bf16x3", "fp8x2"])
def test_split_rank1_integers_exact(prec):
    # A[i][k] = (i mod 7) + 1, B[k][j] = (j mod 5) + 1: every value is exact in
    # both narrow formats (lo parts vanish), so C = K u_i v_j exactly
    M, N, K = 37, 29, 211
    u = np.array([(i % 7) + 1 for i in range(M)], np.float32)
    v = np.array([(j % 5) + 1 for j in range(N)], np.float32)
    A = np.repeat(u[:, None], K, 1)
    B = np.repeat(v[None, :], K, 0)
    assert np.array_equal(C.gemm_split_f64(A, B, prec), K * np.outer(u, v).astype(np.float64))


def test_split_identity_bf16_measures_split_error():
    # I * B = hi(B) + lo(B): within u^2 of B, and strictly better than hi alone
    rng = np.random.default_rng(7)
    N = 96
    B = rng.standard_normal((N, N)).astype(np.float32)
    got = C.gemm_split_f64(np.eye(N, dtype=np.float32), B, "bf16x3")
    b = B.astype(np.float64)
    assert np.all(np.abs(got - b) <= U_BF16 ** 2 * np.abs(b))
    assert np.max(np.abs(got - b) / np.abs(b)) > 0     # bf16x3 does not reproduce FP32 exactly


def _bound(A, B, u, sub_a=None, sub_b=None):
    """Element-wise bound on |split product - A B| for one refinement pass.

    With x = hi + lo + e, |e| <= d_x and |lo| <= l_x, each term's error is
    e_a b + a e_b - e_a e_b + lo_a lo_b, so
    |err_ij| <= sum_k d_a|b| + |a|d_b + d_a d_b + l_a l_b,
    d_x = u^2 |x| + t_x,  l_x = (1 + u)(u |x| + t_x),
    where t_x = half a subnormal spacing divided by the scale (0 for bf16)."""
    a, b = np.abs(A.astype(np.float64)), np.abs(B.astype(np.float64))
    ta = np.zeros((A.shape[0], 1)) if sub_a is None else sub_a[:, None]
    tb = np.zeros((1, B.shape[1])) if sub_b is None else sub_b[None, :]
    da, db = u * u * a + ta, u * u * b + tb
    la, lb = (1 + u) * (u * a + ta), (1 + u) * (u * b + tb)
    K = A.shape[1]
    fp64 = 3 * K * 2.0 ** -52 * (a @ b)               # the oracle's own FP64 sum
    return da @ b + a @ db + da @ db + la @ lb + fp64


@pytest.mark.parametrize("dist", ["uniform", "signed_wide"])
def test_split_bf16x3_error_bound(dist):
    rng = np.random.default_rng(8)
    M, K, N = 40, 300, 33
    if dist == "uniform":
        A, B = rng.random((M, K), np.float32), rng.random((K, N), np.float32)
    else:
        A = (rng.standard_normal((M, K)) * np.exp(rng.uniform(-8, 8, (M, K)))).astype(np.float32)
        B = (rng.standard_normal((K, N)) * np.exp(rng.uniform(-8, 8, (K, N)))).astype(np.float32)
    got = C.gemm_split_f64(A, B, "bf16x3")
    exact = A.astype(np.float64) @ B.astype(np.float64)
    assert np.all(np.abs(got - exact) <= _bound(A, B, U_BF16))


@pytest.mark.parametrize("dist", ["uniform", "signed_wide"])
def test_split_fp8x2_error_bound(dist):
    rng = np.random.default_rng(9)
    M, K, N = 40, 300, 33
    if dist == "uniform":
        A, B = rng.random((M, K), np.float32), rng.random((K, N), np.float32)
    else:   # wide dynamic range inside a row: many elements land on subnormals
        A = (rng.standard_normal((M, K)) * np.exp(rng.uniform(-6, 6, (M, K)))).astype(np.float32)
        B = (rng.standard_normal((K, N)) * np.exp(rng.uniform(-6, 6, (K, N)))).astype(np.float32)
    got = C.gemm_split_f64(A, B, "fp8x2")
    exact = A.astype(np.float64) @ B.astype(np.float64)
    sa = np.array([C.e4m3_scale(x) for x in np.max(np.abs(A), 1)])
    sb = np.array([C.e4m3_scale(x) for x in np.max(np.abs(B), 0)])
    half_sub = SUB_E4M3 / 2
    assert np.all(np.abs(got - exact) <= _bound(A, B, U_E4M3, half_sub / sa, half_sub / sb))
    # and the refinement pass is doing its job: far below one e4m3 rounding
    rel = np.abs(got - exact) / (np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64)))
    assert np.max(rel) < U_E4M3 / 4
