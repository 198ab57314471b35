"""Pins of the FFT function block's oracle (the DFT by its definition):
closed forms that catch a wrong sign of the exponent, swapped real and
imaginary parts or a transposed index, Parseval's identity, the shift
theorem, and the library FFT (numpy.fft) as an independent special case;
for the inverse call also its 1/n scale and the round trip; for the real
call the packing of bins 0 and n/2 and the library's numpy.fft.rfft."""
import numpy as np
import pytest

from oracle.dft import dft_rows, idft_rows, irdft_packed_rows, rdft_packed_rows

import parity


def _interleave(z):
    z = np.atleast_2d(z)
    out = np.empty((z.shape[0], 2 * z.shape[1]))
    out[:, 0::2] = z.real
    out[:, 1::2] = z.imag
    return out


def _complex(x):
    return x[:, 0::2] + 1j * x[:, 1::2]


@pytest.mark.parametrize("n", [1, 2, 4, 8, 64, 1024])
def test_delta_gives_ones(n):
    z = np.zeros(n, complex)
    z[0] = 1
    assert np.array_equal(_complex(dft_rows(_interleave(z))), np.ones((1, n), complex))


@pytest.mark.parametrize("n", [4, 16, 256])
def test_tone_lands_in_its_bin(n):
    j = np.arange(n)
    for m in (1, 3 % n, n // 2, n - 1):
        z = np.exp(2j * np.pi * m * j / n)        # exp(+2 pi i m j / n)
        Z = _complex(dft_rows(_interleave(z)))[0]
        want = np.zeros(n, complex)
        want[m] = n                               # forward transform: peak at +m, not n - m
        assert np.max(np.abs(Z - want)) < 1e-9 * n, (n, m)


def test_imaginary_delta_and_constant():
    n = 4
    z = np.zeros(n, complex)
    z[1] = 1j                                      # x = i delta_1: X[k] = i exp(-2 pi i k / 4) = i (-i)^k
    Z = _complex(dft_rows(_interleave(z)))[0]
    assert np.allclose(Z, [1j, 1, -1j, -1], atol=1e-15)
    c = 0.75 - 2.5j
    Z = _complex(dft_rows(_interleave(np.full(8, c))))[0]
    assert abs(Z[0] - 8 * c) < 1e-13 and np.max(np.abs(Z[1:])) < 1e-13
    # n = 2: sum and difference; n = 1: identity
    Z = _complex(dft_rows(_interleave(np.array([2 + 1j, -3 + 0.5j]))))[0]
    assert np.allclose(Z, [-1 + 1.5j, 5 + 0.5j], rtol=0, atol=1e-15)
    assert np.array_equal(dft_rows(np.array([[1.5, -2.0]])), [[1.5, -2.0]])


def test_parseval_shift_and_library_fft():
    rng = np.random.default_rng(4)
    for n in (2, 8, 128, 512):
        z = rng.standard_normal((5, n)) + 1j * rng.standard_normal((5, n))
        Z = _complex(dft_rows(_interleave(z)))
        assert np.allclose(np.sum(np.abs(Z) ** 2, axis=1), n * np.sum(np.abs(z) ** 2, axis=1), rtol=1e-12)
        ref = np.fft.fft(z, axis=1)
        assert np.max(np.linalg.norm(Z - ref, axis=1) / np.linalg.norm(ref, axis=1)) < 1e-12
        s = 3 % n                                  # circular shift by s multiplies bin k by exp(-2 pi i k s / n)
        Zs = _complex(dft_rows(_interleave(np.roll(z, s, axis=1))))
        k = np.arange(n)
        assert np.allclose(Zs, Z * np.exp(-2j * np.pi * k * s / n), atol=1e-9 * n)


def test_fft_bound_values():
    # the parity bound grows with log2 n and stays at a few u per pass
    u = 2.0 ** -24
    assert parity.rel_fft(1) == 0.0
    assert 6.6 * u < parity.rel_fft(2) < 6.7 * u
    assert 11 * 6.6 * u < parity.rel_fft(2048) < 11 * 6.7 * u
    # a plain FP32 radix-2 FFT (numpy in float32 arithmetic, exact twiddles
    # rounded once) stays inside it
    rng = np.random.default_rng(9)
    for n in (8, 256, 2048):
        z = (rng.standard_normal((4, n)) + 1j * rng.standard_normal((4, n))).astype(np.complex64)
        y = z.copy()
        w = np.exp(-2j * np.pi * np.arange(n // 2) / n).astype(np.complex64)
        ns = 1
        while ns < n:
            j = np.arange(n // 2)
            k = j % ns
            a, b = y[:, j], y[:, j + n // 2] * w[k * (n // (2 * ns))]
            out = np.empty_like(y)
            o = (j - k) * 2 + k
            out[:, o] = a + b
            out[:, o + ns] = a - b
            y, ns = out, ns * 2
        ref = _complex(dft_rows(_interleave(z.astype(complex))))
        err = np.max(np.linalg.norm(y - ref, axis=1) / np.linalg.norm(ref, axis=1))
        assert err < parity.rel_fft(n), (n, err)


@pytest.mark.parametrize("n", [1, 2, 4, 8, 64, 1024])
def test_inverse_of_delta_is_the_scaled_constant(n):
    # x = delta_0: every output 1/n exactly (a power of two); a missing or
    # doubled scale, or the forward transform, would give 1 or n
    z = np.zeros(n, complex)
    z[0] = 1
    assert np.array_equal(_complex(idft_rows(_interleave(z))), np.full((1, n), 1.0 / n, complex))


@pytest.mark.parametrize("n", [4, 16, 256])
def test_inverse_tone_lands_in_the_mirrored_bin(n):
    j = np.arange(n)
    for m in (1, 3 % n, n // 2, n - 1):
        z = np.exp(2j * np.pi * m * j / n)        # exp(+2 pi i m j / n)
        x = _complex(idft_rows(_interleave(z)))[0]
        want = np.zeros(n, complex)
        want[(n - m) % n] = 1                     # inverse: exp(+...) pairs with bin -m, value 1 (scaled by 1/n)
        assert np.max(np.abs(x - want)) < 1e-12, (n, m)


def test_inverse_round_trip_and_library_ifft():
    rng = np.random.default_rng(6)
    for n in (1, 2, 8, 128, 512):
        z = rng.standard_normal((5, n)) + 1j * rng.standard_normal((5, n))
        back = _complex(idft_rows(dft_rows(_interleave(z))))
        assert np.max(np.abs(back - z)) < 1e-12 * max(1, n)
        x = _complex(idft_rows(_interleave(z)))
        ref = np.fft.ifft(z, axis=1)
        assert np.max(np.linalg.norm(x - ref, axis=1) / np.linalg.norm(ref, axis=1)) < 1e-12
    # n = 2 by hand: ((a + b) / 2, (a - b) / 2)
    x = _complex(idft_rows(_interleave(np.array([2 + 1j, -3 + 0.5j]))))[0]
    assert np.allclose(x, [-0.5 + 0.75j, 2.5 + 0.25j], rtol=0, atol=1e-15)


@pytest.mark.parametrize("n", [2, 4, 8, 64, 1024])
def test_real_delta_and_constant(n):
    # delta_0: every bin 1 (packed: X0, X(n/2), then (1, 0) pairs); a
    # constant c: only X0 = n c
    x = np.zeros((1, n))
    x[0, 0] = 1
    want = np.zeros(n)
    want[0] = want[1] = 1
    want[2::2] = 1
    assert np.array_equal(rdft_packed_rows(x)[0], want)
    y = rdft_packed_rows(np.full((1, n), -0.75))[0]
    assert y[0] == -0.75 * n and np.max(np.abs(y[1:])) < 1e-12 * n


@pytest.mark.parametrize("n", [4, 16, 256])
def test_real_tones_land_in_their_packed_slots(n):
    j = np.arange(n)
    for m in range(1, n // 2):
        for f, slot in ((np.cos, 2 * m), (np.sin, 2 * m + 1)):
            y = rdft_packed_rows(f(2 * np.pi * m * j / n)[None, :])[0]
            want = np.zeros(n)
            want[slot] = n / 2 if f is np.cos else -n / 2   # sin: X[m] = -i n/2
            assert np.max(np.abs(y - want)) < 1e-9 * n, (n, m, f.__name__)
    alt = rdft_packed_rows(((-1.0) ** j)[None, :])[0]      # X[n/2] = n, packed second
    want = np.zeros(n)
    want[1] = n
    assert np.max(np.abs(alt - want)) < 1e-9 * n


def test_real_matches_complex_and_library():
    rng = np.random.default_rng(8)
    for n in (2, 8, 128, 2048):
        x = rng.standard_normal((4, n))
        y = rdft_packed_rows(x)
        full = _complex(dft_rows(_interleave(x.astype(complex))))
        ref = np.fft.rfft(x, axis=1)
        for Z in (full[:, : n // 2 + 1], ref):
            assert np.allclose(y[:, 0], Z[:, 0].real, atol=1e-9 * n)
            assert np.allclose(y[:, 1], Z[:, n // 2].real, atol=1e-9 * n)
            assert np.allclose(y[:, 2::2] + 1j * y[:, 3::2], Z[:, 1: n // 2], atol=1e-9 * n)


def test_real_bound_values():
    # sqrt 2 times the half-length complex bound plus 6u; n = 2 is one
    # addition per output (no complex pass)
    u = 2.0 ** -24
    assert parity.rel_rfft(2) == 6 * u
    assert abs(parity.rel_rfft(1024) - (np.sqrt(2) * parity.rel_fft(512) + 6 * u)) < 1e-20


def test_real_inverse_round_trip_and_library():
    # irdft_packed_rows undoes rdft_packed_rows; a packed flat spectrum
    # (all bins 1) is the delta; numpy.fft.irfft of the unpacked bins agrees
    rng = np.random.default_rng(10)
    for n in (2, 4, 64, 1024):
        x = rng.standard_normal((3, n))
        assert np.max(np.abs(irdft_packed_rows(rdft_packed_rows(x)) - x)) < 1e-12 * n
        flat = np.zeros((1, n))
        flat[0, 0] = flat[0, 1] = 1
        flat[0, 2::2] = 1
        want = np.zeros(n)
        want[0] = 1
        assert np.max(np.abs(irdft_packed_rows(flat)[0] - want)) < 1e-12
        p = rdft_packed_rows(x)
        bins = np.zeros((3, n // 2 + 1), complex)
        bins[:, 0], bins[:, n // 2] = p[:, 0], p[:, 1]
        bins[:, 1: n // 2] = p[:, 2::2] + 1j * p[:, 3::2]
        assert np.allclose(irdft_packed_rows(p), np.fft.irfft(bins, n, axis=1), atol=1e-12 * n)
    # n = 2 by hand: [a, b] packed as (X0, X1) = (a + b, a - b)
    assert np.allclose(irdft_packed_rows(np.array([[5.0, -1.0]])), [[2.0, 3.0]], rtol=0, atol=1e-15)
