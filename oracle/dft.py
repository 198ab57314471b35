"""Oracle of the FFT function block (test infrastructure only; parity
pinned by tests/test_oracle_dft.py against closed forms and numpy.fft).

The analysis of Sec. 3.2 (steps 1-2, 1-3) names FFT library calls beside
loop statements as offloadable parts.  The call computes, for each row of n
complex values x[0..n-1] (real and imaginary parts interleaved in a float
row of length 2n), the forward discrete Fourier transform by its definition

    X[k] = sum_{j=0}^{n-1} x[j] * exp(-2 pi i j k / n),   k = 0..n-1.

The inverse call computes, per row, the inverse transform scaled by 1/n,

    x[j] = (1/n) sum_{k=0}^{n-1} X[k] * exp(+2 pi i j k / n),   j = 0..n-1,

so that the inverse of the forward transform gives the row back.

The real call takes rows of n real values and writes each row's spectrum
X[0..n/2] (X[n-k] = conj X[k] for real input) packed into the same n floats:
[X[0], X[n/2], Re X[1], Im X[1], ..., Re X[n/2-1], Im X[n/2-1]] (X[0] and
X[n/2] are real); its inverse call takes such packed rows back to the real
rows, x[j] = (1/n) sum_k X[k] exp(+2 pi i j k / n) over the full
(Hermitian) spectrum.

Evaluated here as those sums in complex double precision (one matrix
product of the row with the n x n matrix of exp(-2 pi i ((j k) mod n) / n),
or its complex conjugate for the inverse; the exponent index is reduced
exactly in integers first).
"""
import numpy as np


def dft_matrix(n):
    jk = np.outer(np.arange(n, dtype=np.int64), np.arange(n, dtype=np.int64)) % n
    return np.exp(-2j * np.pi * jk / n)


def dft_rows(x):
    """Forward DFT of each row of x[R][2n] (interleaved); float64 result of
    the same layout."""
    x = np.asarray(x, np.float64)
    R, m = x.shape
    if m % 2:
        raise ValueError("rows hold interleaved complex values")
    n = m // 2
    z = x[:, 0::2] + 1j * x[:, 1::2]
    Z = z @ dft_matrix(n) if n else z
    out = np.empty((R, m), np.float64)
    out[:, 0::2] = Z.real
    out[:, 1::2] = Z.imag
    return out


def idft_rows(x):
    """Inverse DFT (scaled by 1/n) of each row of x[R][2n] (interleaved);
    float64 result of the same layout."""
    x = np.asarray(x, np.float64)
    R, m = x.shape
    if m % 2:
        raise ValueError("rows hold interleaved complex values")
    n = m // 2
    z = x[:, 0::2] + 1j * x[:, 1::2]
    Z = (z @ np.conj(dft_matrix(n))) / n if n else z
    out = np.empty((R, m), np.float64)
    out[:, 0::2] = Z.real
    out[:, 1::2] = Z.imag
    return out


def rdft_packed_rows(x):
    """DFT of each row of n real values, packed as described above; float64
    result of the same shape."""
    x = np.asarray(x, np.float64)
    R, n = x.shape
    if n < 2 or n % 2:
        raise ValueError("real rows hold an even number of values")
    X = x @ dft_matrix(n)[:, : n // 2 + 1]
    out = np.empty((R, n), np.float64)
    out[:, 0] = X[:, 0].real
    out[:, 1] = X[:, n // 2].real
    out[:, 2::2] = X[:, 1 : n // 2].real
    out[:, 3::2] = X[:, 1 : n // 2].imag
    return out


def irdft_packed_rows(p):
    """Real rows of the packed spectra p[R][n] (the inverse of
    rdft_packed_rows); float64 result of the same shape."""
    p = np.asarray(p, np.float64)
    R, n = p.shape
    if n < 2 or n % 2:
        raise ValueError("packed rows hold an even number of values")
    m = n // 2
    X = np.zeros((R, n), complex)
    X[:, 0] = p[:, 0]
    X[:, m] = p[:, 1]
    X[:, 1:m] = p[:, 2::2] + 1j * p[:, 3::2]
    X[:, m + 1:] = np.conj(X[:, 1:m][:, ::-1])
    return ((X @ np.conj(dft_matrix(n))) / n).real
