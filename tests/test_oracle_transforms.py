"""Pins of the oracle's transforms and differentiation against closed forms, the
textbook DFT, a library FFT and the paper's cot-form differentiation matrix."""
import math

import numpy as np
import pytest

from oracle import oracle as orc

SIZES = [1, 2, 3, 4, 5, 6, 7, 8, 12, 16, 24, 48, 96, 128]


def test_dft_closed_forms():
    # F_N(j, k) = exp(-2 pi i jk / N) (Sec. 2.3): a delta at j0 maps to exp(-2 pi i j0 k/N),
    # and exp(+2 pi i m j / N) maps to N delta_{k m}.
    for n in (5, 8, 12):
        k = np.arange(n)
        for j0 in (0, 1, n - 1):
            x = np.zeros(n, complex)
            x[j0] = 1.0
            np.testing.assert_allclose(orc.dft(x), np.exp(-2j * np.pi * j0 * k / n), atol=1e-14)
        for m in (0, 1, n // 2):
            x = np.exp(2j * np.pi * m * np.arange(n) / n)
            want = np.zeros(n, complex)
            want[m] = n
            np.testing.assert_allclose(orc.dft(x), want, atol=1e-12)
            # sign +1 is the unnormalised inverse
            np.testing.assert_allclose(orc.dft(want, sign=+1) / n, x, atol=1e-14)


@pytest.mark.parametrize("n", SIZES)
def test_fft_matches_textbook_dft(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for sign in (-1, 1):
        ref = orc.dft(x, sign)
        got = orc.fft(x, sign)
        scale = max(1.0, float(np.max(np.abs(ref))))
        assert np.max(np.abs(got - ref)) <= 1e-14 * scale * max(1, math.log2(max(n, 2)))


@pytest.mark.parametrize("n", SIZES)
def test_fft_matches_library_fft(n):
    rng = np.random.default_rng(100 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    np.testing.assert_allclose(orc.fft(x, -1), np.fft.fft(x), rtol=0, atol=1e-13 * max(1, n))
    np.testing.assert_allclose(orc.fft(x, +1), n * np.fft.ifft(x), rtol=0, atol=1e-13 * max(1, n))


@pytest.mark.parametrize("shape", [(4, 6, 8), (8, 8, 8), (12, 4, 6), (16, 8, 2)])
def test_fft3_is_kronecker_of_1d(shape):
    nz, ny, nx = shape
    rng = np.random.default_rng(7)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    A = orc.fft3(a, -1)
    np.testing.assert_allclose(A, np.fft.fftn(a), atol=1e-12)
    back = orc.fft3(A, +1)
    np.testing.assert_allclose(back, a, atol=1e-14)
    # x is the fastest index: a plane wave along x only lights the kx index
    x = np.exp(2j * np.pi * 1 * np.arange(nx) / nx)[None, None, :] * np.ones(shape)
    B = orc.fft3(x, -1)
    assert abs(B[0, 0, 1] - nx * ny * nz) < 1e-9
    B[0, 0, 1] = 0
    assert np.max(np.abs(B)) < 1e-9


def test_wavenumbers_definition():
    # Omega_w = nu_w diag(0, 1, ..., N/2-1, 0, -N/2+1, ..., -1), nu_w = 2 pi / L_w (Sec. 2.3)
    np.testing.assert_allclose(orc.wavenumbers(8, 2 * math.pi), [0, 1, 2, 3, 0, -3, -2, -1])
    np.testing.assert_allclose(orc.wavenumbers(6, 1.0), 2 * math.pi * np.array([0, 1, 2, 0, -2, -1]))
    np.testing.assert_allclose(orc.wavenumbers(4, 4 * math.pi), 0.5 * np.array([0, 1, 0, -1]))
    with pytest.raises(ValueError):
        orc.wavenumbers(5, 1.0)


@pytest.mark.parametrize("n,length", [(4, 2 * math.pi), (6, 1.0), (8, 2.0), (16, 4 * math.pi)])
def test_cot_matrix_equals_fourier_derivative(n, length):
    # The cot-form D_w of Sec. 2.2 and F^{-1} (i Omega_w) F of Sec. 2.3 (Nyquist -> 0) are
    # the same matrix.  Compare the two on random data along each axis of a 3-D array.
    D = orc.dmatrix(n, length)
    rng = np.random.default_rng(n)
    shape = {0: (3, 2, n), 1: (2, n, 3), 2: (n, 3, 2)}
    for axis in range(3):
        f = rng.standard_normal(shape[axis])
        dom = [0.0, 1.0] * 3
        dom[2 * axis + 1] = length
        got = orc.deriv(f, dom, axis)
        want = np.moveaxis(np.tensordot(D, np.moveaxis(f, 2 - axis, 0), axes=(1, 0)), 0, 2 - axis)
        np.testing.assert_allclose(got, want, atol=1e-12 * n)
    # D is skew-symmetric (used in the proofs of Sec. 4)
    np.testing.assert_allclose(D, -D.T, atol=1e-13)


def test_derivative_closed_forms():
    # d/dx sin(nu m x) = nu m cos(nu m x) on the grid; the Nyquist cosine differentiates to 0.
    n, L = 16, 3.0
    nu = 2 * math.pi / L
    x = np.arange(n) * L / n
    for axis in range(3):
        shape = [1, 1, 1]
        shape[2 - axis] = n
        dom = [0.0, 1.0] * 3
        dom[2 * axis + 1] = L
        for m in (1, 3, 7):
            f = np.sin(nu * m * x).reshape(shape)
            got = orc.deriv(np.broadcast_to(f, shape).copy(), dom, axis)
            np.testing.assert_allclose(got.reshape(-1), nu * m * np.cos(nu * m * x), atol=1e-12)
        nyq = np.cos(nu * (n // 2) * x).reshape(shape)
        assert np.max(np.abs(orc.deriv(nyq, dom, axis))) < 1e-12
