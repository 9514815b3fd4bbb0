"""Pins of the oracle's own FFT: brute-force DFT, inversion, Parseval, and the
independent numpy.fft library routine on multi-dimensional arrays."""
import numpy as np
import pytest

LENGTHS = [1, 2, 3, 4, 5, 6, 7, 8, 9, 12, 16, 18, 24, 27, 32, 36, 48, 64, 96, 128, 192]


@pytest.mark.parametrize("n", LENGTHS)
def test_fft_matches_bruteforce_dft(orc, n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for sign in (-1, 1):
        a = orc.fft1d(x, sign)
        b = orc.dft1d(x, sign)
        # textbook definition written out in numpy as a third opinion
        j = np.arange(n)
        M = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
        c = M @ x
        assert np.max(np.abs(a - b)) <= 1e-13 * max(1.0, np.max(np.abs(b)))
        assert np.max(np.abs(a - c)) <= 1e-12 * max(1.0, np.max(np.abs(c)))


@pytest.mark.parametrize("n", [6, 64, 96, 512, 1024])
def test_fft_inverse_and_parseval(orc, n):
    rng = np.random.default_rng(1000 + n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = orc.fft1d(x, -1)
    back = orc.fft1d(X, +1) / n
    assert np.max(np.abs(back - x)) < 1e-14 * np.sqrt(n) * 10
    assert abs(np.sum(np.abs(X) ** 2) / n - np.sum(np.abs(x) ** 2)) < 1e-12 * np.sum(np.abs(x) ** 2)


@pytest.mark.parametrize("shape", [(6, 8, 9), (16, 12), (4, 3, 2)])
def test_fftnd_matches_library(orc, shape):
    rng = np.random.default_rng(7)
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    a = orc.fftnd(x, -1)
    b = np.fft.fftn(x)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))
    a = orc.fftnd(x, +1)
    b = np.fft.ifftn(x) * x.size
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))
