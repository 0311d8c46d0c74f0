"""Pins of the oracle's own Fourier transform (CPU).

The oracle FFT (oracle/fft.c) is checked against things that do not share its
code: the O(N^2) definition of the DFT, NumPy's pocketfft (a library routine),
Parseval's identity, and the spectra of a delta and of a plane wave.
"""
import numpy as np
import pytest

from oracle import fourier as F

SHAPES = [(4, 4, 4), (6, 5, 8), (3, 4, 6), (8, 6, 4), (7, 9, 10), (5, 5, 5)]


@pytest.mark.parametrize("shape", SHAPES)
def test_fft_matches_bruteforce_dft(shape):
    rng = np.random.default_rng(sum(shape))
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    for sign in (-1, 1):
        np.testing.assert_allclose(F.fft3_raw(a, sign), F.dft_bruteforce(a, sign),
                                   rtol=0, atol=1e-11)


@pytest.mark.parametrize("shape", [(12, 18, 16), (32, 24, 27), (10, 14, 22)])
def test_fft_matches_numpy(shape):
    rng = np.random.default_rng(1)
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    np.testing.assert_allclose(F.fft3_raw(a, -1), np.fft.fftn(a), rtol=0, atol=1e-10)
    np.testing.assert_allclose(F.fft3_raw(a, 1), np.fft.ifftn(a) * a.size, rtol=0,
                               atol=1e-10)


def test_fft1_prime_and_composite_lengths():
    rng = np.random.default_rng(2)
    for n in (1, 2, 3, 5, 7, 11, 13, 30, 64, 81, 97, 192):
        a = rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))
        np.testing.assert_allclose(F.fft1_raw(a, -1), np.fft.fft(a, axis=-1), rtol=0,
                                   atol=1e-10 * max(1, n))


@pytest.mark.parametrize("shape", [(6, 8, 10), (4, 6, 9), (8, 8, 8)])
def test_r2c_c2r_round_trip_and_parseval(shape):
    rng = np.random.default_rng(3)
    f = rng.standard_normal(shape)
    X = F.r2c(f)
    assert X.shape == (shape[0], shape[1], shape[2] // 2 + 1)
    np.testing.assert_allclose(F.c2r(X, shape), f, rtol=0, atol=1e-13)
    w = F.half_weights(shape[2])[None, None, :]
    # Parseval: (1/N) sum |f|^2 = sum_G |f(G)|^2 = sum_half c |X|^2
    np.testing.assert_allclose(np.mean(f * f), np.sum(w * np.abs(X) ** 2), rtol=1e-13)
    # the half spectrum is NumPy's rfftn / N
    np.testing.assert_allclose(X, np.fft.rfftn(f) / f.size, rtol=0, atol=1e-15)


def test_delta_and_plane_wave():
    shape = (8, 6, 10)
    N = np.prod(shape)
    d = np.zeros(shape)
    d[0, 0, 0] = 1.0
    np.testing.assert_allclose(F.r2c(d), np.full((8, 6, 6), 1.0 / N), atol=1e-16)
    i0, i1, i2 = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    f = np.cos(2 * np.pi * (2 * i0 / 8 + 1 * i1 / 6 + 3 * i2 / 10))
    X = F.r2c(f)
    expect = np.zeros_like(X)
    expect[2, 1, 3] = 0.5          # only the +G bin lives in the half spectrum
    np.testing.assert_allclose(X, expect, atol=1e-14)


def test_c2r_drops_imaginary_part_of_self_conjugate_planes():
    # the inverse is Re sum_half c X e^{iGr}: an imaginary constant term or an
    # imaginary Nyquist plane contributes nothing
    shape = (4, 4, 6)
    X = np.zeros((4, 4, 4), dtype=complex)
    X[0, 0, 0] = 1j
    X[0, 0, 3] = 1j
    np.testing.assert_allclose(F.c2r(X, shape), 0.0, atol=1e-15)
    X[0, 0, 0] = 2.0
    np.testing.assert_allclose(F.c2r(X, shape), 2.0, atol=1e-15)
