"""Pins of the oracle's Fourier interpolation (multi-step optimisation,
Section "Density optimization strategies"): a trigonometric polynomial in the
source band -- including the cosines that Nyquist samples stand for -- is
reproduced exactly on the finer grid; equal shapes are the identity; the
mean survives; densities keep their electron count."""
import numpy as np
import pytest

from oracle import multistep as MS


def _trig_field(shape, rng, nterms=6, nyquist=True):
    """Coarse-band trigonometric polynomial as a function of fractional
    coordinates; returns a callable f(grid shape) -> samples."""
    n0, n1, n2 = shape
    terms = []
    for _ in range(nterms):
        m = [int(rng.integers(-((n - 1) // 2), (n - 1) // 2 + 1)) for n in shape]
        terms.append((m, rng.normal(), rng.normal()))
    nyq = []
    if nyquist:
        if n0 % 2 == 0:
            nyq.append(((n0 // 2, 0, 0), rng.normal()))
        if n1 % 2 == 0 and n2 % 2 == 0:
            nyq.append(((0, n1 // 2, n2 // 2), rng.normal()))
        if n2 % 2 == 0:
            nyq.append(((1, 0, n2 // 2), rng.normal()))

    def sample(sh):
        x = np.meshgrid(*[np.arange(n) / n for n in sh], indexing="ij")
        out = np.full(sh, 0.7)
        for m, a, b in terms:
            ph = 2 * np.pi * (m[0] * x[0] + m[1] * x[1] + m[2] * x[2])
            out += a * np.cos(ph) + b * np.sin(ph)
        for m, a in nyq:   # products of cosines: the band-edge samples' meaning
            out += a * (np.cos(2 * np.pi * m[0] * x[0]) * np.cos(2 * np.pi * m[1] * x[1]) *
                        np.cos(2 * np.pi * m[2] * x[2]))
        return out
    return sample


@pytest.mark.parametrize("src,dst", [((8, 6, 10), (16, 12, 20)), ((6, 9, 8), (12, 18, 16)),
                                     ((5, 7, 6), (10, 9, 12)), ((8, 8, 8), (8, 16, 12))])
def test_band_limited_field_is_reproduced(src, dst):
    f = _trig_field(src, np.random.default_rng(3))
    got = MS.fourier_interpolate(f(src), dst)
    want = f(dst)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_equal_shape_is_identity():
    rng = np.random.default_rng(5)
    a = rng.normal(size=(6, 8, 10))
    assert np.abs(MS.fourier_interpolate(a, a.shape) - a).max() <= 1e-13


def test_mean_survives_and_out_of_band_content_is_dropped():
    rng = np.random.default_rng(7)
    a = rng.normal(size=(6, 6, 6))
    b = MS.fourier_interpolate(a, (12, 12, 12))
    assert abs(b.mean() - a.mean()) <= 1e-14
    # b is band-limited to the source band: carrying it back by sampling
    # every second point returns a
    assert np.abs(b[::2, ::2, ::2] - a).max() <= 1e-12


def test_density_interpolation_keeps_electrons_and_sign():
    rng = np.random.default_rng(9)
    rho = 0.02 + 0.01 * rng.random((8, 8, 8))
    out = MS.interpolate_density(rho, (16, 16, 16), nelec=12.0, dv=0.5)
    assert out.min() >= 0.0
    assert abs(0.5 * out.sum() - 12.0) <= 1e-12 * 12.0


def test_coarser_destination_is_refused():
    with pytest.raises(ValueError):
        MS.fourier_interpolate(np.zeros((8, 8, 8)), (8, 6, 8))
