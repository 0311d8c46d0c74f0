"""Pins of the oracle's smooth particle-mesh Ewald structure factor (the
paper's method for the ionic structure factor of large cells, Sections
"OFDFT software background" and "Leveraging existing techniques"; the
method of Essmann et al. 1995):

* the cardinal B-splines are the textbook ones: the cubic spline's values at
  the integers, unit integral, symmetry and partition of unity;
* the exponential-spline interpolation is exact for atoms on grid points, so
  PME then equals the exact sum at every frequency;
* for atoms anywhere it converges to the exact sum as the order grows, with
  S(0) = natoms exactly;
* moving every atom by one grid step multiplies S(G) by exp(-2 pi i m / K);
* the reading that the order is even: for odd orders the factor's
  denominator vanishes at the Nyquist frequency."""
import numpy as np
import pytest

from oracle import cell as OC
from oracle import functionals as OF
from oracle import pme as P
from tests.oracle_helpers import box_cell

L = (9.0, 10.0, 11.0)
N = (16, 18, 20)


def freq_fraction(n):
    m0 = OC.mvals(n[0])[:, None, None] / n[0]
    m1 = OC.mvals(n[1])[None, :, None] / n[1]
    m2 = OC.half_mvals(n[2])[None, None, :] / n[2]
    return np.maximum(np.maximum(np.abs(m0), np.abs(m1)), np.abs(m2))


def test_cubic_bspline_values():
    # M_4 at the integers 1, 2, 3: 1/6, 2/3, 1/6 (the cubic B-spline)
    np.testing.assert_allclose(P.bspline(4, np.array([0.0, 1.0, 2.0, 3.0, 4.0])),
                               [0.0, 1 / 6, 2 / 3, 1 / 6, 0.0], atol=1e-15)
    # and its closed form on [0, 1]: x^3 / 6
    x = np.linspace(0, 1, 7)
    np.testing.assert_allclose(P.bspline(4, x), x ** 3 / 6, atol=1e-15)


@pytest.mark.parametrize("n", [4, 6, 10, 16])
def test_bspline_partition_of_unity_symmetry_and_integral(n):
    t = np.linspace(0, 1, 11)[:-1]
    tot = sum(P.bspline(n, t + j) for j in range(n))
    np.testing.assert_allclose(tot, 1.0, atol=1e-14)
    x = np.linspace(0, n, 97)
    np.testing.assert_allclose(P.bspline(n, x), P.bspline(n, n - x), atol=1e-14)
    xs = np.linspace(0, n, 20001)
    assert abs(np.trapezoid(P.bspline(n, xs), xs) - 1.0) < 1e-7


@pytest.mark.parametrize("order", [4, 6, 10])
def test_pme_exact_for_atoms_on_grid_points(order):
    rng = np.random.default_rng(order)
    frac = rng.integers(0, 16, size=(6, 3)) / np.array(N)
    cell = box_cell(L=L, n=N, pos=frac @ np.diag(L))
    atoms = np.arange(6)
    d = P.structure_factor(cell, atoms, order) - P.structure_factor_direct(cell, atoms)
    assert np.abs(d).max() <= 1e-10


def test_pme_converges_to_the_direct_sum():
    rng = np.random.default_rng(3)
    cell = box_cell(L=L, n=N, pos=rng.random((7, 3)) * np.array(L))
    atoms = np.arange(7)
    Sd = P.structure_factor_direct(cell, atoms)
    low = freq_fraction(N) <= 0.125
    errs = []
    for order in (4, 6, 8, 10, 12):
        S = P.structure_factor(cell, atoms, order)
        assert abs(S[0, 0, 0] - 7.0) <= 1e-12
        errs.append(np.abs(S - Sd)[low].max())
    assert all(b < 0.2 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[3] / 7.0 < 1e-8        # order 10


def test_pme_shift_by_one_grid_step():
    rng = np.random.default_rng(5)
    pos = rng.random((5, 3)) * np.array(L)
    atoms = np.arange(5)
    c0 = box_cell(L=L, n=N, pos=pos)
    c1 = box_cell(L=L, n=N, pos=pos + np.array([L[0] / N[0], 0.0, 0.0]))
    S0 = P.structure_factor(c0, atoms, 8)
    S1 = P.structure_factor(c1, atoms, 8)
    ph = np.exp(-2j * np.pi * OC.mvals(N[0]) / N[0])[:, None, None]
    assert np.abs(S1 - S0 * ph).max() <= 1e-12


def test_pme_vext_species_sum():
    # two species: v_ext is the sum of each species' form factor times its
    # own structure factor, and PME reduces to the exact v_ext for atoms on
    # grid points
    rng = np.random.default_rng(11)
    frac = rng.integers(0, 16, size=(5, 3)) / np.array(N)
    cell = OC.Cell(lattice=np.diag(L), n=N, pos=frac @ np.diag(L),
                   species=np.array([0, 1, 0, 1, 1]), Z=[3.0, 2.0], rc=[1.0, 0.8], nelec=12.0)
    np.testing.assert_allclose(P.vext_g(cell, 6), OF.vext_g(cell), rtol=0, atol=1e-11)


def test_odd_order_factor_vanishes_at_nyquist():
    # the reading that fixes the order to even values
    K = 16
    m = np.arange(K)
    for n in (3, 5):
        den = np.exp(2j * np.pi * np.outer(m, np.arange(n - 1)) / K) @ P.bspline(n, np.arange(n - 1) + 1.0)
        assert abs(den[K // 2]) < 1e-14
    for n in (4, 10):
        assert np.all(np.isfinite(P.bfactor(K, n)))
