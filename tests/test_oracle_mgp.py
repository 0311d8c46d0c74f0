"""Pins of the oracle's MGP-family kernels (eq. "MGP"; oracle/mgp.py), CPU.

The paper prints no MGP kernel values (the supplement that defines
eta(q, t) is not part of it), so the absolute kernels are "parity unpinned"
against the paper.  What pins the oracle instead:

* G' (the analytic derivative of the printed G_NL) against 40-digit mpmath
  differentiation of the printed formula, on every branch;
* the paper's t-integral against its integration-by-parts form
  [t^y G]_0^1 - y int t^(y-1) G dt (independent quadrature, in u = t^y) and
  against 30-digit mpmath quadrature;
* x = 0 gives WT exactly; omega(0) = 0; omega -> C_WT G(inf) = -8/5 C_WT;
* the small-eta asymptotes (y = 5/6: J = -(8/3) eta^2 3y/(3y - 2) +
  C eta^(3y) + O(eta^4), C = 3y int_0^inf (G(v) + 8 v^2/3) v^(-3y-1) dv from
  mpmath; y = 5/3: J = -(40/9) eta^2 + (8/9) eta^4 + O(eta^5)), which a wrong
  exponent in eta(q, t) or a dropped chain-rule factor fails;
* the table: node values equal G - I, linear interpolation in between;
* the functional: uniform density gives E_NL = 0, finite differences of the
  MGP potential (WT-type and spline), x = 0 equal to WT.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

from oracle import cell as C
from oracle import functionals as Fn
from oracle import mgp
from tests.oracle_helpers import box_cell, grid_points, smooth_density

mp.mp.dps = 40


def G_mp(x):
    """The printed G_NL in mpmath; above x = 2 through the series
    F = sum_n u^n/((2n-1)(2n+1)), u = 1/x^2, with 1/F - 3 x^2 summed without
    cancellation (-1 - S/P), since the printed form loses digits as x grows."""
    x = mp.mpf(x)
    if x == 0:
        return mp.mpf(0)
    if x == 1:
        return mp.mpf(-2)
    if x > 2:
        u = 1 / (x * x)
        P = mp.nsum(lambda n: u ** (n - 1) / ((2 * n - 1) * (2 * n + 1)), [1, mp.inf])
        S = mp.nsum(lambda n: 3 * u ** (n - 2) / ((2 * n - 1) * (2 * n + 1)), [2, mp.inf])
        return -1 - S / P
    F = mp.mpf(1) / 2 + (1 - x * x) / (4 * x) * mp.log(abs((1 + x) / (1 - x)))
    return 1 / F - 3 * x * x - 1


@pytest.mark.parametrize("e", [1e-3, 0.05, 0.3, 0.499, 0.501, 0.8, 0.999, 1.001, 1.3, 1.499,
                               1.501, 2.5, 10.0, 300.0])
def test_dgnl_against_mpmath(e):
    ref = float(mp.diff(G_mp, mp.mpf(e)))
    assert abs(mgp.dgnl(e) - ref) <= 1e-12 * max(abs(ref), 1e-3 * e), (e, mgp.dgnl(e), ref)


def j_by_parts(eta, y):
    """y int_0^1 t^(y-1) G(eta t^(-1/3)) dt in u = t^y:
    int_0^1 G(eta u^(-1/(3y))) du (the complement of I in G)."""
    g = lambda u: float(Fn.gnl(np.array([eta * u ** (-1.0 / (3.0 * y))]))[0]) if u > 0 else -1.6
    pts = [eta ** (3.0 * y)] if eta < 1.0 else None
    return integrate.quad(g, 0.0, 1.0, points=pts, limit=500, epsabs=1e-15, epsrel=1e-13)[0]


@pytest.mark.parametrize("y", [5.0 / 6.0, 5.0 / 3.0])
@pytest.mark.parametrize("eta", [1e-3, 0.1, 0.5, 0.99, 1.0, 1.01, 1.7, 4.0, 25.0])
def test_integration_by_parts(eta, y):
    I = mgp.correction_integral(eta, y)
    G = float(Fn.gnl(np.array([eta]))[0])
    # [t^y G]_0^1 = G(eta): t^y -> 0 while G stays bounded (-> -8/5)
    assert abs(I - (G - j_by_parts(eta, y))) <= 1e-12, (eta, y)


@pytest.mark.parametrize("y", [5.0 / 6.0, 5.0 / 3.0])
@pytest.mark.parametrize("eta", [0.25, 0.9, 1.0, 2.0])
def test_integral_against_mpmath(eta, y):
    mp.mp.dps = 30
    E, Y = mp.mpf(eta), mp.mpf(y)
    us = E ** (3 * Y) if eta < 1 else mp.mpf(1)
    pts = [0, us / 1000, us / 10, us] + ([1] if eta < 1 else [])
    J = mp.quad(lambda u: G_mp(E * u ** (-1 / (3 * Y))), pts)
    ref = float(G_mp(E) - J)
    mp.mp.dps = 40
    assert abs(mgp.correction_integral(eta, y) - ref) <= 1e-13


def test_x_zero_is_wang_teter_and_limits():
    eta = np.concatenate([np.linspace(0, 6, 601), [10.0, 1e3, 1e6]])
    for y in (5.0 / 6.0, 5.0 / 3.0):
        np.testing.assert_array_equal(mgp.kernel_shape_xy(eta, 0.0, y), Fn.gnl(eta))
    for kind in (mgp.KERNEL_MGP, mgp.KERNEL_MGPA, mgp.KERNEL_MGPG):
        k = mgp.kernel_shape(eta, kind)
        assert k[0] == 0.0                                  # omega(0) = 0
        assert abs(k[-1] + 1.6) < 1e-9                      # G(inf) = -8/5
        w = mgp.kernel(np.array([0.0, 1.0]), 0.9, kind)
        assert w[0] == 0.0
    np.testing.assert_array_equal(mgp.kernel_shape(eta, mgp.KERNEL_WT), Fn.gnl(eta))


def G_plus_quadratic_mp(v):
    """G(v) + 8 v^2/3 without cancellation below v = 1/2: with
    F = 1 - sum_{k>=1} c_k v^(2k) (c_k = 1/((2k-1)(2k+1))), 1/F - 1 = S/F with
    S = sum c_k v^(2k), and S/F - v^2/3 = sum_{k>=2} (c_k + c_(k-1)/3) v^(2k) / F."""
    v = mp.mpf(v)
    if v >= mp.mpf("0.5"):
        return G_mp(v) + 8 * v * v / 3
    c = lambda k: mp.mpf(1) / ((2 * k - 1) * (2 * k + 1))
    F = 1 - mp.nsum(lambda k: c(k) * v ** (2 * k), [1, mp.inf])
    num = mp.nsum(lambda k: (c(k) + c(k - 1) / 3) * v ** (2 * k), [2, mp.inf])
    return num / F


def test_small_eta_asymptote_mgp():
    """y = 5/6 (MGP, MGPA): with a = 1/(3y), J = int_0^1 G(eta u^-a) du; G's
    quadratic term gives -(8/3) eta^2 / (1 - 2a) and the rest, where the
    argument leaves the small-eta range, C eta^(3y) with
    C = 3y int_0^inf (G(v) + 8 v^2/3) v^(-3y-1) dv; the remainder is O(eta^4)."""
    y = 5.0 / 6.0
    mp.mp.dps = 30
    Y = mp.mpf(y)
    f = lambda v: G_plus_quadratic_mp(v) * v ** (-3 * Y - 1)
    Cc = float(3 * Y * mp.quad(f, [0, mp.mpf("0.5"), 1, 2, mp.inf]))
    mp.mp.dps = 40
    for eta in (1e-4, 1e-3, 3e-3, 1e-2):
        J = float(Fn.gnl(np.array([eta]))[0]) - mgp.correction_integral(eta, y)
        ref = -8.0 / 3.0 * eta * eta * 3.0 * y / (3.0 * y - 2.0) + Cc * eta ** (3.0 * y)
        assert abs(J - ref) <= eta ** 4 + 1e-15, (eta, J, ref)


def test_small_eta_asymptote_mgpg():
    """y = 5/3 (MGPG): 3y = 5 > 4, so G's quartic term 8 v^4/45 still
    integrates: J = -(8/3)(5/3) eta^2 + (8/45)(5) eta^4 + O(eta^5)."""
    y = 5.0 / 3.0
    for eta in (3e-3, 1e-2, 3e-2):
        J = float(Fn.gnl(np.array([eta]))[0]) - mgp.correction_integral(eta, y)
        ref = -40.0 / 9.0 * eta * eta + 8.0 / 9.0 * eta ** 4
        assert abs(J - ref) <= 3.0 * eta ** 5 + 1e-15, (eta, J, ref)


def test_table_nodes_and_interpolation():
    y = 5.0 / 6.0
    ja, jb = mgp.j_table(y)
    rng = np.random.default_rng(3)
    for j in rng.integers(0, mgp.TAB_NA + 1, 12):
        e = j * mgp.TAB_H
        assert ja[j] == float(Fn.gnl(np.array([e]))[0]) - mgp.correction_integral(e, y)
        assert mgp.j_interp(np.array([e]), y)[0] == ja[j]
    for k in rng.integers(1, mgp.TAB_NB + 1, 6):
        e = 1.0 / math.sqrt(k * mgp.TAB_WH)
        assert abs(mgp.j_interp(np.array([e]), y)[0] - jb[k]) < 1e-15
    # between nodes: the straight line through the two neighbours, and close
    # to the exact integral
    e = 1.3 * mgp.TAB_H + 0.7
    j = int(e / mgp.TAB_H)
    f = e / mgp.TAB_H - j
    lin = (1 - f) * ja[j] + f * ja[j + 1]
    assert abs(mgp.j_interp(np.array([e]), y)[0] - lin) < 1e-15
    exact = float(Fn.gnl(np.array([e]))[0]) - mgp.correction_integral(e, y)
    assert abs(lin - exact) < 1e-6


def mgp_func(kind, terms=C.WT | C.TF | C.VW, **kw):
    return C.Functional(terms=terms, nl_kernel=kind, **kw)


@pytest.mark.parametrize("kind", [mgp.KERNEL_MGP, mgp.KERNEL_MGPA, mgp.KERNEL_MGPG])
def test_uniform_density_has_no_nonlocal_energy(kind):
    cell = box_cell(n=(8, 8, 10), nelec=6.0)
    rho = np.full(cell.n, cell.nelec / cell.volume)
    r = Fn.energy_potential(cell, mgp_func(kind), rho=rho)
    assert abs(r.e_nl) < 1e-12
    r = Fn.energy_potential(cell, mgp_func(kind, terms=C.SPLINE, nk=6, kf_min=0.3,
                                           kf_max=1.5), rho=rho)
    assert abs(r.e_nl) < 1e-12


@pytest.mark.parametrize("kind", [mgp.KERNEL_MGP, mgp.KERNEL_MGPA, mgp.KERNEL_MGPG])
def test_mgp_potential_finite_difference(kind):
    cell = box_cell(L=(6.0, 7.0, 8.0), n=(8, 8, 10), nelec=24.0)
    rho = smooth_density(cell, seed=2, amp=0.8)
    pts = grid_points(cell)
    h = 1e-5
    dr = (np.cos(pts @ cell.recip[0] + 0.4) + 0.6 * np.sin(pts @ cell.recip[2] - 0.2) +
          0.5 * np.cos(pts @ (cell.recip[1] + cell.recip[0]) + 1.0)) * rho * 0.3
    for func in (mgp_func(kind, terms=C.WT),
                 mgp_func(kind, terms=C.SPLINE, nk=8, kf_min=0.3, kf_max=1.6,
                          nl_mode=C.NL_EXACT)):
        r = Fn.energy_potential(cell, func, rho=rho)
        ep = Fn.energy_potential(cell, func, rho=rho + h * dr).e_nl
        em = Fn.energy_potential(cell, func, rho=rho - h * dr).e_nl
        an = cell.dv * np.sum(r.v * dr)
        assert abs(an) > 1e-2
        assert abs((ep - em) / (2 * h) - an) < 1e-8 * abs(an), (func.terms, kind)


def test_mgp_differs_from_wt_and_variants_differ():
    cell = box_cell(L=(6.0, 7.0, 8.0), n=(8, 8, 10), nelec=6.0)
    rho = smooth_density(cell, seed=5, amp=0.6)
    e = {k: Fn.energy_potential(cell, mgp_func(k, terms=C.WT), rho=rho).e_nl
         for k in (mgp.KERNEL_WT, mgp.KERNEL_MGP, mgp.KERNEL_MGPA, mgp.KERNEL_MGPG)}
    vals = list(e.values())
    assert min(abs(a - b) for i, a in enumerate(vals) for b in vals[i + 1:]) > 1e-6
    # MGPA is the mean of WT and MGP (x = 1/2 with the same y)
    assert abs(e[mgp.KERNEL_MGPA] - 0.5 * (e[mgp.KERNEL_WT] + e[mgp.KERNEL_MGP])) < 1e-12
