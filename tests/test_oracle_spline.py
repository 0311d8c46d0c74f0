"""Pins of the oracle's spline (density-dependent-kernel) nonlocal functional.

Steps s1-s4 of the paper's nonlocal-KEDF section.  Pinned by: the uniform
density (zero energy and potential), exactness of linear interpolation for a
kernel linear in k, reduction to Wang-Teter when every k_F is clamped to one
knot or when there is a single knot, second-order convergence in the knot
spacing against a brute-force per-point kernel, and central finite
differences of the EXACT potential.
"""
import numpy as np
import pytest

from oracle import cell as C
from oracle import functionals as Fn
from oracle.fourier import c2r, r2c
from tests.oracle_helpers import box_cell, grid_points, make_cell, smooth_density
from paper_2002_02985_amd import workloads as W


def spline_func(mode, nk=8, kmin=0.5, kmax=1.6, spacing=C.KNOTS_LOG, **kw):
    return C.Functional(terms=C.SPLINE, nk=nk, kf_min=kmin, kf_max=kmax,
                        knot_spacing=spacing, nl_mode=mode, **kw)


def varied_density(cell, seed=1):
    # k_F spans roughly 0.6 .. 1.3 Bohr^-1
    return smooth_density(cell, seed=seed, amp=0.9, nmodes=3, rho0=0.03)


@pytest.mark.parametrize("mode", [C.NL_S3S4, C.NL_EXACT])
def test_uniform_density_gives_zero(mode):
    cell = box_cell(n=(8, 10, 12), nelec=4.0)
    rho = np.full(cell.n, cell.nelec / cell.volume)
    r = Fn.energy_potential(cell, spline_func(mode), rho=rho)
    assert abs(r.e_nl) < 1e-15
    assert np.abs(r.v).max() < 1e-14


@pytest.mark.parametrize("mode", [C.NL_S3S4, C.NL_EXACT])
def test_linear_in_k_kernel_is_exact(mode):
    cell = box_cell(L=(6.0, 7.0, 8.0), n=(8, 8, 10), nelec=6.0)
    rho = varied_density(cell)
    G2 = C.g2(cell)
    gn = np.sqrt(G2)
    A = Fn.C_WT * Fn.gnl(gn / 2.0)
    B = np.exp(-G2 / 3.0) * (G2 > 0)
    kern = lambda g, k: A + k * B
    func = spline_func(mode, nk=6)
    e, v, g = Fn.spline_nl(cell, func, rho, np.sqrt(rho), gn, kernel=kern)
    a = func.alpha
    kt = np.clip(Fn.kf_of_rho(rho), func.kf_min, func.kf_max)
    rb = r2c(rho ** a)
    phiA = c2r(A * rb, cell.n)
    phiB = c2r(B * rb, cell.n)
    e_bf = cell.dv * np.sum(rho ** a * (phiA + kt * phiB))
    assert abs(e - e_bf) < 1e-13
    if mode == C.NL_S3S4:
        np.testing.assert_allclose(v, 2 * a * rho ** (a - 1) * (phiA + kt * phiB), atol=1e-12)


@pytest.mark.parametrize("mode", [C.NL_S3S4, C.NL_EXACT])
def test_clamped_below_first_knot_equals_wt(mode):
    cell = box_cell(L=(6.0, 7.0, 8.0), n=(8, 8, 10), nelec=6.0)
    rho = varied_density(cell)
    kmin = 2.0   # above every k_F of this density
    sp = Fn.energy_potential(cell, spline_func(mode, nk=5, kmin=kmin, kmax=3.0), rho=rho)
    wt = Fn.energy_potential(cell, C.Functional(terms=C.WT, kf_wt=kmin), rho=rho)
    assert abs(sp.e_nl - wt.e_nl) < 1e-14
    np.testing.assert_allclose(sp.v, wt.v, atol=1e-12)
    np.testing.assert_allclose(sp.g, wt.g, atol=1e-12)


def test_single_knot_all_modes_equal_wt():
    cell = box_cell(L=(6.0, 7.0, 8.0), n=(8, 8, 10), nelec=6.0)
    rho = varied_density(cell)
    wt = Fn.energy_potential(cell, C.Functional(terms=C.WT, kf_wt=0.9), rho=rho)
    for mode in (C.NL_S3S4, C.NL_EXACT):
        sp = Fn.energy_potential(cell, spline_func(mode, nk=1, kmin=0.9, kmax=0.9), rho=rho)
        assert abs(sp.e_nl - wt.e_nl) < 1e-14
        np.testing.assert_allclose(sp.v, wt.v, atol=1e-12)


def test_second_order_convergence_in_knot_spacing():
    # brute force: every grid point gets the WT kernel at its own k_F
    cell = box_cell(L=(5.0, 5.5, 6.0), n=(6, 6, 6), nelec=4.0)
    rho = varied_density(cell, seed=2)
    a = 5.0 / 6.0
    kf = Fn.kf_of_rho(rho)
    kmin, kmax = kf.min() * 0.999, kf.max() * 1.001
    gn = np.sqrt(C.g2(cell))
    rb = r2c(rho ** a)
    e_bf = 0.0
    flat_k = kf.ravel()
    for idx in range(rho.size):
        phi_k = c2r(Fn.C_WT * Fn.gnl(gn / (2 * flat_k[idx])) * rb, cell.n)
        e_bf += rho.ravel()[idx] ** a * phi_k.ravel()[idx]
    e_bf *= cell.dv
    errs = []
    for nk in (5, 9, 17, 33):
        f = spline_func(C.NL_S3S4, nk=nk, kmin=kmin, kmax=kmax, spacing=C.KNOTS_LIN)
        errs.append(abs(Fn.energy_potential(cell, f, rho=rho).e_nl - e_bf))
    # fitted order of convergence in the knot spacing h ~ 1/(nk - 1)
    h = 1.0 / (np.array([5, 9, 17, 33]) - 1.0)
    slope = np.polyfit(np.log(h), np.log(errs), 1)[0]
    assert 1.8 < slope < 2.3, (errs, slope)


@pytest.mark.parametrize("spacing", [C.KNOTS_LOG, C.KNOTS_LIN])
def test_exact_potential_finite_difference(spacing):
    cell = box_cell(L=(6.0, 7.0, 8.0), n=(8, 8, 10), nelec=6.0)
    rho = varied_density(cell, seed=3)
    func = spline_func(C.NL_EXACT, nk=7, kmin=0.4, kmax=1.8, spacing=spacing)
    r = Fn.energy_potential(cell, func, rho=rho)
    d = np.cos(grid_points(cell) @ (cell.recip[0] + cell.recip[2])) * rho * 0.5
    h = 1e-6
    ep = Fn.energy_potential(cell, func, rho=rho + h * d).e_nl
    em = Fn.energy_potential(cell, func, rho=rho - h * d).e_nl
    an = cell.dv * np.sum(r.v * d)
    assert abs((ep - em) / (2 * h) - an) < 1e-6 * abs(an)
    # phi form
    phi = np.sqrt(rho)
    pts = grid_points(cell)
    dp = (np.sin(pts @ cell.recip[1] + 0.3) + 0.5 * np.cos(pts @ (cell.recip[0] - cell.recip[2]) + 1.1)) * phi * 0.1
    ep = Fn.energy_potential(cell, func, phi=phi + h * dp).e_nl
    em = Fn.energy_potential(cell, func, phi=phi - h * dp).e_nl
    an = cell.dv * np.sum(r.g * dp)
    assert abs(an) > 1e-4
    assert abs((ep - em) / (2 * h) - an) < 1e-6 * abs(an)


def test_s3s4_differs_from_exact_but_same_energy():
    cell = box_cell(L=(6.0, 7.0, 8.0), n=(8, 8, 10), nelec=6.0)
    rho = varied_density(cell, seed=4)
    a = Fn.energy_potential(cell, spline_func(C.NL_S3S4), rho=rho)
    b = Fn.energy_potential(cell, spline_func(C.NL_EXACT), rho=rho)
    assert a.e_nl == b.e_nl
    assert np.abs(a.v - b.v).max() > 1e-4


def test_brackets_tie_rules():
    kn = np.array([0.5, 1.0, 2.0])
    kt, j, t, inside = Fn.spline_brackets(kn, np.array([0.1, 0.5, 0.75, 1.0, 2.0, 5.0]))
    np.testing.assert_array_equal(j, [0, 0, 0, 1, 1, 1])
    np.testing.assert_allclose(t, [0, 0, 0.5, 0, 1, 1])
    np.testing.assert_array_equal(inside, [False, False, True, True, False, False])
    np.testing.assert_allclose(C.knots(C.Functional(nk=32, kf_min=0.1, kf_max=3.0))[[0, 31]],
                               [0.1, 3.0], rtol=1e-15)


def test_log_knots_are_a_geometric_progression():
    """Step s1 with geometric spacing: every interior knot is pinned, not only
    the ends.  A geometric progression has a constant ratio and mirror pairs
    whose product is k_min k_max; an arithmetic progression between the same
    ends fails both (and the arithmetic variant is checked by the dual
    properties: constant difference, mirror pairs summing to k_min + k_max)."""
    for nk, lo, hi in [(32, 0.1, 3.0), (7, 0.25, 4.0), (2, 0.5, 2.0)]:
        k = C.knots(C.Functional(nk=nk, kf_min=lo, kf_max=hi, knot_spacing=C.KNOTS_LOG))
        assert len(k) == nk
        ratio = k[1:] / k[:-1]
        np.testing.assert_allclose(ratio, (hi / lo) ** (1.0 / (nk - 1)), rtol=1e-13)
        np.testing.assert_allclose(k * k[::-1], lo * hi, rtol=1e-13)
        # log k is evenly spaced from log k_min to log k_max
        np.testing.assert_allclose(np.log(k), np.linspace(np.log(lo), np.log(hi), nk),
                                   rtol=0, atol=1e-13)
        kl = C.knots(C.Functional(nk=nk, kf_min=lo, kf_max=hi, knot_spacing=C.KNOTS_LIN))
        np.testing.assert_allclose(np.diff(kl), (hi - lo) / (nk - 1), rtol=1e-13)
        np.testing.assert_allclose(kl + kl[::-1], lo + hi, rtol=1e-13)
        if nk > 2:
            # the two progressions really differ inside
            assert np.abs(k[1:-1] - kl[1:-1]).min() > 1e-3


def test_brackets_on_log_knots_match_a_linear_search():
    """Bracket and weight on the 32 geometric knots of the slab workload
    against a plain linear scan over the segments."""
    kn = C.knots(C.Functional(nk=32, kf_min=0.1, kf_max=3.0))
    rng = np.random.default_rng(11)
    kf = np.concatenate([np.exp(rng.uniform(np.log(0.05), np.log(4.0), 2000)), kn,
                         [0.1, 3.0, 0.0, 10.0]])
    kt, j, t, inside = Fn.spline_brackets(kn, kf)
    for x, jj, tt in zip(kf, j, t):
        xc = min(max(x, kn[0]), kn[-1])
        seg = 30
        for s in range(31):
            if kn[s] <= xc < kn[s + 1]:
                seg = s
                break
        assert jj == seg
        assert abs(tt - (xc - kn[seg]) / (kn[seg + 1] - kn[seg])) < 1e-14
        # the hat weights reproduce k~ itself (linear interpolation is exact
        # for a function linear in k)
        assert abs((1 - tt) * kn[seg] + tt * kn[seg + 1] - xc) < 1e-14 * max(1.0, xc)
