"""Pins of the oracle's energy terms (CPU).

Every term is pinned to something other than its own formula: closed forms
(uniform densities, single plane waves), literature constants (Madelung
constants, the Thomas-Fermi constant), arbitrary-precision evaluation of the
printed Lindhard function, radial quadrature of the pseudopotential's
Fourier transform, translation invariance, the Lindhard linear response that
TF + vW + WT must reproduce, and central finite differences of every
potential.
"""
import mpmath
import numpy as np
import pytest
from scipy import integrate, special

from oracle import cell as C
from oracle import functionals as Fn
from oracle.ewald import ewald_energy
from oracle.fourier import c2r, r2c
from tests.oracle_helpers import box_cell, grid_points, make_cell, smooth_density
from paper_2002_02985_amd import workloads as W


def only(terms, **kw):
    return C.Functional(terms=terms, **kw)


# --------------------------------------------------------------- constants
def test_constants_literature_values():
    # C_TF = (3/10)(3 pi^2)^(2/3) = 2.871234..., C_WT = (6/25)(3 pi^2)^(2/3)
    assert abs(Fn.C_TF - 2.871234000188) < 1e-11
    assert abs(Fn.C_WT - 2.296987200151) < 1e-11


# --------------------------------------------------------------- TF
def test_tf_uniform_closed_form():
    cell = make_cell(W.al_fcc_cell(1, (32, 32, 32)))
    rho0 = 12.0 / 7.65 ** 3
    r = Fn.energy_potential(cell, only(C.TF), rho=np.full(cell.n, rho0))
    # C1 uniform density: E_TF = 3.085895 Ha, mu = (5/3) C_TF rho0^(2/3) = 0.428597 Ha
    assert abs(r.e_tf - 3.085895) < 1e-6
    assert abs(r.mu - 0.428597) < 1e-6
    assert r.resid_norm < 1e-14


# --------------------------------------------------------------- vW
def test_vw_uniform_is_zero_and_cosine_closed_form():
    cell = box_cell(n=(12, 10, 16))
    phi0 = 0.2
    r = Fn.energy_potential(cell, only(C.VW), phi=np.full(cell.n, phi0))
    assert abs(r.e_vw) < 1e-15
    pts = grid_points(cell)
    q = 2 * cell.recip[1] + cell.recip[2]
    a = 0.03
    phi = phi0 + a * np.cos(pts @ q)
    r = Fn.energy_potential(cell, only(C.VW), phi=phi)
    assert abs(r.e_vw - a * a * (q @ q) * cell.volume / 4.0) < 1e-13


# --------------------------------------------------------------- Hartree
def test_hartree_plane_wave_closed_form():
    cell = box_cell(n=(12, 10, 16))
    pts = grid_points(cell)
    q = cell.recip[0] - 3 * cell.recip[2]
    rho0, A = 0.02, 0.005
    r = Fn.energy_potential(cell, only(C.HARTREE), rho=rho0 + A * np.cos(pts @ q))
    assert abs(r.e_h - np.pi * cell.volume * A * A / (q @ q)) < 1e-13
    r = Fn.energy_potential(cell, only(C.HARTREE), rho=np.full(cell.n, rho0))
    assert abs(r.e_h) < 1e-15
    # v_H = 4 pi A cos(q.r)/q^2 solves Poisson's equation for the perturbation
    r = Fn.energy_potential(cell, only(C.HARTREE), rho=rho0 + A * np.cos(pts @ q))
    np.testing.assert_allclose(r.v, 4 * np.pi * A / (q @ q) * np.cos(pts @ q), atol=1e-13)


# --------------------------------------------------------------- pseudopotential
def test_pseudopotential_form_factor_by_radial_quadrature():
    # v(G) + 4 pi Z / G^2 must be the transform of Z erfc(r/rc)/r:
    # 4 pi int_0^inf r^2 [Z erfc(r/rc)/r] sin(G r)/(G r) dr
    Z, rc = 3.0, 1.0
    cell = box_cell(Z=Z, rc=rc, pos=[[0, 0, 0]])
    for G in (0.3, 1.0, 2.5, 4.0):
        f = lambda r: 4 * np.pi * Z * special.erfc(r / rc) * np.sin(G * r) / G
        val, _ = integrate.quad(f, 0, 12 * rc, limit=400)
        vg = Fn.vloc_g(cell, np.array([G * G]), 0)[0]
        assert abs((vg + 4 * np.pi * Z / G ** 2) - val) < 1e-9
    # G = 0: int Z erfc(r/rc)/r d^3r = pi Z rc^2
    val, _ = integrate.quad(lambda r: 4 * np.pi * r * Z * special.erfc(r / rc), 0, 12 * rc)
    assert abs(Fn.vloc_g(cell, np.array([0.0]), 0)[0] - val) < 1e-10


def test_single_atom_at_origin_gives_real_form_factor():
    cell = box_cell(pos=[[0.0, 0.0, 0.0]])
    vx = Fn.vext_g(cell)
    G2 = C.g2(cell)
    assert np.abs(vx.imag).max() < 1e-15
    np.testing.assert_allclose(vx.real, Fn.vloc_g(cell, G2, 0) / cell.volume, rtol=1e-14)


def test_vext_translation_by_grid_steps():
    d = W.al_fcc_cell(1, (16, 16, 16), jitter=0.1, seed=4)
    cell = make_cell(d)
    v0 = c2r(Fn.vext_g(cell), cell.n)
    shift = np.array([3, -2, 5])
    d2 = dict(d)
    d2["pos"] = d["pos"] + (shift / np.array(cell.n)) @ cell.lattice
    v1 = c2r(Fn.vext_g(make_cell(d2)), cell.n)
    np.testing.assert_allclose(np.roll(v0, shift, axis=(0, 1, 2)), v1, atol=1e-12)


def test_vext_direct_sum_equals_per_atom_bruteforce():
    # direct structure factor sum vs an independent per-atom accumulation of
    # real-space potentials (each atom's potential is its form factor
    # translated; summing those equals the structure-factor sum)
    d = W.al_fcc_cell(1, (12, 12, 12), jitter=0.2, seed=5)
    cell = make_cell(d)
    vx = c2r(Fn.vext_g(cell), cell.n)
    G = C.gvectors(cell)
    G2 = C.g2(cell)
    acc = np.zeros(cell.n)
    pts = grid_points(cell)
    for a in range(len(cell.pos)):
        # v_a(r) = (1/V) sum_G v(G) e^{iG.(r - R_a)} computed point by point
        ff = Fn.vloc_g(cell, G2, 0) / cell.volume
        w = C.weights(cell)
        ph = np.exp(1j * (np.tensordot(pts, G, axes=([3], [3])) - (G @ cell.pos[a])))
        acc += np.real(np.tensordot(ph, w * ff, axes=([3, 4, 5], [0, 1, 2])))
    np.testing.assert_allclose(vx, acc, atol=1e-11)


# --------------------------------------------------------------- Ewald
@pytest.mark.parametrize("name,basis,ref,tol", [
    ("bcc", [[0, 0, 0], [.5, .5, .5]], 0.895929255682, 1e-11),
    ("fcc", [[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], 0.895873615195, 1e-11),
    ("sc", [[0, 0, 0]], 0.88005944, 1e-8),
])
def test_ewald_madelung_constants(name, basis, ref, tol):
    # point charges in a neutralising background: E/ion = -M Z^2 / r_ws
    a = 2.3
    cell = C.Cell(lattice=np.eye(3) * a, n=(4, 4, 4), pos=np.array(basis) * a,
                  species=np.zeros(len(basis), int), Z=[1.0], rc=[1.0], nelec=len(basis))
    rws = (3 * cell.volume / len(basis) / (4 * np.pi)) ** (1 / 3)
    assert abs(-ewald_energy(cell) / len(basis) * rws - ref) < tol


def test_ewald_split_parameter_independence():
    cell = make_cell(W.al_fcc_cell(1, (8, 8, 8), jitter=0.2, seed=7))
    e = [ewald_energy(cell, eta=x) for x in (0.05, 0.2, 1.0)]
    assert max(e) - min(e) < 1e-11


# --------------------------------------------------------------- Lindhard G_NL
def _gnl_mp(eta):
    mpmath.mp.dps = 60
    e = mpmath.mpf(eta)
    if e == 0:
        return mpmath.mpf(0)
    if e == 1:
        F = mpmath.mpf(1) / 2
    else:
        F = mpmath.mpf(1) / 2 + (1 - e * e) / (4 * e) * mpmath.log(abs((1 + e) / (1 - e)))
    return 1 / F - 3 * e * e - 1


def test_gnl_against_arbitrary_precision_definition():
    etas = np.concatenate([[1e-6, 1e-3, 0.1, 0.5, 0.9, 0.999, 1.001, 1.2, 1.49, 1.5, 1.51,
                            2.0, 3.0, 10.0, 100.0, 1e4],
                           np.random.default_rng(0).uniform(0, 5, 200)])
    got = Fn.gnl(etas)
    ref = np.array([float(_gnl_mp(float(x))) for x in etas])
    assert np.abs(got - ref).max() < 5e-15


def test_gnl_special_values_and_series():
    assert Fn.gnl(np.array([0.0]))[0] == 0.0
    assert abs(Fn.gnl(np.array([1.0]))[0] + 2.0) < 1e-15
    assert abs(Fn.gnl(np.array([1e8]))[0] + 1.6) < 1e-14
    e = 1e-2
    assert abs(Fn.gnl(np.array([e]))[0] - (-8 * e ** 2 / 3 + 8 * e ** 4 / 45 + 104 * e ** 6 / 945)) < 1e-16
    e = 50.0
    assert abs(Fn.gnl(np.array([e]))[0] - (-1.6 - 24 / (175 * e * e) - 8 / (125 * e ** 4))) < 1e-11


# --------------------------------------------------------------- WT
def test_wt_uniform_density_zero():
    cell = box_cell(n=(10, 12, 14), nelec=5.0)
    r = Fn.energy_potential(cell, only(C.WT), rho=np.full(cell.n, cell.nelec / cell.volume))
    assert abs(r.e_nl) < 1e-15
    assert np.abs(r.v).max() < 1e-15


def test_lindhard_response_of_tf_vw_wt():
    # rho = rho0 + eps cos(q.r): Delta E_{TF+vW+WT} = (V eps^2 / 4) (pi^2/k_F) / F(eta)
    # with F the bracket of the printed G_NL (evaluated here in mpmath).
    cell = make_cell(W.al_fcc_cell(1, (32, 32, 32)))
    rho0 = cell.nelec / cell.volume
    kf = (3 * np.pi ** 2 * rho0) ** (1 / 3)
    pts = grid_points(cell)
    q = cell.recip[0]
    func = only(C.TF | C.VW | C.WT)
    e0 = Fn.energy_potential(cell, func, rho=np.full(cell.n, rho0)).e_total

    def de(eps):
        return Fn.energy_potential(cell, func, rho=rho0 + eps * np.cos(pts @ q)).e_total - e0

    eps = 1e-3 * rho0
    k1 = de(eps) / (cell.volume * eps ** 2 / 4)
    k2 = de(eps / 2) / (cell.volume * (eps / 2) ** 2 / 4)
    k_num = (4 * k2 - k1) / 3          # Richardson: removes the eps^2 term of K(eps)
    eta = np.sqrt(q @ q) / (2 * kf)
    mpmath.mp.dps = 40
    e = mpmath.mpf(eta)
    F = 0.5 + (1 - e * e) / (4 * e) * mpmath.log(abs((1 + e) / (1 - e)))
    k_ref = np.pi ** 2 / kf / float(F)
    assert abs(eta - 0.44356) < 1e-5 and abs(float(F) - 0.93159) < 1e-5
    assert abs(k_num / k_ref - 1) < 1e-6


# --------------------------------------------------------------- finite differences
FD_CASES = {
    "tf": C.TF,
    "vw": C.VW,
    "hartree": C.HARTREE,
    "ext": C.EXT,
    "wt": C.WT,
    "all_local": C.TF | C.VW | C.HARTREE | C.EXT,
}


@pytest.mark.parametrize("name", sorted(FD_CASES))
def test_potential_finite_difference(name):
    d = W.al_fcc_cell(1, (12, 12, 12), jitter=0.1, seed=11)
    cell = make_cell(d)
    func = only(FD_CASES[name])
    rho = smooth_density(cell, seed=3)
    rng = np.random.default_rng(4)
    dirn = smooth_density(cell, seed=5) * rng.uniform(0.5, 1.5) - rho  # smooth direction
    r = Fn.energy_potential(cell, func, rho=rho)
    h = 1e-4
    ep = Fn.energy_potential(cell, func, rho=rho + h * dirn).e_total
    em = Fn.energy_potential(cell, func, rho=rho - h * dirn).e_total
    fd = (ep - em) / (2 * h)
    an = cell.dv * np.sum(r.v * dirn)
    assert abs(fd - an) < 1e-7 * max(1.0, abs(an))
    # the phi form: dE/dphi = g
    phi = np.sqrt(rho)
    dphi = np.cos(grid_points(cell) @ cell.recip[1]) * 0.01
    rp = Fn.energy_potential(cell, func, phi=phi + h * dphi).e_total
    rm = Fn.energy_potential(cell, func, phi=phi - h * dphi).e_total
    an = cell.dv * np.sum(r.g * dphi)
    assert abs((rp - rm) / (2 * h) - an) < 1e-7 * max(1.0, abs(an))


def test_residual_and_mu_definitions():
    cell = make_cell(W.al_fcc_cell(1, (12, 12, 12)))
    rho = smooth_density(cell, seed=9)
    r = Fn.energy_potential(cell, only(C.TF | C.VW | C.HARTREE | C.EXT), rho=rho)
    mu = np.sum(r.v * rho) / np.sum(rho)
    assert abs(r.mu - mu) < 1e-12
    R = 2 * np.sqrt(rho) * (r.v - mu)
    assert abs(r.resid_norm - np.sqrt(np.mean(R * R))) < 1e-12
    assert abs(r.nelec_int - cell.nelec) < 1e-12
