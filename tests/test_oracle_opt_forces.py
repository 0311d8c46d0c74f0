"""Pins of the oracle's forces and density optimiser (CPU).

Forces: central finite differences of E_ext + E_ion in the atomic positions
at fixed density, and the vanishing net Ewald force.  Optimiser: jellium
stays uniform with mu = (5/3) C_TF rho0^(2/3); the linear response to a weak
cosine potential; exact electron-count conservation; monotone energy; and the
same minimum from different starting points.
"""
import numpy as np
import pytest

from oracle import cell as C
from oracle import functionals as Fn
from oracle.ewald import eion_forces, ewald_energy, ewald_forces, forces
from oracle.optimize import optimize
from tests.oracle_helpers import box_cell, grid_points, make_cell, smooth_density
from paper_2002_02985_amd import workloads as W


def _e_ext_ion(d, rho):
    cell = make_cell(d)
    r = Fn.energy_potential(cell, C.Functional(terms=C.EXT), rho=rho)
    return r.e_ext + r.e_ion


def test_forces_finite_difference():
    d = W.al_fcc_cell(1, (12, 12, 12), jitter=0.15, seed=21)
    cell = make_cell(d)
    rho = smooth_density(cell, seed=8)
    r = Fn.energy_potential(cell, C.Functional(terms=C.EXT), rho=rho)
    F = forces(cell, r.rho_g)
    h = 1e-5
    for a, k in [(0, 0), (1, 2), (3, 1)]:
        dp = dict(d)
        dp["pos"] = d["pos"].copy()
        dp["pos"][a, k] += h
        dm = dict(d)
        dm["pos"] = d["pos"].copy()
        dm["pos"][a, k] -= h
        fd = -(_e_ext_ion(dp, rho) - _e_ext_ion(dm, rho)) / (2 * h)
        assert abs(fd - F[a, k]) < 1e-7, (a, k, fd, F[a, k])


def test_ewald_forces_finite_difference_and_sum():
    d = W.al_fcc_cell(1, (8, 8, 8), jitter=0.2, seed=22)
    cell = make_cell(d)
    F = ewald_forces(cell)
    assert np.abs(F.sum(axis=0)).max() < 1e-10
    h = 1e-5
    for a, k in [(0, 1), (2, 0)]:
        p = cell.pos.copy()
        p[a, k] += h
        cp = C.Cell(cell.lattice, cell.n, p, cell.species, cell.Z, cell.rc, cell.nelec)
        p2 = cell.pos.copy()
        p2[a, k] -= h
        cm = C.Cell(cell.lattice, cell.n, p2, cell.species, cell.Z, cell.rc, cell.nelec)
        fd = -(ewald_energy(cp) - ewald_energy(cm)) / (2 * h)
        assert abs(fd - F[a, k]) < 1e-8


def test_perfect_lattice_forces_vanish_by_symmetry():
    d = W.al_fcc_cell(1, (16, 16, 16))
    cell = make_cell(d)
    rho = np.full(cell.n, cell.nelec / cell.volume)
    r = Fn.energy_potential(cell, C.Functional(terms=C.EXT), rho=rho)
    assert np.abs(forces(cell, r.rho_g)).max() < 1e-11


def test_jellium_stays_uniform():
    cell = box_cell(L=(6.0, 6.0, 6.0), n=(8, 8, 8), nelec=6.0)
    rho0 = cell.nelec / cell.volume
    rng = np.random.default_rng(5)
    phi0 = np.sqrt(rho0 * (1 + 0.05 * rng.standard_normal(cell.n)))
    out = optimize(cell, C.Functional(terms=C.TF | C.VW), phi0, tol=1e-10, max_iter=200)
    assert out.converged
    rho = out.phi ** 2
    np.testing.assert_allclose(rho, rho0, rtol=1e-8)
    assert abs(out.result.mu - 5.0 / 3.0 * Fn.C_TF * rho0 ** (2.0 / 3.0)) < 1e-9
    assert abs(cell.dv * rho.sum() - cell.nelec) < 1e-12
    assert all(b <= a + 1e-13 for a, b in zip(out.energies, out.energies[1:]))


def test_linear_response_to_weak_cosine_potential():
    cell = box_cell(L=(7.0, 7.0, 7.0), n=(12, 12, 12), nelec=8.0)
    rho0 = cell.nelec / cell.volume
    kf = (3 * np.pi ** 2 * rho0) ** (1 / 3)
    q = cell.recip[0]
    q2 = q @ q
    eps = 1e-4
    vx = np.zeros((12, 12, 7), dtype=complex)
    vx[1, 0, 0] = eps / 2      # v(r) = eps cos(q.r): +q and -q bins carry eps/2
    vx[11, 0, 0] = eps / 2
    func = C.Functional(terms=C.TF | C.VW | C.HARTREE | C.EXT)
    out = optimize(cell, func, np.full(cell.n, np.sqrt(rho0)), tol=1e-11, max_iter=200,
                   vext=vx, e_ion=0.0)
    assert out.converged
    from oracle.fourier import r2c
    drho_q = r2c(out.phi ** 2)[1, 0, 0].real
    k_tf = np.pi ** 2 / kf
    k_vw = q2 / (4 * rho0)
    expect = -(eps / 2) / (k_tf + k_vw + 4 * np.pi / q2)
    assert abs(drho_q / expect - 1) < 1e-3   # O(eps) nonlinearity


def test_optimum_independent_of_start_and_conserves_charge():
    d = W.al_fcc_cell(1, (12, 12, 12), jitter=0.05, seed=1)
    cell = make_cell(d)
    func = C.Functional(terms=C.TF | C.VW | C.HARTREE | C.EXT)
    vx = Fn.vext_g(cell)
    ei = ewald_energy(cell)
    outs = []
    for seed in (1, 2):
        rng = np.random.default_rng(seed)
        phi0 = np.sqrt(cell.nelec / cell.volume * (1 + 0.05 * rng.standard_normal(cell.n)))
        outs.append(optimize(cell, func, phi0, tol=1e-8, max_iter=400, vext=vx, e_ion=ei))
    for o in outs:
        assert o.converged
        assert abs(cell.dv * np.sum(o.phi ** 2) - cell.nelec) < 1e-11
        assert all(b <= a + 1e-12 for a, b in zip(o.energies, o.energies[1:]))
    assert abs(outs[0].result.e_total - outs[1].result.e_total) < 1e-10
    np.testing.assert_allclose(outs[0].phi ** 2, outs[1].phi ** 2, atol=1e-6)
