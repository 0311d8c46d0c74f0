"""Pins of the oracle's real-time TD-OFDFT (Section "Time-Dependent OFDFT",
eqs. "heq" and "cn"):

* a plane wave on a uniform density is an eigenstate of H with energy
  |G|^2/2 + (5/3) C_TF rho0^(2/3) (the kinetic term of eq. "heq" and the TF
  potential; Hartree vanishes for a uniform density), and one
  Crank-Nicolson step multiplies it by (1 - i E dt/2) / (1 + i E dt/2):
  this fixes the sign of the time step and the kinetic convention;
* Crank-Nicolson is unitary for a Hermitian H: the number of electrons is
  conserved, with and without correctors;
* with H fixed, a step of -dt undoes a step of dt;
* the solved step satisfies its linear system when H is applied through the
  FFT rather than the dense matrix;
* Ehrenfest: right after the kick exp(-i k.r) the dipole moves at
  d mu / dt = -k N_e (the current rho grad S with S = -k.r)."""
import numpy as np
import pytest

from oracle import cell as OC
from oracle import functionals as OF
from oracle import tdofdft as TD
from tests.oracle_helpers import box_cell

LOCAL = OC.TF | OC.VW | OC.HARTREE | OC.EXT


def gaussian_cell(n=(12, 12, 12), L=(11.0, 11.0, 11.0), sigma=1.1, nelec=2.0):
    cell = box_cell(L=L, n=n, pos=[[L[0] / 2, L[1] / 2, L[2] / 2]], Z=nelec, rc=1.0,
                    nelec=nelec)
    r = TD.positions(cell) - np.array(L) / 2
    rho = np.exp(-np.einsum("...d,...d->...", r, r) / (2 * sigma ** 2)) + 1e-10
    return cell, rho * nelec / (rho.sum() * cell.dv)


def test_plane_wave_phase_per_step():
    L = (8.0, 9.0, 10.0)
    cell = box_cell(L=L, n=(8, 12, 10), pos=None, nelec=4.0)
    func = OC.Functional(terms=OC.TF | OC.VW | OC.HARTREE)
    rho0 = cell.nelec / cell.volume
    G1 = cell.recip[0] + 2 * cell.recip[2]
    psi0 = TD.kick(cell, np.full(cell.n, rho0), -G1)          # sqrt(rho0) exp(+i G1.r)
    E = 0.5 * G1 @ G1 + 5.0 / 3.0 * OF.C_TF * rho0 ** (2.0 / 3.0)
    dt = 0.07
    psi = psi0
    for _ in range(3):
        psi = TD.step(cell, func, psi, dt, 1, np.zeros((8, 12, 6), complex))
    f = (1 - 0.5j * E * dt) / (1 + 0.5j * E * dt)
    np.testing.assert_allclose(psi, psi0 * f ** 3, rtol=0, atol=1e-12 * np.sqrt(rho0))


@pytest.mark.parametrize("ncorr", [0, 2])
def test_electron_number_is_conserved(ncorr):
    cell, rho = gaussian_cell(n=(10, 10, 12))
    func = OC.Functional(terms=LOCAL)
    psi, _ = TD.propagate(cell, func, TD.kick(cell, rho, [0.05, 0.0, 0.02]), 0.1, 2, ncorr)
    assert abs(cell.dv * np.sum(np.abs(psi) ** 2) - cell.nelec) <= 1e-12 * cell.nelec


def test_fixed_h_step_is_reversible_and_solves_its_system():
    cell, rho = gaussian_cell(n=(8, 10, 12))
    func = OC.Functional(terms=LOCAL)
    v = TD.potential(cell, func, rho, OF.vext_g(cell))
    psi0 = TD.kick(cell, rho, [0.1, -0.05, 0.0])
    dt = 0.2
    psi1 = TD.cn_step(cell, v, psi0, dt)
    lhs = psi1 + 0.5j * dt * TD.apply_h(cell, v, psi1)
    rhs = psi0 - 0.5j * dt * TD.apply_h(cell, v, psi0)
    assert np.abs(lhs - rhs).max() <= 1e-12
    back = TD.cn_step(cell, v, psi1, -dt)
    assert np.abs(back - psi0).max() <= 1e-12


def test_ehrenfest_dipole_velocity_after_the_kick():
    cell, rho = gaussian_cell(n=(12, 12, 12), sigma=1.0)
    func = OC.Functional(terms=LOCAL)
    k = np.array([0.02, 0.0, -0.01])
    mu0 = TD.dipole(cell, rho)
    slopes = []
    for dt in (0.02, 0.01):
        psi = TD.kick(cell, rho, k)
        _, mus = TD.propagate(cell, func, psi, dt, 1, 1)
        slopes.append((mus[0] - mu0) / dt)
    slope = 2 * slopes[1] - slopes[0]          # Richardson: removes the O(dt) term
    np.testing.assert_allclose(slope, -k * cell.nelec, rtol=0, atol=2e-3 * np.abs(k).max() *
                               cell.nelec)
