"""Pins of the oracle's LDA exchange-correlation (E_xc of eq. "efunc", the
Perdew-Zunger parametrisation the paper's applications use): the
high-density coefficient is the random-phase-approximation value
(1 - ln 2)/pi^2; the two branches of the fit meet at r_s = 1 in value and
slope (how the fit was built); Dirac exchange of the uniform gas is
-0.4582/r_s Ha; the potentials are the derivatives of rho eps by finite
differences; the uniform-gas energy is V rho eps."""
import numpy as np
import pytest

from oracle import cell as OC
from oracle import functionals as OF
from tests.oracle_helpers import make_cell
from paper_2002_02985_amd import workloads as W


def test_high_density_coefficient_is_the_rpa_value():
    assert abs(OF.PZ_A - (1.0 - np.log(2.0)) / np.pi ** 2) <= 5e-4 * OF.PZ_A


def test_branches_meet_at_rs_one():
    below, _ = OF.pz_correlation(np.array([1.0 - 1e-12]))
    above, _ = OF.pz_correlation(np.array([1.0]))
    assert abs(below[0] - above[0]) <= 1e-4
    h = 1e-6
    e = lambda r: OF.pz_correlation(np.array([r]))[0][0]
    d_lo = (e(1.0 - h) - e(1.0 - 2 * h)) / h
    d_hi = (e(1.0 + 2 * h) - e(1.0 + h)) / h
    assert abs(d_lo - d_hi) <= 1e-4


def test_dirac_exchange_of_the_uniform_gas():
    rs = np.array([0.5, 1.0, 2.0, 5.0])
    rho = 3.0 / (4.0 * np.pi * rs ** 3)
    eps, _ = OF.lda_xc(rho)
    ec, _ = OF.pz_correlation(rs)
    assert np.abs((eps - ec) * rs - (-0.458165293)).max() <= 1e-8


@pytest.mark.parametrize("rho0", [1e-6, 1e-3, 0.02, 0.3, 5.0])
def test_potential_is_the_derivative(rho0):
    f = lambda r: r * OF.lda_xc(np.array([r]))[0][0]
    h = 1e-6 * rho0
    dfd = (f(rho0 + h) - f(rho0 - h)) / (2 * h)
    _, v = OF.lda_xc(np.array([rho0]))
    assert abs(v[0] - dfd) <= 1e-7 * max(1.0, abs(dfd))


def test_zero_density_and_uniform_energy():
    eps, v = OF.lda_xc(np.array([0.0]))
    assert eps[0] == 0.0 and v[0] == 0.0
    cell = make_cell(W.al_fcc_cell(1, (12, 12, 12)))
    rho0 = 12.0 / cell.volume
    func = OC.Functional(terms=OC.XC)
    r = OF.energy_potential(cell, func, rho=np.full(cell.n, rho0))
    e0, v0 = OF.lda_xc(np.array([rho0]))
    assert abs(r.e_xc - cell.volume * rho0 * e0[0]) <= 1e-12 * abs(r.e_xc)
    assert np.abs(r.v - v0[0]).max() <= 1e-14
    assert abs(r.e_total - r.e_xc) <= 1e-12 * abs(r.e_xc)
