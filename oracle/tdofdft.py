"""Oracle real-time TD-OFDFT (TEST INFRASTRUCTURE ONLY).

Section "Time-Dependent OFDFT" of the paper: the collective orbital psi with
|psi|^2 = rho obeys i d psi / dt = H psi with

    H = -(1/2) nabla^2 + dT_Pauli/drho + v_s,   T_Pauli = T_s - T_vW,

(eq. "heq", adiabatic: the potential is that of the current density), and is
propagated with Crank-Nicolson (eq. "cn") with a predictor-corrector; the
system is displaced at t = 0 by the kick psi = sqrt(rho_0) exp(-i k.r) and
the observable is the dipole mu(t) = int r rho(r, t) dr.

Readings (the paper gives the scheme in words):
* dT_Pauli/drho + v_s is the functional derivative of every term of the
  functional except the von Weizsaecker one (whose coefficient must be 1:
  the Laplacian of H is that term);
* the Crank-Nicolson step follows the time-dependent equation as printed,
  (1 + i dt/2 H) psi(t + dt) = (1 - i dt/2 H) psi(t); the printed eq. "cn"
  has the two signs exchanged, which is the same step for -H;
* predictor: H built from rho(t); each corrector rebuilds H from the
  midpoint density (rho(t) + |psi_trial|^2) / 2 and solves the step again
  from psi(t); "any desired order" is the number of correctors;
* r is the Cartesian position of a grid point, sum_d (i_d / N_d) a_d (no
  wrapping), in the kick and in the dipole.

The linear system of each step is solved exactly: H is formed as a dense
matrix column by column (small grids only) and the system handed to
numpy.linalg.solve.
"""
import dataclasses

import numpy as np

from . import cell as C
from . import functionals as F
from .fourier import c2r, r2c


def positions(cell):
    """Cartesian position of every grid point, shape (N0, N1, N2, 3)."""
    n0, n1, n2 = cell.n
    i0, i1, i2 = np.meshgrid(np.arange(n0) / n0, np.arange(n1) / n1, np.arange(n2) / n2,
                             indexing="ij")
    frac = np.stack([i0, i1, i2], axis=-1)
    return frac @ cell.lattice


def potential(cell, func, rho, vext):
    """dT_Pauli/drho + v_s: the functional derivative of every term but vW."""
    f = dataclasses.replace(func, terms=func.terms & ~C.VW)
    return F.energy_potential(cell, f, rho=rho, vext=vext, e_ion=0.0).v


def laplacian(cell, f):
    """nabla^2 of a real field in the grid's Fourier convention."""
    return c2r(-C.g2(cell) * r2c(f), cell.n)


def apply_h(cell, v, psi):
    """H psi = -(1/2) nabla^2 psi + v psi for complex psi (real and imaginary
    parts transformed separately)."""
    lap = laplacian(cell, psi.real) + 1j * laplacian(cell, psi.imag)
    return -0.5 * lap + v * psi


def dense_h(cell, v):
    """H as an N x N complex matrix (column j = H e_j)."""
    N = cell.npts
    H = np.empty((N, N), dtype=np.complex128)
    e = np.zeros(N)
    for j in range(N):
        e[j] = 1.0
        H[:, j] = apply_h(cell, v, e.reshape(cell.n).astype(np.complex128)).reshape(N)
        e[j] = 0.0
    return H


def cn_step(cell, v, psi, dt):
    """Crank-Nicolson with H fixed: (1 + i dt/2 H) x = (1 - i dt/2 H) psi."""
    N = cell.npts
    H = dense_h(cell, v)
    A = np.eye(N) + 0.5j * dt * H
    b = psi.reshape(N) - 0.5j * dt * (H @ psi.reshape(N))
    return np.linalg.solve(A, b).reshape(cell.n)


def step(cell, func, psi, dt, n_corrector, vext):
    """One time step with the predictor and n_corrector corrector passes."""
    rho_n = np.abs(psi) ** 2
    trial = cn_step(cell, potential(cell, func, rho_n, vext), psi, dt)
    for _ in range(n_corrector):
        rho_mid = 0.5 * (rho_n + np.abs(trial) ** 2)
        trial = cn_step(cell, potential(cell, func, rho_mid, vext), psi, dt)
    return trial


def kick(cell, rho0, k):
    """psi(t = 0) = sqrt(rho_0) exp(-i k.r)."""
    kr = positions(cell) @ np.asarray(k, dtype=np.float64)
    return np.sqrt(rho0) * np.exp(-1j * kr)


def dipole(cell, rho):
    """mu = int r rho dr (3-vector)."""
    r = positions(cell)
    return cell.dv * np.einsum("ijkd,ijk->d", r, rho)


def propagate(cell, func, psi, dt, nsteps, n_corrector, vext=None):
    """nsteps steps; returns the final psi and the dipole after each step."""
    vext = F.vext_g(cell) if vext is None else vext
    mus = []
    for _ in range(nsteps):
        psi = step(cell, func, psi, dt, n_corrector, vext)
        mus.append(dipole(cell, np.abs(psi) ** 2))
    return psi, np.array(mus)
