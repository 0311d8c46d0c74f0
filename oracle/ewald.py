"""Oracle ion-ion energy and ionic forces (TEST INFRASTRUCTURE ONLY).

The paper's total energy (eq. "efunc") is the electronic part; the ion-ion
term needed for a total energy and for forces (the DFTpy+ASE molecular
dynamics of Section "DFTpy+ASE") is the standard Ewald sum of point charges
Z_a in a neutralising background.  The e-ion force is the Hellmann-Feynman
derivative of int v_ext rho at fixed rho.
"""
import itertools

import numpy as np
from scipy.special import erfc

from . import cell as C
from .functionals import vloc_g

PI = np.pi


def _default_eta(cell):
    return (PI / cell.volume ** (1.0 / 3.0)) ** 2


def _charges(cell):
    return cell.Z[cell.species]


def _real_images(cell, eta, tol=1e-17):
    # erfc(sqrt(eta) r) < tol  ->  sqrt(eta) r > ~6.5
    rcut = 6.6 / np.sqrt(eta)
    lat = cell.lattice
    # number of images along each direction: distance between lattice planes
    recip = cell.recip
    nmax = [int(np.ceil(rcut * np.linalg.norm(recip[d]) / (2 * PI))) + 1 for d in range(3)]
    rng = [range(-n, n + 1) for n in nmax]
    L = np.array([np.array(t) @ lat for t in itertools.product(*rng)])
    return L, rcut


def _recip_set(cell, eta):
    gcut = 2.0 * np.sqrt(eta) * 6.6
    b = cell.recip
    lat = cell.lattice
    nmax = [int(np.ceil(gcut * np.linalg.norm(lat[d]) / (2 * PI))) + 1 for d in range(3)]
    rng = [range(-n, n + 1) for n in nmax]
    G = np.array([np.array(t) @ b for t in itertools.product(*rng)])
    G2 = np.einsum("ij,ij->i", G, G)
    keep = (G2 > 0) & (G2 <= gcut * gcut)
    return G[keep], G2[keep]


def ewald_energy(cell, eta=None):
    """E_ion = 1/2 sum_{a,b,L}' Z_a Z_b erfc(sqrt(eta) d)/d
             + (2 pi / V) sum_{G != 0} exp(-G^2/(4 eta)) / G^2 |S(G)|^2
             - sqrt(eta/pi) sum Z_a^2 - pi (sum Z_a)^2 / (2 V eta),
    S(G) = sum_a Z_a exp(i G.R_a).  Independent of eta (split parameter)."""
    if len(cell.pos) == 0:
        return 0.0
    eta = _default_eta(cell) if eta is None else eta
    Z = _charges(cell)
    R = cell.pos
    V = cell.volume
    L, rcut = _real_images(cell, eta)
    e_real = 0.0
    for a in range(len(R)):
        d = R[a][None, None, :] - R[None, :, :] - L[:, None, :]   # (nL, natoms, 3)
        r = np.linalg.norm(d, axis=-1)
        mask = (r > 1e-10) & (r < rcut)
        zz = Z[a] * Z[None, :] * np.ones_like(r)
        e_real += 0.5 * float(np.sum(zz[mask] * erfc(np.sqrt(eta) * r[mask]) / r[mask]))
    G, G2 = _recip_set(cell, eta)
    S = np.exp(1j * (G @ R.T)) @ Z
    e_rec = 2.0 * PI / V * float(np.sum(np.exp(-G2 / (4.0 * eta)) / G2 * np.abs(S) ** 2))
    e_self = -np.sqrt(eta / PI) * float(np.sum(Z * Z))
    e_bg = -PI * float(np.sum(Z)) ** 2 / (2.0 * V * eta)
    return e_real + e_rec + e_self + e_bg


def ewald_forces(cell, eta=None):
    """F_a = -dE_ion/dR_a (natoms x 3)."""
    natoms = len(cell.pos)
    F = np.zeros((natoms, 3))
    if natoms == 0:
        return F
    eta = _default_eta(cell) if eta is None else eta
    Z = _charges(cell)
    R = cell.pos
    V = cell.volume
    L, rcut = _real_images(cell, eta)
    se = np.sqrt(eta)
    for a in range(natoms):
        d = R[a][None, None, :] - R[None, :, :] - L[:, None, :]
        r = np.linalg.norm(d, axis=-1)
        mask = (r > 1e-10) & (r < rcut)
        rr = np.where(mask, r, 1.0)
        mag = erfc(se * rr) / rr ** 2 + 2.0 * se / np.sqrt(PI) * np.exp(-eta * rr * rr) / rr
        coef = np.where(mask, Z[a] * Z[None, :] * mag / rr, 0.0)
        F[a] = np.einsum("lb,lbi->i", coef, d)
    G, G2 = _recip_set(cell, eta)
    ph = np.exp(1j * (G @ R.T))          # (nG, natoms)
    S = ph @ Z
    pref = 4.0 * PI / V * np.exp(-G2 / (4.0 * eta)) / G2
    im = np.imag(ph * np.conj(S)[:, None])   # Im[e^{iG.R_a} conj(S)]
    F += (Z[None, :] * im * pref[:, None]).T @ G
    return F


def eion_forces(cell, rho_g):
    """Hellmann-Feynman e-ion force at fixed rho:
    F_a = sum_half c(m2) G v_{s(a)}(|G|) Im[exp(i G.R_a) rho(G)],
    the exact derivative of int v_ext rho = V sum_half c Re[conj(v_ext(G)) rho(G)]."""
    G = C.gvectors(cell)
    G2 = np.einsum("...i,...i->...", G, G)
    w = C.weights(cell)
    F = np.zeros((len(cell.pos), 3))
    for a in range(len(cell.pos)):
        vs = vloc_g(cell, G2, cell.species[a])
        ph = np.exp(1j * (G @ cell.pos[a]))
        s = w * vs * np.imag(ph * rho_g)
        F[a] = np.tensordot(s, G, axes=([0, 1, 2], [0, 1, 2]))
    return F


def forces(cell, rho_g):
    """Total force on each ion: e-ion (Hellmann-Feynman) plus Ewald."""
    return eion_forces(cell, rho_g) + ewald_forces(cell)
