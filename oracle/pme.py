"""Oracle smooth particle-mesh Ewald structure factor (TEST INFRASTRUCTURE ONLY).

For large cells the paper computes the ionic structure factor with the
smooth particle-mesh Ewald (PME) method of Essmann et al. (J. Chem. Phys. 103,
8577 (1995)), Sections "OFDFT software background" and "Leveraging existing
techniques"; it prints none of the formulas.  This module writes that method
out from its published definition, in plain NumPy loops:

* cardinal B-spline of order n: M_2(x) = 1 - |x - 1| on [0, 2], 0 elsewhere;
  M_n(x) = x/(n-1) M_{n-1}(x) + (n-x)/(n-1) M_{n-1}(x-1);
* Euler exponential spline: for scaled coordinate u = K s (s fractional),
  exp(2 pi i m u / K) ~= b(m) sum_k M_n(u - k) exp(2 pi i m k / K), with
  b(m) = exp(2 pi i (n-1) m / K) / sum_{k=0}^{n-2} M_n(k+1) exp(2 pi i m k / K);
* so the structure factor of this code's sign, S(G) = sum_a exp(-i G.R_a) =
  sum_a exp(-2 pi i m.s_a), is conj(b_0 b_1 b_2)(m) times the unnormalised
  forward DFT of the charge grid Q(k) = sum_a prod_d M_n(u_{a,d} - k_d), the
  B-splines wrapped periodically.

Reading (the paper names the method only): the order n is even, since for odd
n the denominator of b vanishes at the Nyquist frequency m = K/2.
"""
import numpy as np

from . import cell as C
from .fourier import r2c
from .functionals import vloc_g

PI = np.pi


def bspline(n, x):
    """Cardinal B-spline M_n(x) (elementwise), by the two-term recursion."""
    x = np.asarray(x, dtype=np.float64)
    if n == 2:
        return np.where((x >= 0.0) & (x <= 2.0), 1.0 - np.abs(x - 1.0), 0.0)
    return (x * bspline(n - 1, x) + (n - x) * bspline(n - 1, x - 1.0)) / (n - 1)


def bfactor(K, n):
    """b(m) of the exponential spline for m = 0 .. K-1 (complex)."""
    m = np.arange(K)
    k = np.arange(n - 1)
    den = np.exp(2j * PI * np.outer(m, k) / K) @ bspline(n, k + 1.0)
    return np.exp(2j * PI * (n - 1) * m / K) / den


def charge_grid(shape, frac, order):
    """Q(k) = sum_a prod_d M_n(u_{a,d} - k_d), u = K s, wrapped periodically:
    atom a touches the n grid points k_d = floor(u_d) - j, j = 0 .. n-1, with
    weight M_n(u_d - floor(u_d) + j)."""
    K = np.array(shape)
    Q = np.zeros(shape)
    for s in np.asarray(frac, dtype=np.float64):
        u = K * (s - np.floor(s))
        base = np.floor(u).astype(np.int64)
        w = [bspline(order, u[d] - base[d] + np.arange(order)) for d in range(3)]
        idx = [(base[d] - np.arange(order)) % K[d] for d in range(3)]
        Q[np.ix_(idx[0], idx[1], idx[2])] += (w[0][:, None, None] * w[1][None, :, None] *
                                              w[2][None, None, :])
    return Q


def structure_factor(cell, atoms, order):
    """S(G) = sum_{a in atoms} exp(-i G.R_a) on the half spectrum by smooth PME."""
    n0, n1, n2 = cell.n
    frac = cell.fractional()[atoms] if len(atoms) else np.zeros((0, 3))
    Q = charge_grid(cell.n, frac, order)
    F = r2c(Q) * float(n0 * n1 * n2)         # sum_k Q(k) exp(-2 pi i m.k / K)
    b0 = np.conj(bfactor(n0, order))
    b1 = np.conj(bfactor(n1, order))
    b2 = np.conj(bfactor(n2, order))[: n2 // 2 + 1]
    return F * b0[:, None, None] * b1[None, :, None] * b2[None, None, :]


def structure_factor_direct(cell, atoms):
    """The exact sum, S(G) = sum_{a in atoms} exp(-i G.R_a), on the half spectrum."""
    G = C.gvectors(cell)
    S = np.zeros(G.shape[:-1], dtype=np.complex128)
    for a in atoms:
        S += np.exp(-1j * (G @ cell.pos[a]))
    return S


def vext_g(cell, order):
    """v_ext(G) = (1/V) sum_s v_s(|G|) S_s(G) with each species' S_s by PME
    (the local pseudopotential of eq. "efunc")."""
    G = C.gvectors(cell)
    G2 = np.einsum("...i,...i->...", G, G)
    out = np.zeros(G2.shape, dtype=np.complex128)
    for s in range(len(cell.Z)):
        idx = np.nonzero(cell.species == s)[0]
        if idx.size == 0:
            continue
        out += vloc_g(cell, G2, s) * structure_factor(cell, idx, order)
    return out / cell.volume

