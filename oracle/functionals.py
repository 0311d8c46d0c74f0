"""Oracle energy terms and potentials (TEST INFRASTRUCTURE ONLY).

Each function states the passage of the paper it follows.  Everything is FP64
NumPy on the CPU, with the oracle's own FFT (``oracle.fourier``).  Potentials
are functional derivatives: v(r) = dE/drho(r) (density form) and
g(r) = dE/dphi(r) (the psi = sqrt(rho) form of eq. "euler2").
"""
import dataclasses

import numpy as np

from . import cell as C
from .fourier import c2r, r2c

PI = np.pi
# Thomas-Fermi constant (3/10)(3 pi^2)^(2/3): the textbook TF functional that
# the paper names (Table "tlmgp", Section "Linear scalability") without
# printing its formula.
C_TF = 0.3 * (3.0 * PI * PI) ** (2.0 / 3.0)
# Wang-Teter constant (6/25)(3 pi^2)^(2/3), eq. "WT".
C_WT = 6.0 / 25.0 * (3.0 * PI * PI) ** (2.0 / 3.0)


# ---------------------------------------------------------------------------
# LDA exchange-correlation (E_xc of eq. "efunc"; the applications of Section
# "Linear scalability" and the TD-OFDFT section use the Perdew-Zunger
# parametrisation).  Spin-unpolarised homogeneous electron gas at the local
# density: Dirac exchange and the Perdew-Zunger (1981) fit of the
# Ceperley-Alder correlation energy, whose parameters are those published by
# Perdew and Zunger (Phys. Rev. B 23, 5048, Appendix C); the paper cites that
# work and does not print them.
# ---------------------------------------------------------------------------
PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334      # r_s >= 1
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116    # r_s < 1
C_X = -0.75 * (3.0 / PI) ** (1.0 / 3.0)                     # eps_x = C_X rho^(1/3)


def pz_correlation(rs):
    """Correlation energy per electron eps_c(r_s) and its potential
    v_c = eps_c - (r_s/3) d eps_c/d r_s (both Ha), elementwise."""
    rs = np.asarray(rs, dtype=np.float64)
    ec = np.empty_like(rs)
    vc = np.empty_like(rs)
    lo = rs >= 1.0
    r = rs[lo]
    sq = np.sqrt(r)
    den = 1.0 + PZ_BETA1 * sq + PZ_BETA2 * r
    ec[lo] = PZ_GAMMA / den
    vc[lo] = ec[lo] * (1.0 + 7.0 / 6.0 * PZ_BETA1 * sq + 4.0 / 3.0 * PZ_BETA2 * r) / den
    r = rs[~lo]
    lr = np.log(r)
    ec[~lo] = PZ_A * lr + PZ_B + PZ_C * r * lr + PZ_D * r
    vc[~lo] = (PZ_A * lr + (PZ_B - PZ_A / 3.0) + 2.0 / 3.0 * PZ_C * r * lr +
               (2.0 * PZ_D - PZ_C) / 3.0 * r)
    return ec, vc


def lda_xc(rho):
    """eps_xc(rho) (energy per electron) and v_xc = d(rho eps_xc)/d rho;
    both vanish at rho = 0."""
    rho = np.asarray(rho, dtype=np.float64)
    eps = np.zeros_like(rho)
    v = np.zeros_like(rho)
    pos = rho > 0.0
    r3 = np.cbrt(rho[pos])
    ex = C_X * r3
    rs = (3.0 / (4.0 * PI)) ** (1.0 / 3.0) / r3
    ec, vc = pz_correlation(rs)
    eps[pos] = ex + ec
    v[pos] = 4.0 / 3.0 * ex + vc
    return eps, v


# ---------------------------------------------------------------------------
# Lindhard function (Section "New-generation nonlocal KEDFs", the G_NL formula)
# ---------------------------------------------------------------------------
_NSER = 64


def lindhard_F(eta):
    """F(eta) = 1/2 + (1 - eta^2)/(4 eta) ln|(1 + eta)/(1 - eta)|, the bracket
    inverted in G_NL.  F(0) = 1, F(1) = 1/2.

    Written with ln|(1+eta)/(1-eta)| = 2 atanh(eta) for eta < 1 and
    2 atanh(1/eta) for eta > 1; for eta >= 1.5 the equivalent series
    F = sum_{n>=1} x^n / ((2n-1)(2n+1)), x = 1/eta^2, avoids the cancellation
    between 1/2 and the logarithm term.
    """
    eta = np.asarray(eta, dtype=np.float64)
    out = np.empty_like(eta)
    z = eta == 0.0
    lo = (eta > 0.0) & (eta < 1.0)
    one = eta == 1.0
    mid = (eta > 1.0) & (eta < 1.5)
    hi = eta >= 1.5
    out[z] = 1.0
    e = eta[lo]
    out[lo] = 0.5 + (1.0 - e * e) / (2.0 * e) * np.arctanh(e)
    out[one] = 0.5
    e = eta[mid]
    out[mid] = 0.5 - (e * e - 1.0) / (2.0 * e) * np.arctanh(1.0 / e)
    x = 1.0 / (eta[hi] * eta[hi])
    acc = np.zeros_like(x)
    for n in range(_NSER, 0, -1):
        acc = acc * x + 1.0 / ((2.0 * n - 1.0) * (2.0 * n + 1.0))
    out[hi] = x * acc
    return out


def gnl(eta):
    """G_NL(eta) = 1/F(eta) - 3 eta^2 - 1 (the Lindhard-based kernel shape).

    G(0) = 0, G(1) = -2, G(inf) = -8/5.  For eta >= 1.5 the difference
    1/F - 3 eta^2 is formed without cancellation: with x = 1/eta^2,
    F = x P(x) and 3 eta^2 F = 1 + x S(x), so 1/F - 3 eta^2 = -S/P, where
    P = sum_{n>=1} x^(n-1)/((2n-1)(2n+1)) and
    S = sum_{n>=2} 3 x^(n-2)/((2n-1)(2n+1)).
    """
    eta = np.asarray(eta, dtype=np.float64)
    out = np.empty_like(eta)
    hi = eta >= 1.5
    lo = ~hi
    e = eta[lo]
    out[lo] = 1.0 / lindhard_F(e) - 3.0 * e * e - 1.0
    x = 1.0 / (eta[hi] * eta[hi])
    P = np.zeros_like(x)
    S = np.zeros_like(x)
    for n in range(_NSER, 0, -1):
        P = P * x + 1.0 / ((2.0 * n - 1.0) * (2.0 * n + 1.0))
    for n in range(_NSER, 1, -1):
        S = S * x + 3.0 / ((2.0 * n - 1.0) * (2.0 * n + 1.0))
    out[hi] = -1.0 - S / P
    return out


def wt_kernel(gnorm, kf):
    """omega(q) = C_WT G_NL(q / (2 k_F)) (eq. "WT"); omega(0) = 0."""
    return C_WT * gnl(np.asarray(gnorm) / (2.0 * kf))


def nl_kernel(gnorm, kf, kind):
    """The nonlocal kernel omega(|G|; k_F) of the selected family: Wang-Teter
    (eq. "WT") or one of MGP / MGPA / MGPG (eq. "MGP", oracle.mgp)."""
    if kind == 0:
        return wt_kernel(gnorm, kf)
    from . import mgp
    return mgp.kernel(gnorm, kf, kind)


# ---------------------------------------------------------------------------
# External potential through the ionic structure factor
# ---------------------------------------------------------------------------
def vloc_g(cell, gnorm2, species):
    """Local pseudopotential form factor of one species,
    v(G) = -4 pi Z exp(-G^2 rc^2 / 4) / G^2, i.e. the Fourier transform of
    -Z erf(r/rc)/r (per unit volume of the transform).  At G = 0 the
    non-Coulomb remainder pi Z rc^2 is kept (the Coulomb G = 0 part cancels
    against the Hartree and ion-ion background terms)."""
    Z = cell.Z[species]
    rc = cell.rc[species]
    out = np.empty_like(gnorm2)
    nz = gnorm2 > 0
    out[nz] = -4.0 * PI * Z * np.exp(-gnorm2[nz] * rc * rc / 4.0) / gnorm2[nz]
    out[~nz] = PI * Z * rc * rc
    return out


def vext_g(cell):
    """v_ext(G) = (1/V) sum_a v_{s(a)}(|G|) exp(-i G.R_a), the local
    pseudopotential (IONS term, eq. "efunc") through the exact direct
    structure-factor sum (Section "Leveraging existing techniques" discusses
    the structure factor)."""
    G = C.gvectors(cell)
    G2 = np.einsum("...i,...i->...", G, G)
    out = np.zeros(G2.shape, dtype=np.complex128)
    for s in range(len(cell.Z)):
        idx = np.nonzero(cell.species == s)[0]
        if idx.size == 0:
            continue
        sf = np.zeros(G2.shape, dtype=np.complex128)
        for a in idx:
            sf += np.exp(-1j * (G @ cell.pos[a]))
        out += vloc_g(cell, G2, s) * sf
    return out / cell.volume


# ---------------------------------------------------------------------------
# Spline helpers (steps s1, s4)
# ---------------------------------------------------------------------------
def kf_of_rho(rho):
    return np.cbrt(3.0 * PI * PI * rho)


def spline_brackets(kn, kf):
    """Bracket j and linear weight t of k~ = clamp(kf, k_1, k_Nk) on the knot
    set (step s4, linear in k).  An exact knot takes the segment to its right;
    the last knot takes the last segment with t = 1.  Returns
    (kt, j, t, inside) where inside marks points where the clamp is inactive."""
    k1, kn_ = kn[0], kn[-1]
    kt = np.clip(kf, k1, kn_)
    inside = (kf > k1) & (kf < kn_)
    nk = len(kn)
    if nk == 1:
        return kt, np.zeros(kt.shape, dtype=np.int64), np.zeros_like(kt), inside
    j = np.searchsorted(kn, kt, side="right") - 1
    j = np.clip(j, 0, nk - 2)
    t = (kt - kn[j]) / (kn[j + 1] - kn[j])
    return kt, j, t, inside


# ---------------------------------------------------------------------------
# The evaluator
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Result:
    e_tf: float = 0.0
    e_vw: float = 0.0
    e_h: float = 0.0
    e_ext: float = 0.0
    e_nl: float = 0.0
    e_ion: float = 0.0
    e_xc: float = 0.0
    e_total: float = 0.0
    mu: float = 0.0
    nelec_int: float = 0.0
    resid_norm: float = 0.0
    v: np.ndarray = None      # dE/drho with the density floor
    g: np.ndarray = None      # dE/dphi, division-free
    rho_g: np.ndarray = None  # r2c(rho), kept for forces


def _kf_wt(cell, func):
    if func.kf_wt > 0:
        return func.kf_wt
    return (3.0 * PI * PI * cell.nelec / cell.volume) ** (1.0 / 3.0)


def energy_potential(cell, func, rho=None, phi=None, vext=None, e_ion=None):
    """E[rho] and its derivatives for the terms in ``func.terms``.

    The energy is eq. "efunc":
      E = T_TF + T_vW + T_NL + E_H + E_xc + int v_ext rho (+ the constant E_ion),
    with E_xc the LDA (term XC, off by default).
    dE/drho - mu = 0 is eq. "euler"; in the psi form (eq. "euler2") the
    residual is R = dE/dphi - 2 mu phi with mu = int v rho / int rho.
    """
    if (rho is None) == (phi is None):
        raise ValueError("give exactly one of rho, phi")
    if phi is None:
        rho = np.asarray(rho, dtype=np.float64)
        phi = np.sqrt(np.maximum(rho, 0.0))
    else:
        phi = np.asarray(phi, dtype=np.float64)
        rho = phi * phi
    shape = cell.n
    dv = cell.dv
    V = cell.volume
    terms = func.terms
    floor = func.rho_floor
    rho_s = np.maximum(rho, floor)
    phi_fl = np.sqrt(floor)
    sgn = np.where(phi < 0.0, -1.0, 1.0)
    phi_s = sgn * np.maximum(np.abs(phi), phi_fl)
    absphi = np.abs(phi)

    G = C.gvectors(cell)
    G2 = np.einsum("...i,...i->...", G, G)
    gn = np.sqrt(G2)

    res = Result()
    v = np.zeros(shape)
    g = np.zeros(shape)
    res.nelec_int = dv * float(np.sum(rho))
    rho_g = r2c(rho)
    res.rho_g = rho_g

    if terms & C.TF:
        # Thomas-Fermi: C_TF int rho^(5/3), v = (5/3) C_TF rho^(2/3)
        res.e_tf = C_TF * dv * float(np.sum(rho ** (5.0 / 3.0)))
        vt = (5.0 / 3.0) * C_TF * rho ** (2.0 / 3.0)
        v += vt
        g += 2.0 * phi * vt

    if terms & C.VW:
        # von Weizsaecker (lambda = 1 in the paper): (1/2) int |grad phi|^2,
        # the Laplacian by FFT (Introduction; Section "Time-Dependent OFDFT"
        # names it as the term behind -1/2 nabla^2).
        lam = func.lambda_vw
        phi_g = r2c(phi)
        res.e_vw = lam * 0.5 * V * C.gsum(cell, G2 * np.abs(phi_g) ** 2)
        lap = c2r(G2 * phi_g, shape)          # -nabla^2 phi
        g += lam * lap
        v += lam * 0.5 * lap / phi_s

    if terms & C.HARTREE:
        # Hartree: v_H(G) = 4 pi rho(G) / G^2 (G != 0), E_H = 1/2 int v_H rho
        vh_g = np.zeros_like(rho_g)
        nz = G2 > 0
        vh_g[nz] = 4.0 * PI * rho_g[nz] / G2[nz]
        res.e_h = 0.5 * V * C.gsum(cell, np.real(np.conj(vh_g) * rho_g))
        vh = c2r(vh_g, shape)
        v += vh
        g += 2.0 * phi * vh

    if terms & C.EXT:
        vx_g = vext_g(cell) if vext is None else vext
        res.e_ext = V * C.gsum(cell, np.real(np.conj(vx_g) * rho_g))
        vx = c2r(vx_g, shape)
        v += vx
        g += 2.0 * phi * vx
        if e_ion is None:
            from .ewald import ewald_energy
            e_ion = ewald_energy(cell)
        res.e_ion = e_ion

    a, b = func.alpha, func.beta
    if terms & C.WT:
        # Wang-Teter: T_NL = int rho^a (omega * rho^b), eqs. "nl2", "WT",
        # kernel at the average k_F of the cell (or an MGP-family kernel,
        # eq. "MGP", at the same k_F).
        w = nl_kernel(gn, _kf_wt(cell, func), func.nl_kernel)
        phib = c2r(w * r2c(rho ** b), shape)
        phia = c2r(w * r2c(rho ** a), shape) if a != b else phib
        res.e_nl += dv * float(np.sum(rho ** a * phib))
        v += a * rho_s ** (a - 1.0) * phib + b * rho_s ** (b - 1.0) * phia
        g += 2.0 * a * sgn * absphi ** (2.0 * a - 1.0) * phib
        g += 2.0 * b * sgn * absphi ** (2.0 * b - 1.0) * phia

    if terms & C.SPLINE:
        e_nl, vnl, gnl_ = spline_nl(cell, func, rho, phi, gn)
        res.e_nl += e_nl
        v += vnl
        g += gnl_

    if terms & C.XC:
        eps, vxc = lda_xc(rho)
        res.e_xc = dv * float(np.sum(rho * eps))
        v += vxc
        g += 2.0 * phi * vxc

    res.e_total = (res.e_tf + res.e_vw + res.e_h + res.e_ext + res.e_nl + res.e_xc +
                   res.e_ion)
    # chemical potential and Euler-Lagrange residual in the psi form
    sum_rho = float(np.sum(phi * phi))
    res.mu = float(np.sum(g * phi)) / (2.0 * sum_rho) if sum_rho > 0 else 0.0
    R = g - 2.0 * res.mu * phi
    res.resid_norm = float(np.sqrt(np.mean(R * R)))
    res.v = v
    res.g = g
    return res


def spline_nl(cell, func, rho, phi, gn, kernel=None):
    """Density-dependent-kernel (LWT) nonlocal functional with linear splines
    over k_F knots, steps s1-s4 of Section "New-generation nonlocal KEDFs".

    Energy (both modes):
        E = int rho^a(r) sum_i L_i(k~(r)) Phi_i(r),
        Phi_i = F^-1[omega_i F[rho^b]],  omega_i(G) = C_WT G_NL(|G|/(2 k_i))
        (or the MGP-family kernel at k_i: the LMGP functionals),
    with k~ = clamp((3 pi^2 rho)^(1/3), k_1, k_Nk) and L_i the piecewise-linear
    hat functions of k on the knots of step s1.

    Potential, S3S4 (s3 then s4 as printed): the per-knot WT potentials
    interpolated at k~(r): v = sum_i L_i [a rho^(a-1) Phi_i + b rho^(b-1) Psi_i],
    Psi_i = F^-1[omega_i F[rho^a]].
    Potential, EXACT (the functional derivative of the energy above):
        v = a rho^(a-1) sum L_i Phi_i + rho^a (dk~/drho) sum L_i' Phi_i
            + b rho^(b-1) F^-1[sum_i omega_i F[rho^a L_i(k~)]].
    Returns (E_NL, v, g) with g = dE/dphi = 2 phi v written division-free.
    ``kernel(|G|, k)`` replaces omega(|G|; k) (a hook for the spline-exactness
    pin: a kernel linear in k is interpolated exactly).
    """
    shape = cell.n
    dv = cell.dv
    a, b = func.alpha, func.beta
    kn = C.knots(func)
    nk = len(kn)
    floor = func.rho_floor
    rho_s = np.maximum(rho, floor)
    absphi = np.abs(phi)
    sgn = np.where(phi < 0.0, -1.0, 1.0)
    kf = kf_of_rho(rho)
    kt, j, t, inside = spline_brackets(kn, kf)

    rb_g = r2c(rho ** b)
    ra_g = r2c(rho ** a) if (a != b and func.nl_mode == C.NL_S3S4) else None
    v1 = np.zeros(shape)   # sum_i L_i Phi_i
    v2 = np.zeros(shape)   # sum_i L_i' Phi_i
    v3 = np.zeros(shape)   # sum_i L_i Psi_i (S3S4 with a != b)
    hsum = None
    for i in range(nk):
        w = nl_kernel(gn, kn[i], func.nl_kernel) if kernel is None else kernel(gn, kn[i])
        phi_i = c2r(w * rb_g, shape)
        if nk == 1:
            L = np.ones(shape)
            dL = np.zeros(shape)
        else:
            L = np.where(j == i, 1.0 - t, 0.0) + np.where(j + 1 == i, t, 0.0)
            jj = np.clip(j, 0, nk - 2)
            inv_d = 1.0 / (kn[jj + 1] - kn[jj])
            dL = np.where(j == i, -inv_d, 0.0) + np.where(j + 1 == i, inv_d, 0.0)
        v1 += L * phi_i
        v2 += dL * phi_i
        if func.nl_mode == C.NL_EXACT:
            term = w * r2c(rho ** a * L)
            hsum = term if hsum is None else hsum + term
        elif ra_g is not None:
            v3 += L * c2r(w * ra_g, shape)

    e_nl = dv * float(np.sum(rho ** a * v1))
    pa_s = rho_s ** (a - 1.0)
    pb_s = rho_s ** (b - 1.0)
    fa = sgn * absphi ** (2.0 * a - 1.0)   # phi * rho^(a-1), division-free
    fb = sgn * absphi ** (2.0 * b - 1.0)
    if func.nl_mode == C.NL_EXACT:
        A = c2r(hsum, shape)
        dk = np.where(inside, kf / 3.0, 0.0)     # rho * dk~/drho
        v = a * pa_s * v1 + rho ** a * (dk / rho_s) * v2 + b * pb_s * A
        g = 2.0 * (a * fa * v1 + fa * dk * v2 + b * fb * A)
    else:
        psi = v3 if ra_g is not None else v1
        v = a * pa_s * v1 + b * pb_s * psi
        g = 2.0 * (a * fa * v1 + b * fb * psi)
    return e_nl, v, g
