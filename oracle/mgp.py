"""MGP-family kernels of the nonlocal kinetic functional (TEST INFRASTRUCTURE
ONLY: imported by tests/, never by the product library).

Section "New-generation nonlocal KEDFs", eq. "MGP":

    omega_{x,y}(q) = omega_WT(q) - x C_WT int_0^1 dt t^y d/dt G_NL(eta(q, t)),

with (x, y) = (1, 5/6) for MGP, (1/2, 5/6) for MGPA and (1, 5/3) for MGPG
(the parameter sentence after the G_NL formula).

Readings (the paper defers eta(q, t) to a supplement it does not contain):

* eta(q, t) = q / (2 t^(1/3) k_F): the kernel is built by functional
  integration along the uniformly scaled density t rho, whose Fermi
  wavevector is t^(1/3) k_F.  So eta(q, t) = eta t^(-1/3) with
  eta = q / (2 k_F), and the kernel is a function of eta alone:
      omega_{x,y} = C_WT K(eta),  K = G(eta) - x I(eta),
      I(eta) = int_0^1 t^y d/dt G(eta t^(-1/3)) dt.
* Step s2 ("the kernel is calculated at some discrete points of eta ... only
  once", then interpolated): the correction is tabulated once and
  interpolated linearly.  What is tabulated is J = G - I, the part that is
  smooth at eta = 1 where G itself has its logarithmic kink, so that
      K(eta) = (1 - x) G(eta) + x J_lin(eta),
  G evaluated exactly.  Table nodes: eta_j = j / 2048, j = 0 .. 8192 (eta <=
  4); above eta = 4 the variable w = 1 / eta^2 on w_k = k / 16384,
  k = 0 .. 1024 (w = 0 is eta = infinity, where J = G(inf) = -8/5).  J
  depends on y only.

Each node value is the paper's t-integral done by adaptive quadrature
(scipy.integrate.quad): with t = s^3 it reads
    I(eta) = -eta int_0^1 s^(3y-2) G'(eta / s) ds,
split at s = eta where the argument passes 1, and the part below (argument
above 1) rescaled by s = eta r to eta^(3y) times a fixed integral, so that the
quadrature never works on an interval of width eta^3.  G' is the analytic
derivative of the printed G_NL; the integrands are in oracle/mgp.c (called
through scipy's LowLevelCallable), and ``dgnl`` exposes G' for the pins.
"""
import ctypes
import functools
import math
import warnings

import numpy as np
from scipy import LowLevelCallable, integrate

from .functionals import C_WT, gnl

# kernel selectors (the same numbering as the C descriptor's nl_kernel)
KERNEL_WT, KERNEL_MGP, KERNEL_MGPA, KERNEL_MGPG = 0, 1, 2, 3
PARAMS = {KERNEL_MGP: (1.0, 5.0 / 6.0), KERNEL_MGPA: (0.5, 5.0 / 6.0),
          KERNEL_MGPG: (1.0, 5.0 / 3.0)}

TAB_H = 1.0 / 2048.0      # node spacing in eta below eta = 4
TAB_NA = 8192             # intervals in eta
TAB_WH = 1.0 / 16384.0    # node spacing in w = 1/eta^2 above eta = 4
TAB_NB = 1024             # intervals in w

_lib = None


def _load():
    global _lib
    if _lib is None:
        from . import build as _build
        path = _build.build_mgp(force=False)
        lib = ctypes.CDLL(path)
        lib.oracle_dgnl.argtypes = [ctypes.c_double]
        lib.oracle_dgnl.restype = ctypes.c_double
        _lib = lib
    return _lib


def dgnl(e):
    """G'(e), the derivative of the printed G_NL (e > 0, e != 1)."""
    return float(_load().oracle_dgnl(float(e)))


def _callable(name):
    lib = _load()
    fn = getattr(lib, name)
    fn.restype = ctypes.c_double
    fn.argtypes = (ctypes.c_int, ctypes.POINTER(ctypes.c_double))
    return LowLevelCallable(fn)


@functools.lru_cache(maxsize=None)
def _lower_constant(y):
    """int_0^1 -r^(3y-2) G'(1/r) dr (the rescaled part below s = eta)."""
    r, _ = integrate.quad(_callable("oracle_mgp_lower"), 0.0, 1.0, args=(1.0, y),
                          epsabs=1e-14, epsrel=1e-13, limit=500)
    return r


def correction_integral(eta, y):
    """I(eta) = int_0^1 t^y d/dt G(eta t^(-1/3)) dt of eq. "MGP", with
    eta(q, t) = eta t^(-1/3).  (QUADPACK's extrapolation occasionally reports
    round-off at this tolerance; the node values are pinned against
    30-digit mpmath quadrature, so the warning is not shown.)"""
    if eta == 0.0:
        return 0.0
    up = _callable("oracle_mgp_upper")
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        if eta < 1.0:
            hi, _ = integrate.quad(up, eta, 1.0, args=(eta, y), epsabs=1e-14, epsrel=1e-13,
                                   limit=500)
            return hi + eta ** (3.0 * y) * _lower_constant(y)
        val, _ = integrate.quad(up, 0.0, 1.0, args=(eta, y), epsabs=1e-14, epsrel=1e-13,
                                limit=500)
    return val


@functools.lru_cache(maxsize=None)
def j_table(y):
    """Nodes of J = G - I: (values on eta_j = j TAB_H, j <= TAB_NA; values on
    w_k = k TAB_WH, k <= TAB_NB)."""
    ja = np.empty(TAB_NA + 1)
    for j in range(TAB_NA + 1):
        e = j * TAB_H
        ja[j] = float(gnl(np.array([e]))[0]) - correction_integral(e, y)
    jb = np.empty(TAB_NB + 1)
    jb[0] = -8.0 / 5.0
    for k in range(1, TAB_NB + 1):
        e = 1.0 / math.sqrt(k * TAB_WH)
        jb[k] = float(gnl(np.array([e]))[0]) - correction_integral(e, y)
    return ja, jb


def j_interp(eta, y):
    """J_lin(eta): linear interpolation on the table (in eta up to 4, in
    w = 1/eta^2 above)."""
    ja, jb = j_table(y)
    eta = np.asarray(eta, dtype=np.float64)
    out = np.empty_like(eta)
    lo = eta <= 4.0
    out[lo] = np.interp(eta[lo], np.arange(TAB_NA + 1) * TAB_H, ja)
    w = 1.0 / (eta[~lo] * eta[~lo])
    out[~lo] = np.interp(w, np.arange(TAB_NB + 1) * TAB_WH, jb)
    return out


def kernel_shape_xy(eta, x, y):
    """K(eta) = (1 - x) G(eta) + x J_lin(eta) for any (x, y)."""
    eta = np.asarray(eta, dtype=np.float64)
    return (1.0 - x) * gnl(eta) + x * j_interp(eta, y)


def kernel_shape(eta, kind):
    """K(eta) with omega = C_WT K: G_NL for WT, (1 - x) G + x J_lin for the
    MGP family."""
    eta = np.asarray(eta, dtype=np.float64)
    if kind == KERNEL_WT:
        return gnl(eta)
    x, y = PARAMS[kind]
    return kernel_shape_xy(eta, x, y)


def kernel(gnorm, kf, kind):
    """omega(|G|) = C_WT K(|G| / (2 k_F)) for the selected kernel family."""
    return C_WT * kernel_shape(np.asarray(gnorm) / (2.0 * kf), kind)
