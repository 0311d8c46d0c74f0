"""Oracle density optimisation (TEST INFRASTRUCTURE ONLY).

Section "Density optimization strategies": minimise E over phi = sqrt(rho)
(eq. "euler2"), repeating (1) a search direction from nonlinear conjugate
gradients, (2) a line search for the step, (3) the update
phi <- phi cos(theta) + p sin(theta) with p orthogonal to phi and normalised
to N_e (the orthogonal-rotation update, which keeps int rho = N_e exactly).

Reading used here where the paper is not specific: Polak-Ribiere (PR+)
direction on the projected residual R = dE/dphi - 2 mu phi with a restart on
loss of descent; a strong-Wolfe line search (c1 = 1e-4, c2 = 0.1) over theta
by bracketing and cubic interpolation; convergence when
sqrt(mean(R^2)) < tol.
"""
import dataclasses

import numpy as np

from .functionals import energy_potential


@dataclasses.dataclass
class OptResult:
    phi: np.ndarray
    result: object
    iters: int
    evals: int
    converged: bool
    energies: list


def _dot(a, b, dv):
    return dv * float(np.sum(a * b))


def _cubic_min(a, fa, da, b, fb, db):
    """Minimiser of the cubic through (a, fa, da), (b, fb, db); None if none."""
    d1 = da + db - 3.0 * (fa - fb) / (a - b)
    disc = d1 * d1 - da * db
    if disc < 0:
        return None
    d2 = np.sign(b - a) * np.sqrt(disc)
    den = db - da + 2.0 * d2
    if den == 0:
        return None
    return b - (b - a) * (db + d2 - d1) / den


def line_search(fun, f0, d0, theta0, c1=1e-4, c2=0.1, max_evals=20):
    """Strong-Wolfe search for theta > 0 on f(theta); fun(theta) -> (f, df, payload).

    Near convergence energy differences reach the rounding level of E, so the
    sufficient-decrease test also accepts the approximate form
    f <= f0 + eps_f with df <= (2 c1 - 1) df(0) (eps_f = 1e-14 |f0|).
    Returns (theta, f, df, payload, evals)."""
    eps_f = 1e-14 * max(1.0, abs(f0))

    def decrease_ok(a, fa, da):
        return fa <= f0 + c1 * a * d0 or (fa <= f0 + eps_f and da <= (2 * c1 - 1) * d0)

    evals = 0
    a_prev, f_prev, d_prev = 0.0, f0, d0
    a = theta0
    best = None
    while evals < max_evals:
        fa, da, pay = fun(a)
        evals += 1
        if best is None or fa < best[1]:
            best = (a, fa, da, pay)
        if not decrease_ok(a, fa, da) or (evals > 1 and fa > f_prev + eps_f):
            return _zoom(fun, f0, d0, a_prev, f_prev, d_prev, a, fa, da, c2,
                         max_evals - evals, evals, best, decrease_ok, eps_f)
        if abs(da) <= -c2 * d0:
            return a, fa, da, pay, evals
        if da >= 0:
            return _zoom(fun, f0, d0, a, fa, da, a_prev, f_prev, d_prev, c2,
                         max_evals - evals, evals, best, decrease_ok, eps_f)
        # extrapolate
        a_new = _cubic_min(a_prev, f_prev, d_prev, a, fa, da)
        if a_new is None or a_new <= a * 1.1 or a_new > a * 4.0:
            a_new = 2.0 * a
        a_prev, f_prev, d_prev = a, fa, da
        a = a_new
    a, fa, da, pay = best
    return a, fa, da, pay, evals


def _zoom(fun, f0, d0, alo, flo, dlo, ahi, fhi, dhi, c2, budget, evals, best,
          decrease_ok, eps_f):
    for _ in range(max(budget, 0)):
        a = _cubic_min(alo, flo, dlo, ahi, fhi, dhi)
        lo, hi = min(alo, ahi), max(alo, ahi)
        if a is None or not (lo < a < hi):
            a = 0.5 * (alo + ahi)
        else:
            # safeguard: stay clear of the bracket ends
            a = min(max(a, lo + 0.01 * (hi - lo)), hi - 0.01 * (hi - lo))
        fa, da, pay = fun(a)
        evals += 1
        if fa < best[1]:
            best = (a, fa, da, pay)
        if not decrease_ok(a, fa, da) or fa > flo + eps_f:
            ahi, fhi, dhi = a, fa, da
        else:
            if abs(da) <= -c2 * d0:
                return a, fa, da, pay, evals
            if da * (ahi - alo) >= 0:
                ahi, fhi, dhi = alo, flo, dlo
            alo, flo, dlo = a, fa, da
    a, fa, da, pay = best
    return a, fa, da, pay, evals


def optimize(cell, func, phi0, tol=1e-7, max_iter=500, vext=None, e_ion=None):
    """Minimise E[phi^2] at fixed N_e = cell.nelec.  Returns OptResult."""
    dv = cell.dv
    ne = cell.nelec
    phi = np.array(phi0, dtype=np.float64)
    phi *= np.sqrt(ne / _dot(phi, phi, dv))

    def ev(p):
        return energy_potential(cell, func, phi=p, vext=vext, e_ion=e_ion)

    r = ev(phi)
    evals = 1
    energies = [r.e_total]
    R_prev = None
    d_prev = None
    theta_prev = None
    kappa = None          # curvature d2E/dtheta2 seen by the last line search
    converged = False
    it = 0
    for it in range(max_iter):
        R = r.g - 2.0 * r.mu * phi
        if np.sqrt(np.mean(R * R)) < tol:
            converged = True
            break
        if R_prev is None:
            d = -R
        else:
            beta = max(0.0, _dot(R, R - R_prev, dv) / _dot(R_prev, R_prev, dv))
            d = -R + beta * d_prev
        if _dot(d, R, dv) >= 0.0:
            d = -R
        p = d - (_dot(d, phi, dv) / _dot(phi, phi, dv)) * phi
        p *= np.sqrt(ne / _dot(p, p, dv))
        g0 = _dot(r.g, p, dv)          # dE/dtheta at theta = 0
        if g0 >= 0.0:
            d = -R
            p = d - (_dot(d, phi, dv) / _dot(phi, phi, dv)) * phi
            p *= np.sqrt(ne / _dot(p, p, dv))
            g0 = _dot(r.g, p, dv)
        # first trial step: minimiser of the quadratic model with the curvature
        # measured along the previous direction
        if kappa is not None and kappa > 0:
            theta0 = min(1.0, max(1e-12, -g0 / kappa))
        elif theta_prev is not None:
            theta0 = theta_prev
        else:
            theta0 = 0.1

        def fun(th, phi=phi, p=p):
            ph = phi * np.cos(th) + p * np.sin(th)
            rr = ev(ph)
            dth = -phi * np.sin(th) + p * np.cos(th)
            return rr.e_total, _dot(rr.g, dth, dv), (ph, rr)

        th, fth, dth, (phi_new, r_new), ne_ = line_search(fun, r.e_total, g0, theta0)
        evals += ne_
        if fth > r.e_total + 1e-14 * max(1.0, abs(r.e_total)):
            # no decrease along p: stop rather than step uphill
            break
        kappa = (dth - g0) / th if th > 0 else None
        theta_prev = th
        R_prev = R
        d_prev = d
        phi = phi_new
        r = r_new
        energies.append(r.e_total)
    return OptResult(phi=phi, result=r, iters=it, evals=evals, converged=converged,
                     energies=energies)
