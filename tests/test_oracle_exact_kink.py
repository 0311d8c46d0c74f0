"""Why the spline functional is optimised with the S3S4 potential (the
reading of the EXACT variant in the design notes): with linear hat functions
over the k_F knots (steps s1-s4 of the nonlocal-KEDF section), the EXACT
energy is continuous in rho but its derivative is not.  At a point whose
k_F(rho) sits on an interior knot, the slope of the hat functions changes, so
dE/drho there jumps by a finite amount however small the step across the
knot; the Wang-Teter and S3S4 potentials change by O(step).  A gradient
method then meets a non-smooth objective: on a small Mg slab the oracle's
own conjugate-gradient optimiser, run with the EXACT potential, is still
above 5e-5 in RMS residual after 70 iterations and needs several energy
evaluations per line search, while Wang-Teter converges to 1e-7 in fewer
than 100 iterations at under two evaluations per iteration."""
import numpy as np
import pytest

from oracle import cell as C
from oracle import functionals as Fn
from oracle.ewald import ewald_energy
from oracle.optimize import optimize
from paper_2002_02985_amd import workloads as W
from tests.oracle_helpers import box_cell, smooth_density

LOCAL = C.TF | C.VW | C.HARTREE | C.EXT
SPL = dict(nk=12, kf_min=0.1, kf_max=2.5)


def potential_across_knot(func, cell, rho, r0, kj, eps):
    """v(r0) with k_F(rho(r0)) = kj (1 - eps) and kj (1 + eps)."""
    out = []
    for s in (-1.0, 1.0):
        r = rho.copy()
        r[r0] = (kj * (1 + s * eps)) ** 3 / (3 * np.pi ** 2)
        out.append(Fn.energy_potential(cell, func, rho=r).v[r0])
    return out[1] - out[0]


def test_exact_spline_potential_jumps_at_a_knot():
    cell = box_cell(n=(10, 12, 14))
    rho = smooth_density(cell, seed=5, amp=0.4, nmodes=3)
    kn = C.knots(C.Functional(terms=LOCAL | C.SPLINE, **SPL))
    # an interior knot inside the density's k_F range, at a point whose
    # k_F lies near it
    kf = (3 * np.pi ** 2 * rho) ** (1.0 / 3.0)
    j = int(np.argmin(np.abs(kn[1:-1] - np.median(kf)))) + 1
    r0 = np.unravel_index(int(np.argmin(np.abs(kf - kn[j]))), rho.shape)
    funcs = {
        "exact": C.Functional(terms=LOCAL | C.SPLINE, nl_mode=C.NL_EXACT, **SPL),
        "s3s4": C.Functional(terms=LOCAL | C.SPLINE, nl_mode=C.NL_S3S4, **SPL),
        "wt": C.Functional(terms=LOCAL | C.WT),
    }
    # steps of 1e-7 and 1e-8 in k_F across the knot (the smooth change of v
    # is about 30 eps Ha here)
    jumps = {k: [abs(potential_across_knot(f, cell, rho, r0, kn[j], e)) for e in (1e-7, 1e-8)]
             for k, f in funcs.items()}
    # EXACT: the jump stays (the hat slopes change at the knot): ~1.1e-3 Ha
    assert jumps["exact"][1] > 1e-4
    assert jumps["exact"][1] > 0.9 * jumps["exact"][0]
    # smooth potentials: the change shrinks with the step (10x here)
    for k in ("s3s4", "wt"):
        assert jumps[k][1] < 0.2 * jumps[k][0], (k, jumps[k])
        assert jumps[k][1] < 1e-2 * jumps["exact"][1], (k, jumps[k], jumps["exact"])


def slab():
    d = W.mg_hcp_slab((1, 1, 2), n=(12, 20, 36), vacuum=10.0)
    from tests.oracle_helpers import make_cell
    cell = make_cell(d)
    phi0 = np.sqrt(W.gaussian_density(d, sigma=1.5, floor=1e-8))
    return cell, phi0, Fn.vext_g(cell), ewald_energy(cell)


def rms_residual(o):
    R = o.result.g - 2 * o.result.mu * o.phi
    return float(np.sqrt(np.mean(R * R)))


def test_gradient_optimiser_stalls_on_the_exact_spline_energy():
    cell, phi0, vx, ei = slab()
    wt = optimize(cell, C.Functional(terms=LOCAL | C.WT), phi0, tol=1e-7, max_iter=100,
                  vext=vx, e_ion=ei)
    assert wt.converged and wt.evals < 2 * max(wt.iters, 1)
    ex = optimize(cell, C.Functional(terms=LOCAL | C.SPLINE, nl_mode=C.NL_EXACT, **SPL), phi0,
                  tol=1e-7, max_iter=70, vext=vx, e_ion=ei)
    assert not ex.converged
    assert rms_residual(ex) > 5e-5
    assert ex.evals > 3.5 * ex.iters
    # the energy still went down monotonically: the stall is not a bug in
    # the line search but the kinks of the objective
    assert all(b <= a + 1e-12 for a, b in zip(ex.energies, ex.energies[1:]))
