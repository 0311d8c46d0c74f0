"""Lockstep optimisation of several cells (ofdft_optimize_multi): each
member's optimiser is unchanged and its evaluations are merged with the
other members' into batched evaluations, so every result -- energy, residual,
iterations, evaluations and the optimised density -- must equal, bit for bit,
ofdft_optimize on that cell alone.  Members get different tolerances and
iteration limits, so that they leave the group at different times; the
methods are preconditioned CG, plain CG and truncated Newton; Wang-Teter and
spline (S3S4, whose line search works on the derivative only) functionals,
both precisions."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2002_02985_amd import ofdft
from tests.test_gpu_multi import LOCAL, N, cells

pytestmark = pytest.mark.gpu

FUNCS = {
    "wt": (LOCAL | ofdft.TERM_WT, {}),
    "spline": (LOCAL | ofdft.TERM_SPLINE, dict(nk=12, kf_min=0.1, kf_max=2.5)),
}


def densities(cs):
    from paper_2002_02985_amd import workloads as W
    return [W.gaussian_density(c, sigma=1.5, floor=1e-9) for c in cs]


def params_for(prec, method):
    tol = 1e-7 if prec == ofdft.FP64 else 2e-5
    # member 1 stops early on its iteration limit, member 2 on a looser tolerance
    return [(tol, 400, method), (tol, 6, method), (tol * 20, 400, method)]


@pytest.mark.parametrize("method", [ofdft.OPT_PCG, ofdft.OPT_CG, ofdft.OPT_TN])
@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED])
@pytest.mark.parametrize("func", sorted(FUNCS))
def test_lockstep_optimisation_equals_each_alone(func, prec, method):
    if func == "spline" and method == ofdft.OPT_TN:
        pytest.skip("truncated Newton is offered for energy-consistent potentials")
    terms, kw = FUNCS[func]
    cs = cells()
    rhos = densities(cs)
    prm = params_for(prec, method)
    print("case opt multi", func, prec, method, flush=True)
    alone = []
    for c, r, (tol, mi, m) in zip(cs, rhos, prm):
        with ofdft.Grid(c, terms, precision=prec, **kw) as g:
            g.set_density(r)
            res, st = ofdft.ofdft_optimize(g.handle, tol, mi, method=m, allow_noconv=True)
            alone.append((res, st, g.get_density()))
    grids = [ofdft.Grid(c, terms, precision=prec, **kw) for c in cs]
    try:
        for g, r in zip(grids, rhos):
            g.set_density(r)
        rs, sts = ofdft.ofdft_optimize_multi([g.handle for g in grids], prm)
        dens = [g.get_density() for g in grids]
    finally:
        for g in grids:
            g.close()
    for b in range(len(cs)):
        ra, sa, da = alone[b]
        assert sts[b] == sa, (b, sts[b], sa)
        assert rs[b].iters == ra.iters and rs[b].evals == ra.evals, (b, rs[b].iters, ra.iters)
        assert rs[b].e.e_total == ra.e.e_total and rs[b].final_resid == ra.final_resid, b
        assert np.array_equal(dens[b], da), b
    assert sts[1] in (ofdft.OK, ofdft.ENOCONV)


def test_lockstep_refuses_a_grid_without_density():
    """A grid whose resident density was never written is refused (by the
    lockstep call and by the single-grid calls that read that density)."""
    cs = cells()
    g1 = ofdft.Grid(cs[0], LOCAL)
    g2 = ofdft.Grid(cs[1], LOCAL)
    try:
        g1.set_density(densities(cs[:1])[0])
        with pytest.raises(ofdft.OfdftError) as ei:
            ofdft.ofdft_optimize_multi([g1.handle, g2.handle], [(1e-6, 10, ofdft.OPT_PCG)] * 2)
        assert ei.value.status == ofdft.EINVAL
        for call in (lambda: ofdft.ofdft_optimize(g2.handle, 1e-6, 10),
                     lambda: g2.energy_potential(None),
                     lambda: g2.get_density()):
            with pytest.raises(ofdft.OfdftError) as ei:
                call()
            assert ei.value.status == ofdft.EINVAL
    finally:
        g1.close()
        g2.close()
