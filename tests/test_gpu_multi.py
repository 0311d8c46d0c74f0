"""Batched evaluation of several cells of one grid shape
(ofdft_energy_potential_multi) and the server's continuous batching of
energy+potential requests across cells.

Each entry of a batch is a different cell (different lattice, atoms and
electron count on the same 48 x 48 x 64 grid), so the reciprocal-space pass
and the knot kernels must take each cell's own reciprocal vectors, v_ext(G),
kernel table (the Wang-Teter kernel at each cell's average k_F) and E_ion.
Every result must equal, bit for bit, the same grid evaluated alone; one
entry is also compared with the oracle at the parity bars."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import cell as OC
from oracle import functionals as OF
from paper_2002_02985_amd import ofdft
from paper_2002_02985_amd import workloads as W
from tests.oracle_helpers import make_cell

pytestmark = pytest.mark.gpu

LOCAL = ofdft.TERM_TF | ofdft.TERM_VW | ofdft.TERM_HARTREE | ofdft.TERM_EXT
N = (48, 48, 64)


def cells():
    out = []
    for i, (na, sp, L) in enumerate([(13, "Al", None), (8, "Mg", 19.0), (19, "Al", 23.0)]):
        c = W.cluster(na, sp, seed=30 + i, grid=48)
        if L is not None:
            c["lattice"] = np.diag([L, L * 1.05, L * 1.1])   # a different, orthorhombic box
            c["pos"] = c["pos"] - c["pos"].mean(axis=0) + np.array([L / 2, L * 0.525, L * 0.55])
        c["n"] = N
        out.append(c)
    return out


KW = {
    "wt": (LOCAL | ofdft.TERM_WT, {}),
    "spline_s3s4": (LOCAL | ofdft.TERM_SPLINE, dict(nk=12, kf_min=0.1, kf_max=2.5)),
    "spline_exact": (LOCAL | ofdft.TERM_SPLINE,
                     dict(nk=12, kf_min=0.1, kf_max=2.5, nl_mode=ofdft.NL_EXACT)),
    "lmgp": (LOCAL | ofdft.TERM_SPLINE, dict(nk=12, kf_min=0.1, kf_max=2.5,
                                             nl_kernel=ofdft.KERNEL_MGP)),
}


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED, ofdft.MIXED_VW64])
@pytest.mark.parametrize("func", sorted(KW))
def test_multi_cell_batch_equals_each_cell_alone(func, prec):
    terms, kw = KW[func]
    cs = cells()
    rhos = [W.gaussian_density(c, sigma=1.5, floor=1e-9) for c in cs]
    print("case multi", func, prec, flush=True)
    grids = [ofdft.Grid(c, terms, precision=prec, **kw) for c in cs]
    try:
        alone = []
        for g, r in zip(grids, rhos):
            g.set_density(r)
            e, v = g.energy_potential(None)
            alone.append((e.as_dict(), v))
        es, vs = ofdft.ofdft_energy_potential_multi([g.handle for g in grids], [N] * 3)
        # and again in another order (another leader)
        order = [2, 0, 1]
        es2, vs2 = ofdft.ofdft_energy_potential_multi([grids[k].handle for k in order], [N] * 3)
    finally:
        for g in grids:
            g.close()
    for b in range(3):
        ea, va = alone[b]
        eb = es[b].as_dict()
        for k in ea:
            assert eb[k] == ea[k], (func, prec, b, k, eb[k], ea[k])
        assert np.array_equal(vs[b], va), (func, prec, b)
    for j, k in enumerate(order):
        assert es2[j].e_total == alone[k][0]["e_total"]
        assert np.array_equal(vs2[j], alone[k][1])
    if prec == ofdft.FP64:
        # entry 1 (the orthorhombic Mg box) against the oracle
        ro = OF.energy_potential(make_cell(cs[1]), OC.Functional(terms=int(terms), **kw), rho=rhos[1])
        assert abs(es[1].e_total - ro.e_total) <= 1e-10 * abs(ro.e_total)
        m = rhos[1] >= 1e-6
        assert np.abs(vs[1] - ro.v)[m].max() <= 1e-9


def test_multi_refuses_mismatched_grids():
    cs = cells()
    other = dict(cs[0])
    other["n"] = (48, 48, 48)
    g1 = ofdft.Grid(cs[0], LOCAL)
    g2 = ofdft.Grid(other, LOCAL)
    g3 = ofdft.Grid(cs[1], LOCAL | ofdft.TERM_WT)
    try:
        for g in (g1, g2, g3):
            g.set_density(W.uniform_density(g.cell))
        for bad in ([g1.handle, g2.handle], [g1.handle, g3.handle], [g1.handle, g1.handle]):
            with pytest.raises(ofdft.OfdftError) as ei:
                ofdft.ofdft_energy_potential_multi(bad, [None] * len(bad), want_v=False)
            assert ei.value.status == ofdft.EINVAL
    finally:
        for g in (g1, g2, g3):
            g.close()


def test_server_batches_energy_requests_across_cells():
    """One worker slot: while it runs, energy+potential requests of six
    resident cells (one grid shape, two lattices) queue up and are served in
    batches; each result equals the direct grid path."""
    from tests.test_gpu_serve import Server
    base = cells()
    cs = []
    for i in range(6):
        c = dict(base[i % 2])
        c["pos"] = base[i % 2]["pos"] + 0.05 * i
        cs.append(c)
    fd = ofdft.make_functional_desc(LOCAL, precision=ofdft.MIXED_VW64)
    s = Server(max_inflight=1)
    try:
        # make every cell resident with its density
        first = []
        for i, c in enumerate(cs):
            q = {"cell_id": 100 + i, "kind": ofdft.REQ_EP, "cell": c,
                 "rho": W.gaussian_density(c, sigma=1.5, floor=1e-9)}
            first.append((s.submit(q, func=fd), q))
        for t, q in first:
            assert s.result(t, q)[0] == ofdft.OK
        # a long request first, then the energy requests queue behind it
        big = {"cell_id": 999, "kind": ofdft.REQ_OPTIMIZE, "cell": cs[0],
               "rho": W.gaussian_density(cs[0], sigma=1.5, floor=1e-9)}
        tb = s.submit(big, opt=dict(tol=1e-6, max_iter=200), func=fd)
        later = []
        for i, c in enumerate(cs):
            q = {"cell_id": 100 + i, "kind": ofdft.REQ_EP, "cell": c, "rho": None}
            later.append((s.submit(q, func=fd), q))
        res = [s.result(t, q) for t, q in later]
        s.result(tb, big)
        stats = s.stats()
    finally:
        s.close()
    print("batches %d, batched requests %d" % (stats["batches"], stats["batched_requests"]),
          flush=True)
    assert stats["batches"] >= 1 and stats["batched_requests"] >= 2
    for (st, r, v, _), c, (t, q0) in zip(res, cs, first):
        assert st == ofdft.OK
        with ofdft.Grid(c, LOCAL, precision=ofdft.MIXED_VW64) as g:
            e, v_ref = g.energy_potential(q0["rho"])
        assert r.e.e_total == e.e_total
        assert np.array_equal(v, v_ref)


def test_server_batches_optimisation_requests_across_cells():
    """One worker slot: warm-started optimisation requests of six resident
    cells queue behind a long request and are served as lockstep
    optimisations; each result equals ofdft_optimize on the same cell and
    starting density alone."""
    from tests.test_gpu_serve import Server
    base = cells()
    cs = []
    for i in range(6):
        c = dict(base[i % 2])
        c["pos"] = base[i % 2]["pos"] + 0.05 * i
        cs.append(c)
    fd = ofdft.make_functional_desc(LOCAL | ofdft.TERM_WT, precision=ofdft.MIXED_VW64)
    opt = dict(tol=2e-5, max_iter=40)
    s = Server(max_inflight=1)
    ofdft.ofdft_serve_set_batching(s.h, 8, 8)   # lockstep optimisation batches are off by default
    try:
        first = []
        for i, c in enumerate(cs):
            q = {"cell_id": 200 + i, "kind": ofdft.REQ_EP, "cell": c,
                 "rho": W.gaussian_density(c, sigma=1.5 + 0.05 * i, floor=1e-9)}
            first.append((s.submit(q, func=fd), q))
        for t, q in first:
            assert s.result(t, q)[0] == ofdft.OK
        big = {"cell_id": 998, "kind": ofdft.REQ_OPTIMIZE, "cell": cs[0],
               "rho": W.gaussian_density(cs[0], sigma=1.5, floor=1e-9)}
        tb = s.submit(big, opt=dict(tol=1e-6, max_iter=200), func=fd)
        later = []
        for i, c in enumerate(cs):
            q = {"cell_id": 200 + i, "kind": ofdft.REQ_OPTIMIZE, "cell": c, "rho": None}
            later.append((s.submit(q, opt=opt, func=fd), q))
        res = [s.result(t, q) for t, q in later]
        s.result(tb, big)
        stats = s.stats()
    finally:
        s.close()
    print("batches %d, batched requests %d" % (stats["batches"], stats["batched_requests"]),
          flush=True)
    assert stats["batches"] >= 1 and stats["batched_requests"] >= 2
    for (st, r, _, _), c, (t, q0) in zip(res, cs, first):
        assert st in (ofdft.OK, ofdft.ENOCONV)
        with ofdft.Grid(c, LOCAL | ofdft.TERM_WT, precision=ofdft.MIXED_VW64) as g:
            g.set_density(q0["rho"])
            ra, sa = ofdft.ofdft_optimize(g.handle, opt["tol"], opt["max_iter"],
                                          method=ofdft.OPT_CG, allow_noconv=True)
        assert st == sa
        assert r.iters == ra.iters and r.evals == ra.evals
        assert r.e.e_total == ra.e.e_total and r.final_resid == ra.final_resid


def test_serve_set_batching_checks_its_range():
    from tests.test_gpu_serve import Server
    s = Server(max_inflight=1)
    try:
        for bad in ((0, 8), (8, 0), (ofdft.MULTI_MAX + 1, 1)):
            with pytest.raises(ofdft.OfdftError) as ei:
                ofdft.ofdft_serve_set_batching(s.h, *bad)
            assert ei.value.status == ofdft.EINVAL
        ofdft.ofdft_serve_set_batching(s.h, 1, 1)
    finally:
        s.close()
