"""Request server on the GPU: every result is the same alone and in a
concurrent mix, equals the direct grid path (itself pinned to the oracle),
warm starts carry across MD frames, admission respects the memory budget,
and the error codes of submit/poll/cancel."""
import sys
import time

import numpy as np
import pytest

from paper_2002_02985_amd import ofdft
from paper_2002_02985_amd import workloads as W

pytestmark = pytest.mark.gpu

TERMS = ofdft.TERM_TF | ofdft.TERM_VW | ofdft.TERM_HARTREE | ofdft.TERM_EXT
OPT = dict(tol=2e-5, max_iter=60)


def _say(msg):
    print(msg)
    sys.stdout.flush()


def _precision(cell_id):
    return ofdft.FP64 if cell_id % 2 == 0 else ofdft.MIXED


class Server:
    def __init__(self, budget=0, max_inflight=4):
        self.ctx = ofdft.ofdft_ctx_create(0)
        self.h = ofdft.ofdft_server_create(self.ctx, budget, max_inflight)
        self.keep = []

    def submit(self, q, opt=None, func=None):
        cd, keep = ofdft.make_cell_desc(q["cell"])
        fd = func or ofdft.make_functional_desc(TERMS, precision=_precision(q["cell_id"]))
        op = None
        if q["kind"] == ofdft.REQ_OPTIMIZE:
            op = ofdft.OptParams(tol=(opt or OPT)["tol"], max_iter=(opt or OPT)["max_iter"],
                                 method=0, warm=1)
        self.keep.append((cd, fd, op, keep))
        return ofdft.ofdft_serve_submit(self.h, q["cell_id"], q["kind"], cd, fd, op, q["rho"])

    def result(self, t, q):
        assert ofdft.ofdft_serve_wait(self.h, t, 120000) == ofdft.OK
        st, r, v, f = ofdft.ofdft_serve_poll(self.h, t, q["cell"]["n"], len(q["cell"]["species"]))
        return st, r, v, f

    def stats(self):
        return ofdft.ofdft_serve_stats_get(self.h)

    def close(self):
        if self.h:
            ofdft.ofdft_server_destroy(self.h)
            self.h = None
        if self.ctx:
            ofdft.ofdft_ctx_destroy(self.ctx)
            self.ctx = None


def _stream(n=14):
    return W.config_c4(n, seed=7, ntraj=4, min_atoms=13, max_atoms=40, grids=(48, 54, 64), h=0.6)


def _run(reqs, max_inflight, one_at_a_time):
    s = Server(max_inflight=max_inflight)
    try:
        out = {}
        if one_at_a_time:
            for i, q in enumerate(reqs):
                t = s.submit(q)
                out[i] = s.result(t, q)
        else:
            ts = [s.submit(q) for q in reqs]
            for i, (t, q) in enumerate(zip(ts, reqs)):
                out[i] = s.result(t, q)
        return out, s.stats()
    finally:
        s.close()


def test_alone_and_in_the_mix_agree():
    reqs = _stream()
    _say("serve: %d requests, grids %s" % (len(reqs), sorted({q["cell"]["n"][0] for q in reqs})))
    alone, st_a = _run(reqs, 1, True)
    mix, st_m = _run(reqs, 4, False)
    _say("alone p50 %.1f ms; mix p50 %.1f ms p99 %.1f ms" % (st_a["p50_ms"], st_m["p50_ms"],
                                                             st_m["p99_ms"]))
    assert st_m["completed"] == len(reqs) and st_m["failed"] == 0
    nbit = 0
    for i, q in enumerate(reqs):
        sa, ra, va, fa = alone[i]
        sm, rm, vm, fm = mix[i]
        assert sa in (ofdft.OK, ofdft.ENOCONV) and sm == sa, (i, sa, sm)
        na = len(q["cell"]["species"])
        de = abs(ra.e.e_total - rm.e.e_total)
        fp64 = _precision(q["cell_id"]) == ofdft.FP64
        assert de <= (1e-10 * abs(ra.e.e_total) if fp64 else 1e-5 * na), (i, de)
        same = de == 0.0
        if q["kind"] == ofdft.REQ_EP:
            dv = float(np.max(np.abs(va - vm)))
            assert dv <= (1e-9 if fp64 else 1e-4), (i, dv)
            same = same and dv == 0.0
        if q["kind"] == ofdft.REQ_FORCES:
            df = float(np.max(np.abs(fa - fm)))
            assert df <= (1e-9 if fp64 else 1e-4), (i, df)
            same = same and df == 0.0
        if q["kind"] == ofdft.REQ_OPTIMIZE:
            assert ra.iters == rm.iters
        nbit += same
    _say("bit-identical alone vs mix: %d of %d" % (nbit, len(reqs)))


def test_server_matches_direct_grid_path():
    reqs = [q for q in _stream() if q["kind"] != ofdft.REQ_OPTIMIZE][:4]
    s = Server(max_inflight=3)
    try:
        ts = []
        for q in reqs:
            q = dict(q)
            q["rho"] = W.gaussian_density(q["cell"], sigma=1.5, floor=1e-8)
            ts.append((s.submit(q), q))
        for t, q in ts:
            st, r, v, f = s.result(t, q)
            assert st == ofdft.OK
            with ofdft.Grid(q["cell"], TERMS, precision=_precision(q["cell_id"])) as g:
                e, vg = g.energy_potential(q["rho"])
                assert r.e.e_total == e.e_total
                if q["kind"] == ofdft.REQ_EP:
                    assert np.array_equal(v, vg)
                else:
                    g.set_density(q["rho"])
                    assert np.array_equal(f, g.forces())
    finally:
        s.close()


def test_warm_start_across_md_frames():
    base = W.cluster(19, "Al", seed=11, grid=48)
    rng = np.random.default_rng(5)
    frames = [base["pos"]]
    for _ in range(2):
        frames.append(frames[-1] + rng.normal(0.0, 0.05, size=base["pos"].shape))
    fd = ofdft.make_functional_desc(TERMS, precision=ofdft.FP64)
    s = Server(max_inflight=2)
    try:
        res = []
        for k, p in enumerate(frames):
            cell = dict(base)
            cell["pos"] = p
            q = {"cell_id": 0, "kind": ofdft.REQ_OPTIMIZE, "cell": cell,
                 "rho": W.gaussian_density(cell, sigma=1.5, floor=1e-8) if k == 0 else None}
            st, r, _, _ = s.result(s.submit(q, opt=dict(tol=1e-6, max_iter=400), func=fd), q)
            assert st == ofdft.OK
            res.append(r)
        # cold start of the last frame from the Gaussian guess on a fresh grid
        cell = dict(base)
        cell["pos"] = frames[-1]
        q = {"cell_id": 1, "kind": ofdft.REQ_OPTIMIZE, "cell": cell,
             "rho": W.gaussian_density(cell, sigma=1.5, floor=1e-8)}
        st, cold, _, _ = s.result(s.submit(q, opt=dict(tol=1e-6, max_iter=400), func=fd), q)
        assert st == ofdft.OK
        _say("iterations per frame %s, cold %d" % ([r.iters for r in res], cold.iters))
        assert res[-1].iters < cold.iters
        # TF+vW+H+ext is strictly convex in rho: one minimiser
        assert abs(res[-1].e.e_total - cold.e.e_total) < 1e-8 * abs(cold.e.e_total)
        assert s.stats()["resident_cells"] == 2
    finally:
        s.close()


def test_pme_cell_across_md_frames_matches_direct_grid():
    """A cell whose structure factor is taken by smooth PME: each MD frame
    re-spreads the charge grid on the resident cell, and the results equal a
    fresh grid of that frame bit for bit (the fixed-point spread makes PME
    independent of the order in which atoms land)."""
    base = dict(W.cluster(19, "Al", seed=11, grid=48), sf_method=ofdft.SF_PME, pme_order=8)
    rng = np.random.default_rng(9)
    frames = [base["pos"], base["pos"] + rng.normal(0.0, 0.1, size=base["pos"].shape)]
    s = Server(max_inflight=2)
    try:
        for p in frames:
            cell = dict(base, pos=p)
            q = {"cell_id": 0, "kind": ofdft.REQ_EP, "cell": cell,
                 "rho": W.gaussian_density(cell, sigma=1.5, floor=1e-8)}
            st, r, v, _ = s.result(s.submit(q), q)
            assert st == ofdft.OK
            with ofdft.Grid(cell, TERMS, precision=ofdft.FP64) as g:
                e, vg = g.energy_potential(q["rho"])
            assert r.e.e_total == e.e_total and r.e.e_ion == e.e_ion
            assert np.array_equal(v, vg)
        assert s.stats()["resident_cells"] == 1
    finally:
        s.close()


def test_admission_under_a_tight_budget():
    reqs = [q for q in _stream(10)]
    cds = [ofdft.make_cell_desc(q["cell"]) for q in reqs]
    fps = [ofdft.ofdft_footprint_bytes(cd, ofdft.make_functional_desc(
        TERMS, precision=_precision(q["cell_id"])), ofdft.REQ_OPTIMIZE)
        for (cd, _), q in zip(cds, reqs)]
    budget = int(max(fps) * 1.5) + (1 << 20)
    s = Server(budget=budget, max_inflight=4)
    try:
        ts = [s.submit(q) for q in reqs]
        for t, q in zip(ts, reqs):
            st, r, v, f = s.result(t, q)
            assert st in (ofdft.OK, ofdft.ENOCONV)
        stats = s.stats()
        _say("budget %d B, peak %d B, resident %d" % (budget, stats["peak_bytes"],
                                                     stats["resident_cells"]))
        assert stats["peak_bytes"] <= budget
        assert stats["resident_bytes"] <= budget
        assert stats["completed"] == len(reqs)
        assert stats["resident_cells"] < len({q["cell_id"] for q in reqs})   # some were evicted
    finally:
        s.close()


def test_footprint_matches_device_bytes():
    cell = W.cluster(13, "Mg", seed=2, grid=48)
    for prec in (ofdft.FP64, ofdft.MIXED):
        cd, keep = ofdft.make_cell_desc(cell)
        fd = ofdft.make_functional_desc(TERMS, precision=prec)
        want = ofdft.ofdft_footprint_bytes(cd, fd, ofdft.REQ_OPTIMIZE)
        with ofdft.Grid(cell, TERMS, precision=prec) as g:
            rho = W.gaussian_density(cell, sigma=1.5, floor=1e-8)
            g.energy_potential(rho)
            g.set_density(rho)
            g.optimize(tol=1e-4, max_iter=5, allow_noconv=True)
            assert ofdft.ofdft_grid_device_bytes(g.handle) == want
            g.forces()
            # the forces and the force kernel's partial table: the model's
            # FORCES request less its EP request
            extra = (ofdft.ofdft_footprint_bytes(cd, fd, ofdft.REQ_FORCES) -
                     ofdft.ofdft_footprint_bytes(cd, fd, ofdft.REQ_EP))
            assert extra >= 13 * 3 * 8
            assert ofdft.ofdft_grid_device_bytes(g.handle) == want + extra


def test_error_codes():
    q0 = _stream(1)[0]
    s = Server(budget=0, max_inflight=1)
    try:
        bad = dict(q0)
        bad["rho"] = np.full(q0["cell"]["n"], 0.01)
        bad["rho"][1, 2, 3] = np.nan
        with pytest.raises(ofdft.OfdftError) as e:
            s.submit(bad)
        assert e.value.status == ofdft.EINVAL
        tiny = Server(budget=1 << 20, max_inflight=1)   # 1 MiB: below any footprint
        try:
            with pytest.raises(ofdft.OfdftError) as e:
                tiny.submit(q0)
            assert e.value.status == ofdft.ENOMEM
        finally:
            tiny.close()
        assert ofdft.ofdft_serve_poll(s.h, 987654, None, None)[0] == ofdft.ENOTFOUND
        assert ofdft.ofdft_serve_cancel(s.h, 987654) == ofdft.ENOTFOUND
        # a long optimisation, then a queued one behind it: cancel both
        slow = dict(q0)
        slow["kind"] = ofdft.REQ_OPTIMIZE
        t1 = s.submit(slow, opt=dict(tol=1e-14, max_iter=100000))
        t2 = s.submit(slow, opt=dict(tol=1e-14, max_iter=100000))
        time.sleep(0.2)
        assert ofdft.ofdft_serve_cancel(s.h, t2) == ofdft.OK
        assert ofdft.ofdft_serve_cancel(s.h, t1) == ofdft.OK
        for t in (t1, t2):
            assert s.result(t, slow)[0] == ofdft.ECANCELLED
            assert ofdft.ofdft_serve_poll(s.h, t, None, None)[0] == ofdft.ENOTFOUND
        # the server still serves after cancellations
        ok = dict(q0)
        ok["kind"] = ofdft.REQ_EP
        assert s.result(s.submit(ok), ok)[0] == ofdft.OK
        st = s.stats()
        assert st["cancelled"] == 2 and st["running"] == 0 and st["queued"] == 0
    finally:
        s.close()


def test_destroy_with_work_in_flight():
    reqs = _stream(6)
    s = Server(max_inflight=2)
    for q in reqs:
        s.submit(q)
    s.close()   # cancels what is queued, waits for what runs


def test_evicted_density_is_restored():
    """Under a budget of one grid, cell B evicts cell A; A's density is kept in
    host memory and is the warm start when A comes back without a density:
    its optimisation resumes from the converged density (no iterations),
    where a fresh server starts from the uniform density."""
    a = W.cluster(19, "Al", seed=11, grid=48)
    b = W.cluster(13, "Mg", seed=2, grid=48)
    fd = ofdft.make_functional_desc(TERMS, precision=ofdft.FP64)
    cd, keep = ofdft.make_cell_desc(a)
    budget = int(ofdft.ofdft_footprint_bytes(cd, fd, ofdft.REQ_OPTIMIZE) * 1.2)
    opt = dict(tol=1e-6, max_iter=400)

    def run(s, cid, cell, rho):
        q = {"cell_id": cid, "kind": ofdft.REQ_OPTIMIZE, "cell": cell, "rho": rho}
        st, r, _, _ = s.result(s.submit(q, opt=opt, func=fd), q)
        assert st == ofdft.OK
        return r

    s = Server(budget=budget, max_inflight=1)
    try:
        r1 = run(s, 0, a, W.gaussian_density(a, sigma=1.5, floor=1e-8))
        run(s, 1, b, W.gaussian_density(b, sigma=1.5, floor=1e-8))
        assert s.stats()["resident_cells"] == 1          # A was evicted
        r2 = run(s, 0, a, None)
    finally:
        s.close()
    s = Server(budget=budget, max_inflight=1)
    try:
        cold = run(s, 0, a, None)
    finally:
        s.close()
    _say("A: %d iterations, again after eviction %d, uniform start %d" % (
        r1.iters, r2.iters, cold.iters))
    assert r2.iters <= 2 < cold.iters
    assert abs(r2.e.e_total - r1.e.e_total) < 1e-8 * abs(r1.e.e_total)


def test_eviction_with_two_slots_keeps_the_density():
    """Two worker slots under a budget of one grid: while cell B's request
    evicts cell A, an energy request for A (no density of its own) arrives.
    It must wait until A's density has been saved and then start from it: its
    energy is the optimised energy of A, not that of the uniform start."""
    a = W.cluster(19, "Al", seed=11, grid=48)
    b = W.cluster(13, "Mg", seed=2, grid=48)
    fd = ofdft.make_functional_desc(TERMS, precision=ofdft.FP64)
    cd, keep = ofdft.make_cell_desc(a)
    budget = int(ofdft.ofdft_footprint_bytes(cd, fd, ofdft.REQ_OPTIMIZE) * 1.2)
    opt = dict(tol=1e-6, max_iter=400)
    s = Server(budget=budget, max_inflight=2)
    try:
        qa = {"cell_id": 0, "kind": ofdft.REQ_OPTIMIZE, "cell": a,
              "rho": W.gaussian_density(a, sigma=1.5, floor=1e-8)}
        st, r1, _, _ = s.result(s.submit(qa, opt=opt, func=fd), qa)
        assert st == ofdft.OK
        qb = {"cell_id": 1, "kind": ofdft.REQ_OPTIMIZE, "cell": b,
              "rho": W.gaussian_density(b, sigma=1.5, floor=1e-8)}
        qe = {"cell_id": 0, "kind": ofdft.REQ_EP, "cell": a, "rho": None}
        tb = s.submit(qb, opt=opt, func=fd)
        te = s.submit(qe, func=fd)
        st_b, _, _, _ = s.result(tb, qb)
        st_e, re, _, _ = s.result(te, qe)
        stats = s.stats()
    finally:
        s.close()
    _say("A optimised E %.10f; A again after eviction E %.10f; peak %d of budget %d" % (
        r1.e.e_total, re.e.e_total, stats["peak_bytes"], budget))
    assert st_b == ofdft.OK and st_e == ofdft.OK
    assert abs(re.e.e_total - r1.e.e_total) < 1e-8 * abs(r1.e.e_total)
    assert stats["peak_bytes"] <= budget
