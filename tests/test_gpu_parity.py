"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (stated per result):
* FP64 path: relative 1e-10 in every energy term, 1e-9 Ha absolute in the
  potential, 1e-8 Ha/Bohr in forces; FFTs to 1e-12 of the spectrum's scale.
* Mixed path (FP32 fields, FP64 reductions): |dE| <= 1e-5 Ha per atom,
  max |dv| <= 1e-4 Ha on points with rho >= 1e-6, forces <= 1e-4 Ha/Bohr;
  FFTs to 2e-6 of the spectrum's scale.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import cell as OC
from oracle import functionals as OF
from oracle.ewald import ewald_energy, forces as oracle_forces
from oracle.fourier import c2r as o_c2r, r2c as o_r2c
from paper_2002_02985_amd import ofdft
from paper_2002_02985_amd import workloads as W
from tests.gpu_helpers import eval_batch, fft_c2r, fft_r2c
from tests.oracle_helpers import make_cell, smooth_density

pytestmark = pytest.mark.gpu

LOCAL = ofdft.TERM_TF | ofdft.TERM_VW | ofdft.TERM_HARTREE | ofdft.TERM_EXT
ENERGY_KEYS = ("e_tf", "e_vw", "e_h", "e_ext", "e_nl", "e_ion", "e_xc", "e_total")


def oracle_func(terms, **kw):
    return OC.Functional(terms=int(terms), **kw)


def box(n, L=(9.0, 10.0, 11.0), natoms=3, seed=0, Z=2.0):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, size=(natoms, 3)) * np.array(L)
    return {"lattice": np.diag(L), "n": n, "pos": pos, "species": np.zeros(natoms, np.int32),
            "Z": np.array([Z]), "rc": np.array([1.0]), "nelec": Z * natoms}


def tri(n, natoms=3, seed=0, Z=2.0):
    """A skewed (triclinic) cell: the aliased Nyquist frequencies of the
    self-conjugate planes then have partners with a different |G|."""
    lat = np.array([[9.0, 0.0, 0.0], [-3.5, 9.5, 0.0], [1.2, -0.8, 10.5]])
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, size=(natoms, 3)) @ lat
    return {"lattice": lat, "n": n, "pos": pos, "species": np.zeros(natoms, np.int32),
            "Z": np.array([Z]), "rc": np.array([1.0]), "nelec": Z * natoms}


def varied_rho(cell_d, seed=1, amp=0.9, rho0=0.03):
    c = make_cell(cell_d)
    return smooth_density(c, seed=seed, amp=amp, nmodes=3, rho0=rho0)


def compare(e_gpu, v_gpu, ro, rho, natoms, fp64, label=""):
    if fp64:
        for k in ENERGY_KEYS:
            ref = getattr(ro, k)
            assert abs(e_gpu[k] - ref) <= 1e-10 * max(1.0, abs(ref)), (label, k, e_gpu[k], ref)
        assert abs(e_gpu["mu"] - ro.mu) <= 1e-10 * max(1.0, abs(ro.mu))
        np.testing.assert_allclose(v_gpu, ro.v, rtol=0, atol=1e-9, err_msg=label)
    else:
        tol = 1e-5 * max(natoms, 1)
        for k in ENERGY_KEYS:
            assert abs(e_gpu[k] - getattr(ro, k)) <= tol, (label, k, e_gpu[k], getattr(ro, k))
        mask = rho >= 1e-6
        err = np.abs(v_gpu - ro.v)[mask].max()
        assert err <= 1e-4, (label, err)
    # the mixed path rounds the input density to FP32 (relative 6e-8 per value)
    tol_n = 1e-9 if fp64 else 1e-7
    assert abs(e_gpu["nelec_int"] - ro.nelec_int) <= tol_n * ro.nelec_int


# ------------------------------------------------------------------ FFT
FFT_SHAPES = [(12, 18, 16), (24, 16, 12), (6, 4, 4), (32, 32, 32), (18, 27, 54), (96, 96, 96),
              # the 1024-point transforms of the 1024^3 cell on each axis
              (1024, 4, 8), (6, 1024, 4), (8, 6, 1024)]


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED])
@pytest.mark.parametrize("shape", FFT_SHAPES)
def test_fft_pair_against_oracle(shape, prec):
    print("case fft", shape, prec, flush=True)
    cell = box(shape)
    rng = np.random.default_rng(sum(shape))
    nb = 2
    f = rng.standard_normal((nb,) + shape)
    with ofdft.Grid(cell, ofdft.TERM_TF, precision=prec) as g:
        X = fft_r2c(g, f)
        ref = np.stack([o_r2c(f[b]) for b in range(nb)])
        scale = np.abs(ref).max()
        tol = 1e-12 if prec == ofdft.FP64 else 2e-6
        assert np.abs(X - ref).max() <= tol * scale
        # inverse of the oracle spectrum (with imaginary parts on the
        # self-conjugate planes, which the inverse must drop)
        spec = ref.copy()
        spec[:, 0, 0, 0] += 0.3j
        back = fft_c2r(g, spec)
        rref = np.stack([o_c2r(spec[b], shape) for b in range(nb)])
        assert np.abs(back - rref).max() <= tol * np.abs(rref).max() * 4


# ------------------------------------------------------------------ energies
def c1_cell():
    cell, rho = W.config_c1()
    return cell, rho


CASES = {
    "c1_local": (lambda: c1_cell(), LOCAL, {}),
    "c1_wt": (lambda: c1_cell(), LOCAL | ofdft.TERM_WT, {}),
    "box_tf_only": (lambda: (box((12, 18, 16)), None), ofdft.TERM_TF, {}),
    "box_hartree_only": (lambda: (box((12, 18, 16)), None), ofdft.TERM_HARTREE, {}),
    "box_wt": (lambda: (box((24, 16, 12)), None), ofdft.TERM_VW | ofdft.TERM_WT, {}),
    "box_spline_s3s4": (lambda: (box((24, 16, 12)), None), LOCAL | ofdft.TERM_SPLINE,
                        dict(nk=10, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_S3S4)),
    "box_spline_exact": (lambda: (box((24, 16, 12)), None), LOCAL | ofdft.TERM_SPLINE,
                         dict(nk=10, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_EXACT)),
    # (16, 32, 32) and 32^3 run through the fused plane kernels, the others
    # through the separate row and column passes
    "plane_spline_s3s4": (lambda: (box((16, 32, 32)), None), LOCAL | ofdft.TERM_SPLINE,
                          dict(nk=12, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_S3S4)),
    "plane_spline_exact": (lambda: (box((16, 32, 32)), None), LOCAL | ofdft.TERM_SPLINE,
                           dict(nk=12, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_EXACT)),
    "box_spline_lin_exact": (lambda: (box((18, 16, 24)), None), ofdft.TERM_SPLINE,
                             dict(nk=13, kf_min=0.4, kf_max=1.9, knot_spacing=ofdft.KNOTS_LIN,
                                  nl_mode=ofdft.NL_EXACT)),
    # LDA exchange-correlation: with the fixed term sets (plane path) and the
    # general combine (row path), and a dense box whose r_s spans both
    # branches of the correlation fit
    "c1_local_xc": (lambda: c1_cell(), LOCAL | ofdft.TERM_XC, {}),
    "c1_wt_xc": (lambda: c1_cell(), LOCAL | ofdft.TERM_WT | ofdft.TERM_XC, {}),
    "box_spline_s3s4_xc": (lambda: (box((24, 16, 12)), None),
                           LOCAL | ofdft.TERM_SPLINE | ofdft.TERM_XC,
                           dict(nk=10, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_S3S4)),
    "box_xc_dense": (lambda: (box((12, 18, 16), L=(2.5, 2.7, 3.0)), None),
                     ofdft.TERM_TF | ofdft.TERM_XC, {}),
    # 1024-point axes (the million-atom grid's column and knot kernels) at a
    # realistic spacing (0.29 Bohr; on an over-resolved axis the vW Laplacian
    # multiplies FP32 rounding by G_max^2, which grows as the square of the
    # number of points)
    "spline_1024_axis0_s3s4": (lambda: (box((1024, 4, 8), L=(300.0, 6.0, 7.0), natoms=40), None),
                               LOCAL | ofdft.TERM_SPLINE,
                               dict(nk=9, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_S3S4)),
    "spline_1024_axis0_exact": (lambda: (box((1024, 4, 8), L=(300.0, 6.0, 7.0), natoms=40), None),
                                LOCAL | ofdft.TERM_SPLINE,
                                dict(nk=9, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_EXACT)),
    "spline_1024_axis1_s3s4": (lambda: (box((4, 1024, 8), L=(6.0, 300.0, 7.0), natoms=40), None),
                               LOCAL | ofdft.TERM_SPLINE,
                               dict(nk=9, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_S3S4)),
    # MGP-family kernels (eq. "MGP"): the Wang-Teter-type functional at the
    # cell's average k_F (fixed combine, plane path) and the LMGP spline
    # functionals on the row path and the plane path
    "c1_mgp": (lambda: c1_cell(), LOCAL | ofdft.TERM_WT, dict(nl_kernel=ofdft.KERNEL_MGP)),
    "box_wt_mgpa": (lambda: (box((24, 16, 12)), None), LOCAL | ofdft.TERM_WT,
                    dict(nl_kernel=ofdft.KERNEL_MGPA)),
    "box_wt_mgpg": (lambda: (box((24, 16, 12)), None), LOCAL | ofdft.TERM_WT,
                    dict(nl_kernel=ofdft.KERNEL_MGPG)),
    "box_lmgp_s3s4": (lambda: (box((24, 16, 12)), None), LOCAL | ofdft.TERM_SPLINE,
                      dict(nk=10, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_S3S4,
                           nl_kernel=ofdft.KERNEL_MGP)),
    "box_lmgpa_exact": (lambda: (box((24, 16, 12)), None), LOCAL | ofdft.TERM_SPLINE,
                        dict(nk=10, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_EXACT,
                             nl_kernel=ofdft.KERNEL_MGPA)),
    "plane_lmgpg_exact": (lambda: (box((16, 32, 32)), None), LOCAL | ofdft.TERM_SPLINE,
                          dict(nk=12, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_EXACT,
                               nl_kernel=ofdft.KERNEL_MGPG)),
    # triclinic cells, row path and plane path
    "tri_wt": (lambda: (tri((24, 16, 12)), None), LOCAL | ofdft.TERM_WT, {}),
    "tri_spline_s3s4": (lambda: (tri((18, 16, 24)), None), LOCAL | ofdft.TERM_SPLINE,
                        dict(nk=10, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_S3S4)),
    "tri_plane_spline_exact": (lambda: (tri((16, 32, 32)), None), LOCAL | ofdft.TERM_SPLINE,
                               dict(nk=12, kf_min=0.3, kf_max=2.0, nl_mode=ofdft.NL_EXACT)),
}


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED, ofdft.MIXED_VW64])
@pytest.mark.parametrize("name", sorted(CASES))
def test_energy_potential_parity(name, prec):
    print("case energy", name, prec, flush=True)
    mk, terms, kw = CASES[name]
    cell, rho = mk()
    if rho is None:
        rho = varied_rho(cell)
    oc = make_cell(cell)
    ro = OF.energy_potential(oc, oracle_func(terms, **kw), rho=rho)
    with ofdft.Grid(cell, terms, precision=prec, **kw) as g:
        e, v = g.energy_potential(rho)
        compare(e.as_dict(), v, ro, rho, len(cell["species"]), prec == ofdft.FP64, name)
        # resident-density path gives the same numbers
        g.set_density(rho)
        e2, _ = g.energy_potential(None, want_v=False)
        assert e2.e_total == e.e_total


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED])
def test_batch_matches_single(prec):
    cell, _ = c1_cell()
    rhos = [varied_rho(cell, seed=s, amp=0.5, rho0=12 / 7.65 ** 3) for s in range(3)]
    terms = LOCAL | ofdft.TERM_WT
    with ofdft.Grid(cell, terms, precision=prec) as g:
        es, vs = eval_batch(g, rhos)
        for b, rho in enumerate(rhos):
            e1, v1 = g.energy_potential(rho)
            for k in ENERGY_KEYS + ("mu", "resid_norm"):
                assert es[b][k] == getattr(e1, k), (b, k)
            assert np.array_equal(vs[b], v1.astype(vs.dtype)) if prec == ofdft.FP64 else \
                np.abs(vs[b] - v1).max() == 0.0


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED])
def test_input_validation(prec):
    cell, rho = c1_cell()
    with ofdft.Grid(cell, LOCAL, precision=prec) as g:
        bad = rho.copy()
        bad[3, 4, 5] = -1.0
        with pytest.raises(ofdft.OfdftError) as ei:
            g.energy_potential(bad)
        assert ei.value.status == ofdft.EINVAL
        bad[3, 4, 5] = np.nan
        with pytest.raises(ofdft.OfdftError):
            g.energy_potential(bad)
        # a negative value below the smallest FP32 subnormal (it would round
        # to -0 in the mixed path) is refused in both precisions
        bad[3, 4, 5] = -1e-300
        with pytest.raises(ofdft.OfdftError) as ei:
            g.energy_potential(bad)
        assert ei.value.status == ofdft.EINVAL
    bad_cell = dict(cell)
    bad_cell["n"] = (30, 32, 32)
    with pytest.raises(ofdft.OfdftError) as ei:
        ofdft.Grid(bad_cell, LOCAL)
    assert ei.value.status == ofdft.EINVAL


# ------------------------------------------------------------------ forces
@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED])
def test_forces_parity(prec):
    cell = W.al_fcc_cell(1, (24, 24, 24), jitter=0.15, seed=21)
    oc = make_cell(cell)
    rho = smooth_density(oc, seed=8)
    ro = OF.energy_potential(oc, OC.Functional(terms=OC.EXT), rho=rho)
    ref = oracle_forces(oc, ro.rho_g)
    with ofdft.Grid(cell, LOCAL, precision=prec) as g:
        g.set_density(rho)
        F = g.forces()
    tol = 1e-8 if prec == ofdft.FP64 else 1e-4
    assert np.abs(F - ref).max() <= tol, np.abs(F - ref).max()


# ------------------------------------------------------------------ optimiser
def test_optimize_c1_fp64_matches_oracle_minimum():
    from oracle.optimize import optimize as o_opt
    cell, rho = c1_cell()
    oc = make_cell(cell)
    func = OC.Functional(terms=int(LOCAL))
    ref = o_opt(oc, func, np.sqrt(rho), tol=1e-7, max_iter=500, vext=OF.vext_g(oc),
                e_ion=ewald_energy(oc))
    assert ref.converged
    with ofdft.Grid(cell, LOCAL) as g:
        g.set_density(rho)
        r, st = g.optimize(tol=1e-7, max_iter=500)
        assert st == ofdft.OK
        rho_gpu = g.get_density()
    assert r.final_resid < 1e-7
    assert abs(r.e.e_total - ref.result.e_total) < 1e-9
    assert abs(oc.dv * rho_gpu.sum() - cell["nelec"]) < 1e-10
    np.testing.assert_allclose(rho_gpu, ref.phi ** 2, atol=1e-6)


def test_optimize_c1_preconditioned_reaches_the_same_minimum():
    """The preconditioned search direction changes the path, not the
    minimiser (TF+vW+H+ext is strictly convex in rho)."""
    from oracle.optimize import optimize as o_opt
    cell, rho = c1_cell()
    oc = make_cell(cell)
    ref = o_opt(oc, OC.Functional(terms=int(LOCAL)), np.sqrt(rho), tol=1e-7, max_iter=500,
                vext=OF.vext_g(oc), e_ion=ewald_energy(oc))
    with ofdft.Grid(cell, LOCAL) as g:
        g.set_density(rho)
        r, st = g.optimize(tol=1e-7, max_iter=500, method=ofdft.OPT_PCG)
        assert st == ofdft.OK
        g.set_density(rho)
        r0, _ = g.optimize(tol=1e-7, max_iter=500)
    print("c1 iterations: CG %d (%d evals), PCG %d (%d evals)" % (r0.iters, r0.evals, r.iters,
                                                                   r.evals), flush=True)
    assert abs(r.e.e_total - ref.result.e_total) < 1e-9


@pytest.mark.parametrize("name", ["c1_local", "c1_wt", "c1_local_xc"])
def test_truncated_newton_reaches_the_oracle_minimum(name):
    """The truncated-Newton direction changes the path, not the minimiser:
    the oracle's CG minimum (TF+vW+H+ext, with WT or LDA) to 1e-9 Ha in FP64,
    1e-5 Ha/atom mixed."""
    from oracle.optimize import optimize as o_opt
    mk, terms, kw = CASES[name]
    cell, rho = mk()
    oc = make_cell(cell)
    ref = o_opt(oc, oracle_func(terms, **kw), np.sqrt(rho), tol=1e-7, max_iter=800,
                vext=OF.vext_g(oc), e_ion=ewald_energy(oc))
    assert ref.converged
    natoms = len(cell["species"])
    for prec in (ofdft.FP64, ofdft.MIXED):
        with ofdft.Grid(cell, terms, precision=prec, **kw) as g:
            g.set_density(rho)
            tol = 1e-7 if prec == ofdft.FP64 else 2e-5
            r, st = g.optimize(tol=tol, max_iter=300, method=ofdft.OPT_TN)
            g.set_density(rho)
            rp, _ = g.optimize(tol=tol, max_iter=300, method=ofdft.OPT_PCG)
        print("%s %s: TN %d it %d ev, PCG %d it %d ev, dE %.2e" % (
            name, "fp64" if prec == ofdft.FP64 else "mixed", r.iters, r.evals, rp.iters,
            rp.evals, r.e.e_total - ref.result.e_total), flush=True)
        assert st == ofdft.OK
        if prec == ofdft.FP64:
            assert abs(r.e.e_total - ref.result.e_total) < 1e-9
        else:
            assert abs(r.e.e_total - ref.result.e_total) <= 1e-5 * natoms


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED])
def test_preconditioner_speeds_up_a_vacuum_cluster(prec):
    cell = W.cluster(19, "Al", seed=11, grid=48)
    rho = W.gaussian_density(cell, sigma=1.5, floor=1e-8)
    res = {}
    for m in (ofdft.OPT_CG, ofdft.OPT_PCG):
        with ofdft.Grid(cell, LOCAL, precision=prec) as g:
            g.set_density(rho)
            res[m] = g.optimize(tol=1e-5, max_iter=2000, method=m, allow_noconv=True)
    (rc, sc), (rp, sp) = res[ofdft.OPT_CG], res[ofdft.OPT_PCG]
    print("cluster %s: CG %d it %d ev resid %.1e E %.10f; PCG %d it %d ev resid %.1e E %.10f" %
          ("fp64" if prec == ofdft.FP64 else "mixed", rc.iters, rc.evals, rc.final_resid,
           rc.e.e_total, rp.iters, rp.evals, rp.final_resid, rp.e.e_total), flush=True)
    assert sp == ofdft.OK
    assert rp.iters < rc.iters
    if sc == ofdft.OK:
        # both stop at an RMS residual below 1e-5, whose energy error is O(resid^2)
        assert abs(rp.e.e_total - rc.e.e_total) <= (1e-6 if prec == ofdft.FP64 else 1e-4)


def test_spline_s3s4_optimisation_reaches_the_euler_solution():
    """With the interpolated (S3S4) potential the search solves the Euler
    equation: the residual of the returned density is below tol, and a fresh
    evaluation of that density agrees."""
    cell = W.mg_hcp_slab((1, 1, 2), (16, 24, 48), vacuum=8.0)
    rho = W.gaussian_density(cell, sigma=1.5, floor=1e-12)
    kw = dict(nk=16, kf_min=0.1, kf_max=3.0, nl_mode=ofdft.NL_S3S4)
    with ofdft.Grid(cell, LOCAL | ofdft.TERM_SPLINE, precision=ofdft.FP64, **kw) as g:
        g.set_density(rho)
        r, st = g.optimize(tol=1e-6, max_iter=800, method=ofdft.OPT_PCG)
        e, _ = g.energy_potential(None, want_v=False)
    print("slab S3S4: %d iterations, %d evaluations, resid %.2e" % (r.iters, r.evals,
                                                                    r.final_resid), flush=True)
    assert st == ofdft.OK and r.final_resid < 1e-6
    assert e.resid_norm < 1e-6
    assert abs(e.e_total - r.e.e_total) < 1e-9
    assert abs(e.nelec_int - cell["nelec"]) < 1e-9


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED])
@pytest.mark.parametrize("which", ["c2", "c3"])
def test_large_cell_ionic_path_matches(which, prec, monkeypatch):
    """The tiled structure factor and the binned Ewald sum (used from 8192
    atoms on) against the phase-table direct sum and the all-pairs Ewald sum
    on the same cell."""
    if which == "c2":   # bins for the real-space sum (three cut-offs fit across)
        cell, dens = W.config_c2((96, 96, 96), 1)
        rho = dens[0]
    else:               # narrower than three cut-offs: images of all pairs
        cell = W.mg_hcp_slab((6, 4, 9), (96, 96, 144), vacuum=15.0, jitter=0.05, seed=7)
        rho = W.gaussian_density(cell, sigma=1.5, floor=1e-12)
    res = {}
    for large in ("0", "1"):
        monkeypatch.setenv("OFDFT_LARGE_IONS", large)
        with ofdft.Grid(cell, LOCAL, precision=prec) as g:
            e, v = g.energy_potential(rho)
            res[large] = (e.as_dict(), v, ofdft.ofdft_grid_device_bytes(g.handle))
    e0, v0, b0 = res["0"]
    e1, v1, b1 = res["1"]
    print("%s prec %d: e_ext %.3e e_ion %.3e dv %.3e" % (
        which, prec, e1["e_ext"] - e0["e_ext"], e1["e_ion"] - e0["e_ion"],
        float(np.abs(v1 - v0).max())), flush=True)
    tol = 1e-10 if prec == ofdft.FP64 else 1e-5 * len(cell["species"])
    assert abs(e1["e_ion"] - e0["e_ion"]) <= 1e-10 * abs(e0["e_ion"])
    assert abs(e1["e_ext"] - e0["e_ext"]) <= tol * (abs(e0["e_ext"]) if prec == ofdft.FP64 else 1)
    assert float(np.abs(v1 - v0).max()) <= (1e-9 if prec == ofdft.FP64 else 1e-4)
    assert b1 < b0   # no per-atom phase tables


def test_graph_replay_matches_eager():
    """Evaluations replayed from captured HIP graphs give the eager results
    bit for bit, across argument sets and with eager work between replays."""
    cell, rho = c1_cell()
    terms = LOCAL | ofdft.TERM_WT
    xs = [torch.from_numpy(rho).to("cuda:0"), torch.from_numpy(rho * 1.01).to("cuda:0")]
    v = torch.zeros_like(xs[0])
    st = torch.cuda.Stream()
    with ofdft.Grid(cell, terms) as g, torch.cuda.stream(st):
        h = st.cuda_stream
        ref = []
        for x in xs:
            e = ofdft.ofdft_energy_potential_dev(g.handle, x.data_ptr(), v.data_ptr(), h)
            st.synchronize()
            ref.append((e.e_total, e.mu, v.cpu().numpy().copy()))
        ofdft.ofdft_grid_set_graphs(g.handle, True)
        for rep in range(4):
            for k, x in enumerate(xs):
                v.zero_()
                e = ofdft.ofdft_energy_potential_dev(g.handle, x.data_ptr(), v.data_ptr(), h)
                st.synchronize()
                assert e.e_total == ref[k][0] and e.mu == ref[k][1], (rep, k)
                assert np.array_equal(v.cpu().numpy(), ref[k][2]), (rep, k)
                xs[1 - k].mul_(1.0)   # eager work between replays
                st.synchronize()
        # the optimiser runs its evaluations through the graphs as well
        g.set_density(rho)
        r1, s1 = g.optimize(tol=1e-7, max_iter=300, method=ofdft.OPT_PCG)
        ofdft.ofdft_grid_set_graphs(g.handle, False)
        g.set_density(rho)
        r0, s0 = g.optimize(tol=1e-7, max_iter=300, method=ofdft.OPT_PCG)
    assert s1 == s0 == ofdft.OK
    assert r1.e.e_total == r0.e.e_total and r1.iters == r0.iters


PIPE_CASES = ["c1_wt", "box_spline_exact", "plane_spline_s3s4"]


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED])
@pytest.mark.parametrize("name", PIPE_CASES)
def test_pipelined_batch_matches_one_batch(name, prec):
    """A batch split into sub-batches over two streams (2 or 4 of them, the
    last one short) gives every density's energy and potential bit for bit as
    one batch does, launched eagerly and replayed from graphs."""
    mk, terms, kw = CASES[name]
    cell, rho = mk()
    rhos = [varied_rho(cell, seed=s, amp=0.5) * (1.0 + 0.05 * s) for s in range(5)]
    dt = torch.float64 if prec == ofdft.FP64 else torch.float32
    x = torch.from_numpy(np.stack(rhos)).to(dtype=dt, device="cuda:0")
    st = torch.cuda.Stream()
    out = {}
    for pipe in (1, 2, 4):
        print("case pipe", name, prec, pipe, flush=True)
        with ofdft.Grid(cell, terms, precision=prec, **kw) as g, torch.cuda.stream(st):
            ofdft.ofdft_grid_set_pipeline(g.handle, pipe)
            h = st.cuda_stream
            for graphs in (False, True, True):
                ofdft.ofdft_grid_set_graphs(g.handle, graphs)
                v = torch.full_like(x, float("nan"))
                es = ofdft.ofdft_energy_potential_batch_dev(g.handle, 5, x.data_ptr(),
                                                            v.data_ptr(), h)
                st.synchronize()
                got = ([e.e_total for e in es], [e.mu for e in es], v.cpu().numpy())
                if pipe == 1 and not graphs:
                    out["ref"] = got
                    continue
                ref = out["ref"]
                assert got[0] == ref[0] and got[1] == ref[1], (pipe, graphs)
                assert np.array_equal(got[2], ref[2]), (pipe, graphs)
                x.mul_(1.0)   # eager work between replays
                st.synchronize()


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED])
def test_autotuner_keeps_the_result(prec):
    cell, dens = W.config_c2((96, 96, 96), 2)
    dt = torch.float64 if prec == ofdft.FP64 else torch.float32
    x = torch.from_numpy(np.stack(dens)).to(dtype=dt, device="cuda:0")
    v = torch.zeros_like(x)
    h = torch.cuda.current_stream().cuda_stream
    with ofdft.Grid(cell, LOCAL | ofdft.TERM_WT, precision=prec) as g:
        e0 = ofdft.ofdft_energy_potential_batch_dev(g.handle, 2, x.data_ptr(), v.data_ptr(), h)
        res = ofdft.ofdft_grid_tune_dev(g.handle, 2, x.data_ptr(), h)
        e1 = ofdft.ofdft_energy_potential_batch_dev(g.handle, 2, x.data_ptr(), v.data_ptr(), h)
    print("tuned", prec, res, flush=True)
    assert res["candidates"] >= 2 and res["best_ms"] <= res["default_ms"] * 1.0001
    tol = 1e-10 * abs(e0[0].e_total) if prec == ofdft.FP64 else 1e-5 * len(cell["species"])
    for a, b in zip(e0, e1):
        assert abs(a.e_total - b.e_total) <= tol
