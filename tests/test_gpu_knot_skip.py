"""The device-side knot range of the spline functional: the knot passes skip
knots whose hat functions vanish at every grid point, and the results must
be the same, bit for bit, as with every knot transformed (the skipped knots
add exact zeros).  Batches mix densities with narrow and wide k_F ranges, so
that different batch entries skip different knots; row path and plane path,
S3S4 and EXACT, FP64, MIXED and MIXED_VW64."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2002_02985_amd import ofdft
from paper_2002_02985_amd import workloads as W
from tests.gpu_helpers import dev_tensor, stream_handle, torch_dtype
from tests.oracle_helpers import make_cell, smooth_density

pytestmark = pytest.mark.gpu

LOCAL = ofdft.TERM_TF | ofdft.TERM_VW | ofdft.TERM_HARTREE | ofdft.TERM_EXT


def box(n, L=(9.0, 10.0, 11.0), natoms=3, seed=0, Z=2.0):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, size=(natoms, 3)) * np.array(L)
    return {"lattice": np.diag(L), "n": n, "pos": pos, "species": np.zeros(natoms, np.int32),
            "Z": np.array([Z]), "rc": np.array([1.0]), "nelec": Z * natoms}


def densities(cell):
    c = make_cell(cell)
    narrow = smooth_density(c, seed=3, amp=0.05, nmodes=2, rho0=0.02)    # a few knots
    wide = smooth_density(c, seed=4, amp=0.95, nmodes=3, rho0=0.03)      # many knots
    # a cluster-like density with vacuum: k_F clamped at the lowest knot
    vac = W.gaussian_density(cell, sigma=1.2, floor=1e-10)
    return [narrow, wide, vac]


def run(grid, rhos, skip):
    ofdft.ofdft_grid_set_knot_skip(grid.handle, skip)
    dt = torch_dtype(grid)
    x = dev_tensor(np.stack(rhos), dt)
    v = torch.zeros_like(x)
    es = ofdft.ofdft_energy_potential_batch_dev(grid.handle, len(rhos), x.data_ptr(),
                                                v.data_ptr(), stream_handle())
    torch.cuda.synchronize()
    return [e.as_dict() for e in es], v.cpu().numpy()


CASES = {
    "row_s3s4": ((24, 16, 12), ofdft.NL_S3S4),
    "row_exact": ((24, 16, 12), ofdft.NL_EXACT),
    "plane_s3s4": ((16, 32, 32), ofdft.NL_S3S4),
    "plane_exact": ((16, 32, 32), ofdft.NL_EXACT),
}


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED, ofdft.MIXED_VW64])
@pytest.mark.parametrize("case", sorted(CASES))
def test_knot_skip_matches_every_knot(case, prec):
    n, mode = CASES[case]
    cell = box(n)
    rhos = densities(cell)
    print("case knot skip", case, prec, flush=True)
    with ofdft.Grid(cell, LOCAL | ofdft.TERM_SPLINE, precision=prec, nk=24, kf_min=0.1,
                    kf_max=3.0, nl_mode=mode) as g:
        e_on, v_on = run(g, rhos, True)
        e_off, v_off = run(g, rhos, False)
        e_on2, v_on2 = run(g, rhos, True)
    for b in range(len(rhos)):
        for k in ("e_nl", "e_total", "mu", "resid_norm"):
            assert e_on[b][k] == e_off[b][k], (case, b, k, e_on[b][k], e_off[b][k])
            assert e_on2[b][k] == e_on[b][k]
    assert np.array_equal(v_on, v_off), float(np.abs(v_on - v_off).max())
    assert np.array_equal(v_on2, v_on)


def test_knot_skip_on_the_slab_grid():
    """The 256 x 256 x 384 Mg slab (32 knots; the slab's densest point
    brackets knot 23, so about a quarter of the knots are skipped): skipping
    leaves the energy and potential unchanged in MIXED."""
    cell, rho = W.config_c3()
    print("case knot skip slab", flush=True)
    with ofdft.Grid(cell, LOCAL | ofdft.TERM_SPLINE, precision=ofdft.MIXED, nk=32, kf_min=0.1,
                    kf_max=3.0, nl_mode=ofdft.NL_S3S4) as g:
        e_on, v_on = run(g, [rho], True)
        e_off, v_off = run(g, [rho], False)
    assert e_on[0]["e_total"] == e_off[0]["e_total"]
    assert np.array_equal(v_on, v_off)


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED, ofdft.MIXED_VW64])
@pytest.mark.parametrize("case", sorted(CASES))
def test_knot_pipeline_matches_one_stream(case, prec):
    """24 knots = 3 batches: with the knot pipeline the knot transforms of a
    batch run on the grid's second stream into alternating buffers; the
    energies and potentials are the same, bit for bit, as on one stream."""
    n, mode = CASES[case]
    cell = box(n)
    rhos = densities(cell)
    print("case knot pipeline", case, prec, flush=True)
    with ofdft.Grid(cell, LOCAL | ofdft.TERM_SPLINE, precision=prec, nk=24, kf_min=0.1,
                    kf_max=3.0, nl_mode=mode) as g:
        ofdft.ofdft_grid_set_knot_pipeline(g.handle, True)
        e_on, v_on = run(g, rhos, True)
        ofdft.ofdft_grid_set_knot_pipeline(g.handle, False)
        e_off, v_off = run(g, rhos, True)
        ofdft.ofdft_grid_set_knot_pipeline(g.handle, True)
        e_on2, v_on2 = run(g, rhos, True)
    for b in range(len(rhos)):
        for k in e_on[b]:
            assert e_on[b][k] == e_off[b][k], (case, b, k)
            assert e_on2[b][k] == e_on[b][k]
    assert np.array_equal(v_on, v_off)
    assert np.array_equal(v_on2, v_on)
