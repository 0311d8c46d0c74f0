"""The no-allocation entry point ofdft_energy_potential_dev_noalloc against
ofdft_energy_potential_dev on the same grid and density: two calls in a row
on the library's shared static workspace, the second on a smaller grid, and a
grid whose workspace does not fit.  The two entry points run the same
launches, so energies and potentials are compared bit for bit (a stronger
check than the parity bar)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2002_02985_amd import ofdft
from paper_2002_02985_amd import workloads as W
from tests.gpu_helpers import dev_tensor, stream_handle, torch_dtype

pytestmark = pytest.mark.gpu

LOCAL = ofdft.TERM_TF | ofdft.TERM_VW | ofdft.TERM_HARTREE | ofdft.TERM_EXT
KEYS = ("e_tf", "e_vw", "e_h", "e_ext", "e_nl", "e_ion", "e_xc", "e_total", "mu",
        "nelec_int", "resid_norm")


def both(grid, rho):
    dt = torch_dtype(grid)
    x = dev_tensor(rho, dt)
    v_ref = torch.empty_like(x)
    v_na = torch.full_like(x, float("nan"))
    e_ref = ofdft.ofdft_energy_potential_dev(grid.handle, x.data_ptr(), v_ref.data_ptr(),
                                             stream_handle())
    e_na = ofdft.ofdft_energy_potential_dev_noalloc(grid.handle, x.data_ptr(), v_na.data_ptr(),
                                                    stream_handle())
    torch.cuda.synchronize()
    return e_ref.as_dict(), v_ref.cpu().numpy(), e_na.as_dict(), v_na.cpu().numpy()


def check_same(label, e_ref, v_ref, e_na, v_na):
    print("  %s: E %.12f / %.12f, max |dv| %.1e" %
          (label, e_ref["e_total"], e_na["e_total"], float(np.abs(v_ref - v_na).max())),
          flush=True)
    for k in KEYS:
        assert e_na[k] == e_ref[k], (label, k, e_na[k], e_ref[k])
    assert np.array_equal(v_na, v_ref), label


@pytest.mark.parametrize("prec", [ofdft.MIXED, ofdft.FP64, ofdft.MIXED_VW64])
def test_noalloc_matches_the_device_entry_point(prec):
    # call 1: the 96^3 WT cell (108 atoms); call 2: the smaller spline box on
    # 48 x 48 x 64 (a different workspace layout in the same array)
    cell1, dens = W.config_c2(ndens=1)
    cell2 = W.cluster(13, "Al", seed=7, grid=48)
    cell2["n"] = (48, 48, 64)
    rho2 = W.gaussian_density(cell2, sigma=1.5, floor=1e-10)
    print("case noalloc prec %d: 96^3 WT then 48x48x64 spline" % prec, flush=True)
    with ofdft.Grid(cell1, LOCAL | ofdft.TERM_WT, precision=prec) as g1, \
            ofdft.Grid(cell2, LOCAL | ofdft.TERM_SPLINE, precision=prec, nk=12, kf_min=0.1,
                       kf_max=2.5, nl_mode=ofdft.NL_EXACT) as g2:
        check_same("96^3 WT", *both(g1, dens[0]))
        check_same("48x48x64 spline", *both(g2, rho2))
        # and back to the first grid: the stale contents of the shared array
        # from the second call do not leak into the first grid's result
        check_same("96^3 WT again", *both(g1, dens[0]))


def test_noalloc_refuses_a_workspace_beyond_the_scratch():
    cell = W.mg_hcp_slab((2, 1, 2), n=(128, 128, 192), vacuum=8.0)
    rho = W.gaussian_density(cell, sigma=1.5, floor=1e-10)
    print("case noalloc refusal 128x128x192 spline", flush=True)
    with ofdft.Grid(cell, LOCAL | ofdft.TERM_SPLINE, precision=ofdft.FP64, nk=16) as g:
        x = dev_tensor(rho, torch.float64)
        v = torch.empty_like(x)
        with pytest.raises(ofdft.OfdftError) as ei:
            ofdft.ofdft_energy_potential_dev_noalloc(g.handle, x.data_ptr(), v.data_ptr(),
                                                     stream_handle())
        assert ei.value.status == ofdft.EINVAL
        assert "no-allocation scratch" in str(ei.value)
        # the ordinary entry point still works on the same grid
        e = ofdft.ofdft_energy_potential_dev(g.handle, x.data_ptr(), v.data_ptr(),
                                             stream_handle())
        assert np.isfinite(e.e_total)


def test_noalloc_rejects_a_negative_density():
    cell, rho = W.config_c1()
    with ofdft.Grid(cell, LOCAL, precision=ofdft.FP64) as g:
        bad = rho.copy()
        bad[1, 2, 3] = -1.0
        x = dev_tensor(bad, torch.float64)
        with pytest.raises(ofdft.OfdftError) as ei:
            ofdft.ofdft_energy_potential_dev_noalloc(g.handle, x.data_ptr(), None,
                                                     stream_handle())
        assert ei.value.status == ofdft.EINVAL
