"""Grouped column blocks: a block of the reciprocal-space column pass serves
one tile for up to 8 densities of a batch, with the tile's set-up and
per-element operands (1/G^2, G^2, the Wang-Teter kernel) shared.  Every
density's energies and potential must be the same, bit for bit, as with one
density per block (the other autotuner choice), on the fused plane path and
the row/column path, for the Wang-Teter and spline functionals, both
precisions.  The batches are large enough for the launcher to group (it
keeps at least 8192 blocks)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2002_02985_amd import ofdft
from paper_2002_02985_amd import workloads as W
from tests.gpu_helpers import dev_tensor, stream_handle, torch_dtype

pytestmark = pytest.mark.gpu

LOCAL = ofdft.TERM_TF | ofdft.TERM_VW | ofdft.TERM_HARTREE | ofdft.TERM_EXT


def run(grid, x, group):
    ofdft.ofdft_grid_set_col_group(grid.handle, group)
    v = torch.zeros_like(x)
    es = ofdft.ofdft_energy_potential_batch_dev(grid.handle, x.shape[0], x.data_ptr(),
                                                v.data_ptr(), stream_handle())
    torch.cuda.synchronize()
    return [e.as_dict() for e in es], v.cpu().numpy()


# 48^3 and 96^3 take the fused plane kernels; (48, 144, 144) the row and
# column passes (its 144 x 72 plane does not fit in LDS)
CASES = {
    "wt_48": ((48, 48, 48), 128, LOCAL | ofdft.TERM_WT, {}),
    "wt_96": ((96, 96, 96), 64, LOCAL | ofdft.TERM_WT, {}),
    "wt_rows": ((48, 144, 144), 16, LOCAL | ofdft.TERM_WT, {}),
    "spline_48": ((48, 48, 48), 128, LOCAL | ofdft.TERM_SPLINE,
                  dict(nk=12, kf_min=0.1, kf_max=2.5)),
}


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED])
@pytest.mark.parametrize("case", sorted(CASES))
def test_grouped_column_blocks_match_single(case, prec):
    n, nb, terms, kw = CASES[case]
    if prec == ofdft.FP64 and n[0] == 96:
        nb = 32
    cell, dens = W.config_c2(n, nb)
    print("case col group", case, prec, nb, flush=True)
    with ofdft.Grid(cell, terms, precision=prec, **kw) as g:
        x = dev_tensor(np.stack(dens), torch_dtype(g))
        e1, v1 = run(g, x, 1)
        e8, v8 = run(g, x, 8)
    for b in range(nb):
        for k in e1[b]:
            assert e8[b][k] == e1[b][k], (case, prec, b, k, e8[b][k], e1[b][k])
    assert np.array_equal(v8, v1), (case, prec)


def test_col_group_setter_checks_its_range():
    cell, _ = W.config_c2((32, 32, 32), 1)
    with ofdft.Grid(cell, LOCAL) as g:
        for bad in (0, 9, -1):
            with pytest.raises(ofdft.OfdftError) as ei:
                ofdft.ofdft_grid_set_col_group(g.handle, bad)
            assert ei.value.status == ofdft.EINVAL
        ofdft.ofdft_grid_set_col_group(g.handle, 4)


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED])
def test_repeated_batches_are_bit_identical(prec):
    """The same batch evaluated three times gives the same bits (the 96^3
    plane path, with the Wang-Teter combine that ends in 16-byte stores in
    FP64: stores whose data registers were overwritten too soon once left
    wrong low halves in a few thousand points per batch)."""
    nb = 32 if prec == ofdft.FP64 else 64
    cell, dens = W.config_c2((96, 96, 96), nb)
    print("case repeat", prec, nb, flush=True)
    with ofdft.Grid(cell, LOCAL | ofdft.TERM_WT, precision=prec) as g:
        x = dev_tensor(np.stack(dens), torch_dtype(g))
        runs = [run(g, x, 8) for _ in range(3)]
    for e, v in runs[1:]:
        assert np.array_equal(v, runs[0][1]), prec
        assert [d["e_total"] for d in e] == [d["e_total"] for d in runs[0][0]]
