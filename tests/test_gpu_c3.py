"""Full-size parity of the spline nonlocal path: the Mg hcp slab (864 atoms,
15 Bohr vacuum) on its 256 x 256 x 384 grid with N_k = 32 knots, against
the FP64 oracle's energy terms and potential at seeded sample points
(tests/golden/c3_mg864_256x256x384.json, written by make_c3_golden.py from
oracle/ only).  Tolerances: FP64 relative 1e-10 per energy term, 1e-9 Ha in
dE/drho where rho >= 1e-6 (the vacuum holds floor values) and in
dE/dphi = 2 phi v everywhere; mixed with the FP64 von Weizsaecker leg
(MIXED_VW64, the mode for cells with vacuum) 1e-5 Ha/atom, 1e-4 Ha in
dE/drho where rho >= 1e-6 and in dE/dphi everywhere; plain MIXED the same
bars with dE/drho checked where rho >= 1e-3 (its FP32 Laplacian of phi,
divided by phi, is what the FP64 leg removes)."""
import json
import os
import sys

import numpy as np
import pytest

from paper_2002_02985_amd import ofdft
from paper_2002_02985_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "c3_mg864_256x256x384.json")
TERMS = (ofdft.TERM_TF | ofdft.TERM_VW | ofdft.TERM_HARTREE | ofdft.TERM_EXT |
         ofdft.TERM_SPLINE)
KEYS = ("e_tf", "e_vw", "e_h", "e_ext", "e_nl", "e_ion", "e_total")


@pytest.fixture(scope="module")
def c3():
    if not os.path.exists(GOLDEN):
        pytest.skip("golden values not generated")
    with open(GOLDEN) as f:
        gold = json.load(f)
    cell, rho = W.config_c3()
    return cell, rho, gold


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED, ofdft.MIXED_VW64])
@pytest.mark.parametrize("mode", ["s3s4", "exact"])
def test_c3_full_size_against_oracle(c3, mode, prec):
    cell, rho, gold = c3
    print("c3 parity", mode, prec, flush=True)
    ref = gold["modes"][mode]
    idx = np.asarray(gold["sample_index"])
    nl = ofdft.NL_S3S4 if mode == "s3s4" else ofdft.NL_EXACT
    with ofdft.Grid(cell, TERMS, precision=prec, nk=32, kf_min=0.1, kf_max=3.0,
                    nl_mode=nl) as g:
        e, v = g.energy_potential(rho)
    e = e.as_dict()
    vs = v.reshape(-1)[idx]
    vr = np.asarray(ref["v_samples"])
    rs = rho.reshape(-1)[idx]
    de = {k: e[k] - ref["energy"][k] for k in KEYS}
    dv = np.abs(vs - vr)
    print("  dE", {k: "%.2e" % x for k, x in de.items()}, "max dv %.2e" % dv.max(),
          "max dv (rho>=1e-6) %.2e" % dv[rs >= 1e-6].max(),
          "(rho>=1e-4) %.2e" % dv[rs >= 1e-4].max(), "(rho>=1e-3) %.2e" % dv[rs >= 1e-3].max())
    for j in np.argsort(dv)[::-1][:6]:
        print("    rho %.3e v %.6e dv %.2e" % (rs[j], vr[j], dv[j]))
    sys.stdout.flush()
    natoms = len(cell["species"])
    # in the vacuum the density sits at its floor, where v_vW = -lap(phi) / (2 phi_fl)
    # multiplies rounding by 1/phi_fl = 1e6: potentials are compared where rho >= 1e-6
    if prec == ofdft.FP64:
        for k in KEYS:
            assert abs(de[k]) <= 1e-10 * max(1.0, abs(ref["energy"][k])), (k, de[k])
        assert dv[rs >= 1e-6].max() <= 1e-9
        assert (2.0 * np.sqrt(rs) * dv).max() <= 1e-9
    else:
        for k in KEYS:
            assert abs(de[k]) <= 1e-5 * natoms, (k, de[k])
        if prec == ofdft.MIXED_VW64:
            assert dv[rs >= 1e-6].max() <= 1e-4
        else:
            # FP32 transforms leave an absolute error ~1e-5 in lap(phi); divided
            # by phi it reaches 3e-3 Ha at rho = 1e-6, so plain MIXED meets
            # 1e-4 Ha in |dE/drho| on rho >= 1e-3 only
            assert dv[rs >= 1e-3].max() <= 1e-4
        assert (2.0 * np.sqrt(rs) * dv).max() <= 1e-4
    assert abs(e["nelec_int"] - ref["energy"]["nelec_int"]) <= 1e-7 * ref["energy"]["nelec_int"]


def test_c3_modes_share_the_energy(c3):
    """The spline energy is defined once; S3S4 and EXACT differ only in the
    potential."""
    cell, rho, _ = c3
    es = {}
    for nl in (ofdft.NL_S3S4, ofdft.NL_EXACT):
        with ofdft.Grid(cell, TERMS, precision=ofdft.MIXED, nk=32, kf_min=0.1, kf_max=3.0,
                        nl_mode=nl) as g:
            es[nl] = g.energy_potential(rho, want_v=False)[0]
    a, b = es[ofdft.NL_S3S4].e_nl, es[ofdft.NL_EXACT].e_nl
    print("c3 e_nl S3S4 %.12f EXACT %.12f" % (a, b), flush=True)
    assert abs(a - b) <= 1e-6 * abs(a)
