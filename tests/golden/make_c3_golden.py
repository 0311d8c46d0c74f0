"""Writes c3_mg864_256x256x384.json: the FP64 oracle's energy terms and the
potential at seeded sample points for the Mg hcp slab (864 atoms, 15 Bohr
vacuum, 256 x 256 x 384 grid) with TF + vW + Hartree + local pseudopotential
+ the spline nonlocal functional (N_k = 32 log-spaced knots over 0.1-3.0),
in both potential modes (S3S4 and EXACT), at the starting density of that
workload (Gaussian superposition, 1e-12 floor).

Calls only oracle/ (and the seeded input generator).  Runs on the CPU for
about half an hour:  python tests/golden/make_c3_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import cell as OC                     # noqa: E402
from oracle import ewald as OE                    # noqa: E402
from oracle import functionals as OF              # noqa: E402
from paper_2002_02985_amd import workloads as W   # noqa: E402

OUT = os.path.join(HERE, "c3_mg864_256x256x384.json")
NSAMPLE = 256
SAMPLE_SEED = 20020


def sample_index(shape, n=NSAMPLE, seed=SAMPLE_SEED):
    rng = np.random.default_rng(seed)
    return rng.integers(0, int(np.prod(shape)), size=n)


def main():
    t0 = time.time()
    cell, rho = W.config_c3()
    oc = OC.Cell(lattice=cell["lattice"], n=tuple(cell["n"]), pos=cell["pos"],
                 species=cell["species"], Z=cell["Z"], rc=cell["rc"], nelec=cell["nelec"])
    print("density ready %.0f s" % (time.time() - t0), flush=True)
    vext = OF.vext_g(oc)
    print("v_ext(G) ready %.0f s" % (time.time() - t0), flush=True)
    e_ion = OE.ewald_energy(oc)
    print("E_ion ready %.0f s" % (time.time() - t0), flush=True)
    idx = sample_index(cell["n"])
    out = {"workload": "Mg hcp slab 6x4x9 orthorhombic cells (864 atoms) + 15 Bohr vacuum, "
                       "256x256x384, Gaussian superposition (sigma 1.5 Bohr) + 1e-12 floor",
           "terms": "TF|VW|HARTREE|EXT|SPLINE", "nk": 32, "kf_min": 0.1, "kf_max": 3.0,
           "knots": "log", "alpha": 5.0 / 6.0, "beta": 5.0 / 6.0,
           "sample_seed": SAMPLE_SEED, "sample_index": [int(i) for i in idx], "modes": {}}
    terms = OC.TF | OC.VW | OC.HARTREE | OC.EXT | OC.SPLINE
    for name, mode in (("s3s4", OC.NL_S3S4), ("exact", OC.NL_EXACT)):
        func = OC.Functional(terms=terms, nk=32, kf_min=0.1, kf_max=3.0, nl_mode=mode)
        r = OF.energy_potential(oc, func, rho=rho, vext=vext, e_ion=e_ion)
        vs = r.v.reshape(-1)[idx]
        out["modes"][name] = {
            "energy": {k: float(getattr(r, k)) for k in
                       ("e_tf", "e_vw", "e_h", "e_ext", "e_nl", "e_ion", "e_total", "mu",
                        "nelec_int", "resid_norm")},
            "v_samples": [float(x) for x in vs]}
        print("%s done %.0f s: E = %.12f" % (name, time.time() - t0, r.e_total), flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
