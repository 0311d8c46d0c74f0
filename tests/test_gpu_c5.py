"""The million-atom grid (1024^3) against closed forms.

* fcc Al 63^3 conventional cells (1,000,188 atoms, a = 482 Bohr), PME
  structure factor, TF + vW + Hartree + pseudopotential + the spline
  nonlocal functional (32 geometric knots), uniform density rho0 = N_e / V:
  E_TF = C_TF rho0^(5/3) V, E_vW = E_H = E_NL = 0 (no G != 0 component;
  the kernel vanishes at G = 0), E_ext = rho0 sum_a pi Z rc^2 (the G = 0
  remainder of the pseudopotential) and E_ion = -M Z^2 / r_ws per ion with
  the fcc Madelung constant M = 0.895873615195 (r_ws the Wigner-Seitz
  radius).  Bar: 1e-5 Ha/atom in mixed precision.
* The same 1024^3 box without atoms, phi = phi0 + a cos(q x):
  E_vW = a^2 q^2 V / 4 and, for rho = phi^2 = phi0^2 + a^2/2 +
  2 phi0 a cos(q x) + (a^2/2) cos(2 q x), E_H = pi V (4 phi0^2 a^2 + a^4/16) / q^2,
  v = 8 pi phi0 a cos(q x) / q^2 + pi a^2 cos(2 q x) / (2 q^2)
      + a q^2 cos(q x) / (2 phi).
  Bars: FP64 relative 1e-10 in energy and 1e-9 Ha in v; mixed relative 1e-6
  and 1e-4 Ha.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2002_02985_amd import ofdft
from paper_2002_02985_amd import workloads as W
from tests.gpu_helpers import stream_handle

pytestmark = pytest.mark.gpu

C_TF = 0.3 * (3.0 * np.pi ** 2) ** (2.0 / 3.0)
M_FCC = 0.895873615195
N = 1024


def test_million_atom_uniform_density_closed_form():
    cell = W.config_c5()
    cell["sf_method"] = ofdft.SF_PME
    natoms = len(cell["species"])
    V = abs(np.linalg.det(cell["lattice"]))
    rho0 = cell["nelec"] / V
    terms = (ofdft.TERM_TF | ofdft.TERM_VW | ofdft.TERM_HARTREE | ofdft.TERM_EXT |
             ofdft.TERM_SPLINE)
    print("case c5 uniform, %d atoms" % natoms, flush=True)
    with ofdft.Grid(cell, terms, precision=ofdft.MIXED, nk=32, kf_min=0.1, kf_max=3.0,
                    nl_mode=ofdft.NL_S3S4) as g:
        x = torch.full((N, N, N), rho0, dtype=torch.float32, device="cuda:0")
        e = ofdft.ofdft_energy_potential_dev(g.handle, x.data_ptr(), None, stream_handle())
        del x
    e = e.as_dict()
    Z, rc = cell["Z"][0], cell["rc"][0]
    rws = (3.0 * V / natoms / (4.0 * np.pi)) ** (1.0 / 3.0)
    ref = {"e_tf": C_TF * rho0 ** (5.0 / 3.0) * V, "e_vw": 0.0, "e_h": 0.0, "e_nl": 0.0,
           "e_ext": rho0 * natoms * np.pi * Z * rc * rc, "e_ion": -M_FCC * Z * Z / rws * natoms}
    ref["e_total"] = sum(ref.values())
    err = {k: (e[k] - ref[k]) / natoms for k in ref}
    print("  E %.6f (closed form %.6f); per-atom errors %s" %
          (e["e_total"], ref["e_total"], {k: "%.1e" % v for k, v in err.items()}), flush=True)
    for k in ref:
        assert abs(err[k]) <= 1e-5, (k, err[k])
    assert abs(e["nelec_int"] - cell["nelec"]) <= 1e-7 * cell["nelec"]


@pytest.mark.parametrize("prec", [ofdft.FP64, ofdft.MIXED])
def test_1024_cosine_closed_form(prec):
    L = 63 * 7.65
    cell = {"lattice": np.diag([L, L, L]), "n": (N, N, N), "pos": np.zeros((0, 3)),
            "species": np.zeros(0, np.int32), "Z": np.array([3.0]), "rc": np.array([1.0])}
    phi0 = 0.16
    a = 0.3 * phi0
    m = 100
    q = 2.0 * np.pi * m / L
    V = L ** 3
    cell["nelec"] = (phi0 ** 2 + a * a / 2.0) * V
    xs = np.arange(N) * L / N
    phi_x = phi0 + a * np.cos(q * xs)
    rho_x = phi_x ** 2
    v_x = (8.0 * np.pi * phi0 * a * np.cos(q * xs) / q ** 2 +
           np.pi * a * a * np.cos(2.0 * q * xs) / (2.0 * q ** 2) +
           a * q * q * np.cos(q * xs) / (2.0 * phi_x))
    e_vw = a * a * q * q * V / 4.0
    e_h = np.pi * V * (4.0 * phi0 ** 2 * a * a + a ** 4 / 16.0) / q ** 2
    terms = ofdft.TERM_VW | ofdft.TERM_HARTREE
    dt = torch.float64 if prec == ofdft.FP64 else torch.float32
    print("case 1024^3 cosine", prec, flush=True)
    with ofdft.Grid(cell, terms, precision=prec) as g:
        rx = torch.tensor(rho_x, dtype=dt, device="cuda:0")
        x = rx[:, None, None].expand(N, N, N).contiguous()
        v = torch.empty_like(x)
        e = ofdft.ofdft_energy_potential_dev(g.handle, x.data_ptr(), v.data_ptr(),
                                             stream_handle())
        torch.cuda.synchronize()
        vx = torch.tensor(v_x, dtype=torch.float64, device="cuda:0")
        dv = float((v.view(N, -1).double() - vx[:, None]).abs().max().item())
        del x, v
    rel_vw = abs(e.e_vw - e_vw) / e_vw
    rel_h = abs(e.e_h - e_h) / e_h
    print("  E_vW %.10e (%.10e) E_H %.10e (%.10e) rel %.1e %.1e max dv %.2e" %
          (e.e_vw, e_vw, e.e_h, e_h, rel_vw, rel_h, dv), flush=True)
    tol_e, tol_v = (1e-10, 1e-9) if prec == ofdft.FP64 else (1e-6, 1e-4)
    assert rel_vw <= tol_e and rel_h <= tol_e
    assert dv <= tol_v
