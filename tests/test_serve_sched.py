"""Admission policy of the request server (host-only scenario checks), and the
host-only request checks of the C ABI: validation and device footprints."""
import os
import subprocess

import numpy as np
import pytest

from paper_2002_02985_amd import ofdft
from paper_2002_02985_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


# the policy header on its own, and again under AddressSanitizer and
# UndefinedBehaviorSanitizer (host code only, built with the host compiler)
SANITIZE = [[], ["-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]]


@pytest.mark.parametrize("extra", SANITIZE, ids=["plain", "asan_ubsan"])
def test_admission_policy_scenarios(tmp_path, extra):
    exe = str(tmp_path / "sched_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall"] + extra +
                   ["-o", exe, os.path.join(HERE, "sched_check.cpp")], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"


def _descs(cell, **kw):
    cd, keep = ofdft.make_cell_desc(cell)
    terms = kw.pop("terms", ofdft.TERM_TF | ofdft.TERM_VW | ofdft.TERM_HARTREE | ofdft.TERM_EXT)
    return cd, ofdft.make_functional_desc(terms, **kw), keep


def test_footprint_parts():
    cell, _ = W.config_c1()
    cd, fd, keep = _descs(cell)
    N = 32 ** 3
    ep = ofdft.ofdft_footprint_bytes(cd, fd, ofdft.REQ_EP)
    fo = ofdft.ofdft_footprint_bytes(cd, fd, ofdft.REQ_FORCES)
    op = ofdft.ofdft_footprint_bytes(cd, fd, ofdft.REQ_OPTIMIZE)
    # forces: natoms x 3 doubles and the force kernel's per-block partials
    # (32 x 32 rows of 3 segments of 8 k2, 256 per block: 12 blocks)
    assert fo - ep == (4 * 3 + 12 * 4 * 3) * 8
    assert op - ep == 10 * N * 8                # ten FP64 optimiser fields
    # every field-sized buffer is at least: resident rho, 2 staging fields,
    # 4 half spectra (2 N/2+1 complex), v_ext and 3 G tables
    nh = 32 * 32 * 17
    assert ep > (3 * N + 4 * 2 * nh + 2 * nh + 3 * nh) * 8
    cdm, fdm, keepm = _descs(cell, precision=ofdft.MIXED)
    epm = ofdft.ofdft_footprint_bytes(cdm, fdm, ofdft.REQ_EP)
    assert 0.45 * ep < epm < 0.6 * ep           # FP32 fields, FP64 partials and phases


def test_footprint_spline_grows_with_knot_workspace():
    cell, _ = W.config_c1()
    cd, fd, k1 = _descs(cell)
    cds, fds, k2 = _descs(cell, terms=ofdft.TERM_TF | ofdft.TERM_SPLINE)
    cde, fde, k3 = _descs(cell, terms=ofdft.TERM_TF | ofdft.TERM_SPLINE, nl_mode=ofdft.NL_EXACT)
    a = ofdft.ofdft_footprint_bytes(cd, fd, ofdft.REQ_EP)
    b = ofdft.ofdft_footprint_bytes(cds, fds, ofdft.REQ_EP)
    c = ofdft.ofdft_footprint_bytes(cde, fde, ofdft.REQ_EP)
    assert b > a and c - b == 32 ** 3 * 8       # EXACT adds one accumulator field


def test_validate_rejects_bad_requests():
    cell, _ = W.config_c1()
    cd, fd, keep = _descs(cell)
    assert ofdft.ofdft_validate(cd, fd) == ofdft.OK
    bad = dict(cell)
    bad["n"] = (32, 32, 31)
    cdb, fdb, k2 = _descs(bad)
    assert ofdft.ofdft_validate(cdb, fdb) == ofdft.EINVAL
    bad = dict(cell)
    bad["pos"] = np.array(cell["pos"], dtype=float)
    bad["pos"][1, 2] = np.nan
    cdb, fdb, k3 = _descs(bad)
    assert ofdft.ofdft_validate(cdb, fdb) == ofdft.EINVAL
    cdw, fdw, k4 = _descs(cell, terms=ofdft.TERM_WT | ofdft.TERM_SPLINE)
    assert ofdft.ofdft_validate(cdw, fdw) == ofdft.EINVAL
    with pytest.raises(ofdft.OfdftError):
        ofdft.ofdft_footprint_bytes(cd, fd, 7)
