"""CPU checks of the C-ABI library: it loads, exports every function that
include/ofdft.h declares, and its pure host helpers answer without a GPU."""
import ctypes
import os
import re

import pytest

from paper_2002_02985_amd import ofdft

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ofdft.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(ofdft_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ofdft_grid_create", "ofdft_energy_potential", "ofdft_forces",
                     "ofdft_optimize", "ofdft_energy_potential_batch_dev", "ofdft_fft_r2c_dev"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = ofdft.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding wraps each of them
    assert set(declared_functions()) <= set(ofdft._SIGS)


def test_host_helpers():
    assert ofdft.ofdft_abi_version() == 7
    for n in (4, 6, 12, 32, 48, 96, 192, 256, 384, 1024):
        assert ofdft.ofdft_supported_length(n)
    for n in (5, 7, 10, 100, 2048):
        assert not ofdft.ofdft_supported_length(n)


def test_struct_layouts_match_header():
    # field counts of the C structs mirrored in the binding
    assert ctypes.sizeof(ofdft.Energy) == 11 * 8
    assert ctypes.sizeof(ofdft.OptParams) == 8 + 3 * 4 + 4
    assert ofdft.CellDesc.nelec.offset == 9 * 8 + 3 * 4 + 4 + 8 + 8 + 8 + 8 + 8


def test_structure_factor_settings_are_validated_on_the_host():
    import numpy as np
    cell = {"lattice": np.diag([9.0, 10.0, 11.0]), "n": (12, 12, 16),
            "pos": np.array([[1.0, 2.0, 3.0]]), "species": np.zeros(1, np.int32),
            "Z": np.array([3.0]), "rc": np.array([1.0]), "nelec": 3.0}
    f = ofdft.make_functional_desc(ofdft.TERM_TF | ofdft.TERM_EXT)
    for sf, order, want in ((ofdft.SF_DIRECT, 0, ofdft.OK), (ofdft.SF_PME, 0, ofdft.OK),
                            (ofdft.SF_PME, 12, ofdft.OK), (ofdft.SF_PME, 7, ofdft.EINVAL),
                            (ofdft.SF_PME, 2, ofdft.EINVAL), (ofdft.SF_PME, 18, ofdft.EINVAL),
                            (ofdft.SF_PME, 14, ofdft.EINVAL),   # above n[0] = 12
                            (5, 0, ofdft.EINVAL)):
        d, keep = ofdft.make_cell_desc(dict(cell, sf_method=sf, pme_order=order))
        assert ofdft.ofdft_validate(d, f) == want, (sf, order)
    # PME needs no per-atom phase tables: a smaller footprint for many atoms
    rng = np.random.default_rng(0)
    big = dict(cell, pos=rng.random((500, 3)) * 9.0, species=np.zeros(500, np.int32),
               nelec=1500.0)
    sizes = []
    for sf in (ofdft.SF_DIRECT, ofdft.SF_PME):
        d, keep = ofdft.make_cell_desc(dict(big, sf_method=sf))
        sizes.append(ofdft.ofdft_footprint_bytes(d, f, ofdft.REQ_EP))
    assert sizes[1] < sizes[0]
