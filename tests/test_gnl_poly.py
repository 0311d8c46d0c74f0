"""The kernels' polynomial form of G_NL above eta = 1.6 (gnl_poly.hpp).

The G_NL formula of the nonlocal-KEDF section, G = 1/F - 3 eta^2 - 1 with the
Lindhard F, evaluated here at 40 digits (mpmath, no cancellation left at
these eta); the header's degree-16 polynomial in x = 1/eta^2 must agree to
FP64 rounding, the degree-7 one to well inside FP32 rounding, and both with
the oracle's series form.  The header must be what its generator writes.
"""
import importlib.util
import os
import re

import mpmath
import numpy as np

from oracle import functionals as Fn

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2002_02985_amd", "csrc")


def _header():
    text = open(os.path.join(CSRC, "gnl_poly.hpp")).read()
    out = {}
    for name, body in re.findall(r"constexpr double (GNL_X\d+)\[\d+\] = \{([^}]*)\}", text):
        out[name] = [float(v) for v in body.replace("\n", " ").split(",") if v.strip()]
    return out


def _gnl_mp(eta):
    mpmath.mp.dps = 40
    e = mpmath.mpf(eta)
    F = mpmath.mpf(1) / 2 + (1 - e * e) / (4 * e) * mpmath.log((e + 1) / (e - 1))
    return 1 / F - 3 * e * e - 1


def _horner(co, x, dtype):
    x = dtype(x)
    h = dtype(co[-1])
    for v in reversed(co[:-1]):
        h = dtype(h * x + dtype(v))
    return h


ETAS = np.concatenate([np.linspace(1.6, 3.0, 141), np.geomspace(3.0, 1.0e4, 120)])


def test_fp64_polynomial_matches_gnl_to_rounding():
    co = _header()["GNL_X64"]
    assert len(co) == 17
    worst = 0.0
    for eta in ETAS:
        ref = _gnl_mp(eta)
        got = _horner(co, 1.0 / (eta * eta), np.float64)
        worst = max(worst, abs(float(mpmath.mpf(float(got)) - ref)))
    assert worst < 5e-16, worst


def test_fp32_polynomial_matches_gnl():
    co = _header()["GNL_X32"]
    assert len(co) == 8
    worst64 = worst32 = 0.0
    for eta in ETAS:
        ref = _gnl_mp(eta)
        worst64 = max(worst64, abs(float(_horner(co, 1.0 / (eta * eta), np.float64) - ref)))
        x32 = np.float32(1.0) / (np.float32(eta) * np.float32(eta))
        g32 = _horner(co, x32, np.float32)
        # the FP32 kernel rounds eta itself: compare with G at the rounded eta
        worst32 = max(worst32, abs(float(g32) - float(_gnl_mp(float(np.float32(eta))))))
    assert worst64 < 2e-9, worst64      # the approximation itself
    assert worst32 < 5e-7, worst32      # with FP32 arithmetic (ulp of 1.6 is 1.2e-7)


def test_polynomials_agree_with_the_oracle_series():
    h = _header()
    eta = ETAS
    ref = Fn.gnl(eta)
    g64 = np.array([_horner(h["GNL_X64"], 1.0 / (e * e), np.float64) for e in eta])
    assert np.max(np.abs(g64 - ref)) < 5e-16
    # limits: G -> -8/5 as eta -> infinity
    assert abs(_horner(h["GNL_X64"], 0.0, np.float64) + 1.6) < 1e-16
    assert abs(_horner(h["GNL_X32"], 0.0, np.float64) + 1.6) < 1e-9


def test_header_is_the_generators_output():
    spec = importlib.util.spec_from_file_location("gen_gnl_poly", os.path.join(CSRC, "gen_gnl_poly.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    h = _header()
    for name, deg in gen.DEGREES.items():
        co = [float(v) for v in gen.economised(deg)]
        assert co == h[name], name
