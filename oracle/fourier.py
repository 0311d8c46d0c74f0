"""Oracle Fourier transforms (TEST INFRASTRUCTURE ONLY).

Thin ctypes wrapper around ``oracle/fft.c`` (a textbook recursive mixed-radix
transform written for the oracle) plus the real-to-half-spectrum conventions:

    forward:  f(G) = (1/N) sum_r f(r) exp(-i G.r)          -> half spectrum
    inverse:  f(r) = Re sum_{half} c(m2) X(m) exp(i G.r)    c = 1 or 2

The paper computes every reciprocal-space term with 3D FFTs (Section
"Leveraging existing techniques"); these two functions are that transform
pair written out, slowly.  ``dft_bruteforce`` is the O(N^2) definition used
to pin the fast one.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_oracle_fft.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build
            _build.build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_fft3d.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, ctypes.c_int]
        lib.oracle_fft3d.restype = ctypes.c_int
        lib.oracle_fft1d_batch.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_long,
                                           ctypes.c_int]
        lib.oracle_fft1d_batch.restype = ctypes.c_int
        _lib = lib
    return _lib


def fft3_raw(a, sign):
    """Unnormalised 3D DFT of a complex array: sum_j a[j] exp(sign 2 pi i j.k/n)."""
    lib = _load()
    buf = np.ascontiguousarray(a, dtype=np.complex128).copy()
    n0, n1, n2 = buf.shape
    if lib.oracle_fft3d(buf.ctypes.data, n0, n1, n2, int(sign)) != 0:
        raise MemoryError("oracle fft3d allocation failed")
    return buf


def fft1_raw(a, sign):
    """Unnormalised 1D DFT along the last axis."""
    lib = _load()
    buf = np.ascontiguousarray(a, dtype=np.complex128).copy()
    n = buf.shape[-1]
    count = buf.size // n if n else 0
    if lib.oracle_fft1d_batch(buf.ctypes.data, n, count, int(sign)) != 0:
        raise MemoryError("oracle fft1d allocation failed")
    return buf


def half_weights(n2):
    """Multiplicity c(m2) of each half-spectrum plane (1 for m2 = 0 and the
    even-length Nyquist plane, 2 otherwise)."""
    n2h = n2 // 2 + 1
    c = np.full(n2h, 2.0)
    c[0] = 1.0
    if n2 % 2 == 0:
        c[-1] = 1.0
    return c


def r2c(f):
    """Forward transform of a real field to its half spectrum, normalised by 1/N."""
    f = np.asarray(f, dtype=np.float64)
    n0, n1, n2 = f.shape
    full = fft3_raw(f.astype(np.complex128), -1)
    return full[:, :, : n2 // 2 + 1] / float(n0 * n1 * n2)


def c2r(X, shape):
    """Inverse transform of a half spectrum: Re sum_half c(m2) X exp(+i G.r)."""
    n0, n1, n2 = shape
    n2h = n2 // 2 + 1
    X = np.asarray(X, dtype=np.complex128)
    assert X.shape == (n0, n1, n2h)
    full = np.zeros((n0, n1, n2), dtype=np.complex128)
    full[:, :, :n2h] = X * half_weights(n2)[None, None, :]
    return fft3_raw(full, +1).real.copy()


def dft_bruteforce(f, sign=-1):
    """O(N^2) 3D DFT by explicit exponential matrices (pins the fast transform)."""
    a = np.asarray(f, dtype=np.complex128)
    out = a
    for axis, n in enumerate(a.shape):
        j = np.arange(n)
        mat = np.exp(sign * 2j * np.pi * np.outer(j, j) / n)
        out = np.moveaxis(np.tensordot(mat, np.moveaxis(out, axis, 0), axes=(1, 0)), 0, axis)
    return out
