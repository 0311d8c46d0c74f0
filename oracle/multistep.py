"""Multi-step density optimisation, oracle side (TEST INFRASTRUCTURE ONLY).

Section "Density optimization strategies": the density is first optimised on
a coarse grid and the converged density is then interpolated onto a finer
grid, where the optimisation continues.  The paper does not say how it
interpolates; the reading taken here (and by the GPU path) is Fourier
interpolation of phi = sqrt(rho), which keeps rho >= 0:

* the half spectrum of phi on the source grid (forward transform, 1/N) is
  carried to the destination grid frequency by frequency;
* a frequency strictly inside the source band keeps its coefficient;
* the Nyquist coefficient of an even source axis (the samples of a cosine at
  the band edge) is split in halves between +n/2 and -n/2 -- on the stored
  half axis 2 the coefficient at k2 = n2/2 is halved -- so that the cosine it
  stands for is reproduced;
* every other destination frequency is zero, and an axis whose size does not
  change is copied as it is;
* the inverse transform on the destination grid gives phi there; rho = phi^2
  is scaled to the electron count.

Only refinement (destination at least as fine on every axis) is defined.
"""
import numpy as np

from . import fourier as F


def _axis_map(n_src, n_dst):
    """Destination index -> (source index or -1, weight) along a full axis."""
    src = np.full(n_dst, -1, dtype=np.int64)
    w = np.zeros(n_dst)
    for i in range(n_dst):
        m = i if i < (n_dst + 1) // 2 else i - n_dst        # destination frequency
        if n_dst == n_src:
            src[i], w[i] = i, 1.0
        elif n_src % 2 == 0 and abs(m) == n_src // 2:
            src[i], w[i] = n_src // 2, 0.5                  # the source Nyquist, -n/2
        elif 2 * abs(m) < n_src:
            src[i], w[i] = m % n_src, 1.0
    return src, w


def _half_map(n_src, n_dst):
    """Destination half-axis index k >= 0 -> (source index or -1, weight)."""
    nh = n_dst // 2 + 1
    src = np.full(nh, -1, dtype=np.int64)
    w = np.zeros(nh)
    for k in range(nh):
        if n_dst == n_src:
            src[k], w[k] = k, 1.0
        elif n_src % 2 == 0 and 2 * k == n_src:
            src[k], w[k] = k, 0.5
        elif 2 * k < n_src:
            src[k], w[k] = k, 1.0
    return src, w


def fourier_interpolate(f, shape):
    """Band-limited interpolation of the real periodic field f onto `shape`
    (at least as fine as f on every axis)."""
    f = np.asarray(f, dtype=np.float64)
    ns, nd = f.shape, tuple(int(x) for x in shape)
    if any(d < s for s, d in zip(ns, nd)):
        raise ValueError("destination grid coarser than the source")
    X = F.r2c(f)
    s0, w0 = _axis_map(ns[0], nd[0])
    s1, w1 = _axis_map(ns[1], nd[1])
    s2, w2 = _half_map(ns[2], nd[2])
    Y = np.zeros((nd[0], nd[1], nd[2] // 2 + 1), dtype=np.complex128)
    for a in range(nd[0]):
        if s0[a] < 0:
            continue
        for b in range(nd[1]):
            if s1[b] < 0:
                continue
            ok = s2 >= 0
            Y[a, b, ok] = w0[a] * w1[b] * w2[ok] * X[s0[a], s1[b], s2[ok]]
    return F.c2r(Y, nd)


def interpolate_density(rho, shape, nelec, dv):
    """rho on a finer grid: phi = sqrt(rho) interpolated, squared, scaled so
    that dv * sum(rho) = nelec."""
    phi = fourier_interpolate(np.sqrt(np.maximum(rho, 0.0)), shape)
    r = phi * phi
    return r * (nelec / (dv * r.sum()))
