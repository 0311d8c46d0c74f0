"""Small helpers shared by the oracle pin tests (CPU only)."""
import numpy as np

from oracle import cell as C


def make_cell(d, n=None):
    """oracle Cell from a workloads dict (optionally on another grid)."""
    return C.Cell(lattice=d["lattice"], n=d["n"] if n is None else n, pos=d["pos"],
                  species=d["species"], Z=d["Z"], rc=d["rc"], nelec=d["nelec"])


def box_cell(L=(7.0, 8.0, 9.0), n=(12, 12, 16), pos=None, Z=3.0, rc=1.0, nelec=None):
    L = np.asarray(L, dtype=float)
    pos = np.zeros((0, 3)) if pos is None else np.asarray(pos, dtype=float)
    if nelec is None:
        nelec = Z * max(len(pos), 1)
    return C.Cell(lattice=np.diag(L), n=n, pos=pos, species=np.zeros(len(pos), int),
                  Z=[Z], rc=[rc], nelec=nelec)


def grid_points(cell):
    n0, n1, n2 = cell.n
    i0, i1, i2 = np.meshgrid(np.arange(n0), np.arange(n1), np.arange(n2), indexing="ij")
    frac = np.stack([i0 / n0, i1 / n1, i2 / n2], axis=-1)
    return frac @ cell.lattice


def smooth_density(cell, seed=0, amp=0.3, nmodes=4, rho0=None):
    """A strictly positive, band-limited density with int rho = nelec."""
    rng = np.random.default_rng(seed)
    r = grid_points(cell)
    b = cell.recip
    f = np.ones(cell.n)
    for _ in range(nmodes):
        m = rng.integers(-2, 3, size=3)
        G = m @ b
        f += amp / nmodes * np.cos(r @ G + rng.uniform(0, 2 * np.pi))
    f = np.maximum(f, 0.05)
    rho0 = cell.nelec / cell.volume if rho0 is None else rho0
    rho = f * rho0
    rho *= cell.nelec / (cell.dv * rho.sum())
    return rho
