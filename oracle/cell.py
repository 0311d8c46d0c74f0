"""Oracle cell and grid geometry (TEST INFRASTRUCTURE ONLY).

The paper's Grid class carries the lattice vectors and the number of points
per direction, in a real-space and a reciprocal-space flavour (Section
"DFTpy classes").  This is the same information as plain arrays.
"""
import dataclasses

import numpy as np

from .fourier import half_weights

# term bits (same meaning as the C descriptor's bitmask)
TF = 1
VW = 2
HARTREE = 4
EXT = 8
WT = 16
SPLINE = 32
XC = 64

NL_S3S4 = 0
NL_EXACT = 1

KNOTS_LOG = 0
KNOTS_LIN = 1


@dataclasses.dataclass
class Cell:
    lattice: np.ndarray            # 3x3, rows are a_0, a_1, a_2 (Bohr)
    n: tuple                       # (N0, N1, N2)
    pos: np.ndarray                # natoms x 3 Cartesian (Bohr)
    species: np.ndarray            # natoms ints
    Z: np.ndarray                  # valence charge per species
    rc: np.ndarray                 # Gaussian-smearing radius per species (Bohr)
    nelec: float

    def __post_init__(self):
        self.lattice = np.asarray(self.lattice, dtype=np.float64).reshape(3, 3)
        self.n = tuple(int(x) for x in self.n)
        self.pos = np.asarray(self.pos, dtype=np.float64).reshape(-1, 3)
        self.species = np.asarray(self.species, dtype=np.int64).reshape(-1)
        self.Z = np.asarray(self.Z, dtype=np.float64).reshape(-1)
        self.rc = np.asarray(self.rc, dtype=np.float64).reshape(-1)
        self.nelec = float(self.nelec)

    @property
    def volume(self):
        return abs(float(np.linalg.det(self.lattice)))

    @property
    def npts(self):
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def dv(self):
        """Volume element of the grid sum: int f = dv * sum_r f(r)."""
        return self.volume / self.npts

    @property
    def recip(self):
        """Rows b_j with a_i . b_j = 2 pi delta_ij."""
        return 2.0 * np.pi * np.linalg.inv(self.lattice).T

    def fractional(self):
        return self.pos @ np.linalg.inv(self.lattice)


@dataclasses.dataclass
class Functional:
    terms: int = TF | VW | HARTREE | EXT
    lambda_vw: float = 1.0
    alpha: float = 5.0 / 6.0
    beta: float = 5.0 / 6.0
    kf_wt: float = 0.0             # <= 0: (3 pi^2 N_e / V)^(1/3)
    nk: int = 32
    kf_min: float = 0.1
    kf_max: float = 3.0
    knot_spacing: int = KNOTS_LOG
    nl_mode: int = NL_S3S4
    rho_floor: float = 1e-12
    nl_kernel: int = 0             # 0 WT; 1 MGP, 2 MGPA, 3 MGPG (oracle.mgp)


def mvals(n):
    """Integer frequencies m in [-floor(n/2), ceil(n/2) - 1] in FFT order;
    the Nyquist index of an even n takes the negative sign."""
    m = np.arange(n)
    return np.where(m < (n + 1) // 2, m, m - n)


def half_mvals(n2):
    """Frequencies of the half-spectrum planes 0..n2//2 (Nyquist negative)."""
    m = np.arange(n2 // 2 + 1)
    if n2 % 2 == 0:
        m[-1] = -(n2 // 2)
    return m


def gvectors(cell):
    """G vectors of the half spectrum, shape (N0, N1, N2//2+1, 3)."""
    n0, n1, n2 = cell.n
    b = cell.recip
    m0 = mvals(n0)[:, None, None, None]
    m1 = mvals(n1)[None, :, None, None]
    m2 = half_mvals(n2)[None, None, :, None]
    return m0 * b[0] + m1 * b[1] + m2 * b[2]


def g2(cell):
    G = gvectors(cell)
    return np.einsum("...i,...i->...", G, G)


def weights(cell):
    """Half-spectrum multiplicities broadcast to (N0, N1, N2//2+1)."""
    n0, n1, n2 = cell.n
    return np.broadcast_to(half_weights(n2)[None, None, :], (n0, n1, n2 // 2 + 1))


def gsum(cell, x):
    """sum over the full reciprocal set of a real summand given on the half
    spectrum: sum_half c(m2) x."""
    return float(np.sum(weights(cell) * x))


def knots(func):
    """Step s1: the k_F knots, a geometric (default) or arithmetic progression
    from kf_min to kf_max with both ends included."""
    i = np.arange(func.nk, dtype=np.float64)
    if func.nk == 1:
        return np.array([func.kf_min])
    if func.knot_spacing == KNOTS_LOG:
        return func.kf_min * (func.kf_max / func.kf_min) ** (i / (func.nk - 1))
    return func.kf_min + (func.kf_max - func.kf_min) * i / (func.nk - 1)
