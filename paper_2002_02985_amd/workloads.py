"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it only builds atomic
structures and starting densities, as plain NumPy arrays and dicts, from
seeds.  Both the GPU path and the oracle consume its outputs.

Workloads (shapes and structure follow the paper's test systems: fcc Al bulk
cells, an Mg hcp slab with vacuum, Al/Mg clusters in vacuum boxes):

* ``al_fcc_cell``  - fcc Al conventional cubic cells, 4 atoms per cell,
  a = 7.65 Bohr, Z = 3, optional Gaussian jitter of the positions;
* ``mg_hcp_slab`` - Mg hcp in the orthorhombic 4-atom cell (a, sqrt(3) a, c),
  a = 6.066, c = 9.845 Bohr, Z = 2, with vacuum added along z;
* ``cluster``      - the n fcc/hcp lattice sites nearest a seeded centre in a
  cubic vacuum box;
* densities: uniform plus multiplicative noise, or a periodic sum of
  Z-weighted Gaussians (built in reciprocal space with NumPy's FFT, an input
  recipe only) times (1 + noise), renormalised to N_e.
"""
import numpy as np

AL = {"Z": 3.0, "rc": 1.0, "a": 7.65}
MG = {"Z": 2.0, "rc": 1.0, "a": 6.066, "c": 9.845}

# grid sizes 2^a 3^b used for the vacuum-box requests
BOX_GRIDS = (48, 54, 64, 72, 96, 108, 128, 144, 162, 192)


def _cell(lattice, n, pos, species, Z, rc, nelec):
    return {
        "lattice": np.asarray(lattice, dtype=np.float64).reshape(3, 3),
        "n": tuple(int(x) for x in n),
        "pos": np.asarray(pos, dtype=np.float64).reshape(-1, 3),
        "species": np.asarray(species, dtype=np.int32).reshape(-1),
        "Z": np.asarray(Z, dtype=np.float64).reshape(-1),
        "rc": np.asarray(rc, dtype=np.float64).reshape(-1),
        "nelec": float(nelec),
    }


def al_fcc_cell(ncell=1, n=(32, 32, 32), a=AL["a"], jitter=0.0, seed=1):
    """ncell^3 conventional fcc cells of Al (4 atoms each)."""
    basis = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    grid = np.array([[i, j, k] for i in range(ncell) for j in range(ncell)
                     for k in range(ncell)], dtype=np.float64)
    frac = (grid[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    pos = frac * a
    if jitter > 0:
        rng = np.random.default_rng(seed)
        pos = pos + rng.normal(0.0, jitter, size=pos.shape)
    L = a * ncell
    natoms = len(pos)
    return _cell(np.diag([L, L, L]), n, pos, np.zeros(natoms), [AL["Z"]], [AL["rc"]],
                 AL["Z"] * natoms)


def mg_hcp_slab(reps=(6, 4, 9), n=(256, 256, 384), vacuum=15.0, jitter=0.0, seed=3):
    """Mg hcp slab: reps of the orthorhombic 4-atom cell (a, sqrt3 a, c) with
    `vacuum` Bohr added along z and the slab centred in the box."""
    a, c = MG["a"], MG["c"]
    b = np.sqrt(3.0) * a
    basis = np.array([[0.0, 0.0, 0.0], [a / 2, b / 2, 0.0], [2 * a / 3, b / 3, c / 2],
                      [a / 6, 5 * b / 6, c / 2]])
    nx, ny, nz = reps
    cells = np.array([[i * a, j * b, k * c] for i in range(nx) for j in range(ny)
                      for k in range(nz)])
    pos = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    Lz = nz * c + vacuum
    pos[:, 2] += (Lz - nz * c) / 2.0
    if jitter > 0:
        rng = np.random.default_rng(seed)
        pos = pos + rng.normal(0.0, jitter, size=pos.shape)
    natoms = len(pos)
    lat = np.diag([nx * a, ny * b, Lz])
    return _cell(lat, n, pos, np.zeros(natoms), [MG["Z"]], [MG["rc"]], MG["Z"] * natoms)


def box_grid(L, h=0.35, choices=BOX_GRIDS):
    need = L / h
    for g in choices:
        if g >= need:
            return g
    return choices[-1]


def cluster(natoms, species="Al", vacuum=8.0, seed=0, grid=None):
    """The `natoms` lattice sites of bulk Al (fcc) or Mg (hcp) nearest a seeded
    centre, in a cubic box with `vacuum` Bohr on each side."""
    rng = np.random.default_rng(seed)
    if species == "Al":
        a = AL["a"]
        basis = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]]) * a
        cellv = np.diag([a, a, a])
        Z, rc = AL["Z"], AL["rc"]
    else:
        a, c = MG["a"], MG["c"]
        b = np.sqrt(3.0) * a
        basis = np.array([[0.0, 0.0, 0.0], [a / 2, b / 2, 0.0], [2 * a / 3, b / 3, c / 2],
                          [a / 6, 5 * b / 6, c / 2]])
        cellv = np.diag([a, b, c])
        Z, rc = MG["Z"], MG["rc"]
    m = int(np.ceil((natoms / len(basis)) ** (1.0 / 3.0))) + 3
    rng_idx = np.arange(-m, m + 1)
    cells = np.array([[i, j, k] for i in rng_idx for j in rng_idx for k in rng_idx],
                     dtype=np.float64) @ cellv
    sites = (cells[:, None, :] + basis[None, :, :]).reshape(-1, 3)
    centre = rng.uniform(0.0, 1.0, size=3) @ cellv
    d = np.linalg.norm(sites - centre, axis=1)
    pos = sites[np.argsort(d, kind="stable")[:natoms]]
    lo = pos.min(axis=0)
    hi = pos.max(axis=0)
    D = float(np.max(hi - lo))
    L = D + 2.0 * vacuum
    pos = pos - (lo + hi) / 2.0 + L / 2.0
    n = grid if grid is not None else box_grid(L)
    return _cell(np.diag([L, L, L]), (n, n, n), pos, np.zeros(natoms), [Z], [rc],
                 Z * natoms)


def volume(cell):
    return abs(float(np.linalg.det(cell["lattice"])))


def uniform_density(cell, noise=0.0, seed=2):
    """rho0 = N_e / V times (1 + noise * xi), xi ~ N(0, 1) iid per point,
    renormalised to N_e on the grid."""
    n = cell["n"]
    V = volume(cell)
    rho0 = cell["nelec"] / V
    rho = np.full(n, rho0)
    if noise > 0:
        rng = np.random.default_rng(seed)
        rho = rho * (1.0 + noise * rng.standard_normal(n))
        rho = np.maximum(rho, 0.0)
    N = n[0] * n[1] * n[2]
    rho *= cell["nelec"] / (rho.sum() * V / N)
    return rho


def _gaussians_orthorhombic(cell, sigma):
    """The periodic Gaussian sum for a diagonal lattice, where each Gaussian
    is a product of three periodic 1-D Gaussians: rho = sum_a z_a A_a x B_a x
    C_a, contracted with a matrix product per block of x-planes."""
    n = cell["n"]
    L = np.diag(cell["lattice"])
    Zs = cell["Z"][cell["species"]]
    pos = cell["pos"]

    def axis(d):
        x = np.arange(n[d]) * (L[d] / n[d])
        dx = x[None, :] - pos[:, d, None]
        dx -= L[d] * np.round(dx / L[d])
        g = np.zeros_like(dx)
        for img in range(-2, 3):
            g += np.exp(-((dx + img * L[d]) ** 2) / (2.0 * sigma * sigma))
        return g

    A = axis(0) * (Zs / ((2.0 * np.pi) ** 1.5 * sigma ** 3))[:, None]
    B = axis(1)
    C = axis(2)
    rho = np.empty(n)
    step = max(1, int(2 ** 24 // max(1, len(Zs) * n[1])))
    for i0 in range(0, n[0], step):
        i1 = min(n[0], i0 + step)
        AB = A[:, i0:i1, None] * B[:, None, :]            # (na, block, n1)
        rho[i0:i1] = (AB.reshape(len(Zs), -1).T @ C).reshape(i1 - i0, n[1], n[2])
    return rho


def gaussian_superposition(cell, sigma=1.5, floor=0.0):
    """Periodic sum of Z-weighted normalised Gaussians of width sigma centred
    on the atoms.  Diagonal lattices use the separable real-space form; other
    cells are evaluated through the Fourier series on the grid."""
    lat = np.asarray(cell["lattice"])
    if np.count_nonzero(lat - np.diag(np.diag(lat))) == 0 and len(cell["species"]) > 0:
        return np.maximum(_gaussians_orthorhombic(cell, sigma), 0.0) + floor
    n = cell["n"]
    lat = cell["lattice"]
    V = volume(cell)
    b = 2.0 * np.pi * np.linalg.inv(lat).T
    m0 = np.fft.fftfreq(n[0]) * n[0]
    m1 = np.fft.fftfreq(n[1]) * n[1]
    m2 = np.fft.rfftfreq(n[2]) * n[2]
    G = (m0[:, None, None, None] * b[0] + m1[None, :, None, None] * b[1]
         + m2[None, None, :, None] * b[2])
    G2 = np.einsum("...i,...i->...", G, G)
    sf = np.zeros(G2.shape, dtype=np.complex128)
    Zs = cell["Z"][cell["species"]]
    for p, z in zip(cell["pos"], Zs):
        sf += z * np.exp(-1j * (G @ p))
    spec = sf * np.exp(-G2 * sigma * sigma / 2.0) / V
    N = n[0] * n[1] * n[2]
    rho = np.fft.irfftn(spec * N, s=n, axes=(0, 1, 2))
    rho = np.maximum(rho, 0.0) + floor
    return rho


def gaussian_density(cell, sigma=1.5, noise=0.0, seed=1000, floor=0.0, base=None):
    """N_e-normalised rho_atom(r) (1 + noise * xi), xi ~ N(0, 1) iid."""
    rho = gaussian_superposition(cell, sigma, floor) if base is None else base.copy()
    if noise > 0:
        rng = np.random.default_rng(seed)
        rho = rho * (1.0 + noise * rng.standard_normal(rho.shape))
        rho = np.maximum(rho, 0.0)
    n = cell["n"]
    N = n[0] * n[1] * n[2]
    rho *= cell["nelec"] / (rho.sum() * volume(cell) / N)
    return rho


# --------------------------------------------------------------------------
# named configurations
# --------------------------------------------------------------------------
def config_c1():
    """fcc Al 4-atom cubic cell, a = 7.65 Bohr, 32^3, atoms jittered
    N(0, 0.05 Bohr) (seed 1), rho uniform 12 e/cell with 1% noise (seed 2)."""
    cell = al_fcc_cell(1, (32, 32, 32), jitter=0.05, seed=1)
    return cell, uniform_density(cell, 0.01, seed=2)


def config_c2(n=(96, 96, 96), ndens=200, first_seed=1000):
    """fcc Al 3x3x3 conventional cells (108 atoms, a = 22.95 Bohr) on a 96^3
    grid; `ndens` densities from seeds first_seed.. : Gaussian superposition
    (sigma 1.5 Bohr) times (1 + 0.01 xi)."""
    cell = al_fcc_cell(3, n)
    base = gaussian_superposition(cell, 1.5)
    dens = [gaussian_density(cell, noise=0.01, seed=first_seed + s, base=base)
            for s in range(ndens)]
    return cell, dens


def config_c3(n=(256, 256, 384)):
    """Mg hcp slab, 6x4x9 orthorhombic cells (864 atoms) + 15 Bohr vacuum,
    256x256x384 grid; Gaussian superposition plus a 1e-12 floor."""
    cell = mg_hcp_slab((6, 4, 9), n, vacuum=15.0)
    return cell, gaussian_density(cell, sigma=1.5, floor=1e-12)


def config_c4(nreq=512, seed=4242, ntraj=64, min_atoms=13, max_atoms=561, grids=BOX_GRIDS,
              mix=(0.4, 0.3, 0.3), md_step=0.1, h=0.35):
    """Serving request stream: `ntraj` trajectories, each an Al or Mg cluster
    (species with p = 1/2, size ~ U{min_atoms..max_atoms}) in a cubic box with
    8 Bohr of vacuum per side and the smallest grid from `grids` with spacing
    <= h (the largest one if none is fine enough).  `nreq` requests go to seeded trajectories; each request
    is one MD frame of its trajectory (positions R_t + N(0, md_step) per
    step) and is an energy+potential (0), forces (1) or warm-started
    optimisation (2) request with probabilities `mix`.  The first request of
    a trajectory carries the Gaussian-superposition starting density.

    Returns a list of dicts {cell_id, kind, cell, rho (or None), frame}."""
    rng = np.random.default_rng(seed)
    trajs = []
    for t in range(ntraj):
        sp = "Al" if rng.uniform() < 0.5 else "Mg"
        na = int(rng.integers(min_atoms, max_atoms + 1))
        base = cluster(na, sp, seed=seed + 1 + t)
        L = base["lattice"][0, 0]
        g = box_grid(L, h=h, choices=tuple(grids))
        trajs.append(cluster(na, sp, seed=seed + 1 + t, grid=g))
    frames = [0] * ntraj
    pos = [c["pos"].copy() for c in trajs]
    out = []
    for _ in range(nreq):
        t = int(rng.integers(0, ntraj))
        kind = int(rng.choice(3, p=np.asarray(mix, dtype=float)))
        if frames[t] > 0:
            pos[t] = pos[t] + rng.normal(0.0, md_step, size=pos[t].shape)
        cell = dict(trajs[t])
        cell["pos"] = pos[t].copy()
        rho = gaussian_density(cell, sigma=1.5, floor=1e-8) if frames[t] == 0 else None
        out.append({"cell_id": t, "kind": kind, "cell": cell, "rho": rho, "frame": frames[t]})
        frames[t] += 1
    return out


def config_c5(n=(1024, 1024, 1024), jitter=0.0, seed=5, subsample=1):
    """fcc Al 63^3 conventional cells (1,000,188 atoms, a = 482 Bohr) on a
    1024^3 grid, perfect lattice unless jitter > 0; the starting density is
    uniform (N_e / V) and is not built here (8 GiB as doubles).  subsample
    keeps every k-th atom with the electron count scaled to match (a cheaper
    stand-in of the same cell, for sizing the set-up)."""
    cell = al_fcc_cell(63, n, jitter=jitter, seed=seed)
    if subsample > 1:
        keep = np.arange(0, len(cell["species"]), subsample)
        cell["pos"] = cell["pos"][keep]
        cell["species"] = cell["species"][keep]
        cell["nelec"] = AL["Z"] * len(keep)
    return cell
