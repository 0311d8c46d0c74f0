"""ctypes binding of libofdft.so (argument marshalling only).

Every function named ``ofdft_*`` here calls the C entry point of the same name
declared in ``include/ofdft.h``; all computation happens in the library's HIP
kernels.  ``load()`` raises if the library has not been built -- there is no
fallback.  Device arrays are passed as raw pointers (e.g. ``tensor.data_ptr()``
of a torch tensor on the GPU) together with a HIP stream handle.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("OFDFT_LIB", os.path.join(HERE, "libofdft.so"))

OK, PENDING, EINVAL, ENOMEM, EDEVICE, ENOCONV, ECANCELLED, ENOTFOUND = 0, 1, -1, -2, -3, -4, -5, -6
TERM_TF, TERM_VW, TERM_HARTREE, TERM_EXT, TERM_WT, TERM_SPLINE = 1, 2, 4, 8, 16, 32
TERM_XC = 64
KNOTS_LOG, KNOTS_LIN = 0, 1
NL_S3S4, NL_EXACT = 0, 1
FP64, MIXED, MIXED_VW64 = 0, 1, 2
REQ_EP, REQ_FORCES, REQ_OPTIMIZE = 0, 1, 2
OPT_CG, OPT_PCG, OPT_TN = 0, 1, 2
SF_DIRECT, SF_PME = 0, 1
KERNEL_WT, KERNEL_MGP, KERNEL_MGPA, KERNEL_MGPG = 0, 1, 2, 3
MULTI_MAX = 64   # OFDFT_MULTI_MAX: grids per batched call
PASS_NAMES = ["row_fwd", "col1_fwd", "col0_g", "col1_inv", "row_inv", "knot_inv", "knot_col1",
              "knot_row", "exact_fwd", "exact_acc", "finalize", "other", "vw64"]


class CellDesc(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_double * 9), ("n", ctypes.c_int32 * 3),
                ("natoms", ctypes.c_int32), ("pos", ctypes.POINTER(ctypes.c_double)),
                ("species", ctypes.POINTER(ctypes.c_int32)), ("nspecies", ctypes.c_int32),
                ("Z", ctypes.POINTER(ctypes.c_double)), ("rc", ctypes.POINTER(ctypes.c_double)),
                ("nelec", ctypes.c_double), ("sf_method", ctypes.c_int32),
                ("pme_order", ctypes.c_int32)]


class FunctionalDesc(ctypes.Structure):
    _fields_ = [("terms", ctypes.c_uint32), ("lambda_vw", ctypes.c_double),
                ("alpha", ctypes.c_double), ("beta", ctypes.c_double),
                ("kf_wt", ctypes.c_double), ("nk", ctypes.c_int32), ("kf_min", ctypes.c_double),
                ("kf_max", ctypes.c_double), ("knot_spacing", ctypes.c_int32),
                ("nl_mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rho_floor", ctypes.c_double), ("nl_kernel", ctypes.c_int32)]


class Energy(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in
                ("e_tf", "e_vw", "e_h", "e_ext", "e_nl", "e_ion", "e_total", "mu", "nelec_int",
                 "resid_norm", "e_xc")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class OptParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32),
                ("method", ctypes.c_int32), ("warm", ctypes.c_int32)]


class OptResult(ctypes.Structure):
    _fields_ = [("e", Energy), ("iters", ctypes.c_int32), ("evals", ctypes.c_int32),
                ("final_resid", ctypes.c_double)]


class TdParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("n_corrector", ctypes.c_int32),
                ("max_solver_iter", ctypes.c_int32), ("solver_tol", ctypes.c_double)]


class TdStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("solver_iters", ctypes.c_int32),
                ("unconverged_solves", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("max_solver_resid", ctypes.c_double), ("nelec", ctypes.c_double)]


class Request(ctypes.Structure):
    _fields_ = [("cell_id", ctypes.c_uint64), ("kind", ctypes.c_int32),
                ("cell", ctypes.POINTER(CellDesc)), ("func", ctypes.POINTER(FunctionalDesc)),
                ("opt", ctypes.POINTER(OptParams)), ("rho_or_null", ctypes.POINTER(ctypes.c_double))]


class TuneResult(ctypes.Structure):
    _fields_ = [("plane", ctypes.c_int32), ("col_tile_major", ctypes.c_int32),
                ("knot_batch", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double),
                ("pipe", ctypes.c_int32), ("col_group", ctypes.c_int32),
                ("knot_pipe", ctypes.c_int32), ("col_variant", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("cancelled", ctypes.c_uint64),
                ("queued", ctypes.c_int32), ("running", ctypes.c_int32),
                ("resident_cells", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("resident_bytes", ctypes.c_uint64), ("peak_bytes", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_uint64), ("p50_ms", ctypes.c_double),
                ("p99_ms", ctypes.c_double), ("mean_queue_ms", ctypes.c_double),
                ("batches", ctypes.c_uint64), ("batched_requests", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_PP = ctypes.POINTER(ctypes.c_void_p)
_DP = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "ofdft_abi_version": (ctypes.c_int, []),
    "ofdft_last_error": (ctypes.c_char_p, []),
    "ofdft_supported_length": (ctypes.c_int, [ctypes.c_int32]),
    "ofdft_ctx_create": (ctypes.c_int, [ctypes.c_int, _PP]),
    "ofdft_ctx_destroy": (None, [_P]),
    "ofdft_grid_create": (ctypes.c_int, [_P, ctypes.POINTER(CellDesc),
                                         ctypes.POINTER(FunctionalDesc), _PP]),
    "ofdft_grid_destroy": (None, [_P]),
    "ofdft_grid_reserve": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ofdft_grid_device_bytes": (ctypes.c_uint64, [_P]),
    "ofdft_set_density": (ctypes.c_int, [_P, _DP]),
    "ofdft_get_density": (ctypes.c_int, [_P, _DP]),
    "ofdft_energy_potential": (ctypes.c_int, [_P, _DP, _DP, ctypes.POINTER(Energy)]),
    "ofdft_energy_potential_dev": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(Energy)]),
    "ofdft_energy_potential_batch_dev": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P,
                                                        ctypes.POINTER(Energy)]),
    "ofdft_energy_potential_dev_noalloc": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(Energy)]),
    "ofdft_optimize_multi": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "ofdft_energy_potential_multi": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                                    ctypes.POINTER(ctypes.POINTER(ctypes.c_double)),
                                                    ctypes.POINTER(Energy)]),
    "ofdft_fft_r2c_dev": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "ofdft_fft_c2r_dev": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    "ofdft_forces": (ctypes.c_int, [_P, _DP]),
    "ofdft_optimize": (ctypes.c_int, [_P, ctypes.POINTER(OptParams), ctypes.POINTER(OptResult)]),
    "ofdft_validate": (ctypes.c_int, [ctypes.POINTER(CellDesc), ctypes.POINTER(FunctionalDesc)]),
    "ofdft_footprint_bytes": (ctypes.c_int, [ctypes.POINTER(CellDesc),
                                             ctypes.POINTER(FunctionalDesc), ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_uint64)]),
    "ofdft_server_create": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int32, _PP]),
    "ofdft_serve_submit": (ctypes.c_int, [_P, ctypes.POINTER(Request),
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "ofdft_serve_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(OptResult), _DP,
                                        _DP]),
    "ofdft_serve_wait": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.c_int32]),
    "ofdft_serve_cancel": (ctypes.c_int, [_P, ctypes.c_uint64]),
    "ofdft_serve_stats_get": (ctypes.c_int, [_P, ctypes.POINTER(ServeStats)]),
    "ofdft_serve_set_batching": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "ofdft_server_destroy": (None, [_P]),
    "ofdft_grid_set_graphs": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ofdft_grid_interpolate_density": (ctypes.c_int, [_P, _P]),
    "ofdft_optimize_multistep": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int32, _P, _P]),
    "ofdft_td_start": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "ofdft_td_set_psi": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "ofdft_td_get_psi": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "ofdft_td_propagate": (ctypes.c_int, [_P, ctypes.POINTER(TdParams), ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(TdStats)]),
    "ofdft_grid_set_knot_skip": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ofdft_grid_set_col_group": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ofdft_grid_set_col_variant": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ofdft_grid_set_knot_pipeline": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ofdft_grid_set_pipeline": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ofdft_grid_tune_dev": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.POINTER(TuneResult)]),
    "ofdft_grid_tune": (ctypes.c_int, [_P, ctypes.POINTER(TuneResult)]),
    "ofdft_profile_enable": (ctypes.c_int, [_P, ctypes.c_int32]),
    "ofdft_profile_read": (ctypes.c_int, [_P, ctypes.c_int32, _DP,
                                          ctypes.POINTER(ctypes.c_int64)]),
}

_lib = None


def load(path=LIB_PATH):
    """Load libofdft.so; raises OSError if it is missing (build it first)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise OSError("libofdft.so not found at %s: run paper_2002_02985_amd/build.py" % path)
        lib = ctypes.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class OfdftError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("ofdft status %d: %s" % (status, msg))
        self.status = status


def check(status):
    if status not in (OK,):
        raise OfdftError(status, load().ofdft_last_error().decode())
    return status


def _dptr(a):
    return a.ctypes.data_as(_DP)


# ------------------------------------------------------------------ C names
def ofdft_abi_version():
    return load().ofdft_abi_version()


def ofdft_supported_length(n):
    return bool(load().ofdft_supported_length(int(n)))


def ofdft_ctx_create(device=0):
    h = ctypes.c_void_p()
    check(load().ofdft_ctx_create(int(device), ctypes.byref(h)))
    return h


def ofdft_ctx_destroy(ctx):
    load().ofdft_ctx_destroy(ctx)


def make_cell_desc(cell):
    """CellDesc from a workloads dict; returns (desc, keepalive arrays)."""
    lat = np.ascontiguousarray(cell["lattice"], dtype=np.float64).reshape(9)
    pos = np.ascontiguousarray(cell["pos"], dtype=np.float64).reshape(-1)
    spc = np.ascontiguousarray(cell["species"], dtype=np.int32).reshape(-1)
    Z = np.ascontiguousarray(cell["Z"], dtype=np.float64)
    rc = np.ascontiguousarray(cell["rc"], dtype=np.float64)
    d = CellDesc()
    d.lattice[:] = list(lat)
    d.n[:] = [int(x) for x in cell["n"]]
    d.natoms = len(spc)
    d.pos = _dptr(pos)
    d.species = spc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.nspecies = len(Z)
    d.Z = _dptr(Z)
    d.rc = _dptr(rc)
    d.nelec = float(cell["nelec"])
    d.sf_method = int(cell.get("sf_method", SF_DIRECT))
    d.pme_order = int(cell.get("pme_order", 0))
    return d, (lat, pos, spc, Z, rc)


def make_functional_desc(terms, precision=FP64, lambda_vw=1.0, alpha=5.0 / 6.0, beta=5.0 / 6.0,
                         kf_wt=0.0, nk=32, kf_min=0.1, kf_max=3.0, knot_spacing=KNOTS_LOG,
                         nl_mode=NL_S3S4, rho_floor=1e-12, nl_kernel=KERNEL_WT):
    f = FunctionalDesc()
    f.terms = int(terms)
    f.lambda_vw = lambda_vw
    f.alpha = alpha
    f.beta = beta
    f.kf_wt = kf_wt
    f.nk = nk
    f.kf_min = kf_min
    f.kf_max = kf_max
    f.knot_spacing = knot_spacing
    f.nl_mode = nl_mode
    f.precision = precision
    f.rho_floor = rho_floor
    f.nl_kernel = nl_kernel
    return f


def ofdft_grid_create(ctx, cell_desc, func_desc):
    h = ctypes.c_void_p()
    check(load().ofdft_grid_create(ctx, ctypes.byref(cell_desc), ctypes.byref(func_desc),
                                   ctypes.byref(h)))
    return h


def ofdft_grid_destroy(grid):
    load().ofdft_grid_destroy(grid)


def ofdft_grid_reserve(grid, nbatch):
    check(load().ofdft_grid_reserve(grid, int(nbatch)))


def ofdft_grid_device_bytes(grid):
    return int(load().ofdft_grid_device_bytes(grid))


def ofdft_set_density(grid, rho):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    check(load().ofdft_set_density(grid, _dptr(rho)))


def ofdft_get_density(grid, shape):
    out = np.empty(shape, dtype=np.float64)
    check(load().ofdft_get_density(grid, _dptr(out)))
    return out


def ofdft_energy_potential(grid, rho=None, want_v=True, shape=None):
    e = Energy()
    rp = None
    if rho is not None:
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        rp = _dptr(rho)
        shape = rho.shape
    v = np.empty(shape, dtype=np.float64) if want_v else None
    check(load().ofdft_energy_potential(grid, rp, _dptr(v) if want_v else None, ctypes.byref(e)))
    return e, v


def ofdft_energy_potential_dev(grid, d_rho, d_v, stream):
    e = Energy()
    check(load().ofdft_energy_potential_dev(grid, d_rho, d_v, stream, ctypes.byref(e)))
    return e


def ofdft_energy_potential_dev_noalloc(grid, d_rho, d_v, stream):
    e = Energy()
    check(load().ofdft_energy_potential_dev_noalloc(grid, d_rho, d_v, stream, ctypes.byref(e)))
    return e


def ofdft_energy_potential_multi(grids, shapes=None, want_v=True):
    """Batched evaluation of the resident densities of several grids (same
    shape and functional); returns (energies, potentials or None)."""
    n = len(grids)
    harr = (ctypes.c_void_p * n)(*[g.value if isinstance(g, ctypes.c_void_p) else g for g in grids])
    es = (Energy * n)()
    vs = None
    if want_v:
        vs = [np.empty(tuple(sh), dtype=np.float64) for sh in shapes]
        varr = (ctypes.POINTER(ctypes.c_double) * n)(*[_dptr(v) for v in vs])
    else:
        varr = None
    check(load().ofdft_energy_potential_multi(harr, n, varr, es))
    return list(es), vs


def ofdft_energy_potential_batch_dev(grid, nbatch, d_rho, d_v, stream):
    es = (Energy * int(nbatch))()
    check(load().ofdft_energy_potential_batch_dev(grid, int(nbatch), d_rho, d_v, stream, es))
    return list(es)


def ofdft_fft_r2c_dev(grid, nbatch, d_in, d_out, stream):
    check(load().ofdft_fft_r2c_dev(grid, int(nbatch), d_in, d_out, stream))


def ofdft_fft_c2r_dev(grid, nbatch, d_in, d_out, stream):
    check(load().ofdft_fft_c2r_dev(grid, int(nbatch), d_in, d_out, stream))


def ofdft_forces(grid, natoms):
    f = np.empty((natoms, 3), dtype=np.float64)
    check(load().ofdft_forces(grid, _dptr(f)))
    return f


def ofdft_optimize(grid, tol=1e-7, max_iter=1000, method=0, allow_noconv=False):
    p = OptParams(tol=tol, max_iter=max_iter, method=method, warm=0)
    r = OptResult()
    st = load().ofdft_optimize(grid, ctypes.byref(p), ctypes.byref(r))
    if not (st == OK or (allow_noconv and st == ENOCONV)):
        check(st)
    return r, st


def ofdft_optimize_multi(grids, params):
    """Lockstep optimisation of several grids' resident densities; params:
    (tol, max_iter, method) per grid.  Returns ([OptResult], [status])."""
    n = len(grids)
    harr = (ctypes.c_void_p * n)(*[g.value if isinstance(g, ctypes.c_void_p) else g for g in grids])
    ps = (OptParams * n)(*[OptParams(tol=t, max_iter=m, method=k, warm=0) for t, m, k in params])
    rs = (OptResult * n)()
    sts = (ctypes.c_int32 * n)()
    check(load().ofdft_optimize_multi(harr, n, ctypes.cast(ps, ctypes.c_void_p),
                                      ctypes.cast(rs, ctypes.c_void_p),
                                      ctypes.cast(sts, ctypes.c_void_p)))
    return list(rs), list(sts)


def ofdft_grid_interpolate_density(dst, src):
    check(load().ofdft_grid_interpolate_density(dst, src))


def ofdft_optimize_multistep(grids, params, allow_noconv=False):
    """grids: grid handles, coarse to fine; params: (tol, max_iter, method)
    per grid.  Returns ([OptResult per grid], status)."""
    n = len(grids)
    hs = (_P * n)(*grids)
    ps = (OptParams * n)(*[OptParams(tol=t, max_iter=m, method=k, warm=0) for t, m, k in params])
    rs = (OptResult * n)()
    st = load().ofdft_optimize_multistep(hs, n, ps, rs)
    if not (st == OK or (allow_noconv and st == ENOCONV)):
        check(st)
    return list(rs), st


def ofdft_td_start(grid, k):
    """psi = sqrt(resident density) exp(-i k.r) (the kick)."""
    kk = (ctypes.c_double * 3)(*[float(x) for x in k])
    check(load().ofdft_td_start(grid, kk))


def ofdft_td_set_psi(grid, psi):
    re = np.ascontiguousarray(np.real(psi), dtype=np.float64).reshape(-1)
    im = np.ascontiguousarray(np.imag(psi), dtype=np.float64).reshape(-1)
    check(load().ofdft_td_set_psi(grid, _dptr(re), _dptr(im)))


def ofdft_td_get_psi(grid, shape):
    n = int(np.prod(shape))
    re = np.empty(n)
    im = np.empty(n)
    check(load().ofdft_td_get_psi(grid, _dptr(re), _dptr(im)))
    return (re + 1j * im).reshape(shape)


def ofdft_td_propagate(grid, dt, nsteps, n_corrector=1, solver_tol=0.0, max_solver_iter=0):
    """Returns (dipoles nsteps x 3, TdStats)."""
    p = TdParams(float(dt), int(n_corrector), int(max_solver_iter), float(solver_tol))
    mu = np.zeros((max(int(nsteps), 1), 3))
    st = TdStats()
    check(load().ofdft_td_propagate(grid, ctypes.byref(p), int(nsteps), _dptr(mu),
                                    ctypes.byref(st)))
    return mu[:int(nsteps)], st


def ofdft_validate(cell_desc, func_desc):
    """Host-only: returns the status (OK or EINVAL) without raising."""
    return load().ofdft_validate(ctypes.byref(cell_desc), ctypes.byref(func_desc))


def ofdft_footprint_bytes(cell_desc, func_desc, kind):
    b = ctypes.c_uint64()
    check(load().ofdft_footprint_bytes(ctypes.byref(cell_desc), ctypes.byref(func_desc),
                                       int(kind), ctypes.byref(b)))
    return int(b.value)


def ofdft_server_create(ctx, hbm_budget_bytes=0, max_inflight=4):
    h = ctypes.c_void_p()
    check(load().ofdft_server_create(ctx, int(hbm_budget_bytes), int(max_inflight),
                                     ctypes.byref(h)))
    return h


def ofdft_serve_submit(server, cell_id, kind, cell_desc, func_desc, opt=None, rho=None):
    """Returns the ticket; raises on a refused request."""
    q = Request()
    q.cell_id = int(cell_id)
    q.kind = int(kind)
    q.cell = ctypes.pointer(cell_desc)
    q.func = ctypes.pointer(func_desc)
    q.opt = ctypes.pointer(opt) if opt is not None else None
    keep = None
    if rho is not None:
        keep = np.ascontiguousarray(rho, dtype=np.float64)
        q.rho_or_null = _dptr(keep)
    t = ctypes.c_uint64()
    check(load().ofdft_serve_submit(server, ctypes.byref(q), ctypes.byref(t)))
    return int(t.value)


def ofdft_serve_poll(server, ticket, v_shape=None, natoms=None):
    """Returns (status, OptResult, v or None, f or None); status PENDING while running."""
    r = OptResult()
    v = np.full(v_shape, np.nan) if v_shape is not None else None
    f = np.full((natoms, 3), np.nan) if natoms else None
    st = load().ofdft_serve_poll(server, int(ticket), ctypes.byref(r),
                                 _dptr(v) if v is not None else None,
                                 _dptr(f) if f is not None else None)
    return st, r, v, f


def ofdft_serve_wait(server, ticket, timeout_ms=-1):
    return load().ofdft_serve_wait(server, int(ticket), int(timeout_ms))


def ofdft_serve_cancel(server, ticket):
    return load().ofdft_serve_cancel(server, int(ticket))


def ofdft_serve_set_batching(server, max_ep, max_opt):
    check(load().ofdft_serve_set_batching(server, int(max_ep), int(max_opt)))


def ofdft_serve_stats_get(server):
    st = ServeStats()
    check(load().ofdft_serve_stats_get(server, ctypes.byref(st)))
    return st.as_dict()


def ofdft_server_destroy(server):
    load().ofdft_server_destroy(server)


def ofdft_grid_set_graphs(grid, on=True):
    check(load().ofdft_grid_set_graphs(grid, 1 if on else 0))


def ofdft_grid_set_knot_skip(grid, on=True):
    check(load().ofdft_grid_set_knot_skip(grid, 1 if on else 0))


def ofdft_grid_set_col_group(grid, n):
    check(load().ofdft_grid_set_col_group(grid, int(n)))


def ofdft_grid_set_col_variant(grid, variant):
    check(load().ofdft_grid_set_col_variant(grid, int(variant)))


def ofdft_grid_set_knot_pipeline(grid, on=True):
    check(load().ofdft_grid_set_knot_pipeline(grid, 1 if on else 0))


def ofdft_grid_set_pipeline(grid, nsub):
    check(load().ofdft_grid_set_pipeline(grid, int(nsub)))


def ofdft_grid_tune_dev(grid, nbatch, d_rho, stream):
    r = TuneResult()
    check(load().ofdft_grid_tune_dev(grid, int(nbatch), d_rho, stream, ctypes.byref(r)))
    return r.as_dict()


def ofdft_grid_tune(grid):
    r = TuneResult()
    check(load().ofdft_grid_tune(grid, ctypes.byref(r)))
    return r.as_dict()


def ofdft_profile_enable(grid, on=True):
    check(load().ofdft_profile_enable(grid, 1 if on else 0))


def ofdft_profile_read(grid, pass_id):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    check(load().ofdft_profile_read(grid, int(pass_id), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


# ------------------------------------------------------------------ convenience
class Grid:
    """Owns a context and a grid for one cell/functional."""

    def __init__(self, cell, terms, precision=FP64, device=0, ctx=None, **func_kw):
        self.cell = cell
        self.shape = tuple(int(x) for x in cell["n"])
        self.natoms = len(cell["species"])
        self._own_ctx = ctx is None
        self.ctx = ofdft_ctx_create(device) if ctx is None else ctx
        cd, self._keep = make_cell_desc(cell)
        fd = make_functional_desc(terms, precision=precision, **func_kw)
        self.fp64 = precision == FP64
        self.handle = ofdft_grid_create(self.ctx, cd, fd)

    @property
    def field_dtype(self):
        return np.float64 if self.fp64 else np.float32

    def close(self):
        if self.handle:
            ofdft_grid_destroy(self.handle)
            self.handle = None
        if self._own_ctx and self.ctx:
            ofdft_ctx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def energy_potential(self, rho=None, want_v=True):
        return ofdft_energy_potential(self.handle, rho, want_v, self.shape)

    def set_density(self, rho):
        ofdft_set_density(self.handle, rho)

    def get_density(self):
        return ofdft_get_density(self.handle, self.shape)

    def forces(self):
        return ofdft_forces(self.handle, self.natoms)

    def optimize(self, tol=1e-7, max_iter=1000, allow_noconv=False, method=OPT_CG):
        return ofdft_optimize(self.handle, tol, max_iter, method=method,
                              allow_noconv=allow_noconv)
