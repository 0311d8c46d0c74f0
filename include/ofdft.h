/*
 * ofdft.h - C ABI of libofdft.so, an orbital-free DFT energy/potential engine
 * for one AMD MI355X (gfx950).
 *
 * The method is that of Shao, Jiang, Mi, Genova and Pavanello, "DFTpy: An
 * efficient and object-oriented platform for orbital-free DFT simulations"
 * (arXiv:2002.02985).  The library evaluates, on a periodic real-space grid,
 *
 *   E[rho] = T_TF + T_vW + T_NL + E_H + E_xc + int v_ext rho  (+ E_ion)
 *
 * (eq. "efunc"; E_xc the optional LDA term) and its functional derivative
 * v = dE/drho (eqs. "euler", "euler2a"), where T_NL is the Wang-Teter
 * functional (eq. "WT") or the density-dependent-kernel functional evaluated
 * with linear splines over k_F knots (steps s1-s4 of Section
 * "New-generation nonlocal KEDFs"), and minimises E over phi = sqrt(rho) at
 * fixed electron count (eq. "euler2", Section "Density optimization
 * strategies").
 *
 * Conventions
 *   Units: Hartree atomic units (Ha, Bohr).
 *   Grid: n[0] x n[1] x n[2] points, C order (index i2 fastest); point
 *     (i0,i1,i2) sits at r = sum_d (i_d / n_d) a_d, a_d = lattice[d][:].
 *     Every n[d] must be one of the supported FFT lengths (products of 2 and
 *     3 listed by ofdft_supported_length()), n[2] even.
 *   Integrals: int f = (V/N) sum_r f(r).  Fourier coefficients:
 *     f(G) = (1/N) sum_r f(r) exp(-i G.r); the inverse of a half spectrum is
 *     Re sum_half c(m2) X exp(i G.r), c = 1 on the m2 = 0 and m2 = n2/2
 *     planes, 2 elsewhere; Nyquist frequencies take the negative sign.
 *   Fields on the host are double, C order.  Fields passed as device
 *     pointers (the _dev calls) have the grid's field type: double for
 *     OFDFT_FP64 grids, float for OFDFT_MIXED grids.
 *
 * Ownership and errors
 *   Handles are created and owned by the library and released by the
 *   matching _destroy call (NULL is accepted and ignored).  Host arrays
 *   belong to the caller; they are read or written during the call only and
 *   never retained.  Device pointers are borrowed for the duration of the
 *   call on the given stream; the call returns after the stream work it
 *   enqueued has completed.  A grid handle is not thread-safe.
 *   No function aborts: each returns an ofdft_status, and
 *   ofdft_last_error() gives a message for the calling thread.
 *   Non-finite or negative densities give OFDFT_EINVAL.
 *
 * Environment (read when a grid is created; for tests and profiling)
 *   OFDFT_COL_TILE_MAJOR=0|1  fixes the block order of the column passes
 *     (array-major or tile-major), the choice ofdft_grid_tune otherwise makes,
 *     so that a profiled run without the autotuner launches the tuned kernels.
 *   OFDFT_LARGE_IONS=0|1  forces the small-cell (per-atom phase tables) or the
 *     large-cell (tiled sum, binned Ewald) ionic set-up regardless of the atom
 *     count, to compare the two on the same cell.
 */
#ifndef OFDFT_H
#define OFDFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OFDFT_ABI_VERSION 7

typedef struct ofdft_ctx ofdft_ctx;
typedef struct ofdft_grid ofdft_grid;
typedef struct ofdft_server ofdft_server;

typedef enum {
    OFDFT_OK = 0,
    OFDFT_PENDING = 1,
    OFDFT_EINVAL = -1,      /* bad argument, unsupported size, non-finite input */
    OFDFT_ENOMEM = -2,      /* device or host allocation failed                 */
    OFDFT_EDEVICE = -3,     /* HIP runtime error                                */
    OFDFT_ENOCONV = -4,     /* iteration budget exhausted (result still filled) */
    OFDFT_ECANCELLED = -5,
    OFDFT_ENOTFOUND = -6
} ofdft_status;

/* energy terms (bitmask) */
enum {
    OFDFT_TERM_TF = 1,        /* Thomas-Fermi  C_TF int rho^(5/3)                    */
    OFDFT_TERM_VW = 2,        /* von Weizsaecker  (lambda/2) int |grad sqrt(rho)|^2  */
    OFDFT_TERM_HARTREE = 4,   /* 2 pi V sum_{G!=0} |rho(G)|^2 / G^2                  */
    OFDFT_TERM_EXT = 8,       /* int v_ext rho with the local pseudopotential, + E_ion */
    OFDFT_TERM_WT = 16,       /* Wang-Teter nonlocal functional (eqs. "nl2", "WT")    */
    OFDFT_TERM_SPLINE = 32,   /* density-dependent kernel with k_F splines (s1-s4)    */
    OFDFT_TERM_XC = 64        /* LDA exchange-correlation, E_xc of eq. "efunc": Dirac
                                 exchange + Perdew-Zunger (1981) correlation of the
                                 unpolarised electron gas at the local density (the
                                 parametrisation the paper's applications cite)      */
};
enum { OFDFT_KNOTS_LOG = 0, OFDFT_KNOTS_LIN = 1 };
enum { OFDFT_NL_S3S4 = 0, OFDFT_NL_EXACT = 1 };
/* Precision.  FP64: every field, transform and reduction in FP64.
 * MIXED: FP32 fields, transforms and pointwise terms; FP64 energy
 * reductions, electron count, chemical potential and optimiser line search.
 * MIXED_VW64: as MIXED, except that phi's transform pair behind the von
 * Weizsaecker term runs in FP64 (FP32 input, FP64 spectrum, -lambda nabla^2
 * phi returned to the FP32 combine).  v_vW divides that Laplacian by phi, so
 * the FP32 transforms' absolute rounding (about 1e-7 of max |phi|) becomes
 * a potential error of order 1e-5 / phi Ha: MIXED meets 1e-4 Ha in
 * max |dE/drho| where rho >~ 1e-3 (bulk cells), MIXED_VW64 down to
 * rho = 1e-6 (cells with vacuum), at the cost of one FP64 transform pair.
 * Fields passed as device pointers are FP32 in both mixed modes. */
enum { OFDFT_FP64 = 0, OFDFT_MIXED = 1, OFDFT_MIXED_VW64 = 2 };

/* Ionic structure factor S(G) = sum_a exp(-iG.R_a) behind v_ext(G) and the
 * Ewald reciprocal sum.  DIRECT: the exact sum (per-atom phase tables below
 * 8192 atoms, a tiled direct sum from there on).  PME: the smooth
 * particle-mesh Ewald approximation the paper uses for large cells (Sections
 * "OFDFT software background" and "Leveraging existing techniques"; the
 * method of Essmann et al. 1995): each species' atoms spread onto the grid
 * with cardinal B-splines of order pme_order, one forward transform, and the
 * exponential-spline factors; the Ewald split is chosen so that the
 * reciprocal sum ends at half the box.  PME takes the large-cell ionic path
 * at any atom count, where ofdft_forces is not offered.  Its set-up (grid
 * creation, and each change of positions) also allocates, and frees again,
 * N x 8 bytes for the fixed-point charge grid, N x 4 more on a mixed grid
 * and 16 bytes per half-spectrum point with more than one species; these
 * transient bytes are not part of ofdft_footprint_bytes or
 * ofdft_grid_device_bytes. */
enum { OFDFT_SF_DIRECT = 0, OFDFT_SF_PME = 1 };

/* Cell: lattice vectors as rows (Bohr), grid, atoms.  pos is natoms x 3
 * Cartesian Bohr; species[a] indexes Z[] (valence charge) and rc[] (radius of
 * the local pseudopotential v(G) = -4 pi Z exp(-G^2 rc^2 / 4) / G^2, i.e.
 * -Z erf(r/rc)/r, with the non-Coulomb G = 0 value pi Z rc^2).  sf_method is
 * an OFDFT_SF_* value (0, the exact sum, when zero-initialised); pme_order the
 * even B-spline order 4 .. 16, at most every n[d] (0 selects 10). */
typedef struct {
    double lattice[3][3];
    int32_t n[3];
    int32_t natoms;
    const double *pos;
    const int32_t *species;
    int32_t nspecies;
    const double *Z;
    const double *rc;
    double nelec;
    int32_t sf_method;
    int32_t pme_order;
} ofdft_cell_desc;

/* Kernel family of the nonlocal term (WT and SPLINE alike).  WT: eq. "WT",
 * omega = C_WT G_NL(q / (2 k_F)).  MGP, MGPA, MGPG: eq. "MGP",
 * omega_{x,y} = omega_WT - x C_WT int_0^1 t^y d/dt G_NL(eta(q, t)) dt with
 * (x, y) = (1, 5/6), (1/2, 5/6), (1, 5/3), read with eta(q, t) =
 * q / (2 t^(1/3) k_F) (functional integration along the scaled density
 * t rho; the paper defers eta(q, t) to a supplement).  As in step s2, the
 * correction is evaluated once at fixed eta nodes (spacing 1/2048 up to
 * eta = 4, then 1/16384 in 1/eta^2) and interpolated linearly; with SPLINE
 * these are the LMGP functionals. */
enum { OFDFT_KERNEL_WT = 0, OFDFT_KERNEL_MGP = 1, OFDFT_KERNEL_MGPA = 2, OFDFT_KERNEL_MGPG = 3 };

/* Functional.  alpha and beta are the exponents of eq. "nl2"; the GPU path
 * requires alpha == beta.  kf_wt <= 0 selects (3 pi^2 nelec / V)^(1/3) for
 * the Wang-Teter kernel.  Spline knots (step s1): nk values from kf_min to
 * kf_max, geometric (LOG) or arithmetic (LIN), both ends included.
 * nl_mode S3S4 interpolates the per-knot potentials (steps s3, s4 as
 * printed); EXACT returns the functional derivative of the spline energy.
 * rho_floor (default 1e-12) bounds rho^(alpha-1) and 1/sqrt(rho).
 * nl_kernel is an OFDFT_KERNEL_* value (0, Wang-Teter, when zero-initialised). */
typedef struct {
    uint32_t terms;
    double lambda_vw;
    double alpha, beta;
    double kf_wt;
    int32_t nk;
    double kf_min, kf_max;
    int32_t knot_spacing;
    int32_t nl_mode;
    int32_t precision;
    double rho_floor;
    int32_t nl_kernel;
} ofdft_functional_desc;

/* Energies (Ha).  mu = int v rho / int rho; resid_norm = sqrt(mean(R^2)) with
 * R = dE/dphi - 2 mu phi (the residual of eq. "euler2"). */
typedef struct {
    double e_tf, e_vw, e_h, e_ext, e_nl, e_ion, e_total;
    double mu, nelec_int, resid_norm;
    double e_xc;   /* included in e_total */
} ofdft_energy;

int ofdft_abi_version(void);
const char *ofdft_last_error(void);
/* 1 if n is an FFT length the library has kernels for, else 0. */
int ofdft_supported_length(int32_t n);

/* A context is one device and one HIP stream (non-blocking, default
 * priority) on which the grids created from it run. */
ofdft_status ofdft_ctx_create(int device, ofdft_ctx **out);
void ofdft_ctx_destroy(ofdft_ctx *ctx);

/* Host-only checks (no device needed): whether a cell and functional are
 * accepted by ofdft_grid_create, and the device bytes a request of the given
 * kind (OFDFT_REQ_*) needs on a new grid: fixed tables, workspace for one
 * density, host-API staging, plus the optimiser vectors (OPTIMIZE) or the
 * force buffer (FORCES).  These are the figures the server admits by. */
ofdft_status ofdft_validate(const ofdft_cell_desc *cell, const ofdft_functional_desc *func);
ofdft_status ofdft_footprint_bytes(const ofdft_cell_desc *cell,
                                   const ofdft_functional_desc *func, int32_t kind,
                                   uint64_t *bytes);

/* Builds the grid: reciprocal vectors, twiddle tables, the ionic structure
 * factor and v_ext(G) (by the cell's sf_method: the exact direct sum --
 * separable per-atom phases below 8192 atoms, a tiled sum from there on --
 * or smooth PME), the Ewald energy E_ion, and device buffers for one
 * density.  The descriptors are copied. */
ofdft_status ofdft_grid_create(ofdft_ctx *ctx, const ofdft_cell_desc *cell,
                               const ofdft_functional_desc *func, ofdft_grid **out);
void ofdft_grid_destroy(ofdft_grid *grid);
/* Pre-allocates workspace for batched calls of up to nbatch densities. */
ofdft_status ofdft_grid_reserve(ofdft_grid *grid, int32_t nbatch);
/* Bytes of device memory the grid currently holds. */
uint64_t ofdft_grid_device_bytes(const ofdft_grid *grid);

/* Resident density (N doubles, C order), kept on the device in the grid's
 * field type; used by energy_potential(NULL, ...), forces and optimize. */
ofdft_status ofdft_set_density(ofdft_grid *grid, const double *rho_host);
ofdft_status ofdft_get_density(ofdft_grid *grid, double *rho_host);

/* Energy and potential for rho (host, N doubles) or, if rho is NULL, the
 * resident density.  v_out (host, N doubles, may be NULL) receives
 * v = dE/drho; e_out must not be NULL. */
ofdft_status ofdft_energy_potential(ofdft_grid *grid, const double *rho_host,
                                    double *v_out_host, ofdft_energy *e_out);

/* Device variant: d_rho and d_v (may be NULL) are device arrays of N values
 * of the grid's field type, hip_stream a hipStream_t (NULL = the context's
 * own stream). */
ofdft_status ofdft_energy_potential_dev(ofdft_grid *grid, const void *d_rho, void *d_v,
                                        void *hip_stream, ofdft_energy *e_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the device
 * variant above for one density with the evaluation's whole workspace (the
 * spectra, the spline knot spectra and accumulators, the FP64 von Weizsaecker
 * leg's buffers and the partial sums) in a static device array of the library
 * instead of the grid's buffers.  The call allocates nothing: no hipMalloc,
 * hipFree, graph or event; the grid (created earlier) provides its tables.
 * The array holds OFDFT_NOALLOC_SCRATCH_BYTES per device, reserved by the
 * library on every device it runs on until the process ends; its address on
 * a device is resolved by ofdft_ctx_create.  A grid whose one-density
 * workspace is larger (for example a 256x256x384 spline grid: 8 knot spectra
 * of 101 MB) gives OFDFT_EINVAL before anything is launched.  Results are
 * those of ofdft_energy_potential_dev without graphs or pipelining (the same
 * launches).  Every call on a device shares the array, so calls that overlap
 * on one device (on different streams or threads) race; the call returns
 * after its stream work has completed.  Non-finite or negative densities
 * give OFDFT_EINVAL, with e_out left untouched. */
#define OFDFT_NOALLOC_SCRATCH_BYTES (128u * 1024u * 1024u)
ofdft_status ofdft_energy_potential_dev_noalloc(ofdft_grid *grid, const void *d_rho, void *d_v,
                                                void *hip_stream, ofdft_energy *e_out);

/* Batched device variant: nbatch densities of the same cell, stored
 * back to back (nbatch x N values); d_v likewise (may be NULL);
 * e_out has nbatch entries.  Every step of the evaluation runs for the whole
 * batch in each kernel launch. */
ofdft_status ofdft_energy_potential_batch_dev(ofdft_grid *grid, int32_t nbatch,
                                              const void *d_rho, void *d_v,
                                              void *hip_stream, ofdft_energy *e_out);

/* Energy and potential of the resident densities of n different cells in
 * one batched evaluation (the serving loop's batches of requests): every
 * kernel launch processes all n densities, the reciprocal-space terms use
 * each cell's own reciprocal vectors, v_ext(G), kernel table and E_ion.  The
 * grids must share the grid shape, every field of the functional (precision
 * included) and the device; the cells may differ in lattice, atoms and
 * electron count.  grids[0] leads: its workspace (grown to n densities, plus
 * n densities of staging for inputs and potentials), launch schedule and
 * stream serve the batch.  v_out_or_null: NULL, or n pointers each NULL or
 * to N doubles; e_out: n entries.  Each result is the same, bit for bit, as
 * ofdft_energy_potential(grids[b], NULL, ...) with the leader's schedule.
 * 1 <= n <= OFDFT_MULTI_MAX; no grid may appear twice; none may be in use
 * by another thread. */
#define OFDFT_MULTI_MAX 64
ofdft_status ofdft_energy_potential_multi(ofdft_grid *const *grids, int32_t n,
                                          double *const *v_out_or_null, ofdft_energy *e_out);

/* The 3D FFT pair on the grid (the transforms behind every reciprocal-space
 * term): forward d_out = r2c(d_in) as n0 x n1 x (n2/2+1) interleaved complex
 * values, normalised by 1/N; inverse d_out = Re sum_half c X exp(iG.r)
 * (unnormalised).  Device arrays of the grid's field type, nbatch fields. */
ofdft_status ofdft_fft_r2c_dev(ofdft_grid *grid, int32_t nbatch, const void *d_in,
                               void *d_out, void *hip_stream);
ofdft_status ofdft_fft_c2r_dev(ofdft_grid *grid, int32_t nbatch, const void *d_in,
                               void *d_out, void *hip_stream);

/* Forces on the ions (Ha/Bohr, natoms x 3 doubles) for the resident density:
 * F_a = -d(E_ext + E_ion)/dR_a at fixed rho, i.e. the Hellmann-Feynman
 * electron-ion term of the int v_ext rho energy of eq. "efunc" (v_ext the
 * sum of the atoms' local pseudopotentials, Section "DFTpy classes", the
 * IONS functional) plus the Ewald ion-ion term.  This is the force the
 * paper's ASE calculator hands to molecular dynamics (Section "Other
 * Classes and APIs", the DFTpyCalculator; Section "DFTpy+ASE: Dynamics of
 * liquid aluminum") and is exact at the optimised density.  Not offered from
 * 8192 atoms on or with sf_method PME (OFDFT_EINVAL). */
ofdft_status ofdft_forces(ofdft_grid *grid, double *f_out_host);

/* Density optimisation (Section "Density optimization strategies"):
 * nonlinear conjugate gradients (Polak-Ribiere, restarted on loss of
 * descent) on phi = sqrt(rho) with the update phi cos(t) + p sin(t),
 * p orthogonal to phi and normalised to N_e, and a strong-Wolfe line search
 * over t in FP64.  Starts from the resident density (warm start) and leaves
 * the optimised density resident.  Converged when sqrt(mean(R^2)) < tol;
 * OFDFT_ENOCONV (with the result filled in) when max_iter is reached. */
enum {
    OFDFT_OPT_CG = 0,   /* Polak-Ribiere+ on the residual R                          */
    OFDFT_OPT_PCG = 1,  /* the same on z = K R with the reciprocal-space preconditioner
                           K(G) = 1 / (1 + G^2 + 16 pi rho0 / G^2), rho0 = N_e / V, the
                           inverse of the phi-Hessian's vW (G^2) and long-wavelength
                           Hartree (16 pi rho0 / G^2) parts plus a unit shift; K(0) = 1
                           (two extra transforms per iteration)                       */
    OFDFT_OPT_TN = 2    /* truncated Newton (the paper's TN): the direction solves
                           H_T d = -R approximately by CG preconditioned with K, H_T the
                           Hessian of E on the tangent space of the N_e constraint
                           applied by finite differences of dE/dphi (one evaluation per
                           product, at most 20 per iteration, stopped at |r| <=
                           min(1/2, sqrt(rms R)) |R| or on negative curvature); the
                           line search starts at the Newton step                     */
};
typedef struct {
    double tol;
    int32_t max_iter;
    int32_t method;   /* OFDFT_OPT_CG, OFDFT_OPT_PCG or OFDFT_OPT_TN */
    int32_t warm;     /* server requests: start from the resident density */
} ofdft_opt_params;
typedef struct {
    ofdft_energy e;
    int32_t iters, evals;
    double final_resid;
} ofdft_opt_result;
ofdft_status ofdft_optimize(ofdft_grid *grid, const ofdft_opt_params *params,
                            ofdft_opt_result *result);

/* Lockstep optimisation of the resident densities of n different cells (the
 * serving loop's batches of optimisation requests; Section "Density
 * optimization strategies" per cell): each grid runs ofdft_optimize with its
 * own params[b] in a host thread of its own on a stream of its own, and the
 * evaluations the optimisers ask for are merged: an evaluation waits until
 * every member still optimising has asked for one, and they run as one
 * batched evaluation (as ofdft_energy_potential_multi, with phi as input
 * and dE/dphi as output), so every kernel launch serves all members.  Each
 * result is the same, bit for bit, as ofdft_optimize on that grid alone.
 * The grids must satisfy the conditions of ofdft_energy_potential_multi and
 * each hold a resident density; on return each holds its optimised density.
 * statuses[b] receives the member's ofdft_optimize status (OFDFT_OK,
 * OFDFT_ENOCONV, ...; ofdft_last_error() then names the first failing
 * member); the call returns OFDFT_OK when the members ran, OFDFT_EINVAL for
 * bad arguments.  None of the grids may be in use by another thread. */
ofdft_status ofdft_optimize_multi(ofdft_grid *const *grids, int32_t n,
                                  const ofdft_opt_params *params, ofdft_opt_result *results,
                                  ofdft_status *statuses);

/* Multi-step density optimisation (Section "Density optimization
 * strategies": a full optimisation on a coarse grid, the converged density
 * interpolated onto a finer grid, and the optimisation continued there).
 *
 * ofdft_grid_interpolate_density sets dst's resident density from src's:
 * phi = sqrt(rho) of src is Fourier interpolated onto dst's grid -- its half
 * spectrum zero-padded: frequencies strictly inside src's band copied, src's
 * Nyquist coefficient of an even axis split in halves between +-n/2, nothing
 * beyond; an axis of equal size copied -- then squared and scaled to dst's
 * electron count.  Both grids: same device, same precision, the same cell
 * (lattice within 1e-12), dst at least as fine as src on every axis, src
 * with a resident density; else OFDFT_EINVAL.  Synchronous.
 *
 * ofdft_optimize_multistep runs ofdft_optimize on grids[0] (from its
 * resident density) with params[0], then for i = 1 .. ngrids-1 interpolates
 * the result onto grids[i] and optimises there with params[i]; results[i]
 * receives each step's result.  A step that reaches max_iter (OFDFT_ENOCONV)
 * still hands its density on; the return value is the last step's status,
 * or the first other error. */
ofdft_status ofdft_grid_interpolate_density(ofdft_grid *dst, ofdft_grid *src);
ofdft_status ofdft_optimize_multistep(ofdft_grid *const *grids, int32_t ngrids,
                                     const ofdft_opt_params *params, ofdft_opt_result *results);

/* ------------------------------------------------------------------ serving
 * A request server for many cells on one device: energy+potential, force and
 * optimisation requests (the three operations above) are submitted from any
 * thread and run by max_inflight worker slots, each with its own stream, so
 * that requests admitted while others are on the device overlap with them.
 *
 * Residency and warm starts: each cell_id keeps its grid, and with it its
 * density, on the device after a request completes.  A later request with the
 * same cell_id, lattice, grid, species and functional reuses that grid; if
 * only the atom positions changed (successive MD frames) the structure factor,
 * v_ext(G) and E_ion are rebuilt in place and the resident density is the
 * warm start.  Requests of one cell_id run one at a time in submission order.
 *
 * Admission by HBM footprint: a request that needs a new grid is admitted
 * when its footprint (ofdft_footprint_bytes, OPTIMIZE kind, so a resident
 * grid never grows) fits in hbm_budget_bytes next to the resident grids;
 * idle resident grids are evicted least recently used first, those with no
 * queued request before the others.  An evicted cell's density is kept in
 * host memory (N doubles per cell; at most 8 GiB in all, the least recently
 * saved dropped first) and is the starting density when that cell's grid is
 * built again with the same grid shape for a request that brings none
 * (OPTIMIZE with warm = 0 excepted), so warm starts survive eviction.  Until
 * an evicted grid's density has been saved and the grid freed, the grid stays
 * counted against the budget and requests of its cell wait.  A request that cannot fit yet waits, and
 * no later request that needs new memory overtakes it; requests for resident
 * grids still run.  A footprint above the whole budget is refused at submit
 * with OFDFT_ENOMEM.
 *
 * Continuous batching: when a worker takes an energy+potential or (if
 * enabled, ofdft_serve_set_batching) an optimisation request whose cell's
 * grid is resident, it also takes further
 * queued requests of the same kind of other resident cells with the same
 * grid shape and functional (each the earliest queued request of its cell),
 * up to 8, and serves them together -- one batched evaluation
 * (ofdft_energy_potential_multi), or one lockstep optimisation
 * (ofdft_optimize_multi) -- if the leading grid's larger workspace fits in
 * the budget (the growth is counted from the moment the batch is formed);
 * results are the same as alone.
 *
 * Request kinds and results:
 *   EP        energy and potential of rho_or_null, else of the resident
 *             density (a cell with none starts from the uniform density
 *             nelec/V); fills res->e and, at poll, v (N doubles).
 *   FORCES    energy and forces (natoms x 3, Ha/Bohr) of that density;
 *             fills res->e and f.
 *   OPTIMIZE  density optimisation with *opt from rho_or_null if given, else
 *             from the resident density when opt->warm != 0, else from the
 *             uniform density; fills res (OFDFT_ENOCONV if max_iter was hit).
 *   In every kind rho_or_null, when given, becomes the resident density, and
 *   OPTIMIZE leaves the optimised density resident.
 * submit deep-copies the request (descriptors, positions, density) and checks
 * it (OFDFT_EINVAL for a bad descriptor or a non-finite or negative density).
 * poll returns OFDFT_PENDING until the request has finished, then its final
 * status (OK, ENOCONV, ECANCELLED or an error, with ofdft_last_error() set),
 * copies the results into the non-NULL outputs and releases the ticket;
 * unknown or released tickets give OFDFT_ENOTFOUND.  cancel removes a queued
 * request, asks a running optimisation to stop at its next iteration and
 * discards any result: poll then gives OFDFT_ECANCELLED.  submit, poll, wait,
 * cancel and stats are thread-safe.  destroy cancels what is queued, waits
 * for what runs and frees every grid. */
enum { OFDFT_REQ_EP = 0, OFDFT_REQ_FORCES = 1, OFDFT_REQ_OPTIMIZE = 2 };
typedef struct {
    uint64_t cell_id;
    int32_t kind;
    const ofdft_cell_desc *cell;
    const ofdft_functional_desc *func;
    const ofdft_opt_params *opt;   /* OPTIMIZE only */
    const double *rho_or_null;     /* N doubles or NULL */
} ofdft_request;
typedef struct {
    uint64_t submitted, completed, failed, cancelled;
    int32_t queued, running, resident_cells, max_inflight;
    uint64_t resident_bytes, peak_bytes, budget_bytes;
    double p50_ms, p99_ms;          /* submit-to-finish latency of completed requests */
    double mean_queue_ms;           /* submit-to-start                                */
    uint64_t batches;               /* batched evaluations of several cells           */
    uint64_t batched_requests;      /* requests served in them                        */
} ofdft_serve_stats;
ofdft_status ofdft_server_create(ofdft_ctx *ctx, uint64_t hbm_budget_bytes,
                                 int32_t max_inflight, ofdft_server **out);
ofdft_status ofdft_serve_submit(ofdft_server *srv, const ofdft_request *req,
                                uint64_t *ticket);
ofdft_status ofdft_serve_poll(ofdft_server *srv, uint64_t ticket, ofdft_opt_result *res,
                              double *v_or_null, double *f_or_null);
/* Blocks until the request has finished (OFDFT_OK) or timeout_ms has passed
 * (OFDFT_PENDING); does not release the ticket.  timeout_ms < 0 waits
 * without limit. */
ofdft_status ofdft_serve_wait(ofdft_server *srv, uint64_t ticket, int32_t timeout_ms);
ofdft_status ofdft_serve_cancel(ofdft_server *srv, uint64_t ticket);
ofdft_status ofdft_serve_stats_get(ofdft_server *srv, ofdft_serve_stats *out);
/* Largest batch of energy+potential requests and of optimisation requests
 * (continuous batching above; defaults 8 and 1; 1 serves each request alone,
 * at most OFDFT_MULTI_MAX).  Lockstep optimisation batches are off by
 * default: on the mixed serving workload several worker slots running
 * optimisations side by side keep the device busier than one slot running
 * them in lockstep.  Applies to batches formed after the call.
 * OFDFT_EINVAL outside 1..OFDFT_MULTI_MAX. */
ofdft_status ofdft_serve_set_batching(ofdft_server *srv, int32_t max_ep, int32_t max_opt);
void ofdft_server_destroy(ofdft_server *srv);

/* Launch schedule.  An evaluation's launch sequence can be replayed from a HIP
 * graph captured on first use for each argument set (batch size, input,
 * outputs); at most 8 graphs are kept per grid, and they are dropped when the
 * grid's workspace is reallocated.  Graphs need a capturable stream (not the
 * legacy NULL stream) and are not used while per-pass timing is on.
 * ofdft_grid_set_pipeline splits every batch evaluation into nsub
 * sub-batches (nsub >= 1, default 1) that alternate between the caller's
 * stream and the grid's own second stream, forked from and joined back into
 * the caller's; every density's results are the same for any split.  It is
 * not used while per-pass timing is on.
 * The autotuner times the schedule choices -- fused plane kernels or
 * separate row and column passes where both apply, the block order of the
 * column passes, the number of densities a column block serves (one, or a
 * group of up to 8 sharing the tile's set-up and operands; batches of
 * nbatch > 1 on short columns), the number of spline knots per batch, the
 * knot pipeline (below) -- and then, on the fastest of those, the launch
 * shapes the reciprocal-space column pass offers for the axis-0 length
 * (ofdft_grid_set_col_variant) -- on nbatch densities
 * at d_rho (device, the grid's field type; ofdft_grid_tune: the resident
 * density, nbatch 1; a column-pass shape is kept only if it times at least
 * 3% faster than the default one), keeps the fastest for the grid and for every grid of
 * the same shape, precision, functional and batch size created later in the
 * process, and reports it. */
typedef struct {
    int32_t plane, col_tile_major, knot_batch, candidates;
    double best_ms, default_ms;   /* per evaluation call */
    int32_t pipe;                 /* the grid's sub-batch split (not tuned) */
    int32_t col_group;            /* densities per column block (1 or up to 8) */
    int32_t knot_pipe;            /* knot pipeline on (1) or off */
    int32_t col_variant;          /* reciprocal-space column pass shape (0..3) */
} ofdft_tune_result;
ofdft_status ofdft_grid_set_graphs(ofdft_grid *grid, int32_t on);
/* Spline knot range (step s1 on the device; on by default): before the knot
 * loop, one pass over the input finds each density's smallest and largest
 * rho, and with them the knots whose hat functions are non-zero at some
 * point (S3S4: every point's bracket, taken as the interpolation takes it;
 * EXACT: the extremes' brackets and one more knot on each side); the
 * per-knot transforms and the
 * interpolation skip every other knot, whose contributions are exact zeros.
 * Off transforms every knot (the same results: a check of the skipping). */
ofdft_status ofdft_grid_set_knot_skip(ofdft_grid *grid, int32_t on);
/* Densities per column block of the reciprocal-space column pass on batches
 * (the autotuner's choice, set by hand): 1, or up to 8 (a block then takes
 * one tile for up to n densities, its set-up and per-element operands shared;
 * used for columns of at most 8 elements per thread and batches that keep
 * enough blocks).  Results are the same, bit for bit, for every n.
 * OFDFT_EINVAL outside 1..8. */
ofdft_status ofdft_grid_set_col_group(ofdft_grid *grid, int32_t n);
/* Knot pipeline (spline grids with more than 8 knots whose knot spectra take
 * at most 4 GiB, where the grid holds a second knot-spectrum buffer; on by
 * default): knot batch i's transforms run on the grid's second stream into
 * buffer i % 2 while the row pass of batch i - 1 runs on the caller's stream
 * (forked from it and joined back; not used while per-pass timing is on or
 * with a sub-batch split).  Results are the same, bit for bit, either way. */
ofdft_status ofdft_grid_set_knot_pipeline(ofdft_grid *grid, int32_t on);
/* Launch shape of the reciprocal-space column pass (the autotuner's choice,
 * set by hand): bit 0 half the columns per block (twice the blocks), bit 1
 * the transform's radices in reverse order (another Stockham factorisation
 * of the same DFT).  Offered for FP32 passes of lengths 64, 96, 128, 192 and
 * 256 where the shape differs from the default (ofdft_tune_result's
 * col_variant reports what was kept); other lengths, FP64 passes and
 * multi-cell batches use the default shape whatever is set.  Results agree
 * with the default shape to the precision's rounding (the radix order
 * changes the order of the butterflies' sums).  OFDFT_EINVAL outside 0..3. */
ofdft_status ofdft_grid_set_col_variant(ofdft_grid *grid, int32_t variant);
ofdft_status ofdft_grid_set_pipeline(ofdft_grid *grid, int32_t nsub);
ofdft_status ofdft_grid_tune_dev(ofdft_grid *grid, int32_t nbatch, const void *d_rho,
                                 void *hip_stream, ofdft_tune_result *result);
ofdft_status ofdft_grid_tune(ofdft_grid *grid, ofdft_tune_result *result);

/* Per-pass timing of the evaluation pipeline (a profiling aid): when
 * enabled, every kernel launch of the passes below is bracketed by HIP events
 * recorded on the stream it is launched on, and the elapsed times are summed
 * per pass.  Enabling resets the counters. */
enum {
    OFDFT_PASS_ROW_FWD = 0,   /* prologue + axis-2 r2c                          */
    OFDFT_PASS_COL1_FWD,      /* axis-1 forward c2c                             */
    OFDFT_PASS_COL0_G,        /* axis-0 c2c with the reciprocal-space terms     */
    OFDFT_PASS_COL1_INV,      /* axis-1 inverse c2c                             */
    OFDFT_PASS_ROW_INV,       /* axis-2 c2r + combine of the potential          */
    OFDFT_PASS_KNOT_INV,      /* spline: omega_i multiply + axis-0 inverse      */
    OFDFT_PASS_KNOT_COL1,     /* spline: axis-1 inverse of the knot spectra     */
    OFDFT_PASS_KNOT_ROW,      /* spline: axis-2 c2r + interpolation over k_F    */
    OFDFT_PASS_EXACT_FWD,     /* spline EXACT: transforms of rho^a L_i          */
    OFDFT_PASS_EXACT_ACC,     /* spline EXACT: sum_i omega_i F[rho^a L_i]       */
    OFDFT_PASS_FINALIZE,      /* FP64 reductions                                */
    OFDFT_PASS_OTHER,         /* optimiser vector kernels                       */
    OFDFT_PASS_VW64,          /* the FP64 von Weizsaecker leg of MIXED_VW64     */
    OFDFT_NPASS
};
ofdft_status ofdft_profile_enable(ofdft_grid *grid, int32_t on);
ofdft_status ofdft_profile_read(ofdft_grid *grid, int32_t pass, double *total_ms,
                                int64_t *launches);

/* Real-time TD-OFDFT (Section "Time-Dependent OFDFT"): the collective
 * orbital psi, |psi|^2 = rho, obeys i d psi/dt = H psi with
 * H = -(1/2) nabla^2 + v, v = the functional derivative of every term of the
 * grid's functional except von Weizsaecker (dT_Pauli/drho + v_s of eq.
 * "heq", evaluated at the current density; the functional must contain vW
 * with lambda_vw = 1).  Each step solves the Crank-Nicolson system of eq.
 * "cn" in the sign of the time-dependent equation,
 * (1 + i dt/2 H) psi(t + dt) = (1 - i dt/2 H) psi(t), by BiCGSTAB from
 * psi(t); H is first built from rho(t) (predictor), then n_corrector times
 * from the midpoint density (rho(t) + |psi_trial|^2) / 2.  The state lives
 * on the grid (about 23 N field values of device memory).
 *
 * ofdft_td_start: psi = sqrt(resident density) exp(-i k.r), the kick of
 *   strength |k| (Bohr^-1); r = sum_d (i_d / N_d) a_d.
 * ofdft_td_set_psi / ofdft_td_get_psi: psi as two host arrays of N doubles
 *   (real and imaginary parts).
 * ofdft_td_propagate: nsteps steps; dipole_out (may be NULL) receives
 *   mu = int r |psi|^2 dr (3 doubles, Bohr) after each step, nsteps x 3;
 *   stats the solver work, the largest final relative residual
 *   |b - A x| / |b| and int |psi|^2 at the end.  solver_tol <= 0 selects
 *   1e-11 (FP64) or 1e-6 (mixed), max_solver_iter <= 0 selects 200; a solve
 *   that stops above its tolerance is counted, not an error. */
typedef struct {
    double dt;               /* a.u. of time; may be negative (backwards)       */
    int32_t n_corrector;     /* 0 .. 16                                          */
    int32_t max_solver_iter;
    double solver_tol;
} ofdft_td_params;
typedef struct {
    int32_t steps, solver_iters, unconverged_solves, reserved;
    double max_solver_resid;
    double nelec;
} ofdft_td_stats;
ofdft_status ofdft_td_start(ofdft_grid *grid, const double k[3]);
ofdft_status ofdft_td_set_psi(ofdft_grid *grid, const double *re_host, const double *im_host);
ofdft_status ofdft_td_get_psi(ofdft_grid *grid, double *re_host, double *im_host);
ofdft_status ofdft_td_propagate(ofdft_grid *grid, const ofdft_td_params *params, int32_t nsteps,
                                double *dipole_out, ofdft_td_stats *stats);

#ifdef __cplusplus
}
#endif
#endif /* OFDFT_H */
