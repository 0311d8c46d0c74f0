// Host-visible launch interface of the HIP kernels.  Every launcher checks
// its shapes against the kernel's compile-time tiling before it launches and
// returns hipErrorInvalidValue for a length it has no kernel for.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "mgp_table.hpp"

namespace ofdft {

// partial-sum slots (FP64), one row of per-workgroup partials per slot
enum Slot {
    SL_RHO = 0,     // sum rho
    SL_TF,          // sum rho^(5/3)
    SL_H,           // sum_half c |rho(G)|^2 / G^2
    SL_EXT,         // sum_half c Re[conj(v_ext(G)) rho(G)]
    SL_VW,          // sum_half c G^2 |phi(G)|^2
    SL_NL,          // sum rho^alpha Phi  (or rho^alpha v1 for the spline)
    SL_GPHI,        // sum g phi
    SL_GG,          // sum g^2
    SL_PHIPHI,      // sum phi^2
    SL_BAD,         // count of non-finite or negative inputs
    SL_XC,          // sum rho eps_xc(rho)
    SL_AUX0,        // slots for vector reductions
    SL_AUX1,
    SL_AUX2,
    SL_AUX3,
    NSLOT
};

// field kinds of the forward (prologue) kernel
enum FieldKind { FK_RHO = 0, FK_PHI = 1, FK_RHOB = 2, FK_RAW = 3, FK_KNOT = 4 };
// reciprocal-space operations of the axis-0 kernel
// GO_PRECOND: multiply by q0^2 / (G^2 + q0^2 + h / G^2) (q0^2 = precond_q2,
// h = precond_h; 1 at G = 0), the optimiser's reciprocal-space preconditioner
enum GOp { GO_NONE = 0, GO_HEXT = 1, GO_VW = 2, GO_WT = 3, GO_SCALE = 4, GO_PRECOND = 5 };
// epilogues of the inverse row kernel
enum EpiMode { EP_STORE = 0, EP_COMBINE = 1, EP_KNOTS = 2 };

constexpr int MAXKNOTS = 64;
constexpr int MAXKB = 8;     // knots per batch of the spline loop

struct Geom {
    int n0, n1, n2, m, n2h;
    long long N, Nh;            // real points, half-spectrum points per field
    double b[3][3];             // reciprocal vectors (rows)
    double invN;
};

// Nonlocal kernel family (eq. "WT" or eq. "MGP"): omega = C_WT K(eta),
// K = G_NL for Wang-Teter (x = 0), K = (1 - x) G_NL + x J for MGP / MGPA / MGPG,
// J linearly interpolated on the table built in mgp_table.hpp (device copy in
// the kernel's field type; k_gtab reads an FP64 copy).
struct NlKern {
    double x;                   // 0: Wang-Teter
    const void *tab;            // MGP_TAB values of J
};

// k_F knots: the values live in device memory (kernels index them with
// data-dependent brackets, which must not pull a table into registers)
struct Knots {
    int nk;
    int log_spacing;
    double inv_span;            // (nk-1)/ln(k_N/k_1)  or  (nk-1)/(k_N-k_1)
    const double *k;            // device array of nk values
};

// forward row pass: axis-2 r2c of up to 4 fields derived pointwise from the
// input (rho or phi), plus FP64 partials of the prologue.
struct RowFwdArgs {
    const void *in;             // nbatch x N (field type)
    void *out;                  // spectra: out + f * out_fstride + b * Nh
    long long out_fstride;
    int nfields;
    int kind[MAXKB];
    int in_is_phi;
    double beta;                // exponent of FK_RHOB
    double alpha;               // exponent of FK_KNOT (rho^alpha L_i)
    int knot0;                  // FK_KNOT: knot index of field f is knot0 + f
    Knots knots;
    int partials;               // accumulate SL_RHO, SL_TF, SL_BAD
    double *part;               // [nbatch][NSLOT][pstride]
    int pstride;
    const void *twM;            // W_M^n, n < M
    const void *twN;            // W_{n2}^k, k <= M
    const void *tw1;            // W_{n1}^n (plane kernels)
    int in_f32;                 // FP64 kernels: the input is FP32 (the FP64 von
                                // Weizsaecker leg of a mixed-precision grid)
    const int *kneed;           // FK_KNOT fields: per-density knot range (see
                                // launch_knot_range), or null for every knot
};

// Per-entry cell data of a batch whose densities belong to different cells
// of one grid shape and functional (ofdft_energy_potential_multi): the
// cell's reciprocal vectors and its reciprocal-space tables (device array,
// one record per batch entry)
struct CellTab {
    double b[3][3];
    const void *vext;           // half spectrum v_ext(G), field type
    const void *gtab;           // [1/G^2 | G^2 | omega(G)], field type
};

// strided column pass along axis 1 or 0 (c2c), optionally with a fused
// reciprocal-space operation between a forward and an inverse transform
// most densities one column block serves (the autotuner's other choice is 1)
constexpr int COL_GROUP = 8;

struct ColArgs {
    void *data;                 // out; field fb at data + fb * fstride
    const void *src;            // in (may equal data)
    long long fstride;
    long long ncols, inner, outer_stride, elem_stride;
    int inv;                    // direction when the field's op is GO_NONE
    int nbatch;                 // field = blockIdx.y / nbatch
    int op[MAXKB];              // per field op (axis 0 only; zero elsewhere)
    const void *vext;           // half spectrum, field type (GO_HEXT)
    const void *gtab;           // [1/G^2 | G^2 | omega(G)], 3 x Nh values (field type)
    int tile_major;             // block order: 1 tile-major, 0 array-major
    int use_h, use_ext;
    double lambda_vw;
    double kf_wt;               // GO_WT kernel Fermi wavevector
    double precond_q2, precond_h;   // GO_PRECOND
    double *part;
    int pstride;
    const void *tw;             // W_L^n
    Geom g;
    const int *kneed;           // knot spectra: field f is knot knot0 + f; blocks of
    int knot0;                  // knots outside the density's range return at once
    const CellTab *ct;          // reciprocal-space ops of a multi-cell batch: entry b's
                                // b-vectors, v_ext and tables (null: g, vext, gtab)
    int nbb;                    // densities per block: requested (at most
                                // COL_GROUP; 0 or 1 = one), then as launched
    int variant;                // reciprocal-space passes of lengths with variants
                                // (col_variants): bit 0 half the columns per block,
                                // bit 1 the radix order reversed; others ignore it
};

// axis-0 spline kernels: per-knot inverse of omega_i rho^b(G), and the EXACT
// accumulation H += sum_i omega_i F[rho^a L_i]
struct KnotArgs {
    const void *src;            // inv: nbatch arrays; acc: K x nbatch arrays
    void *dst;                  // inv: K x nbatch arrays; acc: nbatch arrays (H)
    long long fstride;
    long long ncols;
    int knot0, K, nbatch;
    int accumulate;             // acc: 0 overwrite H, 1 add into H
    Knots knots;
    const void *tw;
    Geom g;
    NlKern kern;                // kernel family at each knot (tab in field type)
    const int *kneed;           // per-density knot range, or null for every knot
    const CellTab *ct;          // multi-cell batch: entry b's reciprocal vectors (or null)
};

// inverse row pass: axis-2 c2r of up to 4 fields, then a plain store, the
// final combine of the potential, or the spline knot accumulation.
struct RowInvArgs {
    const void *spec;           // field f of batch b at spec + f * spec_fstride + b * Nh
    long long spec_fstride;
    int nfields;
    int mode;
    void *out;                  // EP_STORE: field f of batch b at out + (f * nbatch + b) * N
    const void *in;             // rho or phi (EP_COMBINE / EP_KNOTS)
    int in_is_phi;
    int fld_hext, fld_vw, fld_wt, fld_a;   // field index or -1
    int use_tf, spline, exact;
    int use_xc;                 // LDA exchange-correlation (runtime, any term set)
    double lambda_vw, alpha, floor;
    void *acc1, *acc2;          // spline accumulators sum L_i Phi_i, sum L_i' Phi_i
    int acc_init;               // EP_KNOTS: first knot batch overwrites
    int knot0;
    Knots knots;
    void *v_out, *g_out;        // optional outputs (nbatch x N)
    double *part;
    int pstride;
    int nbatch;
    const void *twM, *twN;
    const void *tw1;            // W_{n1}^n (plane kernels)
    int cf;                     // EP_COMBINE: a fixed term set CF_* below, or 0
    int out_f32;                // EP_STORE of FP64 kernels: out holds FP32 values
    const void *vw_field;       // EP_COMBINE with cf = 0: -lambda nabla^2 phi as a real
                                // field (nbatch x N, field type) computed elsewhere (the
                                // FP64 leg of a mixed grid); fld_vw's spectrum is then unused
    const int *kneed;           // EP_KNOTS: per-density knot range, or null for every
                                // knot (the first batch that meets the range then
                                // initialises the accumulators instead of acc_init)
};

// Term sets of the final combine that have kernels specialised at compile
// time (a set bit = term present); any other set, or a nonlocal term with
// alpha != 5/6, runs the general combine (cf = 0).
enum : int { CB_H = 1, CB_VW = 2, CB_TF = 4, CB_WT = 8, CB_SPL = 16, CB_EXACT = 32, CB_A = 64,
             CB_XC = 128 };   // CB_XC may be added to any of the sets below
constexpr int CF_LOCAL = CB_H | CB_VW | CB_TF;
constexpr int CF_WT = CF_LOCAL | CB_WT;
constexpr int CF_S3S4 = CF_LOCAL | CB_SPL;
constexpr int CF_EXACT = CF_LOCAL | CB_SPL | CB_EXACT | CB_A;

bool length_supported(int L);

// plane kernels (axis-2 and axis-1 fused per (i0, batch) plane) exist for
// the (n1, n2/2) pairs below when the plane fits in LDS; nblocks = n0
template <typename T> bool plane_supported(int n1, int m);
template <typename T> hipError_t launch_plane_fwd(const Geom &g, int nbatch, const RowFwdArgs &a, int &nblocks, hipStream_t s);
template <typename T> hipError_t launch_plane_inv(const Geom &g, const RowInvArgs &a, int &nblocks, hipStream_t s);

// launchers (T = float or double)
template <typename T> hipError_t launch_row_fwd(const Geom &g, int nbatch, const RowFwdArgs &a, int &nblocks, hipStream_t s);
template <typename T> hipError_t launch_col(int L, int nfb, const ColArgs &a, int &nblocks, hipStream_t s);
template <typename T> hipError_t launch_knot_inv(const KnotArgs &a, hipStream_t s);
template <typename T> hipError_t launch_knot_acc(const KnotArgs &a, hipStream_t s);
template <typename T> hipError_t launch_row_inv(const Geom &g, const RowInvArgs &a, int &nblocks, hipStream_t s);
// EP_COMBINE with a fixed term set (a.cf != 0) for the row lengths that have
// it; hipErrorNotSupported for the others (the caller runs the general one)
template <typename T> hipError_t launch_row_combine_fixed(const Geom &g, const RowInvArgs &a, int &nblocks, hipStream_t s);
template <typename T> int row_blocks(const Geom &g);
template <typename T> int col_blocks(int L, long long ncols, int variant = 0);
// the column-pass variants a length offers (bit 0 narrow tile, bit 1 reversed
// radix order; 0 for none), an autotuner choice
template <typename T> int col_variants(int L);

// reciprocal-space tables of a grid: 1/G^2 (0 at G = 0), G^2 and the
// nonlocal kernel C_WT K(|G|/(2 kf)) on the half spectrum, built in FP64
// (kern.tab: the FP64 J table)
template <typename T>
hipError_t launch_gtab(const Geom &g, double kf_wt, const NlKern &kern, void *gtab, hipStream_t s);

// Spline knot range of each density (step s1 on the device): the knots
// whose hat functions can be non-zero at some grid point, kneed[2 b] = first
// and kneed[2 b + 1] = last.  exact_brackets (the S3S4 interpolation, whose
// passes all bracket a point the same way): every grid point's bracket j is
// computed as the interpolation computes it and the range is [min j,
// max j + 1].  Otherwise (EXACT, whose FP64 forward fields bracket through
// another formula): the smallest and largest rho of density b (rho = in or
// in^2 for phi input) bracketed like every grid point and widened by one knot
// on each side.  Knots outside the range add exact zeros, so the spline
// kernels skip them.  part: nbatch x KR_SLOTS x KR_BLOCKS doubles of scratch.
constexpr int KR_BLOCKS = 2048;
constexpr int KR_SLOTS = 4;
template <typename T>
hipError_t launch_knot_range(long long N, int nbatch, const void *in, int in_is_phi,
                             const Knots &kn, int exact_brackets, double *part, int *kneed,
                             hipStream_t s);

// FP64 reductions: sums[b][s] = sum_{i < count.n[s]} part[b][s][i]; the
// counts travel as a kernel argument (the launch sequence of an evaluation
// has no host-to-device copies, so it can be captured in a HIP graph)
struct SlotCounts {
    int n[NSLOT];
};
hipError_t launch_finalize(const double *part, int pstride, const SlotCounts &count, int nbatch,
                           double *sums, hipStream_t s);

// ionic structure factor and v_ext(G), electron-ion forces
template <typename T>
hipError_t launch_vext(const Geom &g, int natoms, const int *spec_off, int nspecies,
                       const double *ph0, const double *ph1, const double *ph2,
                       const double *Z, const double *rc, double volume, void *vext,
                       hipStream_t s);
// atoms sorted by species (spec_off); part: forces_part_doubles(g, natoms)
// doubles of scratch; f_out: 3 natoms doubles
template <typename T>
hipError_t launch_forces(const Geom &g, int natoms, const int *spec_off, int nspecies,
                         const double *ph0, const double *ph1, const double *ph2,
                         const double *Z, const double *rc, const void *rho_g, double *part,
                         double *f_out, hipStream_t s);
long long forces_part_doubles(const Geom &g, int natoms);

// per-axis phase tables exp(-i 2 pi m_d s_d) of every atom (sorted order),
// from fractional coordinates frac[3 a + d] in [0, 1): ph_d[a][i], i < n_d
// (n_2h on axis 2, whose last index is the negative Nyquist frequency)
hipError_t launch_phases(const Geom &g, int natoms, const double *frac, double *ph0, double *ph1,
                         double *ph2, hipStream_t s);

// Ewald sum of point ions q_a in a neutralising background.  Real-space
// images L = sum n_d a_d with |n_d| <= nmax[d] and reciprocal vectors
// G = sum m_d b_d with |m_d| <= gmax[d], G != 0, G^2 <= gcut2 are enumerated
// in the kernels; sf holds one complex S(G) per point of that integer box.
struct EwaldGeom {
    double a;             // splitting parameter
    double rcut2, gcut2;
    int nmax[3], gmax[3];
    double lat[3][3];     // rows a_d
    double b[3][3];       // rows b_d
    double volume;
};
__host__ __device__ inline long long ewald_image_count(const EwaldGeom &e)
{
    return (long long)(2 * e.nmax[0] + 1) * (2 * e.nmax[1] + 1) * (2 * e.nmax[2] + 1);
}
__host__ __device__ inline long long ewald_gbox_count(const EwaldGeom &e)
{
    return (long long)(2 * e.gmax[0] + 1) * (2 * e.gmax[1] + 1) * (2 * e.gmax[2] + 1);
}
// e_atom[a]: atom a's share of the real- and reciprocal-space energy; f (if
// not null): natoms x 3 ion-ion forces.  sf: 2 x ewald_gbox_count doubles.
hipError_t launch_ewald(const EwaldGeom &e, int natoms, const double *pos, const double *q,
                        double *sf, double *e_atom, double *f, hipStream_t s);

// Large cells: tiled structure-factor direct sum writing v_ext(G) and one
// Ewald reciprocal partial per block (sf_tiled_blocks of them; ew_part may be
// null), from species-sorted fractional coordinates; and the real-space Ewald
// sum over a bin list (nc[d] >= 3 bins per direction, each >= rcut wide).
long long sf_tiled_blocks(const Geom &g);
// qbuf: Nh complex FP64 scratch, needed when nspecies > 1
template <typename T>
hipError_t launch_sf_tiled(const Geom &g, const int *spec_off, int nspecies, const double *frac,
                           const double *Z, const double *rc, double volume, double ew_a,
                           double ew_gcut2, void *vext, void *qbuf, double *ew_part,
                           hipStream_t s);
hipError_t launch_ewald_real_cells(const EwaldGeom &e, int natoms, const double *pos,
                                   const double *q, const int *bin_start, const int *bin_of,
                                   const int nc[3], double *e_atom, hipStream_t s);

// Smooth PME structure factor.  Cardinal B-spline of order P: w[j] =
// M_P(t + j) for j = 0 .. P-1, t in [0, 1], from M_2(t) = t, M_2(t + 1) =
// 1 - t and M_k(x) = (x M_{k-1}(x) + (k - x) M_{k-1}(x - 1)) / (k - 1).
template <int P>
__host__ __device__ inline void bspline_fill(double t, double (&w)[P])
{
    w[0] = t;
    w[1] = 1.0 - t;
#pragma unroll
    for (int j = 2; j < P; ++j) w[j] = 0.0;
#pragma unroll
    for (int k = 3; k <= P; ++k) {
        const double r = 1.0 / (k - 1);
#pragma unroll
        for (int j = k - 1; j >= 1; --j) w[j] = ((t + j) * w[j] + (k - t - j) * w[j - 1]) * r;
        w[0] = t * w[0] * r;
    }
}
constexpr int PME_FIX_BITS = 48;   // fractional bits of the fixed-point charge grid
constexpr int PME_MAX_ORDER = 16;
// charge grid q (N unsigned 64-bit fixed-point values, zeroed by the caller)
// += the order-P B-splines of atoms [a_beg, a_beg + natoms) of frac
// (fractional coordinates in [0, 1]); P even, 4 .. 16, at most every n_d
hipError_t launch_pme_spread(const Geom &g, int order, int a_beg, int natoms, const double *frac,
                             unsigned long long *q, hipStream_t s);
// out[i] = q[i] / 2^PME_FIX_BITS as T (out may be q itself when T is double)
template <typename T>
hipError_t launch_pme_to_real(const Geom &g, const unsigned long long *q, void *out, hipStream_t s);
// one species' share of v_ext(G) (and of the Ewald reciprocal sum after the
// last species, one partial per block: pme_finish_blocks of them) from the
// normalised forward transform F of its charge grid; bt: conjugated
// exponential-spline factors b0(0..n0-1), b1(0..n1-1), b2(0..n2/2);
// qbuf: Nh complex FP64, needed unless first and last
int pme_finish_blocks(const Geom &g);
template <typename T>
hipError_t launch_pme_finish(const Geom &g, const void *F, const double2 *bt, double z, double rc,
                             double volume, double ew_a, double ew_gcut2, int first, int last,
                             void *vext, void *qbuf, double *ew_part, hipStream_t s);

// Real-time TD-OFDFT.  Complex vectors are split: n real parts, then n
// imaginary parts.  lattice vectors a_d as rows (9 doubles)
struct TdLattice {
    double a[9];
};
int td_dipole_blocks(const Geom &g);
// rho = wa |a|^2 + wb |b|^2 (b may be null)
template <typename T>
hipError_t launch_td_density(long long n, const void *a, double wa, const void *b, double wb,
                             void *rho, hipStream_t s);
// part[3 * block + c]: per-block sums of r_c rho (td_dipole_blocks blocks)
template <typename T>
hipError_t launch_td_dipole(const Geom &g, const TdLattice &L, const void *rho, double *part,
                            hipStream_t s);
// psi = sqrt(rho) exp(-i k.r)
template <typename T>
hipError_t launch_td_kick(const Geom &g, const TdLattice &L, const double k[3], const void *rho,
                          void *psi, hipStream_t s);
// a diagonal operator c(G) of the complex field on the half spectra of its
// two parts (2 x Nh complex); g2: the grid's G^2 table; q = tau G^2 / 2
enum { TD_KIN = 0,    // c = G^2 / 2
       TD_K = 1,      // c = 1 + i q
       TD_KINV = 2 }; // c = 1 / (1 + i q)
template <typename T>
hipError_t launch_td_spectral(const Geom &g, void *spec, const void *g2, double tau, int mode,
                              hipStream_t s);
// out = z + i tau v u
template <typename T>
hipError_t launch_td_pc_apply(long long n, const void *z, const void *u, const void *v,
                              double tau, void *out, hipStream_t s);
// out = x + i tau (tx + v x)
template <typename T>
hipError_t launch_td_apply(long long n, const void *x, const void *tx, const void *v, double tau,
                           void *out, hipStream_t s);
// z = a x + b y + c w, complex coefficients {re, im}; y, w may be null
template <typename T>
hipError_t launch_td_zlincomb(long long n, void *z, const double a[2], const void *x,
                              const double b[2], const void *y, const double c[2], const void *w,
                              hipStream_t s);

// BiCGSTAB on the device (no host read per dot product).  The solver's
// scalars live in one FP64 array sc[TS_N]; complex numbers are {re, im}.
enum {
    TS_RHO = 0, TS_RHOP = 2, TS_ALPHA = 4, TS_OMEGA = 6,   // complex
    TS_BNORM = 8, TS_RES = 9, TS_DONE = 10, TS_IT = 11, TS_TOL = 12, TS_MAXIT = 13,
    TS_CP = 14,   // p = CP0 r + CP1 p + CP2 v   (3 complex)
    TS_CS = 20,   // s = CS0 r + CS1 v           (2 complex)
    TS_CY = 24,   // y = CY0 y + CY1 p + CY2 s   (3 complex)
    TS_CR = 30,   // r = CR0 s + CR1 t           (2 complex)
    TS_N = 34
};
// the update that follows each pair of dot products
enum { TD_STEP_INIT = 0,   // <b,b>, <r,r>: |b|, the relative residual, done
       TD_STEP_RHO = 1,    // <rh,r>: rho, beta, CP
       TD_STEP_RV = 2,     // <rh,v>: alpha, CS
       TD_STEP_OMEGA = 3,  // <t,s>, <t,t>: omega, CY, CR
       TD_STEP_RR = 4 };   // <r,r>: residual, iteration count, done
int td_dot_blocks(long long n);
// part rows 0, 1 (2, 3): per-block partials of Re, Im <a,b> (<c,d>);
// c, d may be null
template <typename T>
hipError_t launch_td_cdots(long long n, const void *a, const void *b, const void *c,
                           const void *d, double *part, hipStream_t s);
// reduces the partials (td_dot_blocks(n) per row, fixed order) and applies
// step to sc (nothing once sc[TS_DONE] is set)
hipError_t launch_td_scalars(int step, long long n, const double *part, double *sc, hipStream_t s);
// z = c0 x + c1 y + c2 w with the complex coefficients sc[coef ..], skipped
// once sc[TS_DONE] is set; y, w may be null
template <typename T>
hipError_t launch_td_zlincomb_dev(long long n, void *z, const double *sc, int coef, const void *x,
                                  const void *y, const void *w, hipStream_t s);

// vector kernels (optimizer): up to 4 dot products into part slots
template <typename T>
hipError_t launch_dots(long long n, int nd, const void *x0, const void *y0, const void *x1,
                       const void *y1, const void *x2, const void *y2, const void *x3,
                       const void *y3, double *part, int pstride, int &nblocks, hipStream_t s);
// z = a x + b y
template <typename T>
hipError_t launch_lincomb(long long n, void *z, double a, const void *x, double b, const void *y,
                          hipStream_t s);
int dots_blocks(long long n);
// z = sqrt(max(x, 0)) (op 0) or z = x^2 (op 1)
enum { PW_SQRT = 0, PW_SQUARE = 1 };
template <typename T>
hipError_t launch_pointwise(long long n, int op, void *z, const void *x, hipStream_t s);
// destination half spectrum (gd) from a source half spectrum (gs) of a grid
// no finer on any axis: Fourier interpolation (see k_misc.hip)
template <typename T>
hipError_t launch_interp_spec(const Geom &gs, const Geom &gd, const void *src, void *dst,
                              hipStream_t s);

}  // namespace ofdft
