// C ABI of libofdft.so: handles, grid set-up, the evaluation pipeline, forces
// and the density optimiser.  Host code; all field work runs in the HIP
// kernels declared in kernels.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <thread>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ofdft.h"
#include "internal.hpp"
#include "kernels.hpp"

using namespace ofdft;

// ---------------------------------------------------------------- errors
static thread_local std::string g_last_error;

static ofdft_status fail(ofdft_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(e_ == hipErrorOutOfMemory ? OFDFT_ENOMEM : OFDFT_EDEVICE,             \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                   \
    } while (0)

#define ST_TRY(expr)                                                                          \
    do {                                                                                      \
        ofdft_status s_ = (expr);                                                             \
        if (s_ != OFDFT_OK) return s_;                                                        \
    } while (0)

static const double PI = 3.14159265358979323846264338327950288;
static const int NVEC_OPT = 10;   // optimiser vectors per grid
// From this many atoms on, the structure factor is the tiled direct sum
// without per-atom phase tables and the Ewald sum uses bins and the FFT box
// (forces are not offered there: each would cost a full structure factor).
static const int LARGE_IONS = 8192;
static const double C_TF = 2.8712340001881918;

// ---------------------------------------------------------------- handles
struct ofdft_ctx {
    int device;
    hipStream_t stream;
};

enum Pass {
    PS_ROW_FWD = 0,
    PS_COL1_FWD,
    PS_COL0_G,
    PS_COL1_INV,
    PS_ROW_INV,
    PS_KNOT_INV,
    PS_KNOT_COL1,
    PS_KNOT_ROW,
    PS_EXACT_FWD,
    PS_EXACT_ACC,
    PS_FINALIZE,
    PS_OTHER,
    PS_VW64,
    NPASS
};

struct Timer {
    bool on = false;
    std::vector<hipEvent_t> ev;       // pairs
    std::vector<int> kind;
    double ms[NPASS] = {0};
    long long count[NPASS] = {0};
};

// one captured evaluation: its arguments and the executable graph
struct GraphEntry {
    int nb = 0;
    const void *in = nullptr;
    int in_is_phi = 0;
    void *v = nullptr, *gout = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last = 0;
};

struct ofdft_grid {
    ofdft_ctx *ctx = nullptr;
    // copies of the descriptors
    double lattice[3][3];
    int n[3];
    int natoms = 0;
    std::vector<double> pos;
    std::vector<int> species;
    std::vector<int> species_order;   // sorted position -> original atom index
    std::vector<double> Z, rc;
    double nelec = 0;
    ofdft_functional_desc func;
    bool fp64 = true;
    size_t fsz = 8;
    // OFDFT_MIXED_VW64: FP32 fields, with phi's transform pair (the von
    // Weizsaecker term) in FP64 -- tables and workspace of that leg
    bool vw64 = false;
    void *tw0d = nullptr, *tw1d = nullptr, *twMd = nullptr, *twNd = nullptr;
    void *vwspec = nullptr;   // cap * Nh complex FP64
    void *vwout = nullptr;    // cap * N FP32: -lambda nabla^2 phi
    Geom geom;
    double frac[3][3];   // fractional coordinates s_j = sum_i frac[j][i] R_i
    double V = 0, dv = 0;
    Knots knots;
    std::vector<double> knot_host;
    double *d_knots = nullptr;
    double kf_wt = 0;
    double e_ion = 0;
    // nonlocal kernel family: x of eq. "MGP" (0 = Wang-Teter) and the J table
    // (FP64 for the reciprocal-space table, field type for the knot kernels)
    double mgp_x = 0;
    double *d_jtab64 = nullptr;
    void *d_jtab = nullptr;
    // device tables
    void *tw0 = nullptr, *tw1 = nullptr, *twM = nullptr, *twN = nullptr;
    void *vext = nullptr;
    void *gtab = nullptr;    // [1/G^2 | G^2 | omega_WT], 3 x Nh field-type values
    double *ph0 = nullptr, *ph1 = nullptr, *ph2 = nullptr;
    int *d_spec_off = nullptr, *d_atom_species = nullptr;
    double *d_Z = nullptr, *d_rc = nullptr;
    // workspace
    int cap = 0;
    void *spec = nullptr;    // 4 * cap * Nh complex
    void *kspec = nullptr;   // MAXKB * cap * Nh complex (spline)
    void *acc1 = nullptr, *acc2 = nullptr;   // cap * N
    // multi-cell batches led by this grid (ofdft_energy_potential_multi): the
    // per-entry cell records (device and pinned host), the entries' densities
    // and potentials side by side, and the record array of the batch being
    // enqueued (null otherwise)
    CellTab *d_ct = nullptr, *h_ct = nullptr;
    void *batch_in = nullptr, *batch_out = nullptr;
    int batch_cap = 0;
    uint64_t multi_bytes = 0;
    const CellTab *cur_ct = nullptr;
    double *kr_part = nullptr;   // cap * KR_SLOTS * KR_BLOCKS: knot-range partials (spline)
    int *kneed = nullptr;        // cap * 2: each density's knot range (spline)
    bool knot_skip = true;       // spline passes skip knots outside the range
    void *stage_in = nullptr, *stage_out = nullptr;   // cap * N (host API staging)
    double *part = nullptr;
    int pstride = 0;
    double *sums = nullptr;
    double *h_sums = nullptr;   // pinned
    // resident density and optimiser vectors (N each)
    void *rho = nullptr;
    bool rho_set = false;   // the resident density has been written
    void *opt[NVEC_OPT] = {nullptr};
    size_t bytes = 0;
    double *d_forces = nullptr;   // natoms x 3
    double *d_frac = nullptr;     // natoms x 3 fractional coordinates, species-sorted
    double *d_ew_pos = nullptr, *d_ew_q = nullptr, *d_ew_e = nullptr, *d_ew_f = nullptr,
           *d_ew_sf = nullptr;    // Ewald buffers
    Timer timer;
    // tuned launch schedule (see ofdft_grid_tune)
    int tune_col_tile_major = 0;   // block order of the column passes
    int tune_plane = 1;            // fused plane kernels where the plane fits in LDS
    int tune_kb = MAXKB;           // knots per spline batch
    int tune_pipe = 1;             // sub-batches pipelined over two streams
    int tune_col_group = COL_GROUP;   // densities per column block (batches)
    int tune_col_variant = 0;         // reciprocal-space column pass shape (col_variants)
    // second stream of the pipelined evaluation and its events (created on
    // first use)
    hipStream_t s2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr, ev_stagger = nullptr;
    // knot pipeline: a second knot-spectrum buffer (allocated by the rule
    // in knot_pipe_fits) lets a batch's knot transforms run on s2 beside
    // the previous batch's row pass; events fork, ready[2], free[2]
    void *kspec2 = nullptr;
    int tune_knot_pipe = 1;
    hipEvent_t kev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    bool stagger_after_fwd = false;
    const std::atomic<int> *cancel = nullptr;   // checked once per optimiser iteration
    struct EvalBatcher *batcher = nullptr;      // lockstep optimisation: evaluations merged
    hipStream_t opt_stream = nullptr;           // the optimiser's stream (else the context's)
    double precond_q2 = 1.0;                    // optimiser preconditioner q0^2
    bool large_ions = false;                    // tiled structure factor, binned Ewald
    bool use_graphs = false;                    // replay evaluations from HIP graphs
    std::vector<GraphEntry> graphs;
    uint64_t graph_clock = 0;
    int *d_bin_start = nullptr, *d_bin_of = nullptr;
    double *d_ew_part = nullptr;
    int sf_method = OFDFT_SF_DIRECT;            // structure factor of the ionic terms
    int pme_order = 0;                          // B-spline order of the PME spread
    double2 *d_pme_b = nullptr;                 // conjugated exponential-spline factors
    // real-time TD-OFDFT state (ofdft_td_start): one block of split complex
    // vectors, real fields and two half spectra, and the dipole partials
    void *td = nullptr;
    double *d_td_part = nullptr;
    double *d_td_dots = nullptr;   // 4 x td_dot_blocks partials of the solver's dot products
    double *d_td_sc = nullptr;     // the solver's scalars (TS_N)
    double *h_td_sc = nullptr;     // pinned host copy
};

// ---------------------------------------------------------------- helpers
static bool is_supported(int L) { return length_supported(L); }

static ofdft_status dmalloc(ofdft_grid *g, void **p, size_t bytes)
{
    if (*p) return OFDFT_OK;
    hipError_t e = hipMalloc(p, bytes ? bytes : 16);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(OFDFT_ENOMEM, "hipMalloc(" + std::to_string(bytes) + ") failed: " +
                                      hipGetErrorString(e));
    }
    g->bytes += bytes;
    return OFDFT_OK;
}

static void dfree(void *&p)
{
    if (p) (void)hipFree(p);
    p = nullptr;
}

// synchronous upload on the grid's stream (the stream is non-blocking, so no
// implicit ordering with other streams of the process)
static ofdft_status h2d(ofdft_grid *g, void *dst, const void *src, size_t bytes)
{
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, g->ctx->stream));
    HIP_TRY(hipStreamSynchronize(g->ctx->stream));
    return OFDFT_OK;
}

template <typename T>
static std::vector<T> to_type(const double *src, size_t n)
{
    std::vector<T> v(n);
    for (size_t i = 0; i < n; ++i) v[i] = (T)src[i];
    return v;
}

// The MGP J table of exponent y (mgp_table.hpp), built once per process
static const std::vector<double> &mgp_table_cached(double y)
{
    static std::mutex mu;
    static std::map<double, std::vector<double>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(y);
    if (it == cache.end()) it = cache.emplace(y, mgp_build_table(y)).first;
    return it->second;
}

static bool mgp_params(int kernel, double &x, double &y)
{
    switch (kernel) {
    case OFDFT_KERNEL_MGP: x = 1.0; y = 5.0 / 6.0; return true;
    case OFDFT_KERNEL_MGPA: x = 0.5; y = 5.0 / 6.0; return true;
    case OFDFT_KERNEL_MGPG: x = 1.0; y = 5.0 / 3.0; return true;
    default: x = 0.0; y = 0.0; return false;
    }
}

static NlKern nl_kern(const ofdft_grid *g, bool fp64_table)
{
    NlKern k;
    k.x = g->mgp_x;
    k.tab = fp64_table ? (const void *)g->d_jtab64 : g->d_jtab;
    return k;
}

// twiddle table exp(-2 pi i n / L) for n < cnt, built in FP64, stored as
// field type (or as FP64 for the von Weizsaecker leg of a mixed grid)
static ofdft_status upload_twiddles(ofdft_grid *g, void **dst, int L, int cnt, bool as_fp64)
{
    std::vector<double> t(2 * (size_t)cnt);
    for (int i = 0; i < cnt; ++i) {
        const double a = 2.0 * PI * (double)i / (double)L;
        t[2 * i] = std::cos(a);
        t[2 * i + 1] = -std::sin(a);
    }
    ST_TRY(dmalloc(g, dst, (size_t)cnt * 2 * (as_fp64 ? 8 : 4)));
    if (as_fp64) {
        ST_TRY(h2d(g, *dst, t.data(), t.size() * 8));
    } else {
        auto f = to_type<float>(t.data(), t.size());
        ST_TRY(h2d(g, *dst, f.data(), f.size() * 4));
    }
    return OFDFT_OK;
}


// ---------------------------------------------------------------- Ewald (host, FP64)
// E_ion = 1/2 sum' Z_a Z_b erfc(a r)/r + (2 pi / V) sum_{G!=0} e^{-G^2/4a^2}/G^2 |S(G)|^2
//         - a/sqrt(pi) sum Z^2 - pi Q^2 / (2 V a^2),  S(G) = sum Z_a e^{iG.R_a}
// and its forces; point charges in a neutralising background.
// Ewald parameters of a cell: splitting a = 2 sqrt(pi) (n/V^2)^(1/6), real-
// and reciprocal-space cut-offs 6.6/a and 13.2 a, and the integer ranges of
// lattice images and reciprocal vectors that reach them.
static EwaldGeom ewald_geom(const double lat[3][3], const double b[3][3], double V, int na)
{
    EwaldGeom e;
    std::memset(&e, 0, sizeof(e));
    e.a = std::sqrt(PI) * std::pow((double)std::max(na, 1) / (V * V), 1.0 / 6.0) * 2.0;
    const double rcut = 6.6 / e.a, gcut = 2.0 * e.a * 6.6;
    e.rcut2 = rcut * rcut;
    e.gcut2 = gcut * gcut;
    for (int d = 0; d < 3; ++d) {
        // planes of lattice points perpendicular to b_d are 2 pi/|b_d| apart
        const double bn = std::sqrt(b[d][0] * b[d][0] + b[d][1] * b[d][1] + b[d][2] * b[d][2]);
        const double an = std::sqrt(lat[d][0] * lat[d][0] + lat[d][1] * lat[d][1] + lat[d][2] * lat[d][2]);
        e.nmax[d] = (int)std::ceil(rcut * bn / (2 * PI)) + 1;
        e.gmax[d] = (int)std::ceil(gcut * an / (2 * PI)) + 1;
        for (int c = 0; c < 3; ++c) {
            e.lat[d][c] = lat[d][c];
            e.b[d][c] = b[d][c];
        }
    }
    e.volume = V;
    return e;
}

// Ewald parameters for a large cell: the reciprocal sum is taken over the FFT
// box, so its cut-off is the radius of the sphere inscribed in the box,
// min_d pi (n_d - 2) / |a_d|, and a = gcut / 13.2 (or the balanced value if
// that is smaller); bins for the real-space sum are at least 6.6/a wide.
struct LargeEwald {
    EwaldGeom e;
    int nbin[3];
};
static LargeEwald large_ewald(const double lat[3][3], const double b[3][3], double V, int na,
                              const int n[3], bool pme)
{
    LargeEwald L;
    L.e = ewald_geom(lat, b, V, na);
    double gmax = 1e300;
    for (int d = 0; d < 3; ++d) {
        const double an = std::sqrt(lat[d][0] * lat[d][0] + lat[d][1] * lat[d][1] + lat[d][2] * lat[d][2]);
        gmax = std::min(gmax, PI * (n[d] - 2) / an);
    }
    // with PME the reciprocal sum stops at half the box, where the spline
    // interpolation of S(G) is accurate
    const double a = std::min(L.e.a, gmax / (pme ? 26.4 : 13.2));
    const double rcut = 6.6 / a;
    L.e.a = a;
    L.e.rcut2 = rcut * rcut;
    L.e.gcut2 = (13.2 * a) * (13.2 * a);
    for (int d = 0; d < 3; ++d) {
        // width of the cell across the planes spanned by the other two vectors
        const double bn = std::sqrt(b[d][0] * b[d][0] + b[d][1] * b[d][1] + b[d][2] * b[d][2]);
        const double width = 2 * PI / bn;
        L.nbin[d] = std::max(1, (int)std::floor(width / rcut));
        // images for the all-pairs fallback; no reciprocal box there
        L.e.nmax[d] = (int)std::ceil(rcut * bn / (2 * PI)) + 1;
        L.e.gmax[d] = 0;
    }
    return L;
}

static bool use_large_ions(int na, int sf_method)
{
    if (na > 0 && sf_method == OFDFT_SF_PME) return true;
    if (const char *e = std::getenv("OFDFT_LARGE_IONS")) return std::atoi(e) != 0 && na > 0;
    return na >= LARGE_IONS;
}

static int pme_order_of(int order) { return order > 0 ? order : 10; }

// device bytes of the ionic buffers: sorted fractional coordinates, Ewald
// positions, charges, per-atom energies and forces, and S(G) on the box; for
// large cells bins and per-block reciprocal partials instead of S(G) and forces
static uint64_t ion_bytes(const double lat[3][3], int na, int sf_method, const Geom &G)
{
    if (na <= 0) return 0;
    if (use_large_ions(na, sf_method)) {
        const double(*A)[3] = lat;
        const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                           A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
        double b[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
                b[i][j] = 2.0 * PI * (A[i1][j1] * A[i2][j2] - A[i1][j2] * A[i2][j1]) / det;
            }
        const int n[3] = {G.n0, G.n1, G.n2};
        const bool pme = sf_method == OFDFT_SF_PME;
        const LargeEwald L = large_ewald(lat, b, std::fabs(det), na, n, pme);
        const bool binned = L.nbin[0] >= 3 && L.nbin[1] >= 3 && L.nbin[2] >= 3;
        const uint64_t nbins = binned ? (uint64_t)L.nbin[0] * L.nbin[1] * L.nbin[2] : 1;
        const uint64_t recip = pme ? (uint64_t)pme_finish_blocks(G) * 8 +
                                         (uint64_t)(G.n0 + G.n1 + G.n2h) * 16
                                   : (uint64_t)sf_tiled_blocks(G) * 8;
        return (uint64_t)na * (3 + 3 + 1 + 1) * 8 + (uint64_t)na * 4 + (nbins + 1) * 4 + recip +
               (binned ? 0 : 24);
    }
    const double(*A)[3] = lat;
    const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                       A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                       A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    double b[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            b[i][j] = 2.0 * PI * (A[i1][j1] * A[i2][j2] - A[i1][j2] * A[i2][j1]) / det;
        }
    const EwaldGeom e = ewald_geom(lat, b, std::fabs(det), na);
    return (uint64_t)na * (3 + 3 + 1 + 1 + 3) * 8 + (uint64_t)ewald_gbox_count(e) * 24;
}

// E_ion on the device; forces (natoms x 3, original atom order) if asked.
static ofdft_status ewald_device(ofdft_grid *g, double *e_ion, std::vector<double> *forces)
{
    const int na = g->natoms;
    *e_ion = 0.0;
    if (forces) forces->assign(3 * (size_t)na, 0.0);
    if (na == 0) return OFDFT_OK;
    hipStream_t s = g->ctx->stream;
    const EwaldGeom e = ewald_geom(g->lattice, g->geom.b, g->V, na);
    const long long nbox = ewald_gbox_count(e);
    std::vector<double> q(na);
    double Q = 0, Q2 = 0;
    for (int i = 0; i < na; ++i) {
        q[i] = g->Z[g->species[i]];
        Q += q[i];
        Q2 += q[i] * q[i];
    }
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_ew_pos), 3 * (size_t)na * 8));
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_ew_q), (size_t)na * 8));
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_ew_e), (size_t)na * 8));
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_ew_f), 3 * (size_t)na * 8));
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_ew_sf), (size_t)nbox * 24));   // S(G), w(G)
    HIP_TRY(hipMemcpyAsync(g->d_ew_pos, g->pos.data(), 3 * (size_t)na * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(g->d_ew_q, q.data(), (size_t)na * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_ewald(e, na, g->d_ew_pos, g->d_ew_q, g->d_ew_sf, g->d_ew_e,
                         forces ? g->d_ew_f : nullptr, s));
    std::vector<double> ea(na);
    HIP_TRY(hipMemcpyAsync(ea.data(), g->d_ew_e, (size_t)na * 8, hipMemcpyDeviceToHost, s));
    if (forces)
        HIP_TRY(hipMemcpyAsync(forces->data(), g->d_ew_f, 3 * (size_t)na * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double sum = 0.0;
    for (int i = 0; i < na; ++i) sum += ea[i];
    *e_ion = sum - e.a / std::sqrt(PI) * Q2 - PI * Q * Q / (2 * g->V * e.a * e.a);
    return OFDFT_OK;
}

// ---------------------------------------------------------------- timing
static void timer_start(ofdft_grid *g, hipStream_t s, int kind, hipEvent_t &e0)
{
    if (!g->timer.on) return;
    (void)kind;
    (void)hipEventCreate(&e0);
    (void)hipEventRecord(e0, s);
}

static void timer_stop(ofdft_grid *g, hipStream_t s, int kind, hipEvent_t e0)
{
    if (!g->timer.on) return;
    hipEvent_t e1;
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e1, s);
    g->timer.ev.push_back(e0);
    g->timer.ev.push_back(e1);
    g->timer.kind.push_back(kind);
}

static void timer_collect(ofdft_grid *g)
{
    Timer &t = g->timer;
    for (size_t i = 0; i < t.kind.size(); ++i) {
        float ms = 0.f;
        (void)hipEventSynchronize(t.ev[2 * i + 1]);
        if (hipEventElapsedTime(&ms, t.ev[2 * i], t.ev[2 * i + 1]) == hipSuccess) {
            t.ms[t.kind[i]] += ms;
            t.count[t.kind[i]] += 1;
        }
        (void)hipEventDestroy(t.ev[2 * i]);
        (void)hipEventDestroy(t.ev[2 * i + 1]);
    }
    t.ev.clear();
    t.kind.clear();
}

#define TIMED(kind, stmt)                                                                     \
    do {                                                                                      \
        hipEvent_t e0_ = nullptr;                                                             \
        timer_start(g, s, kind, e0_);                                                         \
        hipError_t r_ = (stmt);                                                               \
        timer_stop(g, s, kind, e0_);                                                          \
        if (r_ != hipSuccess)                                                                 \
            return fail(OFDFT_EDEVICE, std::string(#stmt) + ": " + hipGetErrorString(r_));    \
    } while (0)

// ---------------------------------------------------------------- workspace
template <typename T>
static bool use_plane(const ofdft_grid *g)
{
    // (the FP64 spline interpolation epilogue spills registers on planes
    // above 72 x 36: those grids keep the row passes)
    if (sizeof(T) == 8 && (g->func.terms & OFDFT_TERM_SPLINE) && g->geom.n1 * g->geom.m > 72 * 36)
        return false;
    return g->tune_plane && plane_supported<T>(g->geom.n1, g->geom.m);
}

static int max_pstride(const Geom &G, bool fp64)
{
    int rb, c0, c1;
    if (fp64) {
        rb = row_blocks<double>(G);
        c0 = col_blocks<double>(G.n0, (long long)G.n1 * G.n2h);
        c1 = col_blocks<double>(G.n1, (long long)G.n0 * G.n2h);
    } else {
        // the narrow-tile variant of the axis-0 pass (where offered) has the most blocks
        rb = row_blocks<float>(G);
        c0 = std::max(col_blocks<float>(G.n0, (long long)G.n1 * G.n2h),
                      col_blocks<float>(G.n0, (long long)G.n1 * G.n2h, 1));
        c1 = col_blocks<float>(G.n1, (long long)G.n0 * G.n2h);
    }
    return std::max({rb, c0, c1, dots_blocks(G.N), G.n0, 1});
}

// Device bytes of a grid as allocated by this file: fixed tables, workspace
// for `cap` densities, and optionally the host-API staging fields, the
// optimiser vectors and the forces buffer.  Used both to report what a grid
// holds and to size a request before any allocation.
struct BytesModel {
    bool stage = false, opt = false, forces = false;
    bool vw64 = false;   // FP32 grid with the FP64 von Weizsaecker leg
    bool mgp = false;    // MGP-family kernel table
    uint64_t extra = 0;  // buffers of multi-cell batches led by the grid
};
// partial-sum rows: the block counts of the grid's own kernels, and of the
// FP64 passes of a mixed grid's von Weizsaecker leg
static int pstride_of(const Geom &G, bool fp64, bool vw64)
{
    return vw64 ? std::max(max_pstride(G, false), max_pstride(G, true)) : max_pstride(G, fp64);
}
// the knot pipeline's second buffer: spline grids with more than one knot
// batch whose knot spectra take at most 4 GiB (a 256 x 256 x 384 grid: 0.8 GB
// in FP32; the 1024^3 grid's 34 GB are not doubled)
constexpr uint64_t KNOT_PIPE_MAX_BYTES = 4ull << 30;
static bool knot_pipe_fits(int nk, uint64_t kspec_bytes)
{
    return nk > MAXKB && kspec_bytes <= KNOT_PIPE_MAX_BYTES;
}

static uint64_t bytes_model(const Geom &G, size_t fsz, int natoms, int nspecies, int sf_method,
                            uint32_t terms, int nl_mode, int nk, uint64_t cap, uint64_t ions,
                            BytesModel m)
{
    const uint64_t N = (uint64_t)G.N, Nh = (uint64_t)G.Nh, cb = 2 * fsz;
    uint64_t b = 0;
    b += (uint64_t)(G.n0 + G.n1 + G.m + (G.m + 1)) * cb;             // twiddles
    b += Nh * cb;                                                       // v_ext
    b += Nh * 3 * fsz;                                                  // G tables
    if (!use_large_ions(natoms, sf_method))
        b += (uint64_t)natoms * (G.n0 + G.n1 + G.n2h) * 16;             // phase tables
    b += ions;                                                          // coordinates, Ewald
    b += (uint64_t)natoms * 4 + (uint64_t)(nspecies + 1) * 4 + 2 * (uint64_t)nspecies * 8;
    b += (uint64_t)nk * 8;                                              // knots
    if (m.mgp) b += (uint64_t)MGP_TAB * (fsz == 8 ? 8 : 12);           // J tables
    b += N * fsz;                                                       // resident rho
    b += 4 * cap * Nh * cb;                                             // spectra
    if (terms & OFDFT_TERM_SPLINE) {
        b += (uint64_t)MAXKB * cap * Nh * cb;                           // knot spectra
        if (knot_pipe_fits(nk, (uint64_t)MAXKB * cap * Nh * cb))
            b += (uint64_t)MAXKB * cap * Nh * cb;                       // second knot buffer
        b += cap * N * fsz;                                             // accumulator
        if (nl_mode == OFDFT_NL_EXACT) b += cap * N * fsz;
        b += cap * (KR_SLOTS * (uint64_t)KR_BLOCKS * 8 + 2 * 4);        // knot range
    }
    b += cap * NSLOT * (uint64_t)pstride_of(G, fsz == 8, m.vw64) * 8 + cap * NSLOT * 8;   // partials
    if (m.vw64) {
        b += (uint64_t)(G.n0 + G.n1 + G.m + (G.m + 1)) * 16;         // FP64 twiddles
        b += cap * Nh * 16 + cap * N * 4;                              // FP64 spectrum, result
    }
    if (m.stage) b += 2 * N * fsz;
    if (m.opt) b += (uint64_t)NVEC_OPT * N * fsz;
    if (m.forces) b += ((uint64_t)natoms * 3 + (uint64_t)forces_part_doubles(G, natoms)) * 8;
    b += m.extra;
    return b;
}

// captured evaluations refer to the workspace: dropped when it is reallocated
static void graphs_clear(ofdft_grid *g)
{
    for (auto &e : g->graphs) (void)hipGraphExecDestroy(e.exec);
    g->graphs.clear();
}

// device bytes of the per-density workspace that reserve(g, nb) allocates
static uint64_t workspace_bytes(const ofdft_grid *g, int nb)
{
    const Geom &G = g->geom;
    const uint64_t cbytes = 2 * g->fsz;
    const bool spline = g->func.terms & OFDFT_TERM_SPLINE;
    uint64_t b = 4ull * nb * G.Nh * cbytes;
    if (spline) {
        b += (uint64_t)MAXKB * nb * G.Nh * cbytes + (uint64_t)nb * G.N * g->fsz;
        if (knot_pipe_fits(g->knots.nk, (uint64_t)MAXKB * nb * G.Nh * cbytes))
            b += (uint64_t)MAXKB * nb * G.Nh * cbytes;
        if (g->func.nl_mode == OFDFT_NL_EXACT) b += (uint64_t)nb * G.N * g->fsz;
        b += (uint64_t)nb * KR_SLOTS * KR_BLOCKS * sizeof(double) + (uint64_t)nb * 2 * sizeof(int);
    }
    if (g->vw64) b += (uint64_t)nb * G.Nh * 16 + (uint64_t)nb * G.N * 4;
    b += (uint64_t)nb * NSLOT * pstride_of(G, g->fp64, g->vw64) * sizeof(double);
    b += (uint64_t)nb * NSLOT * sizeof(double);
    return b;
}

static ofdft_status reserve(ofdft_grid *g, int nb)
{
    if (nb <= g->cap) return OFDFT_OK;
    graphs_clear(g);
    // drop the old workspace
    dfree(g->spec);
    dfree(g->kspec);
    dfree(g->kspec2);
    dfree(g->acc1);
    dfree(g->acc2);
    dfree(g->stage_in);
    dfree(g->stage_out);
    dfree(g->vwspec);
    dfree(g->vwout);
    dfree(reinterpret_cast<void *&>(g->kr_part));
    dfree(reinterpret_cast<void *&>(g->kneed));
    dfree(reinterpret_cast<void *&>(g->part));
    dfree(reinterpret_cast<void *&>(g->sums));
    if (g->h_sums) (void)hipHostFree(g->h_sums);
    g->h_sums = nullptr;
    g->bytes = 0;   // recounted below together with the fixed tables
    const Geom &G = g->geom;
    const size_t cbytes = 2 * g->fsz;
    const bool spline = g->func.terms & OFDFT_TERM_SPLINE;
    ST_TRY(dmalloc(g, &g->spec, 4 * (size_t)nb * G.Nh * cbytes));
    if (spline) {
        ST_TRY(dmalloc(g, &g->kspec, (size_t)MAXKB * nb * G.Nh * cbytes));
        if (knot_pipe_fits(g->knots.nk, (uint64_t)MAXKB * nb * G.Nh * cbytes))
            ST_TRY(dmalloc(g, &g->kspec2, (size_t)MAXKB * nb * G.Nh * cbytes));
        ST_TRY(dmalloc(g, &g->acc1, (size_t)nb * G.N * g->fsz));
        if (g->func.nl_mode == OFDFT_NL_EXACT)
            ST_TRY(dmalloc(g, &g->acc2, (size_t)nb * G.N * g->fsz));
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->kr_part),
                       (size_t)nb * KR_SLOTS * KR_BLOCKS * sizeof(double)));
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->kneed), (size_t)nb * 2 * sizeof(int)));
    }
    if (g->vw64) {
        ST_TRY(dmalloc(g, &g->vwspec, (size_t)nb * G.Nh * 16));
        ST_TRY(dmalloc(g, &g->vwout, (size_t)nb * G.N * 4));
    }
    g->pstride = pstride_of(G, g->fp64, g->vw64);
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->part),
                   (size_t)nb * NSLOT * g->pstride * sizeof(double)));
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->sums), (size_t)nb * NSLOT * sizeof(double)));
    HIP_TRY(hipHostMalloc((void **)&g->h_sums, (size_t)nb * NSLOT * sizeof(double)));
    g->cap = nb;
    return OFDFT_OK;
}

// ---------------------------------------------------------------- evaluation
struct Layout {
    int s_rho = -1, s_phi = -1, s_rhob = -1, s_h = -1;
    int nfwd = 0, ninv = 0;
};

static Layout layout_of(const ofdft_grid *g)
{
    Layout l;
    const uint32_t t = g->func.terms;
    int idx = 0;
    if (t & (OFDFT_TERM_HARTREE | OFDFT_TERM_EXT)) l.s_rho = idx++;
    if ((t & OFDFT_TERM_VW) && !g->vw64) l.s_phi = idx++;   // else in the FP64 leg
    if (t & (OFDFT_TERM_WT | OFDFT_TERM_SPLINE)) l.s_rhob = idx++;
    l.nfwd = idx;
    l.ninv = (t & OFDFT_TERM_SPLINE) ? idx - 1 : idx;
    if ((t & OFDFT_TERM_SPLINE) && g->func.nl_mode == OFDFT_NL_EXACT) l.s_h = idx++;
    return l;
}

template <typename T>
static ofdft_status col_pass(ofdft_grid *g, hipStream_t s, int axis, void *data, int nfb, int nbatch,
                             int inv, const int *ops, int kind, double *part = nullptr,
                             const void *tw = nullptr, const int *kneed = nullptr, int knot0 = 0,
                             int *nblocks = nullptr)
{
    const Geom &G = g->geom;
    ColArgs a;
    std::memset(&a, 0, sizeof(a));
    a.data = data;
    a.src = data;
    a.fstride = G.Nh;
    a.nbatch = nbatch;
    a.inv = inv;
    a.g = G;
    a.part = part ? part : g->part;
    a.pstride = g->pstride;
    a.vext = g->vext;
    a.gtab = g->gtab;
    a.tile_major = g->tune_col_tile_major;
    a.nbb = g->tune_col_group;
    a.variant = g->tune_col_variant;
    a.use_h = (g->func.terms & OFDFT_TERM_HARTREE) ? 1 : 0;
    a.use_ext = (g->func.terms & OFDFT_TERM_EXT) ? 1 : 0;
    a.lambda_vw = g->func.lambda_vw;
    a.kf_wt = g->kf_wt;
    a.precond_q2 = g->precond_q2;
    a.precond_h = 16.0 * PI * g->nelec / g->V;
    a.kneed = kneed;
    a.knot0 = knot0;
    a.ct = (axis == 0 && ops) ? g->cur_ct : nullptr;
    int L;
    if (axis == 1) {
        L = G.n1;
        a.ncols = (long long)G.n0 * G.n2h;
        a.inner = G.n2h;
        a.outer_stride = (long long)G.n1 * G.n2h;
        a.elem_stride = G.n2h;
        a.tw = tw ? tw : g->tw1;
    } else {
        L = G.n0;
        a.ncols = (long long)G.n1 * G.n2h;
        a.inner = a.ncols;
        a.outer_stride = 0;
        a.elem_stride = (long long)G.n1 * G.n2h;
        a.tw = tw ? tw : g->tw0;
        if (ops)
            for (int f = 0; f < 4; ++f) a.op[f] = ops[f];   // ops has 4 entries
    }
    int nbk = 0;
    TIMED(kind, launch_col<T>(L, nfb, a, nbk, s));
    if (nblocks) *nblocks = nbk;
    return OFDFT_OK;
}

// The fixed term set of the final combine matching these arguments, or 0
// (general combine).  The nonlocal sets assume alpha = 5/6.
static int combine_flavour(const RowInvArgs &rc)
{
    int f = 0;
    if (rc.fld_hext >= 0) f |= CB_H;
    if (rc.fld_vw >= 0) f |= CB_VW;
    if (rc.use_tf) f |= CB_TF;
    if (rc.fld_wt >= 0) f |= CB_WT;
    if (rc.spline) f |= CB_SPL;
    if (rc.exact) f |= CB_EXACT;
    if (rc.fld_a >= 0) f |= CB_A;
    if (f != CF_LOCAL && f != CF_WT && f != CF_S3S4 && f != CF_EXACT) return 0;
    if (f != CF_LOCAL && rc.alpha != 5.0 / 6.0) return 0;
    return rc.use_xc ? (f | CB_XC) : f;
}

static ofdft_status ensure_lane(ofdft_grid *g)
{
    if (g->s2) return OFDFT_OK;
    HIP_TRY(hipStreamCreateWithFlags(&g->s2, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&g->ev_stagger, hipEventDisableTiming));
    for (hipEvent_t &e : g->kev) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return OFDFT_OK;
}

// The workspace of densities b0 .. b0 + nb - 1 of a batch: every per-density
// buffer offset to density b0 (the spectra slots of the sub-batch are laid
// out as for a batch of nb, inside its own share of the workspace).
struct Work {
    char *spec, *kspec, *kspec2;
    void *acc1, *acc2;
    char *vwspec;     // FP64 von Weizsaecker leg: spectrum and result
    void *vwout;
    double *kr_part;  // spline knot range: partials and the per-density range
    int *kneed;
    double *part, *sums, *h_sums;
};

template <typename T>
static Work work_of(const ofdft_grid *g, int b0)
{
    const Geom &G = g->geom;
    const size_t cb = 2 * sizeof(T);
    Work w;
    w.spec = (char *)g->spec + (size_t)4 * b0 * G.Nh * cb;
    w.kspec = g->kspec ? (char *)g->kspec + (size_t)MAXKB * b0 * G.Nh * cb : nullptr;
    w.kspec2 = g->kspec2 ? (char *)g->kspec2 + (size_t)MAXKB * b0 * G.Nh * cb : nullptr;
    w.acc1 = g->acc1 ? (char *)g->acc1 + (size_t)b0 * G.N * sizeof(T) : nullptr;
    w.acc2 = g->acc2 ? (char *)g->acc2 + (size_t)b0 * G.N * sizeof(T) : nullptr;
    w.vwspec = g->vwspec ? (char *)g->vwspec + (size_t)b0 * G.Nh * 16 : nullptr;
    w.vwout = g->vwout ? (char *)g->vwout + (size_t)b0 * G.N * 4 : nullptr;
    w.kr_part = g->kr_part ? g->kr_part + (size_t)b0 * KR_SLOTS * KR_BLOCKS : nullptr;
    w.kneed = g->kneed ? g->kneed + (size_t)b0 * 2 : nullptr;
    w.part = g->part + (size_t)b0 * NSLOT * g->pstride;
    w.sums = g->sums + (size_t)b0 * NSLOT;
    w.h_sums = g->h_sums + (size_t)b0 * NSLOT;
    return w;
}

// The von Weizsaecker term of a mixed grid in FP64 (OFDFT_MIXED_VW64): phi
// from the FP32 input (or sqrt of the FP32 rho) through the FP64 row and
// column passes, lambda G^2 phi(G) with the FP64 energy partial SL_VW on
// axis 0, the inverse passes, and w = -lambda nabla^2 phi stored as FP32 for
// the combine, which divides it by phi.  The transforms' rounding then stays
// about 1e-16 of max |phi| instead of 1e-7, so v_vW = w / (2 phi) keeps its
// accuracy where phi is small (vacuum).  Returns the axis-0 block count
// (the number of SL_VW partials).
static ofdft_status vw_leg(ofdft_grid *g, int nb, const void *d_in, int in_is_phi, hipStream_t s,
                           const Work &w, int &nb_vw)
{
    const Geom &G = g->geom;
    RowFwdArgs rf;
    std::memset(&rf, 0, sizeof(rf));
    rf.in = d_in;
    rf.in_f32 = 1;
    rf.out = w.vwspec;
    rf.out_fstride = (long long)nb * G.Nh;
    rf.nfields = 1;
    rf.kind[0] = FK_PHI;
    rf.in_is_phi = in_is_phi;
    rf.partials = 0;
    rf.part = w.part;
    rf.pstride = g->pstride;
    rf.twM = g->twMd;
    rf.twN = g->twNd;
    rf.tw1 = g->tw1d;
    int nbr = 0;
    TIMED(PS_VW64, launch_row_fwd<double>(G, nb, rf, nbr, s));
    ST_TRY(col_pass<double>(g, s, 1, w.vwspec, nb, nb, 0, nullptr, PS_VW64, w.part, g->tw1d));
    const int ops[4] = {GO_VW, 0, 0, 0};
    ST_TRY(col_pass<double>(g, s, 0, w.vwspec, nb, nb, 0, ops, PS_VW64, w.part, g->tw0d, nullptr,
                            0, &nb_vw));
    ST_TRY(col_pass<double>(g, s, 1, w.vwspec, nb, nb, 1, nullptr, PS_VW64, w.part, g->tw1d));
    RowInvArgs ri;
    std::memset(&ri, 0, sizeof(ri));
    ri.spec = w.vwspec;
    ri.spec_fstride = (long long)nb * G.Nh;
    ri.nfields = 1;
    ri.mode = EP_STORE;
    ri.out = w.vwout;
    ri.out_f32 = 1;
    ri.nbatch = nb;
    ri.twM = g->twMd;
    ri.twN = g->twNd;
    ri.tw1 = g->tw1d;
    ri.fld_hext = ri.fld_vw = ri.fld_wt = ri.fld_a = -1;
    int nbi = 0;
    TIMED(PS_VW64, launch_row_inv<double>(G, ri, nbi, s));
    return OFDFT_OK;
}

template <typename T>
// Enqueues every launch of one evaluation of nb densities on s and the copy
// of their FP64 sums to the pinned host array; no allocation,
// synchronisation or host-to-device copy, so that the sequence can be
// captured in a HIP graph.  d_in, d_v, d_g and w point at the first density.
static ofdft_status eval_enqueue(ofdft_grid *g, int nb, const void *d_in, int in_is_phi, void *d_v,
                                 void *d_g, hipStream_t s, const Work &w, bool knot_lane = true)
{
    const Geom &G = g->geom;
    const Layout l = layout_of(g);
    const uint32_t terms = g->func.terms;
    const bool spline = terms & OFDFT_TERM_SPLINE;
    const bool exact = spline && g->func.nl_mode == OFDFT_NL_EXACT;
    const long long fs = (long long)nb * G.Nh;   // stride between field slots
    char *spec = w.spec;
    const size_t cb = 2 * sizeof(T);
    auto slot_ptr = [&](int sl) { return (void *)(spec + (size_t)sl * fs * cb); };

    // 1. prologue + axis-2 r2c of rho, phi, rho^beta
    RowFwdArgs rf;
    std::memset(&rf, 0, sizeof(rf));
    rf.in = d_in;
    rf.out = spec;
    rf.out_fstride = fs;
    rf.nfields = l.nfwd;
    if (l.s_rho >= 0) rf.kind[l.s_rho] = FK_RHO;
    if (l.s_phi >= 0) rf.kind[l.s_phi] = FK_PHI;
    if (l.s_rhob >= 0) rf.kind[l.s_rhob] = FK_RHOB;
    rf.in_is_phi = in_is_phi;
    rf.beta = g->func.beta;
    rf.alpha = g->func.alpha;
    rf.knots = g->knots;
    rf.partials = 1;
    rf.part = w.part;
    rf.pstride = g->pstride;
    rf.twM = g->twM;
    rf.twN = g->twN;
    rf.tw1 = g->tw1;
    // grids whose (i1, k2) plane fits in LDS fuse passes 1+2 and 4+5
    const bool plane = use_plane<T>(g);
    int nb_row = 0;
    if (plane) TIMED(PS_ROW_FWD, launch_plane_fwd<T>(G, nb, rf, nb_row, s));
    else TIMED(PS_ROW_FWD, launch_row_fwd<T>(G, nb, rf, nb_row, s));
    int nb_vw = 0;
    if (g->vw64) ST_TRY(vw_leg(g, nb, d_in, in_is_phi, s, w, nb_vw));
    if (g->stagger_after_fwd) HIP_TRY(hipEventRecord(g->ev_stagger, s));

    int nb_col0 = 0;
    if (l.nfwd > 0) {
        // 2. axis 1 forward
        if (!plane)
            ST_TRY(col_pass<T>(g, s, 1, spec, l.nfwd * nb, nb, 0, nullptr, PS_COL1_FWD, w.part));
        // 3. axis 0: forward, reciprocal-space term, inverse
        int ops[4] = {0, 0, 0, 0};
        if (l.s_rho >= 0) ops[l.s_rho] = GO_HEXT;
        if (l.s_phi >= 0) ops[l.s_phi] = GO_VW;
        if (l.s_rhob >= 0) ops[l.s_rhob] = spline ? GO_SCALE : GO_WT;
        ST_TRY(col_pass<T>(g, s, 0, spec, l.nfwd * nb, nb, 0, ops, PS_COL0_G, w.part, nullptr,
                           nullptr, 0, &nb_col0));
    }

    // spline loop over knot batches (steps s2-s4)
    if (spline) {
        const int nk = g->knots.nk;
        const int kb = std::max(1, std::min(MAXKB, g->tune_kb));
        // step s1 on the device: each density's range of knots with a
        // non-zero hat somewhere; the knot passes skip the others
        const int *kneed = nullptr;
        if (g->knot_skip && nk > 1) {
            TIMED(PS_KNOT_INV, launch_knot_range<T>(G.N, nb, d_in, in_is_phi, g->knots, !exact,
                                                    w.kr_part,
                                                    w.kneed, s));
            kneed = w.kneed;
        }
        // knot pipeline: batch i's knot transforms (inverse of omega_i
        // rho^beta along axis 0 and axis 1) go to the second stream into
        // buffer i % 2, the row pass (and the EXACT passes) of batch i stay
        // on s and accumulate in order; s waits for the batch's transforms,
        // the second stream for the row pass that last read its buffer
        const bool kpipe = knot_lane && w.kspec2 && g->tune_knot_pipe && !g->timer.on && nk > kb;
        if (kpipe) {
            ST_TRY(ensure_lane(g));
            HIP_TRY(hipEventRecord(g->kev[0], s));
            HIP_TRY(hipStreamWaitEvent(g->s2, g->kev[0], 0));
        }
        for (int k0 = 0, bi = 0; k0 < nk; k0 += kb, ++bi) {
            const int K = std::min(kb, nk - k0);
            char *ks = (kpipe && (bi & 1)) ? w.kspec2 : w.kspec;
            hipStream_t sf = kpipe ? g->s2 : s;
            if (kpipe && bi >= 2) HIP_TRY(hipStreamWaitEvent(sf, g->kev[3 + (bi & 1)], 0));
            KnotArgs ka;
            std::memset(&ka, 0, sizeof(ka));
            ka.src = slot_ptr(l.s_rhob);
            ka.dst = ks;
            ka.fstride = G.Nh;
            ka.ncols = (long long)G.n1 * G.n2h;
            ka.knot0 = k0;
            ka.K = K;
            ka.nbatch = nb;
            ka.knots = g->knots;
            ka.kern = nl_kern(g, false);
            ka.kneed = kneed;
            ka.ct = g->cur_ct;
            ka.tw = g->tw0;
            ka.g = G;
            TIMED(PS_KNOT_INV, launch_knot_inv<T>(ka, sf));
            if (!plane)
                ST_TRY(col_pass<T>(g, sf, 1, ks, K * nb, nb, 1, nullptr, PS_KNOT_COL1, w.part,
                                   nullptr, kneed, k0));
            if (kpipe) {
                HIP_TRY(hipEventRecord(g->kev[1 + (bi & 1)], sf));
                HIP_TRY(hipStreamWaitEvent(s, g->kev[1 + (bi & 1)], 0));
            }
            RowInvArgs ri;
            std::memset(&ri, 0, sizeof(ri));
            ri.spec = ks;
            ri.spec_fstride = fs;
            ri.nfields = K;
            ri.mode = EP_KNOTS;
            ri.in = d_in;
            ri.in_is_phi = in_is_phi;
            ri.exact = exact;
            ri.spline = 1;
            ri.acc1 = w.acc1;
            ri.acc2 = w.acc2;
            ri.acc_init = (k0 == 0);
            ri.kneed = kneed;
            ri.knot0 = k0;
            ri.knots = g->knots;
            ri.nbatch = nb;
            ri.twM = g->twM;
            ri.twN = g->twN;
            ri.tw1 = g->tw1;
            ri.fld_hext = ri.fld_vw = ri.fld_wt = ri.fld_a = -1;
            int nbk = 0;
            if (plane) TIMED(PS_KNOT_ROW, launch_plane_inv<T>(G, ri, nbk, s));
            else TIMED(PS_KNOT_ROW, launch_row_inv<T>(G, ri, nbk, s));
            if (exact) {
                // f_i = rho^a L_i(k~): r2c, axis 1, then axis 0 with omega_i, summed into H
                RowFwdArgs ef = rf;
                ef.out = ks;
                ef.out_fstride = fs;
                ef.nfields = K;
                for (int f = 0; f < K; ++f) ef.kind[f] = FK_KNOT;
                ef.knot0 = k0;
                ef.partials = 0;
                int nbe = 0;
                if (plane) {
                    // (the plane kernel writes every knot's field; those outside
                    // the range are exact zeros, which knot_acc then skips)
                    TIMED(PS_EXACT_FWD, launch_plane_fwd<T>(G, nb, ef, nbe, s));
                } else {
                    ef.kneed = kneed;
                    TIMED(PS_EXACT_FWD, launch_row_fwd<T>(G, nb, ef, nbe, s));
                    ST_TRY(col_pass<T>(g, s, 1, ks, K * nb, nb, 0, nullptr, PS_EXACT_FWD, w.part,
                                       nullptr, kneed, k0));
                }
                KnotArgs kc = ka;
                kc.src = ks;
                kc.dst = slot_ptr(l.s_h);
                kc.accumulate = (k0 > 0);
                TIMED(PS_EXACT_ACC, launch_knot_acc<T>(kc, s));
            }
            if (kpipe) HIP_TRY(hipEventRecord(g->kev[3 + (bi & 1)], s));
        }
        if (exact) {
            ST_TRY(col_pass<T>(g, s, 0, slot_ptr(l.s_h), nb, nb, 1, nullptr, PS_EXACT_ACC, w.part));
            if (!plane)
                ST_TRY(col_pass<T>(g, s, 1, slot_ptr(l.s_h), nb, nb, 1, nullptr, PS_EXACT_ACC, w.part));
        }
    }

    // 4. axis 1 inverse of the fields that return to real space
    if (l.ninv > 0 && !plane)
        ST_TRY(col_pass<T>(g, s, 1, spec, l.ninv * nb, nb, 1, nullptr, PS_COL1_INV, w.part));

    // 5. axis-2 c2r and the final combine
    RowInvArgs rc;
    std::memset(&rc, 0, sizeof(rc));
    rc.spec = spec;
    rc.spec_fstride = fs;
    rc.mode = EP_COMBINE;
    rc.in = d_in;
    rc.in_is_phi = in_is_phi;
    rc.fld_hext = l.s_rho;
    rc.fld_vw = l.s_phi;
    if (g->vw64) {
        rc.fld_vw = 0;   // present; its values come from the FP64 leg
        rc.vw_field = w.vwout;
    }
    rc.fld_wt = (terms & OFDFT_TERM_WT) ? l.s_rhob : -1;
    rc.fld_a = l.s_h;
    rc.use_tf = (terms & OFDFT_TERM_TF) ? 1 : 0;
    rc.use_xc = (terms & OFDFT_TERM_XC) ? 1 : 0;
    rc.spline = spline;
    rc.exact = exact;
    rc.lambda_vw = g->func.lambda_vw;
    rc.alpha = g->func.alpha;
    rc.floor = g->func.rho_floor;
    rc.acc1 = w.acc1;
    rc.acc2 = w.acc2;
    rc.knots = g->knots;
    rc.v_out = d_v;
    rc.g_out = d_g;
    rc.part = w.part;
    rc.pstride = g->pstride;
    rc.nbatch = nb;
    rc.twM = g->twM;
    rc.twN = g->twN;
    rc.tw1 = g->tw1;
    // the fixed term sets have no real-space vW input: the FP64 leg's result
    // goes through the general combine
    rc.cf = g->vw64 ? 0 : combine_flavour(rc);
    int nb_inv = 0;
    if (plane) TIMED(PS_ROW_INV, launch_plane_inv<T>(G, rc, nb_inv, s));
    else TIMED(PS_ROW_INV, launch_row_inv<T>(G, rc, nb_inv, s));

    // 6. fixed-order FP64 sums
    SlotCounts cnt;
    std::memset(&cnt, 0, sizeof(cnt));
    cnt.n[SL_RHO] = cnt.n[SL_TF] = cnt.n[SL_BAD] = nb_row;
    cnt.n[SL_H] = cnt.n[SL_EXT] = (l.s_rho >= 0) ? nb_col0 : 0;
    cnt.n[SL_VW] = g->vw64 ? nb_vw : ((l.s_phi >= 0) ? nb_col0 : 0);
    cnt.n[SL_NL] = cnt.n[SL_GPHI] = cnt.n[SL_GG] = cnt.n[SL_PHIPHI] = nb_inv;
    cnt.n[SL_XC] = (terms & OFDFT_TERM_XC) ? nb_inv : 0;   // written by the LDA combines only
    TIMED(PS_FINALIZE, launch_finalize(w.part, g->pstride, cnt, nb, w.sums, s));
    HIP_TRY(hipMemcpyAsync(w.h_sums, w.sums, (size_t)nb * NSLOT * sizeof(double),
                           hipMemcpyDeviceToHost, s));
    return OFDFT_OK;
}

// Enqueues an evaluation of nb densities as tune_pipe sub-batches that
// alternate between s and the grid's second stream s2 (forked from s and
// joined back into it, so the caller sees the whole evaluation on s).  The
// second lane starts once the first sub-batch's forward pass is done; from
// then on the memory-bound column passes of one sub-batch run beside the
// arithmetic-bound plane passes of the other.  Every density goes through
// the same launches and gives the same results as in one batch.
template <typename T>
static ofdft_status eval_enqueue_pipe(ofdft_grid *g, int nb, const void *d_in, int in_is_phi,
                                      void *d_v, void *d_g, hipStream_t s)
{
    const int pipe = std::max(1, std::min(g->tune_pipe, nb));
    if (pipe == 1 || g->timer.on)
        return eval_enqueue<T>(g, nb, d_in, in_is_phi, d_v, d_g, s, work_of<T>(g, 0));
    ST_TRY(ensure_lane(g));
    const size_t N = (size_t)g->geom.N;
    const int per = (nb + pipe - 1) / pipe;
    HIP_TRY(hipEventRecord(g->ev_fork, s));
    HIP_TRY(hipStreamWaitEvent(g->s2, g->ev_fork, 0));
    for (int j = 0, b0 = 0; b0 < nb; ++j, b0 += per) {
        const int n = std::min(per, nb - b0);
        hipStream_t sj = (j % 2 == 0) ? s : g->s2;
        if (j == 1) HIP_TRY(hipStreamWaitEvent(g->s2, g->ev_stagger, 0));
        const void *in = (const char *)d_in + b0 * N * sizeof(T);
        void *v = d_v ? (char *)d_v + b0 * N * sizeof(T) : nullptr;
        void *gv = d_g ? (char *)d_g + b0 * N * sizeof(T) : nullptr;
        g->stagger_after_fwd = (j == 0);
        const ofdft_status st =
            eval_enqueue<T>(g, n, in, in_is_phi, v, gv, sj, work_of<T>(g, b0), false);
        g->stagger_after_fwd = false;
        ST_TRY(st);
    }
    HIP_TRY(hipEventRecord(g->ev_join, g->s2));
    HIP_TRY(hipStreamWaitEvent(s, g->ev_join, 0));
    return OFDFT_OK;
}

// Replays (capturing on first use) the evaluation for this argument set.
template <typename T>
static ofdft_status eval_graph(ofdft_grid *g, int nb, const void *d_in, int in_is_phi, void *d_v,
                               void *d_g, hipStream_t s)
{
    GraphEntry *hit = nullptr;
    for (auto &e : g->graphs)
        if (e.nb == nb && e.in == d_in && e.in_is_phi == in_is_phi && e.v == d_v && e.gout == d_g)
            hit = &e;
    if (!hit) {
        if (g->graphs.size() >= 8) {   // drop the least recently used
            size_t lru = 0;
            for (size_t i = 1; i < g->graphs.size(); ++i)
                if (g->graphs[i].last < g->graphs[lru].last) lru = i;
            (void)hipGraphExecDestroy(g->graphs[lru].exec);
            g->graphs.erase(g->graphs.begin() + lru);
        }
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        const ofdft_status st = eval_enqueue_pipe<T>(g, nb, d_in, in_is_phi, d_v, d_g, s);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &graph);
        if (st != OFDFT_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        HIP_TRY(e);
        GraphEntry ge;
        ge.nb = nb;
        ge.in = d_in;
        ge.in_is_phi = in_is_phi;
        ge.v = d_v;
        ge.gout = d_g;
        const hipError_t ei = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIP_TRY(ei);
        g->graphs.push_back(ge);
        hit = &g->graphs.back();
    }
    hit->last = ++g->graph_clock;
    HIP_TRY(hipGraphLaunch(hit->exec, s));
    return OFDFT_OK;
}

// Energies, mu and the residual norm of one density from its FP64 sums
static void energies_of(const ofdft_grid *g, const double *S, ofdft_energy &e)
{
    const uint32_t terms = g->func.terms;
    std::memset(&e, 0, sizeof(e));
    e.nelec_int = g->dv * S[SL_RHO];
    if (terms & OFDFT_TERM_TF) e.e_tf = C_TF * g->dv * S[SL_TF];
    if (terms & OFDFT_TERM_VW) e.e_vw = 0.5 * g->func.lambda_vw * g->V * S[SL_VW];
    if (terms & OFDFT_TERM_HARTREE) e.e_h = 2.0 * PI * g->V * S[SL_H];
    if (terms & OFDFT_TERM_EXT) {
        e.e_ext = g->V * S[SL_EXT];
        e.e_ion = g->e_ion;
    }
    if (terms & (OFDFT_TERM_WT | OFDFT_TERM_SPLINE)) e.e_nl = g->dv * S[SL_NL];
    if (terms & OFDFT_TERM_XC) e.e_xc = g->dv * S[SL_XC];
    e.e_total = e.e_tf + e.e_vw + e.e_h + e.e_ext + e.e_nl + e.e_xc + e.e_ion;
    const double spp = S[SL_PHIPHI];
    e.mu = spp > 0 ? S[SL_GPHI] / (2.0 * spp) : 0.0;
    const double r2 = spp > 0 ? S[SL_GG] - S[SL_GPHI] * S[SL_GPHI] / spp : S[SL_GG];
    e.resid_norm = std::sqrt(std::max(0.0, r2) / (double)g->geom.N);
}

template <typename T>
static ofdft_status eval_impl(ofdft_grid *g, int nb, const void *d_in, int in_is_phi, void *d_v,
                              void *d_g, hipStream_t s, ofdft_energy *e_out, double *bad_out)
{
    ST_TRY(reserve(g, nb));
    // graphs on streams that can be captured (not the legacy null stream)
    // and when no per-pass timing is asked for
    if (g->use_graphs && !g->timer.on && s != nullptr) {
        ST_TRY(eval_graph<T>(g, nb, d_in, in_is_phi, d_v, d_g, s));
    } else {
        ST_TRY(eval_enqueue_pipe<T>(g, nb, d_in, in_is_phi, d_v, d_g, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    timer_collect(g);

    double bad = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double *S = g->h_sums + (size_t)b * NSLOT;
        ofdft_energy e;
        energies_of(g, S, e);
        bad += S[SL_BAD];
        if (e_out) e_out[b] = e;
    }
    if (bad_out) *bad_out = bad;
    return OFDFT_OK;
}

static ofdft_status eval_dispatch(ofdft_grid *g, int nb, const void *d_in, int in_is_phi,
                                  void *d_v, void *d_g, hipStream_t s, ofdft_energy *e_out)
{
    // energies reach e_out only when the input was valid
    double bad = 0.0;
    std::vector<ofdft_energy> e((size_t)nb);
    ofdft_status st = g->fp64 ? eval_impl<double>(g, nb, d_in, in_is_phi, d_v, d_g, s, e.data(), &bad)
                              : eval_impl<float>(g, nb, d_in, in_is_phi, d_v, d_g, s, e.data(), &bad);
    if (st != OFDFT_OK) return st;
    if (bad > 0)
        return fail(OFDFT_EINVAL, "input density has " + std::to_string((long long)bad) +
                                      " non-finite or negative values");
    if (e_out) std::copy(e.begin(), e.end(), e_out);
    return OFDFT_OK;
}

// ---------------------------------------------------------------- FFT pair
template <typename T>
// sync: wait for the stream at the end; consume: the inverse may overwrite
// d_in (a scratch spectrum) instead of working on a copy in the workspace
static ofdft_status fft_impl(ofdft_grid *g, int nb, const void *d_in, void *d_out, bool fwd,
                             hipStream_t s, bool sync = true, bool consume = false)
{
    ST_TRY(reserve(g, nb));
    const Geom &G = g->geom;
    if (fwd) {
        RowFwdArgs rf;
        std::memset(&rf, 0, sizeof(rf));
        rf.in = d_in;
        rf.out = d_out;
        rf.out_fstride = 0;
        rf.nfields = 1;
        rf.kind[0] = FK_RAW;
        rf.twM = g->twM;
        rf.twN = g->twN;
        rf.tw1 = g->tw1;
        rf.knots = g->knots;
        int nbk = 0;
        if (use_plane<T>(g)) {
            TIMED(PS_ROW_FWD, launch_plane_fwd<T>(G, nb, rf, nbk, s));
        } else {
            TIMED(PS_ROW_FWD, launch_row_fwd<T>(G, nb, rf, nbk, s));
            ST_TRY(col_pass<T>(g, s, 1, d_out, nb, nb, 0, nullptr, PS_COL1_FWD));
        }
        int ops[4] = {GO_SCALE, 0, 0, 0};
        ST_TRY(col_pass<T>(g, s, 0, d_out, nb, nb, 0, ops, PS_COL0_G));
    } else {
        // inverse: copy the spectrum into the workspace so the caller's input
        // survives, unless it may be consumed
        void *work = consume ? const_cast<void *>(d_in) : g->spec;
        if (!consume)
            HIP_TRY(hipMemcpyAsync(g->spec, d_in, (size_t)nb * G.Nh * 2 * sizeof(T),
                                   hipMemcpyDeviceToDevice, s));
        ST_TRY(col_pass<T>(g, s, 0, work, nb, nb, 1, nullptr, PS_COL0_G));
        const bool plane = use_plane<T>(g);
        if (!plane) ST_TRY(col_pass<T>(g, s, 1, work, nb, nb, 1, nullptr, PS_COL1_INV));
        RowInvArgs ri;
        std::memset(&ri, 0, sizeof(ri));
        ri.spec = work;
        ri.spec_fstride = 0;
        ri.nfields = 1;
        ri.mode = EP_STORE;
        ri.out = d_out;
        ri.nbatch = nb;
        ri.twM = g->twM;
        ri.twN = g->twN;
        ri.tw1 = g->tw1;
        ri.fld_hext = ri.fld_vw = ri.fld_wt = ri.fld_a = -1;
        int nbk = 0;
        if (plane) TIMED(PS_ROW_INV, launch_plane_inv<T>(G, ri, nbk, s));
        else TIMED(PS_ROW_INV, launch_row_inv<T>(G, ri, nbk, s));
    }
    if (sync) {
        HIP_TRY(hipStreamSynchronize(s));
        timer_collect(g);
    }
    return OFDFT_OK;
}

// ---------------------------------------------------------------- grid set-up
// grid sizes of a cell (reciprocal vectors are filled in by grid_setup)
static Geom make_geom(const int32_t n[3])
{
    Geom G;
    std::memset(&G, 0, sizeof(G));
    G.n0 = n[0];
    G.n1 = n[1];
    G.n2 = n[2];
    G.m = n[2] / 2;
    G.n2h = G.m + 1;
    G.N = (long long)G.n0 * G.n1 * G.n2;
    G.Nh = (long long)G.n0 * G.n1 * G.n2h;
    G.invN = 1.0 / (double)G.N;
    return G;
}

static ofdft_status validate(const ofdft_cell_desc *c, const ofdft_functional_desc *f)
{
    if (!c || !f) return fail(OFDFT_EINVAL, "null descriptor");
    for (int d = 0; d < 3; ++d)
        if (!is_supported(c->n[d]))
            return fail(OFDFT_EINVAL, "grid size " + std::to_string(c->n[d]) +
                                          " on axis " + std::to_string(d) + " is not supported");
    if (c->n[2] % 2 != 0 || !is_supported(c->n[2] / 2))
        return fail(OFDFT_EINVAL, "n[2] must be even with n[2]/2 a supported length");
    if (c->natoms < 0 || (c->natoms > 0 && (!c->pos || !c->species)))
        return fail(OFDFT_EINVAL, "bad atom arrays");
    if (c->natoms > 0 && (c->nspecies <= 0 || !c->Z || !c->rc))
        return fail(OFDFT_EINVAL, "bad species arrays");
    for (int a = 0; a < c->natoms; ++a) {
        if (c->species[a] < 0 || c->species[a] >= c->nspecies)
            return fail(OFDFT_EINVAL, "species index out of range");
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(c->pos[3 * a + k])) return fail(OFDFT_EINVAL, "non-finite position");
    }
    if (!(c->nelec > 0)) return fail(OFDFT_EINVAL, "nelec must be positive");
    if (c->sf_method != OFDFT_SF_DIRECT && c->sf_method != OFDFT_SF_PME)
        return fail(OFDFT_EINVAL, "unknown structure-factor method");
    if (c->sf_method == OFDFT_SF_PME) {
        const int P = pme_order_of(c->pme_order);
        if (P < 4 || P > PME_MAX_ORDER || P % 2 != 0)
            return fail(OFDFT_EINVAL, "pme_order must be even, 4 to 16");
        if (P > c->n[0] || P > c->n[1] || P > c->n[2])
            return fail(OFDFT_EINVAL, "pme_order exceeds a grid dimension");
    }
    const uint32_t all = OFDFT_TERM_TF | OFDFT_TERM_VW | OFDFT_TERM_HARTREE | OFDFT_TERM_EXT |
                         OFDFT_TERM_WT | OFDFT_TERM_SPLINE | OFDFT_TERM_XC;
    if (f->terms & ~all) return fail(OFDFT_EINVAL, "unknown term bits");
    if ((f->terms & OFDFT_TERM_WT) && (f->terms & OFDFT_TERM_SPLINE))
        return fail(OFDFT_EINVAL, "WT and SPLINE are exclusive");
    if ((f->terms & (OFDFT_TERM_WT | OFDFT_TERM_SPLINE)) && f->alpha != f->beta)
        return fail(OFDFT_EINVAL, "the GPU path requires alpha == beta");
    if ((f->terms & (OFDFT_TERM_WT | OFDFT_TERM_SPLINE)) && !(f->alpha > 0.5))
        return fail(OFDFT_EINVAL, "alpha must exceed 1/2");
    if (f->nl_kernel < OFDFT_KERNEL_WT || f->nl_kernel > OFDFT_KERNEL_MGPG)
        return fail(OFDFT_EINVAL, "unknown nl_kernel");
    if (f->terms & OFDFT_TERM_SPLINE) {
        if (f->nk < 1 || f->nk > MAXKNOTS) return fail(OFDFT_EINVAL, "nk out of range");
        if (!(f->kf_min > 0) || !(f->kf_max >= f->kf_min) || (f->nk > 1 && !(f->kf_max > f->kf_min)))
            return fail(OFDFT_EINVAL, "bad knot range");
        if (f->nl_mode != OFDFT_NL_S3S4 && f->nl_mode != OFDFT_NL_EXACT)
            return fail(OFDFT_EINVAL, "bad nl_mode");
    }
    if (f->precision != OFDFT_FP64 && f->precision != OFDFT_MIXED &&
        f->precision != OFDFT_MIXED_VW64)
        return fail(OFDFT_EINVAL, "bad precision");
    if (!(f->rho_floor > 0)) return fail(OFDFT_EINVAL, "rho_floor must be positive");
    return OFDFT_OK;
}

static void grid_free(ofdft_grid *g)
{
    graphs_clear(g);
    dfree(g->td);
    dfree(reinterpret_cast<void *&>(g->d_td_part));
    dfree(reinterpret_cast<void *&>(g->d_td_dots));
    dfree(reinterpret_cast<void *&>(g->d_td_sc));
    if (g->h_td_sc) (void)hipHostFree(g->h_td_sc);
    g->h_td_sc = nullptr;
    dfree(g->tw0);
    dfree(g->tw1);
    dfree(g->twM);
    dfree(g->twN);
    dfree(g->tw0d);
    dfree(g->tw1d);
    dfree(g->twMd);
    dfree(g->twNd);
    dfree(g->vwspec);
    dfree(g->vwout);
    dfree(reinterpret_cast<void *&>(g->kr_part));
    dfree(reinterpret_cast<void *&>(g->kneed));
    dfree(g->vext);
    dfree(g->gtab);
    dfree(reinterpret_cast<void *&>(g->ph0));
    dfree(reinterpret_cast<void *&>(g->ph1));
    dfree(reinterpret_cast<void *&>(g->ph2));
    dfree(reinterpret_cast<void *&>(g->d_spec_off));
    dfree(reinterpret_cast<void *&>(g->d_atom_species));
    dfree(reinterpret_cast<void *&>(g->d_Z));
    dfree(reinterpret_cast<void *&>(g->d_rc));
    dfree(reinterpret_cast<void *&>(g->d_knots));
    if (g->d_jtab != (void *)g->d_jtab64) dfree(g->d_jtab);
    g->d_jtab = nullptr;
    dfree(reinterpret_cast<void *&>(g->d_jtab64));
    dfree(g->spec);
    dfree(g->kspec);
    dfree(g->kspec2);
    dfree(g->acc1);
    dfree(g->acc2);
    dfree(g->stage_in);
    dfree(g->stage_out);
    dfree(reinterpret_cast<void *&>(g->part));
    dfree(reinterpret_cast<void *&>(g->sums));
    dfree(reinterpret_cast<void *&>(g->d_forces));
    dfree(reinterpret_cast<void *&>(g->d_frac));
    dfree(reinterpret_cast<void *&>(g->d_ew_pos));
    dfree(reinterpret_cast<void *&>(g->d_ew_q));
    dfree(reinterpret_cast<void *&>(g->d_ew_e));
    dfree(reinterpret_cast<void *&>(g->d_ew_f));
    dfree(reinterpret_cast<void *&>(g->d_ew_sf));
    dfree(reinterpret_cast<void *&>(g->d_bin_start));
    dfree(reinterpret_cast<void *&>(g->d_bin_of));
    dfree(reinterpret_cast<void *&>(g->d_ew_part));
    dfree(reinterpret_cast<void *&>(g->d_pme_b));
    dfree(reinterpret_cast<void *&>(g->d_ct));
    if (g->h_ct) (void)hipHostFree(g->h_ct);
    g->h_ct = nullptr;
    dfree(g->batch_in);
    dfree(g->batch_out);
    dfree(g->rho);
    for (auto &p : g->opt) dfree(p);
    if (g->h_sums) (void)hipHostFree(g->h_sums);
    g->h_sums = nullptr;
    for (hipEvent_t e : g->timer.ev) (void)hipEventDestroy(e);
    g->timer.ev.clear();
    for (hipEvent_t &e : g->kev)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    for (hipEvent_t *e : {&g->ev_fork, &g->ev_join, &g->ev_stagger})
        if (*e) {
            (void)hipEventDestroy(*e);
            *e = nullptr;
        }
    if (g->s2) {
        (void)hipStreamDestroy(g->s2);
        g->s2 = nullptr;
    }
}

// Exponential-spline factors of smooth PME along one axis of K points,
// conjugated for the exp(-iG.R) sign of the structure factor: out[m] =
// conj(b(m)), m = 0 .. cnt-1, with b(m) = exp(2 pi i (P-1) m / K) /
// sum_{k=0}^{P-2} M_P(k+1) exp(2 pi i m k / K).  False if a denominator
// vanishes.
template <int P>
static void bspline_integers(double *out)
{
    double w[P];
    bspline_fill<P>(0.0, w);   // w[j] = M_P(j)
    for (int j = 0; j < P; ++j) out[j] = w[j];
}
static bool pme_bfactors(int order, int K, int cnt, double2 *out)
{
    double M[PME_MAX_ORDER];
    switch (order) {
    case 4: bspline_integers<4>(M); break;
    case 6: bspline_integers<6>(M); break;
    case 8: bspline_integers<8>(M); break;
    case 10: bspline_integers<10>(M); break;
    case 12: bspline_integers<12>(M); break;
    case 14: bspline_integers<14>(M); break;
    case 16: bspline_integers<16>(M); break;
    default: return false;
    }
    for (int m = 0; m < cnt; ++m) {
        double dr = 0.0, di = 0.0;
        for (int k = 0; k <= order - 2; ++k) {
            const double ang = 2.0 * PI * (double)(((long long)m * k) % K) / K;
            dr += M[k + 1] * std::cos(ang);
            di += M[k + 1] * std::sin(ang);
        }
        const double den2 = dr * dr + di * di;
        if (!(den2 > 1e-300)) return false;
        const double ang = 2.0 * PI * (double)(((long long)m * (order - 1)) % K) / K;
        const double nr = std::cos(ang), ni = std::sin(ang);
        out[m] = {(nr * dr + ni * di) / den2, -(ni * dr - nr * di) / den2};
    }
    return true;
}

// Bound on any charge-grid value: atoms contributing to a point have their
// base index floor(n s) within P consecutive points per axis, so they lie in
// two adjacent cells of a partition into cells at least P points wide; each
// atom adds at most 1.
static double pme_grid_bound(const Geom &G, int P, const std::vector<double> &fr)
{
    const int na = (int)(fr.size() / 3);
    const int n[3] = {G.n0, G.n1, G.n2};
    int c[3];
    for (int d = 0; d < 3; ++d) c[d] = std::max(1, n[d] / P);
    std::vector<int> cnt((size_t)c[0] * c[1] * c[2], 0);
    for (int a = 0; a < na; ++a) {
        int ci[3];
        for (int d = 0; d < 3; ++d) {
            int b = (int)std::floor(fr[3 * (size_t)a + d] * n[d]);
            b = std::min(std::max(b, 0), n[d] - 1);
            ci[d] = std::min(b / P, c[d] - 1);
        }
        cnt[((size_t)ci[0] * c[1] + ci[1]) * c[2] + ci[2]]++;
    }
    double worst = 0.0;
    for (int x = 0; x < c[0]; ++x)
        for (int y = 0; y < c[1]; ++y)
            for (int z = 0; z < c[2]; ++z) {
                double t = 0.0;
                for (int dx = 0; dx < 2; ++dx)
                    for (int dy = 0; dy < 2; ++dy)
                        for (int dz = 0; dz < 2; ++dz)
                            t += cnt[(((size_t)(x + dx) % c[0]) * c[1] + (y + dy) % c[1]) * c[2] +
                                     (z + dz) % c[2]];
                worst = std::max(worst, t);
            }
    return worst;
}

// v_ext(G) and the Ewald reciprocal sum by smooth PME: per species, the
// fixed-point charge grid, the grid's forward transform (in the grid's
// precision) into the workspace spectrum, and the spline-factor pass.
template <typename T>
static ofdft_status pme_reciprocal(ofdft_grid *g, const LargeEwald &L,
                                   const std::vector<double> &fr, double *erec)
{
    const Geom &G = g->geom;
    const int na = g->natoms, ns = (int)g->Z.size(), P = g->pme_order;
    hipStream_t s = g->ctx->stream;
    if (na >= (1 << (64 - PME_FIX_BITS - 1)) &&
        pme_grid_bound(G, P, fr) >= (double)(1ull << (64 - PME_FIX_BITS - 1)))
        return fail(OFDFT_EINVAL, "too many atoms within one PME spline window");
    if (!g->d_pme_b) {
        std::vector<double2> bt((size_t)G.n0 + G.n1 + G.n2h);
        if (!pme_bfactors(P, G.n0, G.n0, bt.data()) ||
            !pme_bfactors(P, G.n1, G.n1, bt.data() + G.n0) ||
            !pme_bfactors(P, G.n2, G.n2h, bt.data() + G.n0 + G.n1))
            return fail(OFDFT_EINVAL, "a PME spline factor vanishes");
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_pme_b), bt.size() * sizeof(double2)));
        ST_TRY(h2d(g, g->d_pme_b, bt.data(), bt.size() * sizeof(double2)));
    }
    const int nblk = pme_finish_blocks(G);
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_ew_part), (size_t)nblk * 8));
    ST_TRY(reserve(g, 1));
    std::vector<int> off(ns + 1, 0);
    for (int a = 0; a < na; ++a) off[g->species[a] + 1]++;
    for (int k = 0; k < ns; ++k) off[k + 1] += off[k];
    // transient: the fixed-point grid (converted in place for FP64), its
    // FP32 copy, and sum_s Z_s S_s between species
    void *qfix = nullptr, *qreal = nullptr, *qbuf = nullptr;
    hipError_t e = hipMalloc(&qfix, (size_t)G.N * 8);
    if (e == hipSuccess && !g->fp64) e = hipMalloc(&qreal, (size_t)G.N * sizeof(T));
    if (e == hipSuccess && ns > 1) e = hipMalloc(&qbuf, (size_t)G.Nh * 16);
    ofdft_status st = OFDFT_OK;
    if (e != hipSuccess) st = fail(OFDFT_ENOMEM, "PME charge grid allocation failed");
    void *qr = g->fp64 ? qfix : qreal;
    for (int sp = 0; sp < ns && st == OFDFT_OK; ++sp) {
        e = hipMemsetAsync(qfix, 0, (size_t)G.N * 8, s);
        if (e == hipSuccess)
            e = launch_pme_spread(G, P, off[sp], off[sp + 1] - off[sp], g->d_frac,
                                  (unsigned long long *)qfix, s);
        if (e == hipSuccess) e = launch_pme_to_real<T>(G, (const unsigned long long *)qfix, qr, s);
        if (e != hipSuccess) {
            st = fail(OFDFT_EDEVICE, std::string("PME spread: ") + hipGetErrorString(e));
            break;
        }
        st = fft_impl<T>(g, 1, qr, g->spec, true, s);
        if (st != OFDFT_OK) break;
        e = launch_pme_finish<T>(G, g->spec, g->d_pme_b, g->Z[sp], g->rc[sp], g->V, L.e.a,
                                 L.e.gcut2, sp == 0, sp == ns - 1, g->vext, qbuf, g->d_ew_part, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            st = fail(OFDFT_EDEVICE, std::string("PME finish: ") + hipGetErrorString(e));
    }
    (void)hipStreamSynchronize(s);
    if (qfix) (void)hipFree(qfix);
    if (qreal) (void)hipFree(qreal);
    if (qbuf) (void)hipFree(qbuf);
    ST_TRY(st);
    std::vector<double> part((size_t)nblk);
    HIP_TRY(hipMemcpyAsync(part.data(), g->d_ew_part, part.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double sum = 0.0;
    for (double x : part) sum += x;
    *erec = sum * 2.0 * PI / g->V;
    return OFDFT_OK;
}

// Large cells: v_ext(G) and the Ewald reciprocal sum from the tiled direct
// sum (or smooth PME), the real-space Ewald sum over bins.  fr:
// species-sorted fractional coordinates (already on the device in d_frac).
static ofdft_status setup_ions_large(ofdft_grid *g, const std::vector<int> &order,
                                     const std::vector<double> &fr)
{
    const Geom &G = g->geom;
    const int na = g->natoms, ns = (int)g->Z.size();
    hipStream_t s = g->ctx->stream;
    const bool pme = g->sf_method == OFDFT_SF_PME;
    const LargeEwald L = large_ewald(g->lattice, G.b, g->V, na, g->n, pme);
    double erec = 0.0;
    if (pme) {
        ST_TRY(g->fp64 ? pme_reciprocal<double>(g, L, fr, &erec)
                       : pme_reciprocal<float>(g, L, fr, &erec));
    } else {
        const long long nblk = sf_tiled_blocks(G);
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_ew_part), (size_t)nblk * 8));
        void *qbuf = nullptr;
        if (ns > 1) {
            HIP_TRY(hipMalloc(&qbuf, (size_t)G.Nh * 16));   // released below
        }
        hipError_t err = g->fp64
            ? launch_sf_tiled<double>(G, g->d_spec_off, ns, g->d_frac, g->d_Z, g->d_rc, g->V,
                                      L.e.a, L.e.gcut2, g->vext, qbuf, g->d_ew_part, s)
            : launch_sf_tiled<float>(G, g->d_spec_off, ns, g->d_frac, g->d_Z, g->d_rc, g->V,
                                     L.e.a, L.e.gcut2, g->vext, qbuf, g->d_ew_part, s);
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        if (qbuf) (void)hipFree(qbuf);
        HIP_TRY(err);
        std::vector<double> part((size_t)nblk);
        HIP_TRY(hipMemcpyAsync(part.data(), g->d_ew_part, part.size() * 8, hipMemcpyDeviceToHost,
                               s));
        HIP_TRY(hipStreamSynchronize(s));
        for (double x : part) erec += x;
        erec *= 2.0 * PI / g->V;
    }

    // real space: atoms binned by fractional coordinate, positions wrapped
    // into the cell (counting sort, atoms in bin order); a cell less than
    // three cut-offs wide in some direction sums over images of all pairs
    int nb0 = L.nbin[0], nb1 = L.nbin[1], nb2 = L.nbin[2];
    const bool binned = nb0 >= 3 && nb1 >= 3 && nb2 >= 3;
    if (!binned) nb0 = nb1 = nb2 = 1;
    const int nbins = nb0 * nb1 * nb2;
    std::vector<int> bin(na), start(nbins + 1, 0);
    for (int a = 0; a < na; ++a) {
        const double *f = &fr[3 * (size_t)a];
        const int c0 = std::min(nb0 - 1, (int)(f[0] * nb0));
        const int c1 = std::min(nb1 - 1, (int)(f[1] * nb1));
        const int c2 = std::min(nb2 - 1, (int)(f[2] * nb2));
        bin[a] = (c0 * nb1 + c1) * nb2 + c2;
        start[bin[a] + 1]++;
    }
    for (int k = 0; k < nbins; ++k) start[k + 1] += start[k];
    std::vector<int> fill(start.begin(), start.end() - 1), bin_of(na);
    std::vector<double> pos(3 * (size_t)na), q(na);
    double Q = 0, Q2 = 0;
    for (int a = 0; a < na; ++a) {
        const int slot = fill[bin[a]]++;
        const double *f = &fr[3 * (size_t)a];
        for (int c = 0; c < 3; ++c)
            pos[3 * (size_t)slot + c] =
                f[0] * g->lattice[0][c] + f[1] * g->lattice[1][c] + f[2] * g->lattice[2][c];
        q[slot] = g->Z[g->species[order[a]]];
        bin_of[slot] = bin[a];
        Q += q[slot];
        Q2 += q[slot] * q[slot];
    }
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_ew_pos), pos.size() * 8));
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_ew_q), q.size() * 8));
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_ew_e), q.size() * 8));
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_bin_start), start.size() * 4));
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_bin_of), bin_of.size() * 4));
    ST_TRY(h2d(g, g->d_ew_pos, pos.data(), pos.size() * 8));
    ST_TRY(h2d(g, g->d_ew_q, q.data(), q.size() * 8));
    ST_TRY(h2d(g, g->d_bin_start, start.data(), start.size() * 4));
    ST_TRY(h2d(g, g->d_bin_of, bin_of.data(), bin_of.size() * 4));
    const int nbv[3] = {nb0, nb1, nb2};
    if (binned) {
        HIP_TRY(launch_ewald_real_cells(L.e, na, g->d_ew_pos, g->d_ew_q, g->d_bin_start,
                                        g->d_bin_of, nbv, g->d_ew_e, s));
    } else {
        // the all-pairs kernel with an empty reciprocal box (gmax = 0: G = 0 only)
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_ew_sf), 24));
        HIP_TRY(launch_ewald(L.e, na, g->d_ew_pos, g->d_ew_q, g->d_ew_sf, g->d_ew_e, nullptr, s));
    }
    std::vector<double> ea(na);
    HIP_TRY(hipMemcpyAsync(ea.data(), g->d_ew_e, (size_t)na * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double ereal = 0.0;
    for (double x : ea) ereal += x;
    const double e_ion = ereal + erec - L.e.a / std::sqrt(PI) * Q2 -
                         PI * Q * Q / (2 * g->V * L.e.a * L.e.a);
    g->e_ion = (g->func.terms & OFDFT_TERM_EXT) ? e_ion : 0.0;
    return OFDFT_OK;
}

// Ionic part of the set-up, also rerun when the atoms move (MD frames of a
// resident cell): per-axis phase tables exp(-i 2 pi m_d s_d) for every atom,
// the species-sorted direct sum v_ext(G) = (1/V) sum_a v~(|G|) exp(-iG.R_a)
// of eq. "ie" and the Ewald energy.  Buffers keep their sizes because the atom
// count and species are fixed for a grid.
static ofdft_status setup_ions(ofdft_grid *g)
{
    const Geom &G = g->geom;
    const int na = g->natoms;
    const int ns = (int)g->Z.size();
    hipStream_t s = g->ctx->stream;
    if (na > 0) {
        // atoms sorted by species: the v_ext kernel sums each species' atoms
        // together, and the phase tables and forces use this order
        std::vector<int> order(na);
        for (int a = 0; a < na; ++a) order[a] = a;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return g->species[x] < g->species[y]; });
        std::vector<int> off(ns + 1, 0);
        for (int a = 0; a < na; ++a) off[g->species[a] + 1]++;
        for (int k = 0; k < ns; ++k) off[k + 1] += off[k];
        // fractional coordinates s = inv(A)^T R, wrapped into [0, 1)
        std::vector<double> fr(3 * (size_t)na);
        for (int a = 0; a < na; ++a)
            for (int j = 0; j < 3; ++j) {
                double x = 0;
                for (int i = 0; i < 3; ++i) x += g->pos[3 * order[a] + i] * g->frac[j][i];
                fr[3 * a + j] = x - std::floor(x);
            }
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_frac), fr.size() * sizeof(double)));
        ST_TRY(h2d(g, g->d_frac, fr.data(), fr.size() * sizeof(double)));
        if (!g->large_ions) {
            const int nax[3] = {G.n0, G.n1, G.n2h};
            double **tabs[3] = {&g->ph0, &g->ph1, &g->ph2};
            for (int d = 0; d < 3; ++d)
                ST_TRY(dmalloc(g, reinterpret_cast<void **>(tabs[d]),
                               2 * (size_t)na * nax[d] * sizeof(double)));
            HIP_TRY(launch_phases(G, na, g->d_frac, g->ph0, g->ph1, g->ph2, s));
        }
        std::vector<int> sorted_species(na);
        for (int a = 0; a < na; ++a) sorted_species[a] = g->species[order[a]];
        g->species_order = order;
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_spec_off), (ns + 1) * sizeof(int)));
        ST_TRY(h2d(g, g->d_spec_off, off.data(), (ns + 1) * sizeof(int)));
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_atom_species), na * sizeof(int)));
        ST_TRY(h2d(g, g->d_atom_species, sorted_species.data(), na * sizeof(int)));
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_Z), ns * sizeof(double)));
        ST_TRY(h2d(g, g->d_Z, g->Z.data(), ns * sizeof(double)));
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_rc), ns * sizeof(double)));
        ST_TRY(h2d(g, g->d_rc, g->rc.data(), ns * sizeof(double)));
    }
    ST_TRY(dmalloc(g, &g->vext, (size_t)G.Nh * 2 * g->fsz));
    if (g->large_ions) {
        // fractional coordinates in the species order, for the bins
        std::vector<double> frs(3 * (size_t)na);
        for (int a = 0; a < na; ++a)
            for (int j = 0; j < 3; ++j) {
                double x = 0;
                for (int i = 0; i < 3; ++i) x += g->pos[3 * g->species_order[a] + i] * g->frac[j][i];
                frs[3 * a + j] = x - std::floor(x);
            }
        return setup_ions_large(g, g->species_order, frs);
    }
    if (na > 0) {
        hipError_t e = g->fp64 ? launch_vext<double>(G, na, g->d_spec_off, ns, g->ph0, g->ph1, g->ph2,
                                                     g->d_Z, g->d_rc, g->V, g->vext, s)
                               : launch_vext<float>(G, na, g->d_spec_off, ns, g->ph0, g->ph1, g->ph2,
                                                    g->d_Z, g->d_rc, g->V, g->vext, s);
        HIP_TRY(e);
    } else {
        HIP_TRY(hipMemsetAsync(g->vext, 0, (size_t)G.Nh * 2 * g->fsz, s));
    }
    double e_ion = 0.0;
    ST_TRY(ewald_device(g, &e_ion, nullptr));
    g->e_ion = (g->func.terms & OFDFT_TERM_EXT) ? e_ion : 0.0;
    HIP_TRY(hipStreamSynchronize(s));
    return OFDFT_OK;
}

static ofdft_status grid_setup(ofdft_grid *g, const ofdft_cell_desc *c, const ofdft_functional_desc *f)
{
    std::memcpy(g->lattice, c->lattice, sizeof(g->lattice));
    for (int d = 0; d < 3; ++d) g->n[d] = c->n[d];
    g->natoms = c->natoms;
    g->pos.assign(c->pos, c->pos + 3 * (size_t)c->natoms);
    g->species.assign(c->species, c->species + c->natoms);
    g->Z.assign(c->Z, c->Z + std::max(c->nspecies, 0));
    g->rc.assign(c->rc, c->rc + std::max(c->nspecies, 0));
    g->nelec = c->nelec;
    g->func = *f;
    g->fp64 = f->precision == OFDFT_FP64;
    g->fsz = g->fp64 ? 8 : 4;
    g->vw64 = f->precision == OFDFT_MIXED_VW64 && (f->terms & OFDFT_TERM_VW);

    // geometry: b_j with a_i . b_j = 2 pi delta_ij  (b = 2 pi inv(A)^T)
    const double(*A)[3] = g->lattice;
    const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                       A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                       A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    if (!(std::fabs(det) > 0)) return fail(OFDFT_EINVAL, "singular lattice");
    g->V = std::fabs(det);
    double cof[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            cof[i][j] = A[i1][j1] * A[i2][j2] - A[i1][j2] * A[i2][j1];
        }
    g->geom = make_geom(c->n);
    Geom &G = g->geom;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) G.b[i][j] = 2.0 * PI * cof[i][j] / det;
    g->dv = g->V / (double)G.N;

    // knots (step s1): geometric or arithmetic, both ends included
    std::memset(&g->knots, 0, sizeof(g->knots));
    if (f->terms & OFDFT_TERM_SPLINE) {
        Knots &K = g->knots;
        K.nk = f->nk;
        K.log_spacing = f->knot_spacing == OFDFT_KNOTS_LOG;
        std::vector<double> &k = g->knot_host;
        k.resize(f->nk);
        for (int i = 0; i < f->nk; ++i) {
            const double u = f->nk > 1 ? (double)i / (double)(f->nk - 1) : 0.0;
            k[i] = K.log_spacing ? f->kf_min * std::pow(f->kf_max / f->kf_min, u)
                                 : f->kf_min + (f->kf_max - f->kf_min) * u;
        }
        if (f->nk > 1)
            K.inv_span = K.log_spacing ? (f->nk - 1) / std::log(k[f->nk - 1] / k[0])
                                       : (f->nk - 1) / (k[f->nk - 1] - k[0]);
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_knots), k.size() * sizeof(double)));
        ST_TRY(h2d(g, g->d_knots, k.data(), k.size() * sizeof(double)));
        K.k = g->d_knots;
    }
    g->kf_wt = f->kf_wt > 0 ? f->kf_wt : std::cbrt(3.0 * PI * PI * g->nelec / g->V);

    // MGP-family kernel: the J table in FP64 and in the field type
    double mx = 0.0, my = 0.0;
    if ((f->terms & (OFDFT_TERM_WT | OFDFT_TERM_SPLINE)) && mgp_params(f->nl_kernel, mx, my)) {
        const std::vector<double> &tab = mgp_table_cached(my);
        g->mgp_x = mx;
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_jtab64), tab.size() * 8));
        ST_TRY(h2d(g, g->d_jtab64, tab.data(), tab.size() * 8));
        if (g->fp64) {
            g->d_jtab = g->d_jtab64;
        } else {
            auto tf = to_type<float>(tab.data(), tab.size());
            ST_TRY(dmalloc(g, &g->d_jtab, tf.size() * 4));
            ST_TRY(h2d(g, g->d_jtab, tf.data(), tf.size() * 4));
        }
    }

    // twiddles
    ST_TRY(upload_twiddles(g, &g->tw0, G.n0, G.n0, g->fp64));
    ST_TRY(upload_twiddles(g, &g->tw1, G.n1, G.n1, g->fp64));
    ST_TRY(upload_twiddles(g, &g->twM, G.m, G.m, g->fp64));
    ST_TRY(upload_twiddles(g, &g->twN, G.n2, G.m + 1, g->fp64));
    if (g->vw64) {
        ST_TRY(upload_twiddles(g, &g->tw0d, G.n0, G.n0, true));
        ST_TRY(upload_twiddles(g, &g->tw1d, G.n1, G.n1, true));
        ST_TRY(upload_twiddles(g, &g->twMd, G.m, G.m, true));
        ST_TRY(upload_twiddles(g, &g->twNd, G.n2, G.m + 1, true));
    }


    for (int j = 0; j < 3; ++j)
        for (int i = 0; i < 3; ++i) g->frac[j][i] = cof[j][i] / det;
    ST_TRY(setup_ions(g));
    ST_TRY(dmalloc(g, &g->gtab, 3 * (size_t)G.Nh * g->fsz));
    hipStream_t s = g->ctx->stream;
    HIP_TRY(g->fp64 ? launch_gtab<double>(G, g->kf_wt, nl_kern(g, true), g->gtab, s)
                    : launch_gtab<float>(G, g->kf_wt, nl_kern(g, true), g->gtab, s));
    HIP_TRY(hipStreamSynchronize(s));
    ST_TRY(dmalloc(g, &g->rho, (size_t)G.N * g->fsz));
    return OFDFT_OK;
}

// ---------------------------------------------------------------- host<->device fields
// check_density: refuse non-finite or negative values.  FP64 fields are
// checked by the evaluation's own prologue; for FP32 fields the conversion
// loop checks the FP64 values it visits anyway (a negative value too small
// for FP32 would otherwise arrive as -0 and pass)
// Host fields of an FP32 grid are converted in pinned host memory and copied
// by DMA from and to it: one buffer per direction and calling thread, grown
// to a power of two as larger fields come (at most PIN_MAX floats; larger
// fields go through a pageable vector) and kept for the thread's life, so
// that grids built and dropped by a serving worker reuse its buffers.
constexpr size_t PIN_MAX = size_t(1) << 24;
struct PinStage {
    float *buf[2] = {nullptr, nullptr};
    size_t cap[2] = {0, 0};
};
static thread_local PinStage t_pin;
static float *host_stage(int dir, size_t n, std::vector<float> &fallback)
{
    if (n <= PIN_MAX) {
        if (t_pin.cap[dir] < n) {
            if (t_pin.buf[dir]) (void)hipHostFree(t_pin.buf[dir]);
            t_pin.buf[dir] = nullptr;
            t_pin.cap[dir] = 0;
            size_t c = 1;
            while (c < n) c <<= 1;
            void *p = nullptr;
            if (hipHostMalloc(&p, c * sizeof(float), hipHostMallocDefault) == hipSuccess) {
                t_pin.buf[dir] = (float *)p;
                t_pin.cap[dir] = c;
            }
        }
        if (t_pin.buf[dir]) return t_pin.buf[dir];
    }
    fallback.resize(n);
    return fallback.data();
}

static ofdft_status upload_field(ofdft_grid *g, void *dst, const double *src, size_t n, hipStream_t s,
                                 bool check_density = false)
{
    if (g->fp64) {
        HIP_TRY(hipMemcpyAsync(dst, src, n * 8, hipMemcpyHostToDevice, s));
    } else {
        std::vector<float> fb;
        float *f = host_stage(0, n, fb);
        size_t bad = 0;
        for (size_t i = 0; i < n; ++i) {
            const double x = src[i];
            bad += check_density && !(x >= 0.0 && x <= 1.7976931348623157e308);
            f[i] = (float)x;
        }
        if (bad)
            return fail(OFDFT_EINVAL, "input density has " + std::to_string(bad) +
                                          " non-finite or negative values");
        HIP_TRY(hipMemcpyAsync(dst, f, n * 4, hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    return OFDFT_OK;
}

static ofdft_status download_field(ofdft_grid *g, double *dst, const void *src, size_t n, hipStream_t s)
{
    if (g->fp64) {
        HIP_TRY(hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    } else {
        std::vector<float> fb;
        float *f = host_stage(1, n, fb);
        HIP_TRY(hipMemcpyAsync(f, src, n * 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (size_t i = 0; i < n; ++i) dst[i] = f[i];
    }
    return OFDFT_OK;
}

static hipStream_t pick_stream(ofdft_grid *g, void *hs)
{
    return hs ? (hipStream_t)hs : g->ctx->stream;
}

// ---------------------------------------------------------------- optimiser
// Vectors: 0 phi, 1 p (search direction on the sphere), 2 d (raw direction),
// 3 R (residual), 4 R_prev, 5 g (dE/dphi at phi), 6 phi trial, 7 g trial,
// 8 z = K R (preconditioned residual), 9 z_prev.
enum { V_PHI = 0, V_P, V_D, V_R, V_RP, V_G, V_PT, V_GT, V_Z, V_ZP, NVEC = NVEC_OPT };

struct OptState {
    ofdft_grid *g;
    hipStream_t s;
    long long N;
};

template <typename T>
static ofdft_status dots(OptState &o, int nd, const void *x0, const void *y0, const void *x1,
                         const void *y1, const void *x2, const void *y2, double *out)
{
    ofdft_grid *g = o.g;
    hipStream_t s = o.s;
    int nbk = 0;
    TIMED(PS_OTHER, launch_dots<T>(o.N, nd, x0, y0, x1, y1, x2, y2, nullptr, nullptr, g->part,
                                   g->pstride, nbk, s));
    SlotCounts cnt;
    std::memset(&cnt, 0, sizeof(cnt));
    for (int d = 0; d < nd; ++d) cnt.n[SL_AUX0 + d] = nbk;
    HIP_TRY(launch_finalize(g->part, g->pstride, cnt, 1, g->sums, s));
    HIP_TRY(hipMemcpyAsync(g->h_sums, g->sums, NSLOT * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    timer_collect(g);
    for (int d = 0; d < nd; ++d) out[d] = g->h_sums[SL_AUX0 + d];
    return OFDFT_OK;
}

template <typename T>
static ofdft_status lincomb(OptState &o, void *z, double a, const void *x, double b, const void *y)
{
    ofdft_grid *g = o.g;
    hipStream_t s = o.s;
    TIMED(PS_OTHER, launch_lincomb<T>(o.N, z, a, x, b, y, s));
    return OFDFT_OK;
}

// out = K in with K(G) = q0^2 / (G^2 + q0^2): forward transform, the
// multiply inside the axis-0 pass, inverse transform (grid workspace slot 0)
template <typename T>
static ofdft_status precondition(OptState &o, const void *in, void *out)
{
    ofdft_grid *g = o.g;
    hipStream_t s = o.s;
    const Geom &G = g->geom;
    RowFwdArgs rf;
    std::memset(&rf, 0, sizeof(rf));
    rf.in = in;
    rf.out = g->spec;
    rf.nfields = 1;
    rf.kind[0] = FK_RAW;
    rf.twM = g->twM;
    rf.twN = g->twN;
    rf.tw1 = g->tw1;
    rf.knots = g->knots;
    int nbk = 0;
    const bool plane = use_plane<T>(g);
    if (plane) {
        TIMED(PS_OTHER, launch_plane_fwd<T>(G, 1, rf, nbk, s));
    } else {
        TIMED(PS_OTHER, launch_row_fwd<T>(G, 1, rf, nbk, s));
        ST_TRY(col_pass<T>(g, s, 1, g->spec, 1, 1, 0, nullptr, PS_OTHER));
    }
    int ops[4] = {GO_PRECOND, 0, 0, 0};
    ST_TRY(col_pass<T>(g, s, 0, g->spec, 1, 1, 0, ops, PS_OTHER));
    if (!plane) ST_TRY(col_pass<T>(g, s, 1, g->spec, 1, 1, 1, nullptr, PS_OTHER));
    RowInvArgs ri;
    std::memset(&ri, 0, sizeof(ri));
    ri.spec = g->spec;
    ri.nfields = 1;
    ri.mode = EP_STORE;
    ri.out = out;
    ri.nbatch = 1;
    ri.twM = g->twM;
    ri.twN = g->twN;
    ri.tw1 = g->tw1;
    ri.fld_hext = ri.fld_vw = ri.fld_wt = ri.fld_a = -1;
    if (plane) TIMED(PS_OTHER, launch_plane_inv<T>(G, ri, nbk, s));
    else TIMED(PS_OTHER, launch_row_inv<T>(G, ri, nbk, s));
    return OFDFT_OK;
}

static double cubic_min(double a, double fa, double da, double b, double fb, double db, bool &ok)
{
    const double d1 = da + db - 3.0 * (fa - fb) / (a - b);
    const double disc = d1 * d1 - da * db;
    ok = false;
    if (disc < 0) return 0;
    const double d2 = (b > a ? 1.0 : -1.0) * std::sqrt(disc);
    const double den = db - da + 2.0 * d2;
    if (den == 0) return 0;
    ok = true;
    return b - (b - a) * (db + d2 - d1) / den;
}

// The optimiser's evaluation of phi (dE/dphi to gout): directly, or, in a
// lockstep optimisation, merged with the other members' evaluations
static ofdft_status opt_eval(ofdft_grid *g, const void *phi, void *gout, hipStream_t s,
                            ofdft_energy *e);

// Truncated-Newton direction (Section "Density optimization strategies":
// the paper's TN, a line-search Newton-CG method) on the tangent space of
// the constraint <phi, phi> dv = N_e: preconditioned CG on H_T d = -R with
// H_T v = P[(g(phi + h v) - g(phi)) / h - 2 mu v], P the projector orthogonal
// to phi and h a finite-difference step relative to |phi| / |v|; stopped at
// |r| <= min(1/2, sqrt(|R|_rms)) |R| (the forcing sequence of Newton-CG), on
// negative curvature (the first iteration then returns the preconditioned
// steepest descent direction) or after max_inner products.  On entry V_R
// holds R and V_Z holds K R; on return V_D holds d.  Each product is one
// evaluation.  Vectors: r in V_RP, z in V_Z, p in V_ZP, H p in V_P, the
// displaced phi and its gradient in V_PT and V_GT.
template <typename T>
static ofdft_status tn_direction(OptState &o, void **v, const ofdft_energy &E, int &evals)
{
    ofdft_grid *g = o.g;
    hipStream_t s = o.s;
    const int max_inner = 20;
    const double eta_fd = g->fp64 ? 1e-6 : 1e-3;
    double w[3];
    ST_TRY(dots<T>(o, 3, v[V_Z], v[V_PHI], v[V_PHI], v[V_PHI], v[V_R], v[V_R], w));
    const double pp = w[1], rr0 = w[2];
    if (!(pp > 0) || !(rr0 > 0)) return fail(OFDFT_EINVAL, "degenerate Newton system");
    ST_TRY(lincomb<T>(o, v[V_Z], -1.0, v[V_Z], w[0] / pp, v[V_PHI]));   // z = P K r, r = -R
    ST_TRY(lincomb<T>(o, v[V_RP], -1.0, v[V_R], 0.0, nullptr));
    ST_TRY(lincomb<T>(o, v[V_ZP], 1.0, v[V_Z], 0.0, nullptr));          // p = z
    ST_TRY(lincomb<T>(o, v[V_D], 0.0, v[V_Z], 0.0, nullptr));           // d = 0
    ST_TRY(dots<T>(o, 1, v[V_RP], v[V_Z], nullptr, nullptr, nullptr, nullptr, w));
    double rz = w[0];
    const double eta = std::min(0.5, std::sqrt(E.resid_norm));
    for (int j = 0; j < max_inner; ++j) {
        ST_TRY(dots<T>(o, 1, v[V_ZP], v[V_ZP], nullptr, nullptr, nullptr, nullptr, w));
        if (!(w[0] > 0)) break;
        const double h = eta_fd * std::sqrt(pp / w[0]);
        ST_TRY(lincomb<T>(o, v[V_PT], 1.0, v[V_PHI], h, v[V_ZP]));
        ofdft_energy Et;
        ST_TRY(opt_eval(g, v[V_PT], v[V_GT], s, &Et));
        ++evals;
        ST_TRY(lincomb<T>(o, v[V_P], 1.0 / h, v[V_GT], -1.0 / h, v[V_G]));
        ST_TRY(lincomb<T>(o, v[V_P], 1.0, v[V_P], -2.0 * E.mu, v[V_ZP]));
        ST_TRY(dots<T>(o, 2, v[V_P], v[V_PHI], v[V_ZP], v[V_P], nullptr, nullptr, w));
        ST_TRY(lincomb<T>(o, v[V_P], 1.0, v[V_P], -w[0] / pp, v[V_PHI]));   // H_T p
        const double pAp = w[1];   // p is orthogonal to phi
        if (!(pAp > 0)) {
            if (j == 0) ST_TRY(lincomb<T>(o, v[V_D], 1.0, v[V_ZP], 0.0, nullptr));
            break;
        }
        const double alpha = rz / pAp;
        ST_TRY(lincomb<T>(o, v[V_D], 1.0, v[V_D], alpha, v[V_ZP]));
        ST_TRY(lincomb<T>(o, v[V_RP], 1.0, v[V_RP], -alpha, v[V_P]));
        ST_TRY(dots<T>(o, 1, v[V_RP], v[V_RP], nullptr, nullptr, nullptr, nullptr, w));
        if (std::sqrt(w[0]) <= eta * std::sqrt(rr0)) break;
        ST_TRY(precondition<T>(o, v[V_RP], v[V_Z]));
        ST_TRY(dots<T>(o, 1, v[V_Z], v[V_PHI], nullptr, nullptr, nullptr, nullptr, w));
        ST_TRY(lincomb<T>(o, v[V_Z], 1.0, v[V_Z], -w[0] / pp, v[V_PHI]));
        ST_TRY(dots<T>(o, 1, v[V_RP], v[V_Z], nullptr, nullptr, nullptr, nullptr, w));
        const double beta = w[0] / rz;
        rz = w[0];
        ST_TRY(lincomb<T>(o, v[V_ZP], 1.0, v[V_Z], beta, v[V_ZP]));
    }
    return OFDFT_OK;
}

template <typename T>
static ofdft_status optimize_impl(ofdft_grid *g, const ofdft_opt_params *prm, ofdft_opt_result *res)
{
    hipStream_t s = g->opt_stream ? g->opt_stream : g->ctx->stream;
    const Geom &G = g->geom;
    OptState o{g, s, G.N};
    ST_TRY(reserve(g, 1));
    for (int i = 0; i < NVEC; ++i) ST_TRY(dmalloc(g, &g->opt[i], (size_t)G.N * sizeof(T)));
    void **v = g->opt;
    const double dv = g->dv, ne = g->nelec;
    const int max_iter = prm->max_iter;
    const double tol = prm->tol;
    const bool tn = prm->method == OFDFT_OPT_TN;
    const bool precond = prm->method == OFDFT_OPT_PCG || tn;
    // The line search brackets and refines a root of dE/dtheta = <g, dphi/dtheta>
    // without comparing energies (a) when the potential is not the derivative
    // of the energy: the S3S4 spline potential interpolates per-knot
    // potentials, and the search then solves the Euler equation along the
    // line; (b) on the mixed path, where energy differences near convergence
    // fall below the FP32 rounding of the large Hartree and electron-ion
    // terms while the FP64 dot products of the derivative stay reliable.
    const bool deriv_only =
        !g->fp64 || ((g->func.terms & OFDFT_TERM_SPLINE) && g->func.nl_mode == OFDFT_NL_S3S4);
    std::memset(res, 0, sizeof(*res));

    // phi = sqrt(rho_resident), normalised to N_e
    TIMED(PS_OTHER, launch_pointwise<T>(G.N, PW_SQRT, v[V_PHI], g->rho, s));
    double pp;
    ST_TRY(dots<T>(o, 1, v[V_PHI], v[V_PHI], nullptr, nullptr, nullptr, nullptr, &pp));
    if (!(pp > 0)) return fail(OFDFT_EINVAL, "resident density is zero");
    ST_TRY(lincomb<T>(o, v[V_PHI], std::sqrt(ne / (dv * pp)), v[V_PHI], 0.0, nullptr));

    ofdft_energy E;
    ST_TRY(opt_eval(g, v[V_PHI], v[V_G], s, &E));
    int evals = 1, iter = 0;
    bool have_prev = false, converged = false;
    double kappa = -1.0, theta_prev = -1.0;
    const double c1 = 1e-4, c2 = 0.1;
    for (iter = 0; iter < max_iter; ++iter) {
        if (E.resid_norm < tol) {
            converged = true;
            break;
        }
        if (g->cancel && g->cancel->load(std::memory_order_relaxed))
            return fail(OFDFT_ECANCELLED, "optimisation cancelled");
        // R = g - 2 mu phi; z = K R with the preconditioner, else z = R
        ST_TRY(lincomb<T>(o, v[V_R], 1.0, v[V_G], -2.0 * E.mu, v[V_PHI]));
        const int Z = precond ? V_Z : V_R, ZP = precond ? V_ZP : V_RP;
        if (precond) ST_TRY(precondition<T>(o, v[V_R], v[V_Z]));
        double dd[3];
        if (tn) {
            ST_TRY(tn_direction<T>(o, v, E, evals));
        } else if (have_prev) {
            // Polak-Ribiere+: beta = max(0, <z, R - R_prev> / <z_prev, R_prev>)
            ST_TRY(dots<T>(o, 3, v[Z], v[V_R], v[Z], v[V_RP], v[ZP], v[V_RP], dd));
            const double beta = std::max(0.0, (dd[0] - dd[1]) / dd[2]);
            ST_TRY(lincomb<T>(o, v[V_D], -1.0, v[Z], beta, v[V_D]));
        } else {
            ST_TRY(lincomb<T>(o, v[V_D], -1.0, v[Z], 0.0, nullptr));
        }
        double q[3];
        for (int attempt = 0; attempt < 2; ++attempt) {
            ST_TRY(dots<T>(o, 3, v[V_D], v[V_R], v[V_D], v[V_PHI], v[V_PHI], v[V_PHI], q));
            if (q[0] >= 0.0 && attempt == 0) {   // not a descent direction: restart
                if (tn) ST_TRY(precondition<T>(o, v[V_R], v[V_Z]));   // TN used V_Z
                ST_TRY(lincomb<T>(o, v[V_D], -1.0, v[Z], 0.0, nullptr));
                continue;
            }
            break;
        }
        // p = d - (<d,phi>/<phi,phi>) phi, scaled to <p,p> dv = N_e
        ST_TRY(lincomb<T>(o, v[V_P], 1.0, v[V_D], -q[1] / q[2], v[V_PHI]));
        double pq[2];
        ST_TRY(dots<T>(o, 2, v[V_P], v[V_P], v[V_G], v[V_P], nullptr, nullptr, pq));
        if (!(pq[0] > 0)) break;
        const double sc = std::sqrt(ne / (dv * pq[0]));
        ST_TRY(lincomb<T>(o, v[V_P], sc, v[V_P], 0.0, nullptr));
        const double d0 = dv * pq[1] * sc;   // dE/dtheta at 0
        if (!(d0 < 0)) break;

        double theta0 = (kappa > 0) ? std::min(1.0, std::max(1e-12, -d0 / kappa))
                                    : (theta_prev > 0 ? theta_prev : 0.1);
        // TN: the Newton step phi + d is theta = |P d| / |phi| along the rotation
        if (tn) theta0 = std::min(1.0, std::max(1e-12, std::sqrt(pq[0] / q[2])));
        const double f0 = E.e_total;
        // energy differences below the evaluation's rounding level are not
        // trusted: there the search accepts on the derivative conditions
        const double eps_f = (g->fp64 ? 1e-14 : 1e-8) * std::max(1.0, std::fabs(f0));
        // trial evaluation at theta: phi_t = phi cos + p sin; returns E and dE/dtheta
        double last_theta = -1.0;
        ofdft_energy Et;
        auto trial = [&](double th, double &f, double &df) -> ofdft_status {
            ST_TRY(lincomb<T>(o, v[V_PT], std::cos(th), v[V_PHI], std::sin(th), v[V_P]));
            ST_TRY(opt_eval(g, v[V_PT], v[V_GT], s, &Et));
            ++evals;
            double gd[2];
            ST_TRY(dots<T>(o, 2, v[V_GT], v[V_PHI], v[V_GT], v[V_P], nullptr, nullptr, gd));
            f = Et.e_total;
            df = dv * (-std::sin(th) * gd[0] + std::cos(th) * gd[1]);
            last_theta = th;
            return OFDFT_OK;
        };
        auto decrease_ok = [&](double a, double fa, double da) {
            if (deriv_only) return true;
            return fa <= f0 + c1 * a * d0 || (fa <= f0 + eps_f && da <= (2 * c1 - 1) * d0);
        };
        // next trial inside (lo, hi): cubic interpolation of (f, df), or the
        // secant on df when energies are not compared
        auto interp = [&](double a0, double f0_, double d0_, double a1, double f1, double d1,
                          bool &ok) {
            if (!deriv_only) return cubic_min(a0, f0_, d0_, a1, f1, d1, ok);
            ok = d1 != d0_;
            return ok ? a0 - d0_ * (a1 - a0) / (d1 - d0_) : 0.0;
        };
        double best_d = 1e300;
        // strong-Wolfe search: bracket, then zoom with safeguarded cubic steps
        double a_lo = 0.0, f_lo = f0, d_lo = d0, a_hi = 0, f_hi = 0, d_hi = 0;
        double a = theta0, best_a = -1, best_f = 1e300;
        bool done = false, zoom = false;
        int budget = 20;
        double fa = 0, da = 0;
        auto note_best = [&](double a_, double f_, double d_) {
            if (deriv_only ? std::fabs(d_) < best_d : f_ < best_f) {
                best_f = f_;
                best_d = std::fabs(d_);
                best_a = a_;
            }
        };
        for (int k = 0; k < budget && !done && !zoom; ++k) {
            ST_TRY(trial(a, fa, da));
            note_best(a, fa, da);
            if (!decrease_ok(a, fa, da) || (!deriv_only && k > 0 && fa > f_lo + eps_f)) {
                a_hi = a; f_hi = fa; d_hi = da; zoom = true; break;
            }
            if (std::fabs(da) <= -c2 * d0) { done = true; break; }
            if (da >= 0) {
                a_hi = a_lo; f_hi = f_lo; d_hi = d_lo;
                a_lo = a; f_lo = fa; d_lo = da;
                zoom = true;
                break;
            }
            bool ok;
            double an = interp(a_lo, f_lo, d_lo, a, fa, da, ok);
            if (!ok || an <= a * 1.1 || an > a * 4.0) an = 2.0 * a;
            a_lo = a; f_lo = fa; d_lo = da;
            a = an;
        }
        if (zoom) {
            for (int k = 0; k < budget && !done; ++k) {
                const double lo = std::min(a_lo, a_hi), hi = std::max(a_lo, a_hi);
                bool ok;
                double an = interp(a_lo, f_lo, d_lo, a_hi, f_hi, d_hi, ok);
                if (!ok || !(an > lo && an < hi)) an = 0.5 * (a_lo + a_hi);
                else an = std::min(std::max(an, lo + 0.01 * (hi - lo)), hi - 0.01 * (hi - lo));
                a = an;
                ST_TRY(trial(a, fa, da));
                note_best(a, fa, da);
                if (!decrease_ok(a, fa, da) || (!deriv_only && fa > f_lo + eps_f)) {
                    a_hi = a; f_hi = fa; d_hi = da;
                } else {
                    if (std::fabs(da) <= -c2 * d0) { done = true; break; }
                    if (da * (a_hi - a_lo) >= 0) { a_hi = a_lo; f_hi = f_lo; d_hi = d_lo; }
                    a_lo = a; f_lo = fa; d_lo = da;
                }
            }
        }
        if (!done) {
            // fall back to the best point seen
            if (!deriv_only && !(best_f <= f0 + eps_f)) break;
            if (deriv_only && !(best_d < std::fabs(d0))) break;
            if (best_a != last_theta) ST_TRY(trial(best_a, fa, da));
            a = best_a;
        }
        kappa = (da - d0) / a;
        theta_prev = a;
        // accept: phi <- phi_t, g <- g_t, R_prev <- R
        std::swap(v[V_PHI], v[V_PT]);
        std::swap(v[V_G], v[V_GT]);
        std::swap(v[V_R], v[V_RP]);
        if (precond) std::swap(v[V_Z], v[V_ZP]);
        have_prev = true;
        E = Et;
    }
    if (!converged && E.resid_norm < tol) converged = true;
    // leave the optimised density resident: rho = phi^2
    TIMED(PS_OTHER, launch_pointwise<T>(G.N, PW_SQUARE, g->rho, v[V_PHI], s));
    HIP_TRY(hipStreamSynchronize(s));
    g->rho_set = true;
    res->e = E;
    res->iters = iter;
    res->evals = evals;
    res->final_resid = E.resid_norm;
    if (!converged) return fail(OFDFT_ENOCONV, "optimisation did not reach the tolerance");
    return OFDFT_OK;
}

// Multi-step optimisation (Section "Density optimization strategies"): the
// resident density of dst from that of src, by Fourier interpolation of
// phi = sqrt(rho) onto dst's grid (at least as fine on every axis), squared
// and scaled to dst's electron count.  Runs on src's stream; both grids are
// idle when it returns.
template <typename T>
static ofdft_status interp_impl(ofdft_grid *dst, ofdft_grid *src)
{
    hipStream_t s = src->ctx->stream;
    const Geom &Gs = src->geom, &Gd = dst->geom;
    HIP_TRY(hipStreamSynchronize(dst->ctx->stream));
    ST_TRY(dmalloc(src, &src->opt[V_PHI], (size_t)Gs.N * sizeof(T)));
    ST_TRY(dmalloc(dst, &dst->opt[V_PHI], (size_t)Gd.N * sizeof(T)));
    ST_TRY(dmalloc(dst, &dst->rho, (size_t)Gd.N * sizeof(T)));
    ofdft_grid *g = src;   // per-pass timing of the src grid
    TIMED(PS_OTHER, launch_pointwise<T>(Gs.N, PW_SQRT, src->opt[V_PHI], src->rho, s));
    ST_TRY(fft_impl<T>(src, 1, src->opt[V_PHI], src->spec, true, s));
    // the padded spectrum goes to dst's workspace slot 1; the inverse copies
    // it to slot 0 and transforms there
    void *slot1 = (char *)dst->spec + (size_t)Gd.Nh * 2 * sizeof(T);
    TIMED(PS_OTHER, launch_interp_spec<T>(Gs, Gd, src->spec, slot1, s));
    ST_TRY(fft_impl<T>(dst, 1, slot1, dst->opt[V_PHI], false, s));
    OptState o{dst, s, Gd.N};
    double pp = 0.0;
    ST_TRY(dots<T>(o, 1, dst->opt[V_PHI], dst->opt[V_PHI], nullptr, nullptr, nullptr, nullptr, &pp));
    if (!(pp > 0)) return fail(OFDFT_EINVAL, "interpolated density is zero");
    ST_TRY(lincomb<T>(o, dst->opt[V_PHI], std::sqrt(dst->nelec / (dst->dv * pp)), dst->opt[V_PHI],
                      0.0, nullptr));
    g = dst;
    TIMED(PS_OTHER, launch_pointwise<T>(Gd.N, PW_SQUARE, dst->rho, dst->opt[V_PHI], s));
    HIP_TRY(hipStreamSynchronize(s));
    dst->rho_set = true;
    return OFDFT_OK;
}

static ofdft_status interpolate_density(ofdft_grid *dst, ofdft_grid *src)
{
    if (!dst || !src) return fail(OFDFT_EINVAL, "null grid");
    if (dst == src) return fail(OFDFT_EINVAL, "source and destination are the same grid");
    if (src->ctx->device != dst->ctx->device)
        return fail(OFDFT_EINVAL, "grids on different devices");
    if (src->fp64 != dst->fp64) return fail(OFDFT_EINVAL, "grids of different precision");
    for (int i = 0; i < 3; ++i) {
        if (dst->n[i] < src->n[i])
            return fail(OFDFT_EINVAL, "destination grid coarser than the source on an axis");
        for (int j = 0; j < 3; ++j)
            if (std::fabs(dst->lattice[i][j] - src->lattice[i][j]) >
                1e-12 * (1.0 + std::fabs(src->lattice[i][j])))
                return fail(OFDFT_EINVAL, "grids of different cells");
    }
    if (!src->rho_set) return fail(OFDFT_EINVAL, "source grid has no resident density");
    HIP_TRY(hipSetDevice(src->ctx->device));
    graphs_clear(dst);
    return src->fp64 ? interp_impl<double>(dst, src) : interp_impl<float>(dst, src);
}

// ================================================================ autotuner
// The launch schedule of an evaluation has free choices: the fused plane
// kernels or separate row and column passes (where the plane fits in LDS),
// the block order of the column passes, densities per column block, the
// number of spline knots per batch and the knot pipeline.  The tuner times
// every combination on the caller's batch, then, on the fastest, the shapes
// the reciprocal-space column pass offers for its length (half the columns
// per block, the reversed radix order, both), and keeps the fastest; results
// are shared by all grids of the same shape, precision, functional and batch
// size in the process.
struct TuneVal {
    int plane, tile_major, kb, pipe, cgrp, kpipe, cvar;
};
using TuneKey = std::tuple<int, int, int, int, uint32_t, int, int, int>;
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneVal> g_tune_cache;

static TuneKey tune_key(const ofdft_grid *g, int nb)
{
    return TuneKey(g->n[0], g->n[1], g->n[2], g->func.precision,
                   g->func.terms | ((uint32_t)g->func.nl_kernel << 16), g->func.nl_mode,
                   (g->func.terms & OFDFT_TERM_SPLINE) ? g->func.nk : 0, nb);
}

static void tune_apply_cached(ofdft_grid *g, int nb)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(tune_key(g, nb));
    if (it == g_tune_cache.end()) return;
    g->tune_plane = it->second.plane;
    g->tune_col_tile_major = it->second.tile_major;
    g->tune_kb = it->second.kb;
    g->tune_pipe = it->second.pipe;
    g->tune_col_group = it->second.cgrp;
    g->tune_knot_pipe = it->second.kpipe;
    g->tune_col_variant = it->second.cvar;
    graphs_clear(g);
}

static ofdft_status eval_dispatch(ofdft_grid *g, int nb, const void *d_in, int in_is_phi,
                                  void *d_v, void *d_g, hipStream_t s, ofdft_energy *e_out);

static ofdft_status tune_impl(ofdft_grid *g, int nb, const void *d_in, hipStream_t s,
                              ofdft_tune_result *out)
{
    ST_TRY(reserve(g, nb));
    const bool plane_ok = g->fp64 ? plane_supported<double>(g->geom.n1, g->geom.m)
                                  : plane_supported<float>(g->geom.n1, g->geom.m);
    const bool spline = g->func.terms & OFDFT_TERM_SPLINE;
    std::vector<TuneVal> cand;
    for (int pl : {1, 0}) {
        if (!pl && !plane_ok) continue;
        for (int tm : {0, 1})
            for (int kb : {MAXKB, MAXKB / 2})
                for (int cg : {COL_GROUP, 1})
                    for (int kp : {1, 0})
                        if ((spline || kb == MAXKB) && (nb > 1 || cg == COL_GROUP) &&
                            (g->kspec2 || kp == 1))
                            cand.push_back({pl, tm, kb, g->tune_pipe, cg, kp});
    }
    std::vector<ofdft_energy> e((size_t)nb);
    auto apply = [&](const TuneVal &c) {
        g->tune_plane = c.plane;
        g->tune_col_tile_major = c.tile_major;
        g->tune_kb = c.kb;
        g->tune_pipe = c.pipe;
        g->tune_col_group = c.cgrp;
        g->tune_knot_pipe = c.kpipe;
        g->tune_col_variant = c.cvar;
        graphs_clear(g);
    };
    // median of three timed calls after one warm-up
    auto time_of = [&](const TuneVal &c, double &ms) -> ofdft_status {
        apply(c);
        ST_TRY(eval_dispatch(g, nb, d_in, 0, nullptr, nullptr, s, e.data()));
        double t[3];
        for (double &x : t) {
            const auto t0 = std::chrono::steady_clock::now();
            ST_TRY(eval_dispatch(g, nb, d_in, 0, nullptr, nullptr, s, e.data()));
            x = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
        std::sort(t, t + 3);
        ms = t[1];
        return OFDFT_OK;
    };
    double best = 1e300, dflt = 0.0;
    TuneVal pick = cand[0];
    for (size_t c = 0; c < cand.size(); ++c) {
        double ms;
        ST_TRY(time_of(cand[c], ms));
        if (c == 0) dflt = ms;
        if (ms < best) {
            best = ms;
            pick = cand[c];
        }
    }
    // the column pass's shapes, on the fastest schedule; a shape replaces
    // the default one only if it is faster by TUNE_SHAPE_MARGIN (short
    // calls time within a few percent of each other, and a shape picked on
    // noise alone measured slower under concurrent streams)
    constexpr double TUNE_SHAPE_MARGIN = 0.97;
    const int vm = g->fp64 ? col_variants<double>(g->geom.n0) : col_variants<float>(g->geom.n0);
    int ncand = (int)cand.size();
    const TuneVal base = pick;
    const double base_ms = best;
    for (int v = 1; v <= 3; ++v) {
        if ((v & vm) != v) continue;
        TuneVal c = base;
        c.cvar = v;
        double ms;
        ST_TRY(time_of(c, ms));
        ++ncand;
        if (ms < best && ms < base_ms * TUNE_SHAPE_MARGIN) {
            best = ms;
            pick = c;
        }
    }
    apply(pick);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[tune_key(g, nb)] = pick;
    }
    if (out) {
        out->plane = pick.plane;
        out->col_tile_major = pick.tile_major;
        out->knot_batch = pick.kb;
        out->candidates = (int32_t)ncand;
        out->best_ms = best;
        out->default_ms = dflt;
        out->pipe = pick.pipe;
        out->col_group = pick.cgrp;
        out->knot_pipe = pick.kpipe;
        out->col_variant = pick.cvar;
    }
    return OFDFT_OK;
}

// ================================================================ internal
namespace ofdft_internal {

ofdft_status set_positions(ofdft_grid *g, const double *pos)
{
    if (!g || (g->natoms > 0 && !pos)) return fail(OFDFT_EINVAL, "null argument");
    for (int i = 0; i < 3 * g->natoms; ++i)
        if (!std::isfinite(pos[i])) return fail(OFDFT_EINVAL, "non-finite position");
    HIP_TRY(hipSetDevice(g->ctx->device));
    g->pos.assign(pos, pos + 3 * (size_t)g->natoms);
    return setup_ions(g);
}

void bind_context(ofdft_grid *g, ofdft_ctx *ctx) { g->ctx = ctx; }

void set_cancel(ofdft_grid *g, const std::atomic<int> *flag) { g->cancel = flag; }

void set_error(const std::string &msg) { g_last_error = msg; }

int ctx_device(const ofdft_ctx *ctx) { return ctx->device; }

bool has_tuning(const ofdft_grid *g)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune_cache.count(tune_key(g, 1)) > 0;
}

uint64_t multi_growth_bytes(const ofdft_grid *g, int n)
{
    uint64_t grow = 0;
    if (n > g->cap) grow += workspace_bytes(g, n) - (g->cap > 0 ? workspace_bytes(g, g->cap) : 0);
    if (n > g->batch_cap) {
        const uint64_t staging = (uint64_t)n * (2ull * g->geom.N * g->fsz + sizeof(CellTab));
        if (staging > g->multi_bytes) grow += staging - g->multi_bytes;
    }
    return grow;
}

}  // namespace ofdft_internal


// ---------------------------------------------------------------- TD-OFDFT
// Real-time propagation of the collective orbital (Section "Time-Dependent
// OFDFT"): i d psi/dt = H psi with H = -(1/2) nabla^2 + v, v the functional
// derivative of every term but von Weizsaecker (dT_Pauli/drho + v_s of eq.
// "heq", adiabatic), Crank-Nicolson steps (eq. "cn", with the signs of the
// time-dependent equation: (1 + i dt/2 H) psi(t+dt) = (1 - i dt/2 H) psi(t))
// solved by BiCGSTAB, and corrector passes that rebuild H from the midpoint
// density (rho(t) + |psi_trial|^2) / 2.
enum { TV_PSI = 0, TV_TRIAL, TV_B, TV_R, TV_RH, TV_P, TV_V, TV_S, TV_T, TV_KIN, NTV };
struct TdBufs {
    void *vec[NTV];          // split complex vectors, 2N values each
    void *rho_n, *rho, *veff;  // real fields, N values each
    void *spec;              // two half spectra, 2 Nh complex
};
static uint64_t td_bytes(const Geom &G, size_t fsz)
{
    return ((uint64_t)NTV * 2 * G.N + 3 * (uint64_t)G.N + 4 * (uint64_t)G.Nh) * fsz;
}
static TdBufs td_bufs(ofdft_grid *g)
{
    const Geom &G = g->geom;
    char *p = static_cast<char *>(g->td);
    TdBufs b;
    for (int k = 0; k < NTV; ++k) {
        b.vec[k] = p;
        p += 2 * (size_t)G.N * g->fsz;
    }
    b.rho_n = p;
    p += (size_t)G.N * g->fsz;
    b.rho = p;
    p += (size_t)G.N * g->fsz;
    b.veff = p;
    p += (size_t)G.N * g->fsz;
    b.spec = p;
    return b;
}
static const void *im_part(const ofdft_grid *g, const void *x)
{
    return static_cast<const char *>(x) + (size_t)g->geom.N * g->fsz;
}

// complex dot products <a, b> = sum conj(a) b over the split vectors
template <typename T>
static ofdft_status td_cdot(ofdft_grid *g, hipStream_t s, const void *a, const void *b,
                            std::complex<double> *out)
{
    int nbk = 0;
    const void *ai = im_part(g, a), *bi = im_part(g, b);
    HIP_TRY(launch_dots<T>(g->geom.N, 4, a, b, ai, bi, a, bi, ai, b, g->part, g->pstride, nbk, s));
    SlotCounts cnt;
    std::memset(&cnt, 0, sizeof(cnt));
    for (int d = 0; d < 4; ++d) cnt.n[SL_AUX0 + d] = nbk;
    HIP_TRY(launch_finalize(g->part, g->pstride, cnt, 1, g->sums, s));
    HIP_TRY(hipMemcpyAsync(g->h_sums, g->sums, NSLOT * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const double *h = g->h_sums + SL_AUX0;
    *out = {h[0] + h[1], h[2] - h[3]};
    return OFDFT_OK;
}

template <typename T>
static hipError_t td_lin(ofdft_grid *g, hipStream_t s, void *z, std::complex<double> a,
                         const void *x, std::complex<double> b = 0.0, const void *y = nullptr,
                         std::complex<double> c = 0.0, const void *w = nullptr)
{
    const double ca[2] = {a.real(), a.imag()}, cb[2] = {b.real(), b.imag()},
                 cc[2] = {c.real(), c.imag()};
    return launch_td_zlincomb<T>(g->geom.N, z, ca, x, cb, y, cc, w, s);
}

// out = c(G) x for a diagonal operator of the complex field (TD_KIN: the
// kinetic operator; TD_K / TD_KINV: 1 + i tau G^2/2 and its inverse), through
// the forward and inverse transforms of the two parts (no host wait)
template <typename T>
static ofdft_status td_kapply(ofdft_grid *g, const TdBufs &B, hipStream_t s, const void *x,
                              void *out, double tau, int mode)
{
    const Geom &G = g->geom;
    ST_TRY(fft_impl<T>(g, 2, x, B.spec, true, s, false));
    const void *g2 = static_cast<const char *>(g->gtab) + (size_t)G.Nh * g->fsz;
    HIP_TRY(launch_td_spectral<T>(G, B.spec, g2, tau, mode, s));
    ST_TRY(fft_impl<T>(g, 2, B.spec, out, false, s, false, true));   // B.spec is scratch
    return OFDFT_OK;
}

// out = x + i tau H x with the potential in veff (tau = +-dt/2)
template <typename T>
static ofdft_status td_apply(ofdft_grid *g, const TdBufs &B, hipStream_t s, const void *x,
                             void *out, double tau)
{
    ST_TRY(td_kapply<T>(g, B, s, x, B.vec[TV_KIN], tau, TD_KIN));
    HIP_TRY(launch_td_apply<T>(g->geom.N, x, B.vec[TV_KIN], B.veff, tau, out, s));
    return OFDFT_OK;
}

// out = A K^-1 z = z + i tau veff (K^-1 z), K = 1 + i tau G^2/2: the system
// matrix A = K + i tau veff right-preconditioned with its kinetic part (one
// transform pair per product, as for A itself)
template <typename T>
static ofdft_status td_apply_pc(ofdft_grid *g, const TdBufs &B, hipStream_t s, const void *z,
                                void *out, double tau)
{
    ST_TRY(td_kapply<T>(g, B, s, z, B.vec[TV_KIN], tau, TD_KINV));
    HIP_TRY(launch_td_pc_apply<T>(g->geom.N, z, B.vec[TV_KIN], B.veff, tau, out, s));
    return OFDFT_OK;
}

// veff = v[rho] of every term but vW (the grid's functional otherwise)
template <typename T>
static ofdft_status td_potential(ofdft_grid *g, const TdBufs &B, hipStream_t s, const void *rho)
{
    const uint32_t terms = g->func.terms;
    const bool graphs = g->use_graphs;
    graphs_clear(g);
    g->use_graphs = false;
    g->func.terms = terms & ~(uint32_t)OFDFT_TERM_VW;
    ofdft_energy e;
    ofdft_status st = eval_dispatch(g, 1, rho, 0, B.veff, nullptr, s, &e);
    g->func.terms = terms;
    g->use_graphs = graphs;
    return st;
}

// (1 + i tau H) x = b by BiCGSTAB on A K^-1 y = b, x = K^-1 y (right
// preconditioning with the kinetic part K = 1 + i tau G^2/2, exact in
// reciprocal space): the residual b - A x is the unpreconditioned one, and
// the iteration starts from the guess in x.  The scalars stay on the device
// (k_td_scalars after each pair of dot products; the linear combinations
// read their coefficients there and stop once the solve is done), and the
// host reads them once per iteration to decide whether to go on.  Each
// iteration runs in full (no exit after its first half-step): a residual
// that vanishes there gives omega = 0 and r = s, and the solve ends at the
// iteration's end.
template <typename T>
static ofdft_status td_solve(ofdft_grid *g, const TdBufs &B, hipStream_t s, double tau,
                             const void *b, void *x, int maxit, double tol, int *iters,
                             double *relres)
{
    void *r = B.vec[TV_R], *rh = B.vec[TV_RH], *p = B.vec[TV_P], *v = B.vec[TV_V],
         *sv = B.vec[TV_S], *t = B.vec[TV_T];
    const long long N = g->geom.N;
    double *sc = g->d_td_sc, *part = g->d_td_dots, *h = g->h_td_sc;
    void *y = x;                                   // y = K x, in place
    ST_TRY(td_kapply<T>(g, B, s, x, y, tau, TD_K));
    ST_TRY(td_apply_pc<T>(g, B, s, y, t, tau));
    HIP_TRY(td_lin<T>(g, s, r, 1.0, b, -1.0, t));
    HIP_TRY(td_lin<T>(g, s, rh, 1.0, r));
    HIP_TRY(hipMemsetAsync(p, 0, 2 * (size_t)N * g->fsz, s));
    HIP_TRY(hipMemsetAsync(v, 0, 2 * (size_t)N * g->fsz, s));
    h[TS_TOL] = tol;
    h[TS_MAXIT] = maxit;
    HIP_TRY(hipMemcpyAsync(sc + TS_TOL, h + TS_TOL, 2 * sizeof(double), hipMemcpyHostToDevice, s));
    HIP_TRY(launch_td_cdots<T>(N, b, b, r, r, part, s));
    HIP_TRY(launch_td_scalars(TD_STEP_INIT, N, part, sc, s));
    auto read = [&]() -> ofdft_status {
        HIP_TRY(hipMemcpyAsync(h, sc, TS_N * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        return OFDFT_OK;
    };
    ST_TRY(read());
    while (h[TS_DONE] == 0.0) {
        HIP_TRY(launch_td_cdots<T>(N, rh, r, nullptr, nullptr, part, s));
        HIP_TRY(launch_td_scalars(TD_STEP_RHO, N, part, sc, s));
        HIP_TRY(launch_td_zlincomb_dev<T>(N, p, sc, TS_CP, r, p, v, s));
        ST_TRY(td_apply_pc<T>(g, B, s, p, v, tau));
        HIP_TRY(launch_td_cdots<T>(N, rh, v, nullptr, nullptr, part, s));
        HIP_TRY(launch_td_scalars(TD_STEP_RV, N, part, sc, s));
        HIP_TRY(launch_td_zlincomb_dev<T>(N, sv, sc, TS_CS, r, v, nullptr, s));
        ST_TRY(td_apply_pc<T>(g, B, s, sv, t, tau));
        HIP_TRY(launch_td_cdots<T>(N, t, sv, t, t, part, s));
        HIP_TRY(launch_td_scalars(TD_STEP_OMEGA, N, part, sc, s));
        HIP_TRY(launch_td_zlincomb_dev<T>(N, y, sc, TS_CY, y, p, sv, s));
        HIP_TRY(launch_td_zlincomb_dev<T>(N, r, sc, TS_CR, sv, t, nullptr, s));
        HIP_TRY(launch_td_cdots<T>(N, r, r, nullptr, nullptr, part, s));
        HIP_TRY(launch_td_scalars(TD_STEP_RR, N, part, sc, s));
        ST_TRY(read());
    }
    ST_TRY(td_kapply<T>(g, B, s, y, x, tau, TD_KINV));   // x = K^-1 y
    *iters = (int)h[TS_IT];
    *relres = h[TS_RES];
    return OFDFT_OK;
}

template <typename T>
static ofdft_status td_dipole(ofdft_grid *g, const TdBufs &B, hipStream_t s, const void *rho,
                              double mu[3])
{
    TdLattice L;
    for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) L.a[3 * i + c] = g->lattice[i][c];
    const int nb = td_dipole_blocks(g->geom);
    HIP_TRY(launch_td_dipole<T>(g->geom, L, rho, g->d_td_part, s));
    std::vector<double> h(3 * (size_t)nb);
    HIP_TRY(hipMemcpyAsync(h.data(), g->d_td_part, h.size() * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int k = 0; k < nb; ++k) acc += h[3 * (size_t)k + c];
        mu[c] = acc * g->dv;
    }
    return OFDFT_OK;
}

static ofdft_status td_alloc(ofdft_grid *g)
{
    ST_TRY(reserve(g, 2));
    ST_TRY(dmalloc(g, &g->td, td_bytes(g->geom, g->fsz)));
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_td_part),
                   3 * (size_t)td_dipole_blocks(g->geom) * sizeof(double)));
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_td_dots),
                   4 * (size_t)td_dot_blocks(g->geom.N) * sizeof(double)));
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_td_sc), TS_N * sizeof(double)));
    if (!g->h_td_sc) HIP_TRY(hipHostMalloc((void **)&g->h_td_sc, TS_N * sizeof(double)));
    return OFDFT_OK;
}

template <typename T>
static ofdft_status td_start_impl(ofdft_grid *g, const double k[3])
{
    hipStream_t s = g->ctx->stream;
    if (!g->rho_set) return fail(OFDFT_EINVAL, "the grid has no resident density");
    ST_TRY(td_alloc(g));
    const TdBufs B = td_bufs(g);
    TdLattice L;
    for (int i = 0; i < 3; ++i)
        for (int c = 0; c < 3; ++c) L.a[3 * i + c] = g->lattice[i][c];
    HIP_TRY(launch_td_kick<T>(g->geom, L, k, g->rho, B.vec[TV_PSI], s));
    HIP_TRY(hipStreamSynchronize(s));
    return OFDFT_OK;
}

template <typename T>
static ofdft_status td_propagate_impl(ofdft_grid *g, const ofdft_td_params *prm, int nsteps,
                                      double *mu_out, ofdft_td_stats *st)
{
    hipStream_t s = g->ctx->stream;
    const TdBufs B = td_bufs(g);
    const Geom &G = g->geom;
    const double tau = 0.5 * prm->dt;
    const double tol = prm->solver_tol > 0 ? prm->solver_tol : (g->fp64 ? 1e-11 : 1e-6);
    const int maxit = prm->max_solver_iter > 0 ? prm->max_solver_iter : 200;
    std::memset(st, 0, sizeof(*st));
    for (int n = 0; n < nsteps; ++n) {
        void *psi = B.vec[TV_PSI], *trial = B.vec[TV_TRIAL], *b = B.vec[TV_B];
        HIP_TRY(launch_td_density<T>(G.N, psi, 1.0, nullptr, 0.0, B.rho_n, s));
        const void *rho_h = B.rho_n;
        for (int c = 0; c <= prm->n_corrector; ++c) {
            if (c > 0) {
                HIP_TRY(launch_td_density<T>(G.N, psi, 0.5, trial, 0.5, B.rho, s));
                rho_h = B.rho;
            }
            ST_TRY(td_potential<T>(g, B, s, rho_h));
            ST_TRY(td_apply<T>(g, B, s, psi, b, -tau));                  // (1 - i tau H) psi
            if (c == 0) HIP_TRY(td_lin<T>(g, s, trial, 1.0, psi));       // guess: psi(t)
            int it = 0;
            double res = 0.0;
            ST_TRY(td_solve<T>(g, B, s, tau, b, trial, maxit, tol, &it, &res));
            st->solver_iters += it;
            st->max_solver_resid = std::max(st->max_solver_resid, res);
            if (res > tol) st->unconverged_solves++;
        }
        HIP_TRY(td_lin<T>(g, s, psi, 1.0, trial));
        HIP_TRY(launch_td_density<T>(G.N, psi, 1.0, nullptr, 0.0, B.rho, s));
        if (mu_out) ST_TRY(td_dipole<T>(g, B, s, B.rho, mu_out + 3 * (size_t)n));
        st->steps++;
    }
    std::complex<double> nn;
    ST_TRY(td_cdot<T>(g, s, B.vec[TV_PSI], B.vec[TV_PSI], &nn));
    st->nelec = nn.real() * g->dv;
    return OFDFT_OK;
}

// ================================================================ C ABI
// ---------------------------------------------------------------- multi-cell batches
// Whether two grids can share a launch sequence: the same grid shape,
// functional (every field) and device.  The cells may differ (lattice, atoms,
// electron count): the reciprocal-space pass and the knot kernels take each
// entry's own reciprocal vectors and tables.
static bool batchable(const ofdft_grid *a, const ofdft_grid *b)
{
    const ofdft_functional_desc &x = a->func, &y = b->func;
    return a->ctx->device == b->ctx->device && a->n[0] == b->n[0] && a->n[1] == b->n[1] &&
           a->n[2] == b->n[2] && x.terms == y.terms && x.lambda_vw == y.lambda_vw &&
           x.alpha == y.alpha && x.beta == y.beta && x.nk == y.nk && x.kf_min == y.kf_min &&
           x.kf_max == y.kf_max && x.knot_spacing == y.knot_spacing && x.nl_mode == y.nl_mode &&
           x.precision == y.precision && x.rho_floor == y.rho_floor && x.nl_kernel == y.nl_kernel;
}

// One evaluation of n cells' densities, led by grids[0], whose workspace,
// twiddles and schedule serve the whole batch, on stream s.  Inputs: in[b]
// (device, the grid's field type; rho, or phi with in_is_phi) or, with in
// null, each grid's resident density.  Outputs: potentials copied to the host
// (v_host[b] not null) or dE/dphi to device arrays (g_dev[b] not null).  The
// caller has finished all work on the inputs.
template <typename T>
static ofdft_status eval_multi_core(ofdft_grid *const *grids, int n, const void *const *in,
                                    int in_is_phi, double *const *v_host, void *const *g_dev,
                                    hipStream_t s, ofdft_energy *e_out)
{
    ofdft_grid *g = grids[0];
    const Geom &G = g->geom;
    const size_t fb = (size_t)G.N * sizeof(T);
    ST_TRY(reserve(g, n));
    if (g->batch_cap < n) {
        g->bytes -= g->multi_bytes;
        dfree(reinterpret_cast<void *&>(g->d_ct));
        dfree(g->batch_in);
        dfree(g->batch_out);
        if (g->h_ct) (void)hipHostFree(g->h_ct);
        g->h_ct = nullptr;
        g->batch_cap = 0;
        g->multi_bytes = 0;
        const uint64_t before = g->bytes;
        ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_ct), (size_t)n * sizeof(CellTab)));
        ST_TRY(dmalloc(g, &g->batch_in, (size_t)n * fb));
        ST_TRY(dmalloc(g, &g->batch_out, (size_t)n * fb));
        HIP_TRY(hipHostMalloc((void **)&g->h_ct, (size_t)n * sizeof(CellTab)));
        g->multi_bytes = g->bytes - before;
        g->batch_cap = n;
    }
    bool want_v = false, want_g = false;
    for (int b = 0; b < n; ++b) {
        const ofdft_grid *x = grids[b];
        const void *src = in ? in[b] : (x->rho_set ? x->rho : nullptr);
        if (!src) return fail(OFDFT_EINVAL, "a grid of the batch has no resident density");
        CellTab &c = g->h_ct[b];
        std::memcpy(c.b, x->geom.b, sizeof(c.b));
        c.vext = x->vext;
        c.gtab = x->gtab;
        HIP_TRY(hipMemcpyAsync((char *)g->batch_in + b * fb, src, fb, hipMemcpyDeviceToDevice, s));
        want_v |= v_host && v_host[b];
        want_g |= g_dev && g_dev[b];
    }
    HIP_TRY(hipMemcpyAsync(g->d_ct, g->h_ct, (size_t)n * sizeof(CellTab), hipMemcpyHostToDevice, s));
    g->cur_ct = g->d_ct;
    const ofdft_status st =
        eval_enqueue<T>(g, n, g->batch_in, in_is_phi, want_v ? g->batch_out : nullptr,
                        want_g ? g->batch_out : nullptr, s, work_of<T>(g, 0));
    g->cur_ct = nullptr;
    ST_TRY(st);
    for (int b = 0; b < n; ++b)
        if (g_dev && g_dev[b])
            HIP_TRY(hipMemcpyAsync(g_dev[b], (const char *)g->batch_out + b * fb, fb,
                                   hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    timer_collect(g);
    double bad = 0.0;
    std::vector<ofdft_energy> e((size_t)n);
    for (int b = 0; b < n; ++b) {
        const double *S = g->h_sums + (size_t)b * NSLOT;
        energies_of(grids[b], S, e[b]);
        bad += S[SL_BAD];
    }
    if (bad > 0)
        return fail(OFDFT_EINVAL, "a density of the batch has " + std::to_string((long long)bad) +
                                      " non-finite or negative values");
    for (int b = 0; b < n; ++b)
        if (v_host && v_host[b])
            ST_TRY(download_field(g, v_host[b], (const char *)g->batch_out + b * fb, (size_t)G.N, s));
    std::copy(e.begin(), e.end(), e_out);
    return OFDFT_OK;
}

// The resident densities of n cells (ofdft_energy_potential_multi): the
// members' densities were last written on their own contexts' streams
template <typename T>
static ofdft_status eval_multi(ofdft_grid *const *grids, int n, double *const *v_host,
                               ofdft_energy *e_out)
{
    hipStream_t s = grids[0]->ctx->stream;
    for (int b = 0; b < n; ++b)
        if (grids[b]->ctx->stream != s) HIP_TRY(hipStreamSynchronize(grids[b]->ctx->stream));
    return eval_multi_core<T>(grids, n, nullptr, 0, v_host, nullptr, s, e_out);
}

// ---------------------------------------------------------------- lockstep optimisation
// Several grids optimised together (ofdft_optimize_multi), each in a host
// thread of its own on a stream of its own: the optimisers are unchanged, and
// each evaluation a member asks for waits until every member still optimising
// has asked for one; the last to arrive runs them all as one batched
// evaluation (the kernels of one evaluation then serve every member) and
// wakes the others.  A member that finishes leaves the group (which may
// complete a waiting batch).  The results are those of each grid optimised
// alone: the batched evaluation is the same, bit for bit, per density.
struct EvalBatcher {
    struct Req {
        ofdft_grid *g;
        const void *in;
        void *gout;
        ofdft_energy *e;
        ofdft_status st;
        std::string err;
    };
    std::mutex mu;
    std::condition_variable cv;
    int active = 0;
    uint64_t generation = 0;
    std::vector<Req *> waiting;
    uint64_t batches = 0, merged = 0;
    // runs the waiting requests (lock held); every member waiting is blocked,
    // so the leader's workspace and stream are free
    void run()
    {
        const int n = (int)waiting.size();
        std::vector<ofdft_grid *> gs((size_t)n);
        std::vector<const void *> in((size_t)n);
        std::vector<void *> out((size_t)n);
        std::vector<ofdft_energy> e((size_t)n);
        for (int b = 0; b < n; ++b) {
            gs[b] = waiting[b]->g;
            in[b] = waiting[b]->in;
            out[b] = waiting[b]->gout;
        }
        ofdft_grid *L = gs[0];
        hipStream_t s = L->opt_stream ? L->opt_stream : L->ctx->stream;
        ofdft_status st;
        if (n == 1) {
            st = eval_dispatch(L, 1, in[0], 1, nullptr, out[0], s, e.data());
        } else {
            st = L->fp64 ? eval_multi_core<double>(gs.data(), n, in.data(), 1, nullptr, out.data(),
                                                   s, e.data())
                         : eval_multi_core<float>(gs.data(), n, in.data(), 1, nullptr, out.data(),
                                                  s, e.data());
        }
        const std::string err = st == OFDFT_OK ? std::string() : std::string(ofdft_last_error());
        for (int b = 0; b < n; ++b) {
            waiting[b]->st = st;
            waiting[b]->err = err;
            if (st == OFDFT_OK) *waiting[b]->e = e[b];
        }
        batches++;
        merged += n;
        waiting.clear();
        generation++;
        cv.notify_all();
    }
    ofdft_status eval(ofdft_grid *g, const void *in, void *gout, ofdft_energy *e)
    {
        Req r{g, in, gout, e, OFDFT_OK, std::string()};
        std::unique_lock<std::mutex> lk(mu);
        waiting.push_back(&r);
        const uint64_t gen = generation;
        if ((int)waiting.size() == active) run();
        else cv.wait(lk, [&] { return generation != gen; });
        if (r.st != OFDFT_OK) return fail(r.st, r.err);
        return OFDFT_OK;
    }
    void leave()
    {
        std::lock_guard<std::mutex> lk(mu);
        active--;
        if (!waiting.empty() && (int)waiting.size() == active) run();
    }
};

static ofdft_status opt_eval(ofdft_grid *g, const void *phi, void *gout, hipStream_t s,
                             ofdft_energy *e)
{
    if (!g->batcher) return eval_dispatch(g, 1, phi, 1, nullptr, gout, s, e);
    // the member's vector is complete before another thread's stream reads it
    HIP_TRY(hipStreamSynchronize(s));
    return g->batcher->eval(g, phi, gout, e);
}

static ofdft_status check_opt_params(const ofdft_opt_params *params)
{
    if (!(params->tol > 0) || params->max_iter < 0) return fail(OFDFT_EINVAL, "bad parameters");
    if (params->method != OFDFT_OPT_CG && params->method != OFDFT_OPT_PCG &&
        params->method != OFDFT_OPT_TN)
        return fail(OFDFT_EINVAL, "unknown optimisation method");
    return OFDFT_OK;
}

// ---------------------------------------------------------------- no-allocation evaluation
// The workspace of ofdft_energy_potential_dev_noalloc (spectra, spline knot
// spectra and accumulators, the FP64 leg's buffers, partial sums) for callers
// that cannot allocate device memory.  Host code never uses this array's name
// as an address: each device's copy is resolved once with hipGetSymbolAddress
// (in ofdft_ctx_create, with that device current) and only that pointer is
// passed to kernels.  Every call on a device shares its copy; calls that
// overlap on one device race.  Nothing in it needs to start at zero: every
// buffer is written before it is read within one evaluation (the first knot
// batch overwrites the accumulators, and the final sums read only the partials
// that the evaluation's own blocks wrote).
static __device__ __align__(256) unsigned char scratch[OFDFT_NOALLOC_SCRATCH_BYTES];
static constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

static ofdft_status scratch_resolve(int device)
{
    if (device < 0 || device >= SCRATCH_MAX_DEVICES)
        return fail(OFDFT_EINVAL, "device index beyond the no-allocation scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return OFDFT_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(OFDFT_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                       hipGetErrorString(e));
    g_scratch_ptr[device] = p;
    return OFDFT_OK;
}

static void *scratch_of(int device)
{
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

// Carves the one-density workspace of a grid out of the scratch array
// (256-byte aligned pieces); returns the bytes needed, and fills w when they
// fit.
template <typename T>
static size_t scratch_work(const ofdft_grid *g, char *base, Work &w)
{
    const Geom &G = g->geom;
    const size_t cb = 2 * sizeof(T);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off += (bytes + 255) & ~(size_t)255;
        return p;
    };
    std::memset(&w, 0, sizeof(w));
    w.spec = take((size_t)4 * G.Nh * cb);
    if (g->func.terms & OFDFT_TERM_SPLINE) {
        w.kspec = take((size_t)MAXKB * G.Nh * cb);
        w.acc1 = take((size_t)G.N * sizeof(T));
        if (g->func.nl_mode == OFDFT_NL_EXACT) w.acc2 = take((size_t)G.N * sizeof(T));
        w.kr_part = (double *)take((size_t)KR_SLOTS * KR_BLOCKS * sizeof(double));
        w.kneed = (int *)take((size_t)2 * sizeof(int));
    }
    if (g->vw64) {
        w.vwspec = take((size_t)G.Nh * 16);
        w.vwout = take((size_t)G.N * 4);
    }
    w.part = (double *)take((size_t)NSLOT * g->pstride * sizeof(double));
    w.sums = (double *)take((size_t)NSLOT * sizeof(double));
    return off;
}

template <typename T>
static ofdft_status eval_noalloc(ofdft_grid *g, const void *d_rho, void *d_v, hipStream_t s,
                                 ofdft_energy *e_out)
{
    char *base = (char *)scratch_of(g->ctx->device);
    if (!base)
        return fail(OFDFT_EDEVICE, "no-allocation scratch not resolved for this device");
    Work w;
    const size_t need = scratch_work<T>(g, base, w);
    if (need > (size_t)OFDFT_NOALLOC_SCRATCH_BYTES)
        return fail(OFDFT_EINVAL, "the workspace of one evaluation on this grid needs " +
                                      std::to_string(need) + " bytes; the no-allocation scratch holds " +
                                      std::to_string((size_t)OFDFT_NOALLOC_SCRATCH_BYTES));
    double hs[NSLOT];
    w.h_sums = hs;
    // no per-pass timing (it creates events) and no graphs or second stream
    const bool timer = g->timer.on;
    g->timer.on = false;
    const ofdft_status st = eval_enqueue<T>(g, 1, d_rho, 0, d_v, nullptr, s, w);
    g->timer.on = timer;
    ST_TRY(st);
    HIP_TRY(hipStreamSynchronize(s));
    ofdft_energy e;
    energies_of(g, hs, e);
    if (hs[SL_BAD] > 0)
        return fail(OFDFT_EINVAL, "input density has " + std::to_string((long long)hs[SL_BAD]) +
                                      " non-finite or negative values");
    *e_out = e;
    return OFDFT_OK;
}

extern "C" {

int ofdft_abi_version(void) { return OFDFT_ABI_VERSION; }

const char *ofdft_last_error(void) { return g_last_error.c_str(); }

int ofdft_supported_length(int32_t n) { return is_supported(n) ? 1 : 0; }

ofdft_status ofdft_ctx_create(int device, ofdft_ctx **out)
{
    if (!out) return fail(OFDFT_EINVAL, "null output pointer");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(OFDFT_EINVAL, "no such device");
    HIP_TRY(hipSetDevice(device));
    // library set-up per device: the address of this device's copy of the
    // no-allocation scratch array
    ST_TRY(scratch_resolve(device));
    ofdft_ctx *c = new (std::nothrow) ofdft_ctx;
    if (!c) return fail(OFDFT_ENOMEM, "host allocation failed");
    c->device = device;
    hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete c;
        return fail(OFDFT_EDEVICE, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
    }
    *out = c;
    return OFDFT_OK;
}

void ofdft_ctx_destroy(ofdft_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipStreamDestroy(ctx->stream);
    delete ctx;
}

ofdft_status ofdft_grid_create(ofdft_ctx *ctx, const ofdft_cell_desc *cell,
                               const ofdft_functional_desc *func, ofdft_grid **out)
{
    if (!ctx || !out) return fail(OFDFT_EINVAL, "null argument");
    *out = nullptr;
    ST_TRY(validate(cell, func));
    HIP_TRY(hipSetDevice(ctx->device));
    ofdft_grid *g = new (std::nothrow) ofdft_grid;
    if (!g) return fail(OFDFT_ENOMEM, "host allocation failed");
    g->ctx = ctx;
    if (const char *e = std::getenv("OFDFT_COL_TILE_MAJOR")) g->tune_col_tile_major = std::atoi(e);
    g->sf_method = cell->sf_method;
    g->pme_order = pme_order_of(cell->pme_order);
    g->large_ions = use_large_ions(cell->natoms, cell->sf_method);
    ofdft_status st = grid_setup(g, cell, func);
    if (st == OFDFT_OK) st = reserve(g, 1);
    if (st == OFDFT_OK) tune_apply_cached(g, 1);
    if (st != OFDFT_OK) {
        grid_free(g);
        delete g;
        return st;
    }
    *out = g;
    return OFDFT_OK;
}

void ofdft_grid_destroy(ofdft_grid *grid)
{
    if (!grid) return;
    (void)hipSetDevice(grid->ctx->device);
    (void)hipStreamSynchronize(grid->ctx->stream);
    grid_free(grid);
    delete grid;
}

ofdft_status ofdft_grid_reserve(ofdft_grid *grid, int32_t nbatch)
{
    if (!grid || nbatch < 1) return fail(OFDFT_EINVAL, "bad argument");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    return reserve(grid, nbatch);
}

uint64_t ofdft_grid_device_bytes(const ofdft_grid *grid)
{
    if (!grid) return 0;
    BytesModel m;
    m.stage = grid->stage_in != nullptr || grid->stage_out != nullptr;
    m.opt = grid->opt[0] != nullptr;
    m.forces = grid->d_forces != nullptr;
    m.vw64 = grid->vw64;
    m.mgp = grid->d_jtab64 != nullptr;
    m.extra = grid->multi_bytes;
    uint64_t b = bytes_model(grid->geom, grid->fsz, grid->natoms, (int)grid->Z.size(),
                             grid->sf_method, grid->func.terms, grid->func.nl_mode,
                             (grid->func.terms & OFDFT_TERM_SPLINE) ? grid->func.nk : 0,
                             (uint64_t)grid->cap,
                             ion_bytes(grid->lattice, grid->natoms, grid->sf_method, grid->geom), m);
    if (m.stage && !(grid->stage_in && grid->stage_out)) b -= (uint64_t)grid->geom.N * grid->fsz;
    if (grid->td)
        b += td_bytes(grid->geom, grid->fsz) +
             3 * (uint64_t)td_dipole_blocks(grid->geom) * sizeof(double);
    return b;
}

ofdft_status ofdft_validate(const ofdft_cell_desc *cell, const ofdft_functional_desc *func)
{
    return validate(cell, func);
}

ofdft_status ofdft_footprint_bytes(const ofdft_cell_desc *cell, const ofdft_functional_desc *func,
                                   int32_t kind, uint64_t *bytes)
{
    if (!bytes) return fail(OFDFT_EINVAL, "null output pointer");
    *bytes = 0;
    ST_TRY(validate(cell, func));
    if (kind < OFDFT_REQ_EP || kind > OFDFT_REQ_OPTIMIZE) return fail(OFDFT_EINVAL, "bad request kind");
    const Geom G = make_geom(cell->n);
    BytesModel m;
    m.stage = true;
    m.opt = kind == OFDFT_REQ_OPTIMIZE;
    m.forces = kind == OFDFT_REQ_FORCES;
    m.vw64 = func->precision == OFDFT_MIXED_VW64 && (func->terms & OFDFT_TERM_VW);
    m.mgp = (func->terms & (OFDFT_TERM_WT | OFDFT_TERM_SPLINE)) &&
            func->nl_kernel != OFDFT_KERNEL_WT;
    *bytes = bytes_model(G, func->precision == OFDFT_FP64 ? 8 : 4, cell->natoms, cell->nspecies,
                         cell->sf_method, func->terms, func->nl_mode,
                         (func->terms & OFDFT_TERM_SPLINE) ? func->nk : 0, 1,
                         ion_bytes(cell->lattice, cell->natoms, cell->sf_method, G), m);
    return OFDFT_OK;
}

ofdft_status ofdft_set_density(ofdft_grid *grid, const double *rho_host)
{
    if (!grid || !rho_host) return fail(OFDFT_EINVAL, "null argument");
    const long long N = grid->geom.N;
    for (long long i = 0; i < N; ++i)
        if (!std::isfinite(rho_host[i]) || rho_host[i] < 0)
            return fail(OFDFT_EINVAL, "density has non-finite or negative values");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    ST_TRY(upload_field(grid, grid->rho, rho_host, (size_t)N, grid->ctx->stream));
    grid->rho_set = true;
    return OFDFT_OK;
}

ofdft_status ofdft_get_density(ofdft_grid *grid, double *rho_host)
{
    if (!grid || !rho_host) return fail(OFDFT_EINVAL, "null argument");
    if (!grid->rho_set) return fail(OFDFT_EINVAL, "the grid has no resident density");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    return download_field(grid, rho_host, grid->rho, (size_t)grid->geom.N, grid->ctx->stream);
}

ofdft_status ofdft_energy_potential(ofdft_grid *grid, const double *rho_host, double *v_out_host,
                                    ofdft_energy *e_out)
{
    if (!grid || !e_out) return fail(OFDFT_EINVAL, "null argument");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    const size_t N = (size_t)grid->geom.N;
    hipStream_t s = grid->ctx->stream;
    if (rho_host) {
        // non-finite or negative values are counted by the evaluation itself
        // (its prologue partials), which then fails with OFDFT_EINVAL
        ST_TRY(dmalloc(grid, &grid->stage_in, N * grid->fsz));
        ST_TRY(upload_field(grid, grid->stage_in, rho_host, N, s, true));
    }
    if (!rho_host && !grid->rho_set) return fail(OFDFT_EINVAL, "the grid has no resident density");
    const void *d_in = rho_host ? grid->stage_in : grid->rho;
    void *d_v = nullptr;
    if (v_out_host) {
        ST_TRY(dmalloc(grid, &grid->stage_out, N * grid->fsz));
        d_v = grid->stage_out;
    }
    ST_TRY(eval_dispatch(grid, 1, d_in, 0, d_v, nullptr, s, e_out));
    if (v_out_host) ST_TRY(download_field(grid, v_out_host, d_v, N, s));
    return OFDFT_OK;
}

ofdft_status ofdft_energy_potential_dev(ofdft_grid *grid, const void *d_rho, void *d_v,
                                        void *hip_stream, ofdft_energy *e_out)
{
    return ofdft_energy_potential_batch_dev(grid, 1, d_rho, d_v, hip_stream, e_out);
}

ofdft_status ofdft_energy_potential_dev_noalloc(ofdft_grid *grid, const void *d_rho, void *d_v,
                                                void *hip_stream, ofdft_energy *e_out)
{
    if (!grid || !d_rho || !e_out) return fail(OFDFT_EINVAL, "bad argument");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    hipStream_t s = pick_stream(grid, hip_stream);
    return grid->fp64 ? eval_noalloc<double>(grid, d_rho, d_v, s, e_out)
                      : eval_noalloc<float>(grid, d_rho, d_v, s, e_out);
}

ofdft_status ofdft_energy_potential_multi(ofdft_grid *const *grids, int32_t n,
                                          double *const *v_out_or_null, ofdft_energy *e_out)
{
    if (!grids || !e_out || n < 1 || n > OFDFT_MULTI_MAX) return fail(OFDFT_EINVAL, "bad argument");
    for (int b = 0; b < n; ++b) {
        if (!grids[b]) return fail(OFDFT_EINVAL, "null grid in the batch");
        if (!batchable(grids[0], grids[b]))
            return fail(OFDFT_EINVAL, "grids of a batch need the same shape, functional and device");
        for (int c = 0; c < b; ++c)
            if (grids[c] == grids[b]) return fail(OFDFT_EINVAL, "a grid appears twice in the batch");
    }
    HIP_TRY(hipSetDevice(grids[0]->ctx->device));
    return grids[0]->fp64 ? eval_multi<double>(grids, n, v_out_or_null, e_out)
                          : eval_multi<float>(grids, n, v_out_or_null, e_out);
}

ofdft_status ofdft_energy_potential_batch_dev(ofdft_grid *grid, int32_t nbatch, const void *d_rho,
                                              void *d_v, void *hip_stream, ofdft_energy *e_out)
{
    if (!grid || !d_rho || !e_out || nbatch < 1) return fail(OFDFT_EINVAL, "bad argument");
    if (nbatch > 65535) return fail(OFDFT_EINVAL, "nbatch too large");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    return eval_dispatch(grid, nbatch, d_rho, 0, d_v, nullptr, pick_stream(grid, hip_stream), e_out);
}

ofdft_status ofdft_fft_r2c_dev(ofdft_grid *grid, int32_t nbatch, const void *d_in, void *d_out,
                               void *hip_stream)
{
    if (!grid || !d_in || !d_out || nbatch < 1 || nbatch > 65535)
        return fail(OFDFT_EINVAL, "bad argument");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    hipStream_t s = pick_stream(grid, hip_stream);
    return grid->fp64 ? fft_impl<double>(grid, nbatch, d_in, d_out, true, s)
                      : fft_impl<float>(grid, nbatch, d_in, d_out, true, s);
}

ofdft_status ofdft_fft_c2r_dev(ofdft_grid *grid, int32_t nbatch, const void *d_in, void *d_out,
                               void *hip_stream)
{
    if (!grid || !d_in || !d_out || nbatch < 1 || nbatch > 65535)
        return fail(OFDFT_EINVAL, "bad argument");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    hipStream_t s = pick_stream(grid, hip_stream);
    return grid->fp64 ? fft_impl<double>(grid, nbatch, d_in, d_out, false, s)
                      : fft_impl<float>(grid, nbatch, d_in, d_out, false, s);
}

ofdft_status ofdft_forces(ofdft_grid *grid, double *f_out_host)
{
    if (!grid || !f_out_host) return fail(OFDFT_EINVAL, "null argument");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    const int na = grid->natoms;
    if (na == 0) return OFDFT_OK;
    if (grid->large_ions)
        return fail(OFDFT_EINVAL, "forces are available for cells below " +
                                      std::to_string(LARGE_IONS) +
                                      " atoms with the direct structure factor");
    ofdft_grid *g = grid;
    if (!g->rho_set) return fail(OFDFT_EINVAL, "the grid has no resident density");
    hipStream_t s = g->ctx->stream;
    ST_TRY(reserve(g, 1));
    // rho(G) of the resident density into the workspace spectrum
    ofdft_status st = g->fp64 ? fft_impl<double>(g, 1, g->rho, g->spec, true, s)
                              : fft_impl<float>(g, 1, g->rho, g->spec, true, s);
    ST_TRY(st);
    // the forces and the partial-force table of the tiled kernel
    const size_t nfd = 3 * (size_t)na + (size_t)forces_part_doubles(g->geom, na);
    ST_TRY(dmalloc(g, reinterpret_cast<void **>(&g->d_forces), nfd * sizeof(double)));
    double *d_f = g->d_forces, *d_part = g->d_forces + 3 * (size_t)na;
    const int ns = (int)g->Z.size();
    hipError_t e = g->fp64 ? launch_forces<double>(g->geom, na, g->d_spec_off, ns, g->ph0, g->ph1,
                                                   g->ph2, g->d_Z, g->d_rc, g->spec, d_part, d_f, s)
                           : launch_forces<float>(g->geom, na, g->d_spec_off, ns, g->ph0, g->ph1,
                                                  g->ph2, g->d_Z, g->d_rc, g->spec, d_part, d_f, s);
    std::vector<double> fs(3 * (size_t)na);
    if (e == hipSuccess) e = hipMemcpyAsync(fs.data(), d_f, fs.size() * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    HIP_TRY(e);
    std::vector<double> fe;
    double e_ion = 0.0;
    ST_TRY(ewald_device(g, &e_ion, &fe));
    for (int a = 0; a < na; ++a) {
        const int orig = g->species_order[a];
        for (int k = 0; k < 3; ++k) f_out_host[3 * orig + k] = fs[3 * a + k] + fe[3 * orig + k];
    }
    return OFDFT_OK;
}


ofdft_status ofdft_td_start(ofdft_grid *grid, const double k[3])
{
    if (!grid || !k) return fail(OFDFT_EINVAL, "null argument");
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(k[c])) return fail(OFDFT_EINVAL, "non-finite kick");
    if (!(grid->func.terms & OFDFT_TERM_VW) || grid->func.lambda_vw != 1.0)
        return fail(OFDFT_EINVAL, "TD-OFDFT needs the von Weizsaecker term with lambda = 1 "
                                  "(the Laplacian of the Hamiltonian)");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    return grid->fp64 ? td_start_impl<double>(grid, k) : td_start_impl<float>(grid, k);
}

ofdft_status ofdft_td_propagate(ofdft_grid *grid, const ofdft_td_params *params, int32_t nsteps,
                                double *dipole_out, ofdft_td_stats *stats)
{
    if (!grid || !params || !stats || nsteps < 0) return fail(OFDFT_EINVAL, "bad argument");
    if (!grid->td) return fail(OFDFT_EINVAL, "no TD state: call ofdft_td_start first");
    if (!std::isfinite(params->dt) || params->dt == 0.0 || params->n_corrector < 0 ||
        params->n_corrector > 16 || params->max_solver_iter < 0 || !(params->solver_tol >= 0))
        return fail(OFDFT_EINVAL, "bad TD parameters");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    return grid->fp64 ? td_propagate_impl<double>(grid, params, nsteps, dipole_out, stats)
                      : td_propagate_impl<float>(grid, params, nsteps, dipole_out, stats);
}

ofdft_status ofdft_td_get_psi(ofdft_grid *grid, double *re_host, double *im_host)
{
    if (!grid || !re_host || !im_host) return fail(OFDFT_EINVAL, "null argument");
    if (!grid->td) return fail(OFDFT_EINVAL, "no TD state: call ofdft_td_start first");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    const size_t N = (size_t)grid->geom.N;
    const TdBufs B = td_bufs(grid);
    hipStream_t s = grid->ctx->stream;
    ST_TRY(download_field(grid, re_host, B.vec[TV_PSI], N, s));
    return download_field(grid, im_host, im_part(grid, B.vec[TV_PSI]), N, s);
}

ofdft_status ofdft_td_set_psi(ofdft_grid *grid, const double *re_host, const double *im_host)
{
    if (!grid || !re_host || !im_host) return fail(OFDFT_EINVAL, "null argument");
    const size_t N = (size_t)grid->geom.N;
    for (size_t i = 0; i < N; ++i)
        if (!std::isfinite(re_host[i]) || !std::isfinite(im_host[i]))
            return fail(OFDFT_EINVAL, "non-finite psi");
    if (!(grid->func.terms & OFDFT_TERM_VW) || grid->func.lambda_vw != 1.0)
        return fail(OFDFT_EINVAL, "TD-OFDFT needs the von Weizsaecker term with lambda = 1");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    ST_TRY(td_alloc(grid));
    const TdBufs B = td_bufs(grid);
    hipStream_t s = grid->ctx->stream;
    ST_TRY(upload_field(grid, B.vec[TV_PSI], re_host, N, s));
    return upload_field(grid, const_cast<void *>(im_part(grid, B.vec[TV_PSI])), im_host, N, s);
}

ofdft_status ofdft_optimize(ofdft_grid *grid, const ofdft_opt_params *params, ofdft_opt_result *result)
{
    if (!grid || !params || !result) return fail(OFDFT_EINVAL, "null argument");
    ST_TRY(check_opt_params(params));
    if (!grid->rho_set) return fail(OFDFT_EINVAL, "the grid has no resident density");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    return grid->fp64 ? optimize_impl<double>(grid, params, result)
                      : optimize_impl<float>(grid, params, result);
}

ofdft_status ofdft_optimize_multi(ofdft_grid *const *grids, int32_t n,
                                  const ofdft_opt_params *params, ofdft_opt_result *results,
                                  ofdft_status *statuses)
{
    if (!grids || !params || !results || !statuses || n < 1 || n > OFDFT_MULTI_MAX)
        return fail(OFDFT_EINVAL, "bad argument");
    for (int b = 0; b < n; ++b) {
        if (!grids[b]) return fail(OFDFT_EINVAL, "null grid in the batch");
        if (!batchable(grids[0], grids[b]))
            return fail(OFDFT_EINVAL, "grids of a batch need the same shape, functional and device");
        for (int c = 0; c < b; ++c)
            if (grids[c] == grids[b]) return fail(OFDFT_EINVAL, "a grid appears twice in the batch");
        if (!grids[b]->rho_set)
            return fail(OFDFT_EINVAL, "a grid of the batch has no resident density");
        ST_TRY(check_opt_params(&params[b]));
    }
    const int dev = grids[0]->ctx->device;
    HIP_TRY(hipSetDevice(dev));
    for (int b = 0; b < n; ++b) HIP_TRY(hipStreamSynchronize(grids[b]->ctx->stream));
    std::vector<hipStream_t> streams((size_t)n, nullptr);
    for (int b = 0; b < n; ++b) {
        const hipError_t e = hipStreamCreateWithFlags(&streams[b], hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (int c = 0; c < b; ++c) (void)hipStreamDestroy(streams[c]);
            return fail(OFDFT_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));
        }
    }
    EvalBatcher B;
    B.active = n;
    std::vector<std::string> errs((size_t)n);
    for (int b = 0; b < n; ++b) {
        grids[b]->batcher = &B;
        grids[b]->opt_stream = streams[b];
    }
    auto member = [&](int b) {
        (void)hipSetDevice(dev);
        ofdft_grid *g = grids[b];
        const ofdft_status st = g->fp64 ? optimize_impl<double>(g, &params[b], &results[b])
                                        : optimize_impl<float>(g, &params[b], &results[b]);
        statuses[b] = st;
        if (st != OFDFT_OK) errs[b] = ofdft_last_error();
        B.leave();
    };
    std::vector<std::thread> threads;
    threads.reserve((size_t)n - 1);
    for (int b = 1; b < n; ++b) threads.emplace_back(member, b);
    member(0);
    for (auto &t : threads) t.join();
    for (int b = 0; b < n; ++b) {
        (void)hipStreamSynchronize(streams[b]);
        (void)hipStreamDestroy(streams[b]);
        grids[b]->batcher = nullptr;
        grids[b]->opt_stream = nullptr;
    }
    for (int b = 0; b < n; ++b)
        if (statuses[b] != OFDFT_OK) {
            g_last_error = "member " + std::to_string(b) + ": " + errs[b];
            break;
        }
    return OFDFT_OK;
}

ofdft_status ofdft_grid_interpolate_density(ofdft_grid *dst, ofdft_grid *src)
{
    return interpolate_density(dst, src);
}

ofdft_status ofdft_optimize_multistep(ofdft_grid *const *grids, int32_t ngrids,
                                     const ofdft_opt_params *params, ofdft_opt_result *results)
{
    if (!grids || !params || !results || ngrids < 1) return fail(OFDFT_EINVAL, "null argument");
    for (int i = 0; i < ngrids; ++i)
        if (!grids[i]) return fail(OFDFT_EINVAL, "null grid");
    ofdft_status last = OFDFT_OK;
    for (int i = 0; i < ngrids; ++i) {
        if (i > 0) ST_TRY(interpolate_density(grids[i], grids[i - 1]));
        last = ofdft_optimize(grids[i], &params[i], &results[i]);
        if (last != OFDFT_OK && last != OFDFT_ENOCONV) return last;
    }
    return last;
}

ofdft_status ofdft_grid_set_graphs(ofdft_grid *grid, int32_t on)
{
    if (!grid) return fail(OFDFT_EINVAL, "null argument");
    grid->use_graphs = on != 0;
    if (!grid->use_graphs) graphs_clear(grid);
    return OFDFT_OK;
}

ofdft_status ofdft_grid_set_knot_skip(ofdft_grid *grid, int32_t on)
{
    if (!grid) return fail(OFDFT_EINVAL, "null grid");
    if ((on != 0) != grid->knot_skip) graphs_clear(grid);
    grid->knot_skip = on != 0;
    return OFDFT_OK;
}

ofdft_status ofdft_grid_set_knot_pipeline(ofdft_grid *grid, int32_t on)
{
    if (!grid) return fail(OFDFT_EINVAL, "null grid");
    if ((on != 0) != (grid->tune_knot_pipe != 0)) graphs_clear(grid);
    grid->tune_knot_pipe = on != 0;
    return OFDFT_OK;
}

ofdft_status ofdft_grid_set_col_group(ofdft_grid *grid, int32_t n)
{
    if (!grid) return fail(OFDFT_EINVAL, "null grid");
    if (n < 1 || n > COL_GROUP) return fail(OFDFT_EINVAL, "column group outside 1..8");
    if (n != grid->tune_col_group) graphs_clear(grid);
    grid->tune_col_group = n;
    return OFDFT_OK;
}

ofdft_status ofdft_grid_set_col_variant(ofdft_grid *grid, int32_t variant)
{
    if (!grid) return fail(OFDFT_EINVAL, "null grid");
    if (variant < 0 || variant > 3) return fail(OFDFT_EINVAL, "column variant outside 0..3");
    if (variant != grid->tune_col_variant) graphs_clear(grid);
    grid->tune_col_variant = variant;
    return OFDFT_OK;
}

ofdft_status ofdft_grid_set_pipeline(ofdft_grid *grid, int32_t nsub)
{
    if (!grid) return fail(OFDFT_EINVAL, "null grid");
    if (nsub < 1) return fail(OFDFT_EINVAL, "nsub must be at least 1");
    grid->tune_pipe = nsub;
    graphs_clear(grid);
    return OFDFT_OK;
}

ofdft_status ofdft_grid_tune_dev(ofdft_grid *grid, int32_t nbatch, const void *d_rho,
                                 void *hip_stream, ofdft_tune_result *result)
{
    if (!grid || !d_rho || nbatch < 1 || nbatch > 65535) return fail(OFDFT_EINVAL, "bad argument");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    return tune_impl(grid, nbatch, d_rho, pick_stream(grid, hip_stream), result);
}

ofdft_status ofdft_grid_tune(ofdft_grid *grid, ofdft_tune_result *result)
{
    if (!grid) return fail(OFDFT_EINVAL, "null argument");
    if (!grid->rho_set) return fail(OFDFT_EINVAL, "the grid has no resident density");
    HIP_TRY(hipSetDevice(grid->ctx->device));
    return tune_impl(grid, 1, grid->rho, grid->ctx->stream, result);
}

// per-pass timing with HIP events on the launch stream
ofdft_status ofdft_profile_enable(ofdft_grid *grid, int32_t on)
{
    if (!grid) return fail(OFDFT_EINVAL, "null argument");
    grid->timer.on = on != 0;
    graphs_clear(grid);
    for (int i = 0; i < NPASS; ++i) {
        grid->timer.ms[i] = 0;
        grid->timer.count[i] = 0;
    }
    return OFDFT_OK;
}

ofdft_status ofdft_profile_read(ofdft_grid *grid, int32_t pass, double *total_ms, int64_t *launches)
{
    if (!grid || pass < 0 || pass >= NPASS || !total_ms || !launches)
        return fail(OFDFT_EINVAL, "bad argument");
    *total_ms = grid->timer.ms[pass];
    *launches = grid->timer.count[pass];
    return OFDFT_OK;
}

}  // extern "C"
