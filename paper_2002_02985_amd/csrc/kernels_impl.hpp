// HIP kernels of the orbital-free DFT evaluation (templated on the field
// type T = float | double and on the FFT length).  Included by the
// per-precision translation units, which instantiate the launchers.
//
// One energy+potential evaluation is five field passes plus a reduction:
//   1. row_fwd   axis-2 r2c of rho, phi and rho^beta computed pointwise from
//                the input (Thomas-Fermi partials fused);
//   2. col       axis-1 forward c2c;
//   3. col       axis-0 forward c2c, reciprocal-space term (Hartree + local
//                pseudopotential, von Weizsaecker Laplacian, Wang-Teter
//                kernel), axis-0 inverse c2c -- per field, with the
//                reciprocal-space energy partials;
//   4. col       axis-1 inverse c2c;
//   5. row_inv   axis-2 c2r of all fields and the final combine of the
//                potential v = dE/drho and of g = dE/dphi, with the
//                nonlocal energy and chemical-potential partials;
//   6. finalize  fixed-order FP64 sums of the per-workgroup partials.
// The spline functional adds, per batch of knots, an axis-0 kernel that
// applies omega_i(|G|) and inverts, the axis-1 inverse, and an axis-2 c2r
// that interpolates over k_F at every point (steps s2-s4).
#pragma once
#include <cmath>
#include <type_traits>

#include "fft_core.hpp"
#include "gnl_poly.hpp"
#include "kernels.hpp"

namespace ofdft {

constexpr int NT = 256;
constexpr double PI_D = 3.14159265358979323846264338327950288;
constexpr double THREE_PI2 = 29.608813203268075856503472999628;  // 3 pi^2
constexpr double C_TF_D = 2.8712340001881918;   // (3/10)(3 pi^2)^(2/3)
constexpr double C_WT_D = 2.2969872001505534;   // (6/25)(3 pi^2)^(2/3)

// complex elements per block of the column and row passes (tile sizes)
template <typename T> struct Cfg;
template <> struct Cfg<float> {
    static constexpr int COL_ELEMS = 8192;
    static constexpr int ROW_ELEMS = 2048;
};
template <> struct Cfg<double> {
    static constexpr int COL_ELEMS = 2048;
    static constexpr int ROW_ELEMS = 1024;
};

constexpr int pow2_floor(int x)
{
    int p = 1;
    while (p * 2 <= x) p *= 2;
    return p;
}
// at most 16 columns per block: smaller tiles keep more blocks in flight per
// CU, which measured faster than 32-wide tiles on both the 96-point and the
// 256-point column passes
constexpr int COL_PMAX = 16;
// grouped column blocks (COL_GROUP densities, sharing the tile's set-up
// and operands) only while the launch keeps at least COL_MIN_BLOCKS blocks
constexpr long long COL_MIN_BLOCKS = 8192;
template <typename T, int L> constexpr int col_P()
{
    int p = pow2_floor(Cfg<T>::COL_ELEMS / L);
    if (p > COL_PMAX) p = COL_PMAX;
    if (p < 4) p = 4;
    if (p > NT) p = NT;
    return p;
}
// column passes with no reciprocal-space operation hold no per-element
// registers besides the transform and take twice as many columns (the
// 1024-point passes of the 10^6-atom cell: 128-byte row segments instead of
// 64-byte ones, measured faster; the other lengths reach the 16-column cap
// either way)
template <typename T, int L> constexpr int col_P_plain()
{
    int p = pow2_floor(2 * Cfg<T>::COL_ELEMS / L);
    if (p > COL_PMAX) p = COL_PMAX;
    if (p < 4) p = 4;
    if (p > NT) p = NT;
    return p;
}
// columns per block and threads per block of the knot kernels: the column
// tile, except for 1024-point columns, which take the wide tile of the
// plain column passes (16 columns: the eight knot spectra are written in
// 128-byte row segments instead of 64-byte ones) with 1024 threads
template <typename T, int L> constexpr int knot_P()
{
    return L >= 1024 ? col_P_plain<T, L>() : col_P<T, L>();
}
// threads per block of the column kernel: 256, and more for long columns,
// whose L x P tile fills so much LDS that one or two blocks fit on a CU (a
// 1024-point, 16-column tile takes 128 KB): L P / 16 rounded down to a power
// of two, clamped to 256 .. 1024, keeps about 16 elements per thread.  (The
// knot kernels of 8-column tiles stay at 256: with more threads their
// per-knot registers spill at two blocks per CU, which measured slower.)
template <typename T, int L, int P> constexpr int col_NT()
{
    int t = pow2_floor(L * P / 16);
    if (t < NT) t = NT;
    if (t > 1024) t = 1024;
    return t;
}
// grouped column kernels are built for the column lengths whose operands
// take at most 8 registers per thread (the batched small grids)
template <typename T, int L> constexpr bool col_grouped()
{
    return L * col_P<T, L>() / col_NT<T, L, col_P<T, L>()>() <= 8;
}
template <typename T, int L> constexpr int knot_NT()
{
    return knot_P<T, L>() != col_P<T, L>() ? col_NT<T, L, knot_P<T, L>()>() : NT;
}
template <typename T, int M> constexpr int row_P()
{
    int p = pow2_floor(Cfg<T>::ROW_ELEMS / M);
    return p < 1 ? 1 : p;
}

// ---------------------------------------------------------------- math
__device__ __forceinline__ float d_cbrt(float x) { return cbrtf(x); }
__device__ __forceinline__ double d_cbrt(double x) { return cbrt(x); }
__device__ __forceinline__ float d_pow(float x, float e) { return powf(x, e); }
__device__ __forceinline__ double d_pow(double x, double e) { return pow(x, e); }
__device__ __forceinline__ float d_log(float x) { return logf(x); }
__device__ __forceinline__ double d_log(double x) { return log(x); }
__device__ __forceinline__ float d_log1p(float x) { return log1pf(x); }
__device__ __forceinline__ double d_log1p(double x) { return log1p(x); }
__device__ __forceinline__ float d_sqrt(float x) { return sqrtf(x); }
__device__ __forceinline__ double d_sqrt(double x) { return sqrt(x); }
// FP32: the hardware square root (1 ulp) without the correctly rounded
// fix-up sequence; FP64: the correctly rounded one
__device__ __forceinline__ float d_sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double d_sqrt_fast(double x) { return sqrt(x); }
// 1/x: FP32 the hardware reciprocal (1 ulp), FP64 the division
__device__ __forceinline__ float d_rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double d_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ bool d_finite(float x) { return isfinite(x); }
__device__ __forceinline__ bool d_finite(double x) { return isfinite(x); }
// base-2 logarithm and power: the hardware transcendental instructions for
// FP32 fields (about 1 ulp), the library functions for FP64
__device__ __forceinline__ float d_log2(float x) { return __builtin_amdgcn_logf(x); }
__device__ __forceinline__ double d_log2(double x) { return log2(x); }
__device__ __forceinline__ float d_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ double d_exp2(double x) { return exp2(x); }
// max for operands that are never NaN: the IEEE-754 2019 maximum (one
// instruction; fmaxf would first quiet both operands)
__device__ __forceinline__ float d_fmax(float x, float y) { return __builtin_elementwise_maximum(x, y); }
__device__ __forceinline__ double d_fmax(double x, double y) { return __builtin_fmax(x, y); }
template <typename T> __device__ __forceinline__ T neg_inf() { return -__builtin_huge_valf(); }
template <> __device__ __forceinline__ double neg_inf<double>() { return -__builtin_huge_val(); }
constexpr double LOG2_3PI2 = 4.8879547596657937775;   // log2(3 pi^2)
constexpr double KF_C = 3.0936677262801355;   // (3 pi^2)^(1/3)

// Lindhard kernel shape G_NL(eta) = 1/F - 3 eta^2 - 1 with
// F = 1/2 + (1 - eta^2)/(4 eta) ln|(1 + eta)/(1 - eta)| (the G_NL formula of
// the nonlocal-KEDF section).  The logarithm is taken as log1p of
// 2 eta/(1 - eta) or 2/(eta - 1); from eta = 1.6 on, where 1/F - 3 eta^2
// would cancel, G_NL is a polynomial in x = 1/eta^2 (gnl_poly.hpp: the
// Chebyshev economisation of G = -1 - S/P with F = x P(x) and
// 3 eta^2 F = 1 + x S(x), P and S the series of the logarithm in 1/eta;
// degree 7 in FP32, 16 in FP64, each within its precision's rounding).
template <typename T>
__device__ __forceinline__ T gnl_dev(T eta)
{
    if (!(eta > T(0))) return T(0);
    if (eta == T(1)) return T(-2);
    // FP32: quotients by the hardware reciprocal (1 ulp); FP64: divisions.
    // Below 1.6 one expression serves both sides of eta = 1 (the operands
    // selected per lane, so a wave whose lanes straddle eta = 1 runs one
    // logarithm): ln|(1 + eta)/(1 - eta)| = log1p(2 eta / (1 - eta)) below 1,
    // log1p(2 / (eta - 1)) above, and (1 - eta^2) changes sign.
    if (eta < T(GNL_POLY_ETA)) {
        const bool lo = eta < T(1);
        const T d = lo ? T(1) - eta : eta - T(1);
        const T num = lo ? T(2) * eta : T(2);
        const T m = lo ? (T(1) - eta) * (T(1) + eta) : -((eta - T(1)) * (eta + T(1)));
        T F = T(0.5) + m * d_rcp(T(4) * eta) * d_log1p(num * d_rcp(d));
        return d_rcp(F) - T(3) * eta * eta - T(1);
    }
    const T x = d_rcp(eta * eta);
    constexpr const double *C = sizeof(T) == 8 ? GNL_X64 : GNL_X32;
    constexpr int DEG = sizeof(T) == 8 ? GNL_X64_DEG : GNL_X32_DEG;
    T h = T(C[DEG]);
#pragma unroll
    for (int k = DEG - 1; k >= 0; --k) h = h * x + T(C[k]);
    return h;
}

// K(eta) of the kernel family (omega = C_WT K): G_NL for Wang-Teter; for the
// MGP family (1 - x) G_NL + x J with J interpolated linearly on its table
// (in eta up to 4, in w = 1/eta^2 above; the node rule of mgp_table.hpp)
template <typename T>
__device__ __forceinline__ T nl_kernel_dev(T eta, const NlKern &k)
{
    if (k.x == 0.0) return gnl_dev<T>(eta);
    const T *tab = (const T *)k.tab;
    T j;
    if (eta <= T(4)) {
        const T s = eta * T(MGP_SA);
        int i = (int)s;
        i = i > MGP_NA - 1 ? MGP_NA - 1 : i;
        const T f = s - T(i);
        j = tab[i] + f * (tab[i + 1] - tab[i]);
    } else {
        const T s = d_rcp(eta * eta) * T(MGP_SB);
        int i = (int)s;
        i = i > MGP_NB - 1 ? MGP_NB - 1 : i;
        const T f = s - T(i);
        const T *tb = tab + MGP_NA + 1;
        j = tb[i] + f * (tb[i + 1] - tb[i]);
    }
    const T x = T(k.x);
    return k.x == 1.0 ? j : (T(1) - x) * gnl_dev<T>(eta) + x * j;
}

// k_F = (3 pi^2 rho)^(1/3), clamped to the knot range; bracket j and linear
// weight t on the knots (step s4).  An exact knot belongs to the segment on
// its right; the last knot to the last segment with t = 1.  kat(i) is knot i
// in T.
template <typename T, class KAT>
__device__ __forceinline__ void knot_bracket_at(T kf, int nk, int log_spacing, double inv_span,
                                                const KAT &kat, int &j, T &t, bool &inside)
{
    const T k1 = kat(0), kN = kat(nk - 1);
    inside = kf > k1 && kf < kN;
    const T kt = kf < k1 ? k1 : (kf > kN ? kN : kf);
    if (nk == 1) {
        j = 0;
        t = T(0);
        return;
    }
    T s = log_spacing ? T(inv_span) * d_log(kt / k1) : T(inv_span) * (kt - k1);
    int jj = (int)floor(s);
    jj = jj < 0 ? 0 : (jj > nk - 2 ? nk - 2 : jj);
    if (kt < kat(jj) && jj > 0) jj -= 1;
    else if (jj < nk - 2 && kt >= kat(jj + 1)) jj += 1;
    j = jj;
    const T kj = kat(jj), kj1 = kat(jj + 1);
    t = (kt - kj) / (kj1 - kj);
}
// knots read from the device array
template <typename T>
__device__ __forceinline__ void knot_bracket_kf(T kf, const Knots &kn, int &j, T &t, bool &inside)
{
    knot_bracket_at(kf, kn.nk, kn.log_spacing, kn.inv_span, [&](int i) { return T(kn.k[i]); }, j,
                    t, inside);
}
// knots already converted to T, in LDS
template <typename T>
__device__ __forceinline__ void knot_bracket_tab(T kf, int nk, int log_spacing, double inv_span,
                                                 const T *ktab, int &j, T &t, bool &inside)
{
    knot_bracket_at(kf, nk, log_spacing, inv_span, [&](int i) { return ktab[i]; }, j, t, inside);
}

// rho^(-1/6) in FP64 without the FP64 logarithm and exponential (dozens of
// instructions each), in integer and FP64 multiply-add instructions only.
// The estimate takes log2 rho as linear in the high word of its bits
// (exponent and top 20 mantissa bits; off by at most 0.086) and forms the
// high word of y from -log2(rho)/6, shifted by 0.05 so that the estimate is
// within 3.5% of rho^(-1/6); five Newton steps on f(y) = y^-6 - rho,
// y <- y (7 - rho y^6) / 6, each taking a relative error e to about
// -3.5 e^2, leave the FP64 rounding (3.5e-2 -> 4.3e-3 -> 6.5e-5 -> 1.5e-8 ->
// 7.6e-16).  rho must be >= 0; below the smallest normal double the result
// is 0 (every power of rho the terms use is then below 1e-51).
__device__ __forceinline__ double rsixth(double rho)
{
    constexpr int B = 1023 << 20;                 // high word of 1.0
    constexpr int SHIFT = 52429;                  // 0.05 * 2^20
    const int hi = (int)(__double_as_longlong(rho) >> 32);
    const int yh = B - (hi - B) / 6 - SHIFT;
    double y = __longlong_as_double((long long)yh << 32);
#pragma unroll
    for (int it = 0; it < 5; ++it) {
        const double y2 = y * y;
        y = y * (7.0 - rho * (y2 * y2 * y2)) * (1.0 / 6.0);
    }
    return rho >= 0x1p-1022 ? y : 0.0;
}

// k_F = (3 pi^2 rho)^(1/3) from log2(rho)
template <typename T>
__device__ __forceinline__ T kf_from_log2(T lu)
{
    return d_exp2((T(LOG2_3PI2) + lu) * T(1.0 / 3.0));
}

// An opaque copy of the thread index (an empty asm with a register operand,
// no memory access): index arithmetic derived from it is recomputed where it
// is used rather than hoisted out of per-field loops and kept live.
__device__ __forceinline__ int opaque(int t)
{
    asm volatile("" : "+v"(t));
    return t;
}
__device__ __forceinline__ float opaque_v(float x)
{
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ double opaque_v(double x)
{
    asm volatile("" : "+v"(x));
    return x;
}
template <typename T>
__device__ __forceinline__ cpx<T> opaque(cpx<T> z)
{
    asm volatile("" : "+v"(z.x), "+v"(z.y));
    return z;
}

// signed grid frequency of index i on an axis of n points (Nyquist negative)
__device__ __forceinline__ int freq(int i, int n) { return i < (n + 1) / 2 ? i : i - n; }

template <typename T>
__device__ __forceinline__ T gvec2(const Geom &g, int m0, int m1, int m2)
{
    // the (m1, m2) part first: in the column passes it is the same for every
    // element of a column and is computed once
    const T gx = T(m0) * T(g.b[0][0]) + (T(m1) * T(g.b[1][0]) + T(m2) * T(g.b[2][0]));
    const T gy = T(m0) * T(g.b[0][1]) + (T(m1) * T(g.b[1][1]) + T(m2) * T(g.b[2][1]));
    const T gz = T(m0) * T(g.b[0][2]) + (T(m1) * T(g.b[1][2]) + T(m2) * T(g.b[2][2]));
    return gx * gx + gy * gy + gz * gz;
}

// (c / d, c % d) for the column c = c0 + p of a block tile (c0 the tile's
// first column, block-uniform; 0 <= p < the tile width): the division once
// per tile in 32 bits, then wrap steps per lane (at most p / d + 1)
__device__ __forceinline__ void tile_divmod(unsigned c0, unsigned p, unsigned d, unsigned &q,
                                            unsigned &r)
{
    q = c0 / d;
    r = c0 - q * d + p;
    while (r >= d) {
        r -= d;
        ++q;
    }
}

__device__ __forceinline__ double *part_ptr(double *part, int b, int slot, int pstride)
{
    return part + ((long long)b * NSLOT + slot) * pstride;
}

// ================================================================ row forward
// Axis-2 r2c of P rows per block.  The input is read once into registers;
// the fields (rho, phi, rho^beta, or rho^alpha L_i(k~) for the EXACT spline)
// are derived pointwise and transformed one after the other through LDS.
template <typename T, int M>
__global__ __launch_bounds__(NT) void k_row_fwd(RowFwdArgs a, Geom g)
{
    constexpr int P = row_P<T, M>();
    constexpr int PS = P + 1;
    constexpr int PAIRS = P * M;
    constexpr int PER = (PAIRS + NT - 1) / NT;
    __shared__ cpx<T> buf[M * PS];
    __shared__ double red[3 * NT / 64];
    const int tid = threadIdx.x;
    const int b = blockIdx.y;
    const long long nrows = (long long)g.n0 * g.n1;
    const long long r0 = (long long)blockIdx.x * P;
    const T *in = (const T *)a.in + (long long)b * g.N;
    const cpx<T> *twM = (const cpx<T> *)a.twM;
    const cpx<T> *twN = (const cpx<T> *)a.twN;
    // EXACT spline fields rho^a L_i: knots outside the density's range are
    // zero everywhere (their spectra are not needed by the later passes)
    const bool knots = a.nfields > 0 && a.kind[0] == FK_KNOT;
    int klo = 0, khi = 1 << 30;
    if (knots && a.kneed) {
        klo = a.kneed[2 * b];
        khi = a.kneed[2 * b + 1];
        if (a.knot0 > khi || a.knot0 + a.nfields - 1 < klo) return;
    }
    // knot fields: the knots in T, in LDS for the per-point brackets
    __shared__ T knl[MAXKNOTS];
    if (knots) {
        if (tid < a.knots.nk) knl[tid] = T(a.knots.k[tid]);   // nk <= MAXKNOTS <= NT
        __syncthreads();
    }

    cpx<T> x[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * NT;
        x[q] = {T(0), T(0)};
        if (idx < PAIRS) {
            const int p = idx / M, n = idx % M;
            const long long row = r0 + p;
            if (row < nrows) {
                if constexpr (sizeof(T) == 8) {
                    if (a.in_f32) {
                        // FP32 input of the FP64 von Weizsaecker leg
                        const float2 v = ((const float2 *)((const float *)a.in +
                                                           (long long)b * g.N + row * g.n2))[n];
                        x[q] = {T(v.x), T(v.y)};
                    } else {
                        x[q] = ((const cpx<T> *)(in + row * g.n2))[n];
                    }
                } else {
                    x[q] = ((const cpx<T> *)(in + row * g.n2))[n];
                }
            }
        }
    }
    // derived values: u = rho, w = phi, z = rho^beta  (or, for knot fields,
    // u = rho^alpha, w = t, jj = bracket)
    // FP64 passes that need neither the partials nor rho^beta nor the knot
    // weights (the von Weizsaecker leg: phi only) skip the FP64 logarithm
    // and exponential; FP32 passes always evaluate them
    bool need_lu = sizeof(T) == 4 || a.partials || knots;
    for (int f = 0; f < a.nfields; ++f) need_lu |= a.kind[f] == FK_RHOB;
    const bool sixth = sizeof(T) == 8 && a.alpha == 5.0 / 6.0 && a.beta == 5.0 / 6.0;
    cpx<T> u[PER], w[PER], z[PER];
    int jj[PER][2];
    double sums[3] = {0.0, 0.0, 0.0};   // sum rho, sum rho^(5/3), bad count
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * NT;
        const bool live = idx < PAIRS && r0 + idx / M < nrows;
        const T xv[2] = {x[q].x, x[q].y};
        T uu[2], ww[2], zz[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const T v = xv[c];
            const bool ok = d_finite(v) && (a.in_is_phi || v >= T(0));
            const T rho = a.in_is_phi ? v * v : (v > T(0) ? v : T(0));
            if (sixth) {
                // FP64, alpha = beta = 5/6: every power from y = rho^(-1/6)
                // (rho^(2/3) = rho y^2, k_F = KF_C rho y^4, rho^(5/6) = rho y)
                const T y = need_lu ? T(rsixth((double)rho)) : T(0);
                if (live && a.partials) {
                    if (!ok) {
                        sums[2] += 1.0;
                    } else {
                        sums[0] += (double)rho;
                        sums[1] += (double)(rho * (rho * (y * y)));
                    }
                }
                if (knots) {
                    T t;
                    bool inside;
                    const T y2 = y * y;
                    knot_bracket_tab(T(KF_C) * rho * (y2 * y2), a.knots.nk, a.knots.log_spacing,
                                     a.knots.inv_span, knl, jj[q][c], t, inside);
                    uu[c] = rho * y;
                    ww[c] = t;
                    zz[c] = T(0);
                } else {
                    uu[c] = a.in_is_phi ? v * v : v;
                    ww[c] = a.in_is_phi ? v : d_sqrt(rho);
                    zz[c] = rho * y;
                }
                continue;
            }
            const T lu = (need_lu && rho > T(0)) ? d_log2(rho) : neg_inf<T>();
            if (live && a.partials) {
                if (!ok) {
                    sums[2] += 1.0;
                } else {
                    sums[0] += (double)rho;
                    sums[1] += (double)(rho * d_exp2(lu * T(2.0 / 3.0)));
                }
            }
            if (knots) {
                T t;
                bool inside;
                knot_bracket_tab(kf_from_log2(lu), a.knots.nk, a.knots.log_spacing,
                                 a.knots.inv_span, knl, jj[q][c], t, inside);
                uu[c] = d_exp2(T(a.alpha) * lu);
                ww[c] = t;
                zz[c] = T(0);
            } else {
                uu[c] = a.in_is_phi ? v * v : v;
                ww[c] = a.in_is_phi ? v : d_sqrt(rho);
                zz[c] = need_lu ? d_exp2(T(a.beta) * lu) : T(0);
            }
        }
        u[q] = {uu[0], uu[1]};
        w[q] = {ww[0], ww[1]};
        z[q] = {zz[0], zz[1]};
    }
    if (a.partials) {
        block_sums<NT, 3>(sums, red, tid);
        if (tid == 0) {
            part_ptr(a.part, b, SL_RHO, a.pstride)[blockIdx.x] = sums[0];
            part_ptr(a.part, b, SL_TF, a.pstride)[blockIdx.x] = sums[1];
            part_ptr(a.part, b, SL_BAD, a.pstride)[blockIdx.x] = sums[2];
        }
    }
    for (int f = 0; f < a.nfields; ++f) {
        const int kind = a.kind[f];
        const int knot = a.knot0 + f;
        if (knots && (knot < klo || knot > khi)) continue;   // uniform in the block
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + q * NT;
            if (idx < PAIRS) {
                const int p = idx / M, n = idx % M;
                cpx<T> val;
                if (kind == FK_RHO || kind == FK_RAW) val = u[q];
                else if (kind == FK_PHI) val = w[q];
                else if (kind == FK_RHOB) val = z[q];
                else {
                    const T tv[2] = {w[q].x, w[q].y};
                    const T uv[2] = {u[q].x, u[q].y};
                    T o[2];
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        const int j = jj[q][c];
                        const T L = a.knots.nk == 1 ? T(1)
                                                    : (j == knot ? T(1) - tv[c]
                                                                 : (j + 1 == knot ? tv[c] : T(0)));
                        o[c] = L * uv[c];
                    }
                    val = {o[0], o[1]};
                }
                buf[n * PS + p] = val;
            }
        }
        __syncthreads();
        lds_fft<T, M, false, P, NT, PS>(buf, twM, tid);
        // unpack the half-length complex transform into the r2c half spectrum:
        // X[k] = (Z[k] + conj Z[M-k])/2 - i W^k (Z[k] - conj Z[M-k])/2
        cpx<T> *out = (cpx<T> *)a.out + f * a.out_fstride + (long long)b * g.Nh;
        constexpr int OUTS = P * (M + 1);
        for (int o = tid; o < OUTS; o += NT) {
            const int p = o / (M + 1), k = o % (M + 1);
            const long long row = r0 + p;
            if (row < nrows) {
                const cpx<T> zk = buf[(k == M ? 0 : k) * PS + p];
                const cpx<T> zm = cconj(buf[(k == 0 ? 0 : M - k) * PS + p]);
                const cpx<T> e = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y + zm.y)};
                const cpx<T> d = {T(0.5) * (zk.x - zm.x), T(0.5) * (zk.y - zm.y)};
                const cpx<T> wd = cmul(twN[k], d);
                out[row * g.n2h + k] = {e.x + wd.y, e.y - wd.x};
            }
        }
        __syncthreads();
    }
}

// ================================================================ columns
// Block order: array-major (consecutive blocks take adjacent tiles of one
// array, which keeps DRAM pages open) or tile-major (consecutive blocks take
// one tile of every (field, density) array, which keeps the tile's share of
// the reciprocal-space tables in L2).
// MC: a multi-cell batch (per-entry reciprocal vectors and tables from a.ct)
template <typename T, int L, int P, bool MC = false, bool GRP = false, int PV = 0>
__global__ __launch_bounds__((col_NT<T, L, P>())) void k_col(ColArgs a, int nfb, int ntiles)
{
    constexpr int NT = col_NT<T, L, P>();   // this kernel's block size
    constexpr int RSTEP = NT / P;
    constexpr int PER = (L + RSTEP - 1) / RSTEP;
    static_assert(NT % P == 0, "tile width must divide the block");
    static_assert(!(GRP && MC), "a multi-cell batch has one density per block");
    __shared__ cpx<T> buf[L * P];
    __shared__ cpx<T> tws[L];     // W_L^n, read by every stage
    __shared__ double red[NT];
    const int tid = threadIdx.x;
    // a block serves one tile of one field for the densities b0 .. b1 - 1
    // (GRP: a.nbb of them, else one; nfb counts (field, group) pairs): the
    // tile's set-up and its per-element operands are shared by the group
    const int nbb = GRP && a.nbb > 1 ? a.nbb : 1;
    const int nbg = (a.nbatch + nbb - 1) / nbb;
    const int fg = a.tile_major ? (int)(blockIdx.x % (unsigned)nfb)
                                : (int)(blockIdx.x / (unsigned)ntiles);
    const int tile = a.tile_major ? (int)(blockIdx.x / (unsigned)nfb)
                                  : (int)(blockIdx.x % (unsigned)ntiles);
    const int field = fg / nbg;
    const int b0 = (fg % nbg) * nbb;
    const int b1 = b0 + nbb < a.nbatch ? b0 + nbb : a.nbatch;
    const int p = tid % P;
    // column indices in 32 bits (a field holds fewer than 2^32 elements)
    const unsigned c0 = (unsigned)tile * (unsigned)P;
    const unsigned c = c0 + (unsigned)p;
    const bool cvalid = c < (unsigned)a.ncols;
    unsigned cq, cr;
    tile_divmod(c0, (unsigned)p, (unsigned)a.inner, cq, cr);
    const unsigned cbase = cvalid ? cq * (unsigned)a.outer_stride + cr : 0u;
    const cpx<T> *tw = tws;
    const int op = field < MAXKB ? a.op[field] : GO_NONE;

    for (int i = tid; i < L; i += NT) tws[i] = ((const cpx<T> *)a.tw)[i];
    // the first stage of a transform reads element n of this thread's column
    // from memory and the last one writes it back (the stages assign
    // pencil p = tid % P to this thread, as NT is a multiple of P)
    // a column past the end reads column 0 and writes nothing
    const unsigned cofs = cvalid ? cbase : 0u;
    const unsigned es = (unsigned)a.elem_stride;
    // the wide-tile instantiation (P > col_P) serves plain passes only; the
    // default and the narrow (autotuner variant) tiles carry the operations
    constexpr bool OPS = P <= col_P<T, L>();
    Geom g = a.g;
    const void *vext_b = a.vext, *gtab_b = a.gtab;
    if constexpr (MC) {
        vext_b = a.ct[b0].vext;
        gtab_b = a.ct[b0].gtab;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) g.b[i][j] = a.ct[b0].b[i][j];
    }
    unsigned u1, u2;
    tile_divmod(c0, (unsigned)p, (unsigned)g.n2h, u1, u2);
    const int i1 = cvalid ? (int)u1 : 0;
    const int k2 = cvalid ? (int)u2 : 0;
    const int m1 = freq(i1, g.n1);
    const int m2 = (k2 == g.m) ? -g.m : k2;
    // the per-element operand of the field's reciprocal-space operation
    // (element n of column c is the half-spectrum point e = n * ncols + c on
    // axis 0): 1/G^2 (Hartree+ion; 0 at G = 0), G^2 (vW), the Wang-Teter
    // kernel, the preconditioner factor (1 at G = 0), 1 (scale)
    auto operand = [&](int q) -> T {
        const int n = tid / P + q * RSTEP;
        if (n >= L || !cvalid) return T(0);
        const unsigned e = (unsigned)n * (unsigned)a.ncols + c;
        if (op == GO_WT) return ((const T *)gtab_b + 2 * a.g.Nh)[(size_t)e];
        if (op == GO_SCALE) return T(1);
        const T G2 = gvec2<T>(g, freq(n, L), m1, m2);
        if (op == GO_HEXT) return G2 > T(0) ? d_rcp(G2) : T(0);
        if (op == GO_VW) return G2;
        const T q2 = T(a.precond_q2);   // GO_PRECOND
        return G2 > T(0) ? q2 / (G2 + q2 + T(a.precond_h) / G2) : T(1);
    };
    // grouped: the operands are kept in LDS (registers held across the
    // densities would cost occupancy); the first transform's barrier
    // publishes them
    __shared__ T opl[GRP && OPS ? L * P : 1];
    if constexpr (GRP && OPS) {
        if (op != GO_NONE) {
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int n = tid / P + q * RSTEP;
                if (n < L) opl[n * P + p] = operand(q);
            }
        }
    }
    constexpr bool MULTI = make_plan(L, sizeof(T) == 4).n >= 2;
    const double wgt = (k2 == 0 || k2 == g.m) ? 1.0 : 2.0;
    const T invN = T(g.invN);
    const T fourpi = T(4.0 * PI_D);
#pragma unroll 1
    for (int b = b0; b < b1; ++b) {
        if (a.kneed) {
            // a knot spectrum outside the density's knot range is not needed
            const int kn = a.knot0 + field;
            if (kn < a.kneed[2 * b] || kn > a.kneed[2 * b + 1]) continue;   // uniform
        }
        const long long fb = (long long)field * a.nbatch + b;
        const cpx<T> *src = (const cpx<T> *)a.src + fb * a.fstride;
        cpx<T> *dst = (cpx<T> *)a.data + fb * a.fstride;
        // per density, everything that depends on the thread is derived from
        // an opaque copy of its index: recomputed here rather than hoisted
        // out of the loop and held in registers
        const int tl = GRP ? opaque(tid) : tid;
        const int pl = tl % P;
        const unsigned cl = c0 + (unsigned)pl;
        const bool cv = cl < (unsigned)a.ncols;
        unsigned co = cofs;
        if constexpr (GRP) {
            unsigned q1, r1;
            tile_divmod(c0, (unsigned)pl, (unsigned)a.inner, q1, r1);
            co = cv ? q1 * (unsigned)a.outer_stride + r1 : 0u;
        }
        auto ld = [&](unsigned n, unsigned) { return src[(size_t)(co + n * es)]; };
        auto st = [&](unsigned n, unsigned, cpx<T> v) {
            if (cv) dst[(size_t)(co + n * es)] = v;
        };
        if (!OPS || op == GO_NONE) {
            if constexpr (MULTI) {
                // starts and ends with a barrier
                if (a.inv) lds_fft_io<T, L, true, P, NT, P, 1, PV>(buf, tw, tl, ld, st);
                else lds_fft_io<T, L, false, P, NT, P, 1, PV>(buf, tw, tl, ld, st);
                continue;
            } else {
                lds_sync();
                for (int n = tl / P; n < L; n += RSTEP) buf[n * P + pl] = ld(n, pl);
                lds_sync();
                if (a.inv) lds_fft<T, L, true, P, NT, P, 1, PV>(buf, tw, tl);
                else lds_fft<T, L, false, P, NT, P, 1, PV>(buf, tw, tl);
            }
        } else if constexpr (OPS) {
            // v_ext(G) of the Hartree+ion field, fetched now so that its
            // latency overlaps the forward transform
            cpx<T> pre[PER];
            if (op == GO_HEXT && a.use_ext) {
                const cpx<T> *vx = (const cpx<T> *)vext_b;
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int n = tl / P + q * RSTEP;
                    pre[q] = (n < L && cv) ? vx[(size_t)((unsigned)n * (unsigned)a.ncols + cl)]
                                           : cpx<T>{T(0), T(0)};
                }
            }
            // axis 0: element n is i0, column c is (i1, k2)
            lds_fft_src<T, L, false, P, NT, P, 1, PV>(buf, tw, tl, ld);
            const int t = opaque(tl);
            double s0 = 0.0, s1 = 0.0;
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int n = t / P + q * RSTEP;
                if (n >= L || !cv) continue;
                T w;
                if constexpr (GRP) w = opl[n * P + pl];
                else w = operand(q);
                const cpx<T> F = cscale(buf[n * P + pl], invN);
                cpx<T> o;
                if (op == GO_HEXT) {
                    s0 += wgt * (double)((F.x * F.x + F.y * F.y) * w);
                    o = a.use_h ? cscale(F, fourpi * w) : cpx<T>{T(0), T(0)};
                    if (a.use_ext) {
                        const cpx<T> v = pre[q];
                        s1 += wgt * (double)(v.x * F.x + v.y * F.y);
                        o = cadd(o, v);
                    }
                } else if (op == GO_VW) {
                    s0 += wgt * (double)(w * (F.x * F.x + F.y * F.y));
                    o = cscale(F, T(a.lambda_vw) * w);
                } else if (op == GO_SCALE) {
                    o = F;
                } else {   // GO_WT, GO_PRECOND
                    o = cscale(F, w);
                }
                buf[n * P + pl] = o;
            }
            if (op == GO_HEXT || op == GO_VW) {
                double ss[2] = {s0, s1};
                block_sums<NT, 2>(ss, red, tl);
                if (tl == 0) {
                    if (op == GO_HEXT) {
                        part_ptr(a.part, b, SL_H, a.pstride)[tile] = ss[0];
                        part_ptr(a.part, b, SL_EXT, a.pstride)[tile] = ss[1];
                    } else {
                        part_ptr(a.part, b, SL_VW, a.pstride)[tile] = ss[0];
                    }
                }
            }
            lds_sync();
            if (op != GO_SCALE) {
                lds_fft_dst<T, L, true, P, NT, P, 1, PV>(buf, tw, tl, st);   // ends with a barrier
                continue;
            }
        }
        for (int n = tl / P; n < L; n += RSTEP) st(n, pl, buf[n * P + pl]);
        lds_sync();
    }
}

// ================================================================ spline, axis 0
// Step s2/s3: for knots i = knot0 .. knot0+K-1, Phi_i(G) = omega_i(|G|) rho^b(G)
// with omega_i = C_WT G_NL(|G| / (2 k_i)), then the axis-0 inverse.
template <typename T, int L>
__global__ __launch_bounds__((knot_NT<T, L>())) void k_knot_inv(KnotArgs a)
{
    constexpr int P = knot_P<T, L>();
    constexpr int NT = knot_NT<T, L>();   // this kernel's block size
    constexpr int RSTEP = NT / P;
    constexpr int PER = (L + RSTEP - 1) / RSTEP;
    __shared__ cpx<T> buf[L * P];
    __shared__ cpx<T> tws[L];
    const int tid = threadIdx.x;
    const int b = blockIdx.y;
    // knots outside the density's range (their hats vanish at every point)
    // are not transformed; a batch entirely outside it returns at once
    int klo = 0, khi = 1 << 30;
    if (a.kneed) {
        klo = a.kneed[2 * b];
        khi = a.kneed[2 * b + 1];
        if (a.knot0 > khi || a.knot0 + a.K - 1 < klo) return;
    }
    const int p = tid % P;
    const unsigned c0 = (unsigned)blockIdx.x * (unsigned)P;
    const unsigned c = c0 + (unsigned)p;   // 32-bit column index
    const bool cvalid = c < (unsigned)a.ncols;
    Geom g = a.g;
    if (a.ct) {   // multi-cell batch: this entry's reciprocal vectors
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) g.b[i][j] = a.ct[b].b[i][j];
    }
    const unsigned es32 = (unsigned)g.n1 * (unsigned)g.n2h;
    const unsigned cofs = cvalid ? (unsigned)c : 0u;   // past the end: column 0, not written
    const cpx<T> *src = (const cpx<T> *)a.src + b * a.fstride;
    for (int i = tid; i < L; i += NT) tws[i] = ((const cpx<T> *)a.tw)[i];
    const cpx<T> *tw = tws;
    unsigned u1, u2;
    tile_divmod(c0, (unsigned)p, (unsigned)g.n2h, u1, u2);
    const int i1 = cvalid ? (int)u1 : 0;
    const int k2 = cvalid ? (int)u2 : 0;
    const int m1 = freq(i1, g.n1);
    const int m2 = (k2 == g.m) ? -g.m : k2;
    cpx<T> xs[PER];
    T gn[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int n = tid / P + q * RSTEP;
        xs[q] = {T(0), T(0)};
        gn[q] = T(0);
        if (n < L && cvalid) {
            xs[q] = src[(size_t)(c + (unsigned)n * es32)];
            gn[q] = d_sqrt(gvec2<T>(g, freq(n, L), m1, m2));
        }
    }
    for (int kk = 0; kk < a.K; ++kk) {
        if (a.knot0 + kk < klo || a.knot0 + kk > khi) continue;   // uniform in the block
        const T inv2k = T(0.5 / a.knots.k[a.knot0 + kk]);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int n = tid / P + q * RSTEP;
            if (n < L) buf[n * P + p] = cscale(xs[q], T(C_WT_D) * nl_kernel_dev<T>(gn[q] * inv2k, a.kern));
        }
        __syncthreads();
        // the last stage writes this thread's column (pencil p) to memory
        cpx<T> *dst = (cpx<T> *)a.dst + ((long long)kk * a.nbatch + b) * a.fstride;
        lds_fft_dst<T, L, true, P, NT, P, 1>(buf, tw, tid, [&](unsigned n, unsigned, cpx<T> v) {
            if (cvalid) dst[(size_t)(cofs + n * es32)] = v;
        });
    }
}

// EXACT mode: H(G) (+)= sum_{kk} omega_{knot0+kk}(|G|) F[rho^a L_i](G), where the
// K inputs have had the axis-2 r2c and axis-1 forward passes; this kernel does
// the axis-0 forward transform and the normalisation.
template <typename T, int L>
__global__ __launch_bounds__((knot_NT<T, L>())) void k_knot_acc(KnotArgs a)
{
    constexpr int P = knot_P<T, L>();
    constexpr int NT = knot_NT<T, L>();   // this kernel's block size
    constexpr int RSTEP = NT / P;
    constexpr int PER = (L + RSTEP - 1) / RSTEP;
    __shared__ cpx<T> buf[L * P];
    const int tid = threadIdx.x;
    const int b = blockIdx.y;
    // knots outside the density's range contribute exact zeros: skipped; the
    // first batch that meets the range overwrites H
    int klo = 0, khi = 1 << 30;
    bool add_to_h = a.accumulate != 0;
    if (a.kneed) {
        klo = a.kneed[2 * b];
        khi = a.kneed[2 * b + 1];
        if (a.knot0 > khi || a.knot0 + a.K - 1 < klo) return;
        add_to_h = a.knot0 > klo;
    }
    const int p = tid % P;
    const unsigned c0 = (unsigned)blockIdx.x * (unsigned)P;
    const unsigned c = c0 + (unsigned)p;   // 32-bit column index
    const bool cvalid = c < (unsigned)a.ncols;
    Geom g = a.g;
    if (a.ct) {   // multi-cell batch: this entry's reciprocal vectors
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) g.b[i][j] = a.ct[b].b[i][j];
    }
    const unsigned es32 = (unsigned)g.n1 * (unsigned)g.n2h;
    const unsigned cofs = cvalid ? (unsigned)c : 0u;   // past the end: column 0, not written
    const cpx<T> *tw = (const cpx<T> *)a.tw;
    unsigned u1, u2;
    tile_divmod(c0, (unsigned)p, (unsigned)g.n2h, u1, u2);
    const int i1 = cvalid ? (int)u1 : 0;
    const int k2 = cvalid ? (int)u2 : 0;
    const int m1 = freq(i1, g.n1);
    const int m2 = (k2 == g.m) ? -g.m : k2;
    const T invN = T(g.invN);
    cpx<T> acc[PER];
    T gn[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int n = tid / P + q * RSTEP;
        acc[q] = {T(0), T(0)};
        gn[q] = (n < L && cvalid) ? d_sqrt(gvec2<T>(g, freq(n, L), m1, m2)) : T(0);
    }
    for (int kk = 0; kk < a.K; ++kk) {
        if (a.knot0 + kk < klo || a.knot0 + kk > khi) continue;   // uniform in the block
        // the first stage reads this thread's column (pencil p) from memory
        const cpx<T> *src = (const cpx<T> *)a.src + ((long long)kk * a.nbatch + b) * a.fstride;
        lds_fft_src<T, L, false, P, NT, P, 1>(buf, tw, tid,
                                              [&](unsigned n, unsigned) { return src[(size_t)(cofs + n * es32)]; });
        const T inv2k = T(0.5 / a.knots.k[a.knot0 + kk]);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int n = tid / P + q * RSTEP;
            if (n < L) {
                const T w = T(C_WT_D) * nl_kernel_dev<T>(gn[q] * inv2k, a.kern) * invN;
                const cpx<T> v = buf[n * P + p];
                acc[q].x += w * v.x;
                acc[q].y += w * v.y;
            }
        }
        __syncthreads();
    }
    cpx<T> *dst = (cpx<T> *)a.dst + (long long)b * a.fstride;
    if (cvalid) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int n = tid / P + q * RSTEP;
            if (n < L) {
                cpx<T> v = acc[q];
                const size_t e = c + (unsigned)n * es32;
                if (add_to_h) v = cadd(v, dst[e]);
                dst[e] = v;
            }
        }
    }
}

// ================================================================ step s4
// Interpolation of the knot-i potential Phi_i at a pair of points with
// brackets j[c] and weights t[c]: v1 += L_i Phi_i with L_i = 1 - t at knot j
// and t at knot j + 1; for EXACT, v2 collects Phi_{j+1} - Phi_j (the knot
// slope without its 1/(k_{j+1} - k_j), applied once per knot batch by
// knot_slope_scale).  One knot (nk = 1): L = 1, no slope.
template <typename T>
__device__ __forceinline__ void knot_interp(const int (&j)[2], const T (&t)[2], int i, int nk,
                                            int exact, cpx<T> z, cpx<T> &v1, cpx<T> &v2)
{
    const T ph[2] = {z.x, z.y};
    T w1[2], d2[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const bool e0 = j[c] == i, e1 = j[c] + 1 == i;
        w1[c] = nk == 1 ? T(1) : (e0 ? T(1) - t[c] : (e1 ? t[c] : T(0)));
        d2[c] = nk == 1 ? T(0) : (e0 ? -ph[c] : (e1 ? ph[c] : T(0)));
    }
    v1.x += w1[0] * ph[0];
    v1.y += w1[1] * ph[1];
    if (exact) {
        v2.x += d2[0];
        v2.y += d2[1];
    }
}

template <typename T>
__device__ __forceinline__ void knot_slope_scale(const Knots &kn, const int (&j)[2], cpx<T> &v2)
{
    if (kn.nk == 1) return;
    v2.x *= T(1.0 / (kn.k[j[0] + 1] - kn.k[j[0]]));
    v2.y *= T(1.0 / (kn.k[j[1] + 1] - kn.k[j[1]]));
}

// ================================================================ LDA xc
// Exchange-correlation of the unpolarised homogeneous electron gas at the
// local density (E_xc of eq. "efunc"): Dirac exchange eps_x = C_X rho^(1/3)
// and the Perdew-Zunger (1981) fit of the correlation energy in
// r_s = (3/(4 pi rho))^(1/3), with the parameters Perdew and Zunger published
// (the parametrisation the paper's applications use).  r3 = rho^(1/3).
// eps = eps_x + eps_c, v = d(rho eps)/d rho = (4/3) eps_x + eps_c -
// (r_s/3) d eps_c/d r_s; both 0 at rho = 0.
constexpr double XC_CX = -0.7385587663820223;   // -(3/4)(3/pi)^(1/3)
constexpr double XC_RS = 0.6203504908994001;    // (3/(4 pi))^(1/3)
constexpr double PZ_G = -0.1423, PZ_B1 = 1.0529, PZ_B2 = 0.3334;             // r_s >= 1
constexpr double PZ_A = 0.0311, PZ_B = -0.048, PZ_C = 0.0020, PZ_D = -0.0116;  // r_s < 1

template <typename T>
__device__ __forceinline__ void lda_xc_point(T rho, T r3, T &eps, T &v)
{
    if (!(rho > T(0))) {
        eps = T(0);
        v = T(0);
        return;
    }
    const T ex = T(XC_CX) * r3;
    const T rs = T(XC_RS) * d_rcp(r3);
    T ec, vc;
    if (rs >= T(1)) {
        const T sq = d_sqrt_fast(rs);
        const T iden = d_rcp(T(1) + T(PZ_B1) * sq + T(PZ_B2) * rs);
        ec = T(PZ_G) * iden;
        vc = ec * (T(1) + T(7.0 / 6.0 * PZ_B1) * sq + T(4.0 / 3.0 * PZ_B2) * rs) * iden;
    } else {
        const T lr = d_log(rs);
        ec = T(PZ_A) * lr + T(PZ_B) + T(PZ_C) * rs * lr + T(PZ_D) * rs;
        vc = T(PZ_A) * lr + T(PZ_B - PZ_A / 3.0) + T(2.0 / 3.0 * PZ_C) * rs * lr +
             T((2.0 * PZ_D - PZ_C) / 3.0) * rs;
    }
    eps = ex + ec;
    v = T(4.0 / 3.0) * ex + vc;
}

// ================================================================ final combine
// Per-point combine of the real-space fields into v = dE/drho and
// g = dE/dphi (eqs. "euler", "euler2"), with the FP64 partial sums of
// rho^alpha Phi (E_NL), g phi, g^2 and phi^2.  Inputs per point: x (rho or
// phi), hv = v_H + v_ext, wv = -lambda nabla^2 phi, nl = the WT potential
// Phi or the EXACT spline field A (exclusive), s1/s2 = the spline
// accumulators sum_i L_i Phi_i and sum_i L_i' Phi_i.
//
// CF = 0 takes the term set from the arguments and any alpha.  A non-zero CF
// fixes the term set at compile time (CF_* in kernels.hpp; the host picks one
// when the functional matches it exactly) and, when a nonlocal term is present, alpha
// = 5/6 (the WT and spline exponents of the paper's kernels), so that every
// power of rho the terms need comes from two exponentials:
//   p = rho^(1/6):              phi = p^3, rho^(1/3) = p^2, rho^(2/3) = p^4,
//                               rho^(5/6) = p^5, k_F = (3 pi^2)^(1/3) p^2
//   q = max(rho, floor)^(-1/6): rho_s^(-1/6) = q, rho_s^(-1/2) = q^3,
//                               rho_s^(-1) = q^6

template <typename T>
struct CombineConst {
    T alpha, floor_rho, lfloor, k_lo, k_hi;
    T yfloor;   // floor^(-1/6) (FP64 fixed term sets)
};

template <typename T>
__device__ __forceinline__ CombineConst<T> combine_const(const RowInvArgs &a)
{
    CombineConst<T> c;
    c.alpha = T(a.alpha);
    c.floor_rho = T(a.floor);
    c.lfloor = d_log2(c.floor_rho);
    c.yfloor = c.floor_rho > T(0) ? d_exp2(c.lfloor * T(-1.0 / 6.0)) : __builtin_huge_val();
    c.k_lo = a.spline ? T(a.knots.k[0]) : T(0);
    c.k_hi = a.spline ? T(a.knots.k[a.knots.nk - 1]) : T(0);
    return c;
}

// partial sums of the combine: rho^a Phi, g phi, g^2, phi^2 and, with the
// LDA term (always in the general combine), rho eps_xc
template <int CF> constexpr int combine_nsum() { return (CF == 0 || (CF & CB_XC)) ? 5 : 4; }

// PH: 1 = x is phi, 0 = x is rho (both fixed at compile time, fixed term
// sets only), -1 = taken from the arguments.  S: the type of the partial
// sums (double; the fixed term sets also take T, a thread's own few points,
// which the caller adds to its FP64 sums).
template <typename T, int CF, int PH = -1, typename S = double>
__device__ __forceinline__ void combine_point(const RowInvArgs &a, const CombineConst<T> &cc, T x,
                                              T hv, T wv, T nl, T s1, T s2, T &vo, T &go,
                                              S (&sums)[combine_nsum<CF>()])
{
    static_assert(PH == -1 || CF != 0, "the general combine reads the input kind at run time");
    static_assert(CF != 0 || sizeof(S) == 8, "the general combine sums in FP64");
    const bool in_phi = PH < 0 ? a.in_is_phi != 0 : PH == 1;
    T phi, rho;
    if (in_phi) {
        phi = x;
        rho = phi * phi;
    } else {
        // with a fixed input kind a negative density is not clamped: the
        // evaluation's prologue counts it and the call fails
        rho = PH == 0 ? x : (x > T(0) ? x : T(0));
        phi = T(0);
    }
    // FP64 fixed term sets take p and q from rho^(-1/6) (rsixth) instead
    // of the FP64 logarithm and exponentials
    constexpr bool NEWTON = CF != 0 && sizeof(T) == 8;
    T lu = T(0), lr = T(0);
    if constexpr (NEWTON) {
    } else if constexpr (PH >= 0) {
        // rho >= 0 here and log2(0) = -inf: no branch for empty points;
        // rho_s = max(rho, floor) in the log domain
        lu = d_log2(rho);
        lr = d_fmax(lu, cc.lfloor);
    } else {
        lu = rho > T(0) ? d_log2(rho) : neg_inf<T>();
        lr = rho >= cc.floor_rho ? lu : cc.lfloor;
    }
    T vv = T(0), gg = T(0);
    if constexpr (CF != 0) {
        constexpr T AL = T(5.0 / 6.0);
        T p, q;
        if constexpr (NEWTON) {
            // p = rho^(1/6) = rho y^5, q = max(rho, floor)^(-1/6)
            const double y = rsixth((double)rho);
            const double y2 = y * y;
            p = T(rho * (y2 * y2 * y));
            q = T(rho >= cc.floor_rho && y > 0.0 ? y : cc.yfloor);
        } else {
            p = d_exp2(lu * T(1.0 / 6.0));
            q = d_exp2(lr * T(-1.0 / 6.0));
        }
        const T p2 = p * p;
        if (!in_phi) phi = p2 * p;
        // phi = rho^(1/2) >= 0 when the input is rho
        const T sgn = PH == 0 ? T(1) : (phi < T(0) ? T(-1) : T(1));
        const T p4 = p2 * p2;
        const T q3 = q * q * q;
        // every fixed set the host picks holds H+ext, vW and TF: the sums
        // start from them
        if constexpr ((CF & CB_H) && (CF & CB_VW) && (CF & CB_TF)) {
            const T vt = T(5.0 / 3.0 * C_TF_D) * p4;
            const T ht = hv + vt;
            vv = ht + (PH == 0 ? T(0.5) : T(0.5) * sgn) * wv * q3;
            gg = wv + T(2) * phi * ht;
        } else {
            if constexpr ((CF & CB_H) != 0) {
                vv += hv;
                gg += T(2) * phi * hv;
            }
            if constexpr ((CF & CB_VW) != 0) {
                vv += T(0.5) * wv * sgn * q3;
                gg += wv;
            }
            if constexpr ((CF & CB_TF) != 0) {
                const T vt = T(5.0 / 3.0 * C_TF_D) * p4;
                vv += vt;
                gg += T(2) * phi * vt;
            }
        }
        if constexpr ((CF & CB_XC) != 0) {
            T eps, vx;
            lda_xc_point(rho, p2, eps, vx);
            vv += vx;
            gg += T(2) * phi * vx;
            sums[4] += (S)(rho * eps);
        }
        if constexpr ((CF & (CB_WT | CB_A | CB_SPL)) != 0) {
            const T ra = p4 * p;         // rho^a
            const T fa_ = sgn * p2;      // phi rho^(a-1)
            if constexpr ((CF & CB_WT) != 0) {
                vv += T(2) * AL * q * nl;
                gg += T(4) * AL * fa_ * nl;
                sums[0] += (S)(ra * nl);
            }
            if constexpr ((CF & CB_A) != 0) {
                vv += AL * q * nl;
                gg += T(2) * AL * fa_ * nl;
            }
            if constexpr ((CF & CB_SPL) != 0) {
                sums[0] += (S)(ra * s1);
                if constexpr ((CF & CB_EXACT) == 0) {
                    vv += T(2) * AL * q * s1;
                    gg += T(4) * AL * fa_ * s1;
                } else {
                    const T kf = T(KF_C) * p2;
                    const T dk = (kf > cc.k_lo && kf < cc.k_hi) ? kf * T(1.0 / 3.0) : T(0);
                    vv += AL * q * s1 + ra * dk * (q3 * q3) * s2;
                    gg += T(2) * (AL * fa_ * s1 + fa_ * dk * s2);
                }
            }
        }
    } else {
        if (!a.in_is_phi) phi = d_sqrt(rho);
        const T sgn = phi < T(0) ? T(-1) : T(1);
        const T alpha = cc.alpha;
        const bool has_wt = a.fld_wt >= 0, has_a = a.fld_a >= 0;
        T ra = T(0), ra1 = T(0), fa_ = T(0);
        if (a.spline || has_wt || has_a) {
            ra = d_exp2(alpha * lu);                   // rho^a
            ra1 = d_exp2((alpha - T(1)) * lr);         // rho_s^(a-1)
            fa_ = sgn * d_exp2((alpha - T(0.5)) * lu); // phi rho^(a-1)
        }
        if (a.fld_hext >= 0) {                         // v_H + v_ext
            vv += hv;
            gg += T(2) * phi * hv;
        }
        if (a.fld_vw >= 0) {                           // -lambda nabla^2 phi
            vv += T(0.5) * wv * sgn * d_exp2(T(-0.5) * lr);
            gg += wv;
        }
        if (has_wt) {                                  // Wang-Teter Phi
            vv += T(2) * alpha * ra1 * nl;
            gg += T(4) * alpha * fa_ * nl;
            sums[0] += (double)(ra * nl);
        }
        if (has_a) {                                   // EXACT: F^-1[sum_i omega_i F[rho^a L_i]]
            vv += alpha * ra1 * nl;
            gg += T(2) * alpha * fa_ * nl;
        }
        if (a.use_tf) {
            const T vt = T(5.0 / 3.0 * C_TF_D) * d_exp2(lu * T(2.0 / 3.0));
            vv += vt;
            gg += T(2) * phi * vt;
        }
        if (a.use_xc) {
            T eps, vx;
            lda_xc_point(rho, d_exp2(lu * T(1.0 / 3.0)), eps, vx);
            vv += vx;
            gg += T(2) * phi * vx;
            sums[4] += (double)(rho * eps);
        }
        if (a.spline) {
            sums[0] += (double)(ra * s1);
            if (!a.exact) {
                vv += T(2) * alpha * ra1 * s1;
                gg += T(4) * alpha * fa_ * s1;
            } else {
                const T kf = kf_from_log2(lu);
                const T dk = (kf > cc.k_lo && kf < cc.k_hi) ? kf * T(1.0 / 3.0) : T(0);
                vv += alpha * ra1 * s1 + ra * dk * d_exp2(-lr) * s2;
                gg += T(2) * (alpha * fa_ * s1 + fa_ * dk * s2);
            }
        }
    }
    sums[1] += (S)gg * (S)phi;
    sums[2] += (S)gg * (S)gg;
    sums[3] += (S)phi * (S)phi;
    vo = vv;
    go = gg;
}

// ================================================================ row inverse
// c2r of one block of half-spectrum rows into buf (z[n] = f[2n] + i f[2n+1],
// element n of row p at buf[n * PS + p]):
// Z[k] = (X[k] + conj X[M-k]) + i (X[k] - conj X[M-k]) conj(W^k), k < M, with
// the imaginary parts of X[0] and X[M] dropped (Re of the inverse).
template <typename T, int M, int P, int PS>
__device__ __forceinline__ void c2r_rows(cpx<T> *buf, const cpx<T> *__restrict__ spec,
                                         long long r0, long long nrows, int n2h,
                                         const cpx<T> *__restrict__ twM,
                                         const cpx<T> *__restrict__ twN, int tid)
{
    constexpr int PAIRS = P * M;
    for (int o = tid; o < PAIRS; o += NT) {
        const int p = o / M, k = o % M;
        const long long row = r0 + p;
        cpx<T> z = {T(0), T(0)};
        if (row < nrows) {
            const cpx<T> *x = spec + row * n2h;
            cpx<T> xk = x[k];
            cpx<T> xm = x[M - k];
            if (k == 0) {
                xk.y = T(0);
                xm.y = T(0);
            }
            const cpx<T> s = {xk.x + xm.x, xk.y - xm.y};   // X[k] + conj X[M-k]
            const cpx<T> d = {xk.x - xm.x, xk.y + xm.y};   // X[k] - conj X[M-k]
            const cpx<T> dw = cmul(d, cconj(twN[k]));
            z = {s.x - dw.y, s.y + dw.x};                  // s + i dw
        }
        buf[k * PS + p] = z;
    }
    __syncthreads();
    lds_fft<T, M, true, P, NT, PS>(buf, twM, tid);
}

// c2r of the knot passes: NPEN pencils, pencil pp < P row r0 + pp of sa,
// pencil P <= pp < 2P the same row of sb (zeros without sb); element n of
// pencil pp at buf[n * ES + pp].  With NPEN = 2P two knots' rows go through
// one transform, twice the butterflies per Stockham stage of a one-spectrum
// pass, so that the stages of short rows keep more waves busy between
// barriers.  Each load pair (X[k], X[M-k]), k = 0 .. M/2, gives Z[k] and
// Z[M-k]; every load of the pass is issued before the first is used (one
// memory latency per pass rather than one per item), and twN is read from
// LDS.
template <typename T, int M, int P, int NPEN, int ES, int CH>
__device__ __forceinline__ void c2r_knot_chunk(cpx<T> *buf, const cpx<T> *__restrict__ sa,
                                               const cpx<T> *__restrict__ sb, long long r0,
                                               long long nrows, int n2h, const cpx<T> *twN,
                                               int tid, int q0)
{
    constexpr int H = M / 2 + 1;
    constexpr int ITEMS = NPEN * H;
    cpx<T> xk[CH], xm[CH];
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int o = tid + (q0 + c) * NT;
        const int pp = o / H, k = o % H;
        const int p = pp < P ? pp : pp - P;
        const cpx<T> *spec = pp < P ? sa : sb;
        xk[c] = {T(0), T(0)};
        xm[c] = {T(0), T(0)};
        if ((ITEMS % NT == 0 || o < ITEMS) && spec && r0 + p < nrows) {
            const cpx<T> *x = spec + (r0 + p) * n2h;
            xk[c] = x[k];
            xm[c] = x[M - k];
        }
    }
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        const int o = tid + (q0 + c) * NT;
        if (ITEMS % NT != 0 && o >= ITEMS) continue;
        const int pp = o / H, k = o % H;
        cpx<T> xa = xk[c], xb = xm[c];
        if (k == 0) {
            xa.y = T(0);
            xb.y = T(0);
        }
        // Z[k] = (X[k] + conj X[M-k]) + i (X[k] - conj X[M-k]) conj(W^k)
        const cpx<T> s0 = {xa.x + xb.x, xa.y - xb.y};
        const cpx<T> d0 = {xa.x - xb.x, xa.y + xb.y};
        const cpx<T> w0 = cmul(d0, cconj(twN[k]));
        buf[k * ES + pp] = {s0.x - w0.y, s0.y + w0.x};
        // Z[M-k] from the same pair, X[M-k] and X[k] exchanged
        if (k > 0 && 2 * k != M) {
            const cpx<T> s1 = {xb.x + xa.x, xb.y - xa.y};
            const cpx<T> d1 = {xb.x - xa.x, xb.y + xa.y};
            const cpx<T> w1 = cmul(d1, cconj(twN[M - k]));
            buf[(M - k) * ES + pp] = {s1.x - w1.y, s1.y + w1.x};
        }
    }
}
// The loads of a pass go out in NCH chunks (one for the S3S4 epilogue; two
// where the EXACT epilogue's second accumulator leaves fewer registers).
template <typename T, int M, int P, int NPEN, int ES, int NCH>
__device__ __forceinline__ void c2r_knot_rows(cpx<T> *buf, const cpx<T> *__restrict__ sa,
                                              const cpx<T> *__restrict__ sb, long long r0,
                                              long long nrows, int n2h, const cpx<T> *twM,
                                              const cpx<T> *twN, int tid)
{
    constexpr int PI = (NPEN * (M / 2 + 1) + NT - 1) / NT;
    constexpr int CH = (PI + NCH - 1) / NCH;
    // per-item indices recomputed per pass, not hoisted out of the pass loop
    tid = opaque(tid);
    c2r_knot_chunk<T, M, P, NPEN, ES, CH>(buf, sa, sb, r0, nrows, n2h, twN, tid, 0);
    if constexpr (PI > CH)
        c2r_knot_chunk<T, M, P, NPEN, ES, PI - CH>(buf, sa, sb, r0, nrows, n2h, twN, tid, CH);
    __syncthreads();
    lds_fft<T, M, true, NPEN, NT, ES>(buf, twM, tid);
}

// The knot epilogue is instantiated with CF = CB_SPL (S3S4) or CB_SPL |
// CB_EXACT and asks for at least 4 resident waves per SIMD (128 VGPRs):
// measured faster than the 3 its unconstrained allocation allows.
constexpr int ROW_KNOTS_MINW = 4;
template <int MODE, int CF> constexpr int row_inv_minw()
{
    return MODE != EP_KNOTS ? 1 : ROW_KNOTS_MINW;
}
static_assert(MAXKNOTS <= NT, "the knot tables are filled by one load per thread");
template <typename T, int M, int CF, int MODE>
__global__ __launch_bounds__(NT, (row_inv_minw<MODE, CF>())) void k_row_inv(RowInvArgs a, Geom g)
{
    constexpr int P = row_P<T, M>();
    constexpr int PS = P + 1;
    constexpr int PAIRS = P * M;
    constexpr int PER = (PAIRS + NT - 1) / NT;
    // the knot epilogue transforms two knots' rows at once (c2r_knot_rows)
    // for rows of up to 256 complex points (longer rows have enough
    // butterflies per stage, and the pair's registers would spill)
    constexpr bool PAIR = MODE == EP_KNOTS && M <= 256;
    constexpr bool KN = MODE == EP_KNOTS;
    __shared__ cpx<T> buf[M * (PAIR ? 2 * P + 1 : PS)];
    __shared__ double red[5 * NT / 64];
    // knot passes: twM and twN (M + 1 entries) and the knots in LDS, and the
    // passes some point of the block needs, one bit per pass and wave
    __shared__ cpx<T> twl[KN ? 2 * M + 1 : 1];
    __shared__ T knl[KN ? MAXKNOTS : 1];
    __shared__ unsigned needw[KN ? NT / 64 : 1];
    const int tid = threadIdx.x;
    const int b = blockIdx.y;
    const long long nrows = (long long)g.n0 * g.n1;
    const long long r0 = (long long)blockIdx.x * P;
    const cpx<T> *twM = (const cpx<T> *)a.twM;
    const cpx<T> *twN = (const cpx<T> *)a.twN;
    auto spec_of = [&](int f) {
        return (const cpx<T> *)a.spec + f * a.spec_fstride + (long long)b * g.Nh;
    };
    // pair q of this thread: row p = idx / M, element n = idx % M
    bool valid[PER];
    long long offs[PER];
    int lds_at[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int idx = tid + q * NT;
        const int p = idx / M, n = idx % M;
        valid[q] = idx < PAIRS && r0 + p < nrows;
        offs[q] = valid[q] ? (r0 + p) * g.n2 + 2 * n : 0;
        lds_at[q] = n * PS + p;
    }

    // one instantiation per mode, so that each holds only the registers its
    // own epilogue needs (the fixed term sets, CF != 0, are combines)
    if constexpr (MODE == EP_STORE) {
        for (int f = 0; f < a.nfields; ++f) {
            c2r_rows<T, M, P, PS>(buf, spec_of(f), r0, nrows, g.n2h, twM, twN, tid);
            const long long fo = ((long long)f * a.nbatch + b) * g.N;
            bool done = false;
            if constexpr (sizeof(T) == 8) {
                if (a.out_f32) {
                    // the FP64 von Weizsaecker leg hands its result to the
                    // FP32 combine
                    float *outf = (float *)a.out + fo;
#pragma unroll
                    for (int q = 0; q < PER; ++q)
                        if (valid[q]) {
                            const cpx<T> v = buf[lds_at[q]];
                            *(float2 *)(outf + offs[q]) = make_float2((float)v.x, (float)v.y);
                        }
                    done = true;
                }
            }
            if (!done) {
                T *out = (T *)a.out + fo;
#pragma unroll
                for (int q = 0; q < PER; ++q)
                    if (valid[q]) *(cpx<T> *)(out + offs[q]) = buf[lds_at[q]];
            }
            __syncthreads();
        }
        return;
    }

    // a knot batch entirely outside the density's knot range adds nothing;
    // the first batch that meets it initialises the accumulators
    bool acc_init = a.acc_init != 0;
    int klo = 0, khi = 1 << 30;   // knots transformed for this density
    if constexpr (MODE == EP_KNOTS) {
        if (a.kneed) {
            klo = a.kneed[2 * b];
            khi = a.kneed[2 * b + 1];
            if (a.knot0 > khi || a.knot0 + a.nfields - 1 < klo) return;
            acc_init = a.knot0 <= klo;
        }
    }

    // input density (rho or phi) for this block's pairs
    const T *in = (const T *)a.in + (long long)b * g.N;
    cpx<T> xin[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q)
        xin[q] = valid[q] ? *(const cpx<T> *)(in + offs[q]) : cpx<T>{T(0), T(0)};

    if constexpr (MODE == EP_KNOTS) {
        // step s4 for this batch of knots: v1 += L_i Phi_i, v2 += L_i' Phi_i
        // (v2 for EXACT only, fixed at compile time by CF)
        constexpr bool exact = (CF & CB_EXACT) != 0;
        const int nk = a.knots.nk;
        constexpr int TWQ = (2 * M + 1 + NT - 1) / NT;
#pragma unroll
        for (int q = 0; q < TWQ; ++q) {
            const int i = tid + q * NT;
            if (i < 2 * M + 1) twl[i] = i < M ? twM[i] : twN[i - M];
        }
        if (tid < nk) knl[tid] = T(a.knots.k[tid]);   // nk <= MAXKNOTS <= NT
        __syncthreads();
        // per point: knot brackets (two 8-bit fields per pair, nk <= 64) and
        // weights.  The pair's row, element and validity are recomputed
        // from an opaque copy of the thread index where they are used
        // instead of being held in registers across the passes.
        auto pair_at = [&](int q, int t, int &p, int &n) {
            const int idx = t + q * NT;
            p = idx / M;
            n = idx % M;
            return idx < PAIRS && r0 + p < nrows;
        };
        unsigned jp[PER];
        T tt[PER][2];
        cpx<T> v1[PER], v2[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const T vv[2] = {xin[q].x, xin[q].y};
            int jq[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const T rho = a.in_is_phi ? vv[c] * vv[c] : (vv[c] > T(0) ? vv[c] : T(0));
                const T lu = rho > T(0) ? d_log2(rho) : neg_inf<T>();
                bool inside;
                knot_bracket_tab(kf_from_log2(lu), nk, a.knots.log_spacing, a.knots.inv_span, knl,
                                 jq[c], tt[q][c], inside);
            }
            jp[q] = (unsigned)jq[0] | ((unsigned)jq[1] << 8);
            v1[q] = {T(0), T(0)};
            v2[q] = {T(0), T(0)};
        }
        auto jj_of = [&](int q, int (&j)[2]) {
            j[0] = (int)(jp[q] & 0xffu);
            j[1] = (int)(jp[q] >> 8);
        };
        // knots f and f + 1 per pass (PAIR, else one); a pass is skipped if
        // no point of this block uses its knots (a knot used by none adds
        // exact zeros).  Bit f / KS of need: pass f, for the whole block
        // after one reduction.
        constexpr int KS = PAIR ? 2 : 1;
        constexpr int NCH = exact ? 2 : 1;
        unsigned need = 0;
        {
            const int t = opaque(tid);
            for (int f = 0; f < a.nfields; f += KS) {
                const int i = a.knot0 + f;
                const int ihi = i + (PAIR && f + 1 < a.nfields ? 1 : 0);
                bool nf = false;
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    int p, n, j[2];
                    jj_of(q, j);
                    nf |= pair_at(q, t, p, n) &&
                          (nk == 1 || (j[0] >= i - 1 && j[0] <= ihi) || (j[1] >= i - 1 && j[1] <= ihi));
                }
                need |= nf ? 1u << (f / KS) : 0u;
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) need |= (unsigned)__shfl_xor((int)need, off);
        if ((tid & 63) == 0) needw[tid >> 6] = need;
        __syncthreads();
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) need |= needw[w];
        constexpr int PS2 = 2 * P + 1;
        for (int f = 0; f < a.nfields; f += KS) {
            if (!((need >> (f / KS)) & 1u)) continue;
            const int i = a.knot0 + f;
            const bool two = PAIR && f + 1 < a.nfields;
            // a pass's partner knot outside the transformed range reads as
            // zeros (its weight is zero at every point of this density)
            const bool ina = i >= klo && i <= khi, inb = two && i + 1 >= klo && i + 1 <= khi;
            if constexpr (PAIR)
                c2r_knot_rows<T, M, P, 2 * P, PS2, NCH>(buf, ina ? spec_of(f) : nullptr,
                                                        inb ? spec_of(f + 1) : nullptr, r0,
                                                        nrows, g.n2h, twl, twl + M, tid);
            else
                c2r_knot_rows<T, M, P, P, PS, NCH>(buf, spec_of(f), nullptr, r0, nrows, g.n2h,
                                                   twl, twl + M, tid);
            const int t = opaque(tid);
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                int p, n, j[2];
                if (!pair_at(q, t, p, n)) continue;
                jj_of(q, j);
                if constexpr (PAIR) {
                    const int at2 = n * PS2 + p;
                    knot_interp(j, tt[q], i, nk, exact, buf[at2], v1[q], v2[q]);
                    if (two) knot_interp(j, tt[q], i + 1, nk, exact, buf[at2 + P], v1[q], v2[q]);
                } else {
                    knot_interp(j, tt[q], i, nk, exact, buf[n * PS + p], v1[q], v2[q]);
                }
            }
            __syncthreads();
        }
        if constexpr (exact) {
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                int j[2];
                jj_of(q, j);
                knot_slope_scale(a.knots, j, v2[q]);
            }
        }
        // accumulators: every load issued before the first add
        T *acc1 = (T *)a.acc1 + (long long)b * g.N;
        T *acc2 = exact ? (T *)a.acc2 + (long long)b * g.N : nullptr;
        const int t = opaque(tid);
        long long po[PER];
        bool ok[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            int p, n;
            ok[q] = pair_at(q, t, p, n);
            po[q] = ok[q] ? (r0 + p) * g.n2 + 2 * n : 0;
        }
        if (!acc_init) {
            cpx<T> o1[PER];
#pragma unroll
            for (int q = 0; q < PER; ++q)
                o1[q] = ok[q] ? *(const cpx<T> *)(acc1 + po[q]) : cpx<T>{T(0), T(0)};
#pragma unroll
            for (int q = 0; q < PER; ++q) v1[q] = cadd(v1[q], o1[q]);
            if constexpr (exact) {
#pragma unroll
                for (int q = 0; q < PER; ++q)
                    o1[q] = ok[q] ? *(const cpx<T> *)(acc2 + po[q]) : cpx<T>{T(0), T(0)};
#pragma unroll
                for (int q = 0; q < PER; ++q) v2[q] = cadd(v2[q], o1[q]);
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (!ok[q]) continue;
            *(cpx<T> *)(acc1 + po[q]) = v1[q];
            if constexpr (exact) *(cpx<T> *)(acc2 + po[q]) = v2[q];
        }
        return;
    }

    // EP_COMBINE: v = dE/drho and g = dE/dphi from all terms
    cpx<T> fh[PER], fl[PER], fn[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) fh[q] = fl[q] = fn[q] = {T(0), T(0)};
    // with vw_field set (general combine only: the host picks CF = 0 for it)
    // the von Weizsaecker term arrives in real space
    const bool vwf = CF == 0 && a.vw_field != nullptr;
    const int flds[4] = {a.fld_hext, vwf ? -1 : a.fld_vw, a.fld_wt, a.fld_a};
    for (int s = 0; s < 4; ++s) {
        if (flds[s] < 0) continue;
        c2r_rows<T, M, P, PS>(buf, spec_of(flds[s]), r0, nrows, g.n2h, twM, twN, tid);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (!valid[q]) continue;
            const cpx<T> z = buf[lds_at[q]];
            if (s == 0) fh[q] = z;
            else if (s == 1) fl[q] = z;
            else fn[q] = z;   // WT Phi or the EXACT field A (exclusive)
        }
        __syncthreads();
    }
    if constexpr (CF == 0) {
        if (vwf) {
            const T *vw = (const T *)a.vw_field + (long long)b * g.N;
#pragma unroll
            for (int q = 0; q < PER; ++q)
                if (valid[q]) fl[q] = *(const cpx<T> *)(vw + offs[q]);
        }
    }
    const T *acc1 = a.spline ? (const T *)a.acc1 + (long long)b * g.N : nullptr;
    const T *acc2 = (a.spline && a.exact) ? (const T *)a.acc2 + (long long)b * g.N : nullptr;
    T *vout = a.v_out ? (T *)a.v_out + (long long)b * g.N : nullptr;
    T *gout = a.g_out ? (T *)a.g_out + (long long)b * g.N : nullptr;
    const CombineConst<T> cc = combine_const<T>(a);
    double sums[combine_nsum<CF>()] = {};   // rho^a Phi, g phi, g^2, phi^2 (, rho eps_xc)
    // the input kind (phi or rho) is fixed per launch: compiled in for the
    // fixed term sets
    auto points = [&](auto ph) {
        constexpr int PH = decltype(ph)::value;
        // a fixed term set sums a thread's few points in T first
        using S = std::conditional_t<CF != 0, T, double>;
        S ts[combine_nsum<CF>()] = {};
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if (!valid[q]) continue;
            cpx<T> a1 = {T(0), T(0)}, a2 = {T(0), T(0)};
            if (acc1) a1 = *(const cpx<T> *)(acc1 + offs[q]);
            if (acc2) a2 = *(const cpx<T> *)(acc2 + offs[q]);
            cpx<T> vo, go;
            combine_point<T, CF, PH, S>(a, cc, xin[q].x, fh[q].x, fl[q].x, fn[q].x, a1.x, a2.x,
                                        vo.x, go.x, ts);
            combine_point<T, CF, PH, S>(a, cc, xin[q].y, fh[q].y, fl[q].y, fn[q].y, a1.y, a2.y,
                                        vo.y, go.y, ts);
            if (vout) *(cpx<T> *)(vout + offs[q]) = vo;
            if (gout) *(cpx<T> *)(gout + offs[q]) = go;
        }
#pragma unroll
        for (int k = 0; k < combine_nsum<CF>(); ++k) sums[k] = (double)ts[k];
    };
    if constexpr (CF != 0) {
        if (a.in_is_phi) points(std::integral_constant<int, 1>());
        else points(std::integral_constant<int, 0>());
    } else {
        points(std::integral_constant<int, -1>());
    }
    block_sums<NT, combine_nsum<CF>()>(sums, red, tid);
    if (tid == 0) {
        part_ptr(a.part, b, SL_NL, a.pstride)[blockIdx.x] = sums[0];
        part_ptr(a.part, b, SL_GPHI, a.pstride)[blockIdx.x] = sums[1];
        part_ptr(a.part, b, SL_GG, a.pstride)[blockIdx.x] = sums[2];
        part_ptr(a.part, b, SL_PHIPHI, a.pstride)[blockIdx.x] = sums[3];
        if constexpr (combine_nsum<CF>() == 5)
            part_ptr(a.part, b, SL_XC, a.pstride)[blockIdx.x] = sums[combine_nsum<CF>() - 1];
    }
}

// ================================================================ plane kernels
// For grids whose (i1, k2) plane fits in LDS, one block handles a whole
// i0-plane of one density: the axis-2 r2c of every row and the axis-1 c2c of
// every column run back to back on the same padded buffer (element (i1, k)
// at buf[k * A + i1], A odd), so the spectrum needs one HBM round trip less
// per field; the inverse side mirrors it and ends in the combine or in the
// spline interpolation.
template <int N1> constexpr int plane_A() { return (N1 % 2 == 0) ? N1 + 1 : N1; }
template <int N1, int M> constexpr int plane_NT() { return 1024; }
// minimum resident waves per SIMD the compiler must allow: two 1024-thread
// blocks per CU for FP32 (64 VGPRs), one for FP64
template <typename T> constexpr int plane_minw() { return sizeof(T) == 4 ? 8 : 4; }
// FP32: the kernels also stage the input plane in LDS (two blocks per CU
// share its 160 KB, so a block stays within 96 KB); FP64: one block per CU,
// the input plane is read again from memory where it is needed (it stays in
// L2 between the reads) and the block may take all 160 KB
template <typename T> constexpr bool plane_stage_x() { return sizeof(T) == 4; }
template <typename T, int N1, int M> constexpr bool plane_fits()
{
    // the padded plane, the staged input plane (N1 x 2M reals) if any and
    // the twiddles (N1 + 2M + 1 complex)
    const long long reals = (long long)(M + 1) * plane_A<N1>() * 2 +
                            (plane_stage_x<T>() ? (long long)N1 * 2 * (M + 1) : 0) +
                            2LL * (N1 + 2 * M + 1);
    // FP64 planes larger than 96 x 48 spill registers at one 1024-thread
    // block per CU; those grids keep the row and column passes
    return reals * (long long)sizeof(T) <= (plane_stage_x<T>() ? 98304 : 155648) &&
           (plane_stage_x<T>() || N1 * M <= 96 * 48);
}

// X[k] from Z[k] and Z[M-k] (r2c unpack), W^k = twN[k]
template <typename T>
__device__ __forceinline__ cpx<T> r2c_unpack(cpx<T> zk, cpx<T> zmk, cpx<T> w)
{
    const cpx<T> zm = cconj(zmk);
    const cpx<T> e = {T(0.5) * (zk.x + zm.x), T(0.5) * (zk.y + zm.y)};
    const cpx<T> d = {T(0.5) * (zk.x - zm.x), T(0.5) * (zk.y - zm.y)};
    const cpx<T> wd = cmul(w, d);
    return {e.x + wd.y, e.y - wd.x};
}

// Z[k] from X[k] and X[M-k] (c2r pack), W^k = twN[k]
template <typename T>
__device__ __forceinline__ cpx<T> c2r_pack(cpx<T> xk, cpx<T> xm, cpx<T> w)
{
    const cpx<T> s = {xk.x + xm.x, xk.y - xm.y};
    const cpx<T> d = {xk.x - xm.x, xk.y + xm.y};
    const cpx<T> dw = cmul(d, cconj(w));
    return {s.x - dw.y, s.y + dw.x};
}

// copies the twiddle tables of both axes and of the r2c (un)pack into LDS:
// [W_N1^n, n < N1 | W_M^n, n < M | W_2M^k, k <= M]
template <typename T, int N1, int M, int NTP>
__device__ __forceinline__ void stage_plane_twiddles(cpx<T> *tws, const void *tw1, const void *twM,
                                                     const void *twN, int tid)
{
    for (int i = tid; i < N1 + 2 * M + 1; i += NTP)
        tws[i] = i < N1 ? ((const cpx<T> *)tw1)[i]
                        : (i < N1 + M ? ((const cpx<T> *)twM)[i - N1]
                                      : ((const cpx<T> *)twN)[i - N1 - M]);
}

template <typename T, int N1, int M>
__global__ __launch_bounds__((plane_NT<N1, M>()), (plane_minw<T>())) void k_plane_fwd(RowFwdArgs a, Geom g)
{
    constexpr int NTP = plane_NT<N1, M>();
    constexpr int A = plane_A<N1>();
    constexpr int PAIRS = N1 * M;
    constexpr int PER = (PAIRS + NTP - 1) / NTP;
    __shared__ cpx<T> buf[(M + 1) * A];
    constexpr bool STX = plane_stage_x<T>();
    __shared__ cpx<T> xs[STX ? N1 * M : 1];   // the input plane, read once from HBM
    __shared__ cpx<T> tws[N1 + 2 * M + 1];   // twiddles of both axes and the r2c unpack
    __shared__ double red[3 * NTP / 64];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x, b = blockIdx.y;
    const cpx<T> *in = (const cpx<T> *)((const T *)a.in + (long long)b * g.N +
                                        (long long)i0 * N1 * g.n2);
    stage_plane_twiddles<T, N1, M, NTP>(tws, a.tw1, a.twM, a.twN, tid);
    const cpx<T> *tw1 = tws;
    const cpx<T> *twM = tws + N1;
    const cpx<T> *twN = tws + N1 + M;

    constexpr unsigned S = sizeof(cpx<T>);
    const BufRes rin = buf_res(in, PAIRS * S);
    cpx<T> x[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const unsigned idx = (unsigned)(tid + q * NTP);
        x[q] = idx < (unsigned)PAIRS ? bld<cpx<T>>(rin, (unsigned)tid * S, (unsigned)(q * NTP) * S)
                                     : cpx<T>{T(0), T(0)};
        if constexpr (STX) {
            if (idx < (unsigned)PAIRS) xs[idx] = x[q];
        }
    }
    lds_sync();
    const bool knots = a.nfields > 0 && a.kind[0] == FK_KNOT;
    if (a.partials) {
        double sums[3] = {0.0, 0.0, 0.0};
        auto count = [&](auto ph) {
            constexpr bool P = decltype(ph)::value;
            T ts[2] = {T(0), T(0)};   // a thread's few points, summed in T
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                if (tid + q * NTP >= PAIRS) continue;
                const T xv[2] = {x[q].x, x[q].y};
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const T v = xv[c];
                    const bool ok = d_finite(v) && (P || v >= T(0));
                    if (!ok) {
                        sums[2] += 1.0;
                        continue;
                    }
                    const T rho = P ? v * v : v;   // >= 0; log2(0) = -inf
                    ts[0] += rho;
                    if constexpr (sizeof(T) == 8) {
                        const double y = rsixth(rho);   // rho^(2/3) = rho y^2
                        ts[1] += rho * (rho * (y * y));
                    } else {
                        ts[1] += rho * d_exp2(d_log2(rho) * T(2.0 / 3.0));
                    }
                }
            }
            sums[0] = (double)ts[0];
            sums[1] = (double)ts[1];
        };
        if (a.in_is_phi) count(std::true_type());
        else count(std::false_type());
        if constexpr (3 * NTP * sizeof(double) <= sizeof(buf))
            block_sums_lds<NTP, 3>(sums, (double *)buf, red, tid);
        else
            block_sums<NTP, 3>(sums, red, tid);
        if (tid == 0) {
            part_ptr(a.part, b, SL_RHO, a.pstride)[i0] = sums[0];
            part_ptr(a.part, b, SL_TF, a.pstride)[i0] = sums[1];
            part_ptr(a.part, b, SL_BAD, a.pstride)[i0] = sums[2];
        }
    }
#pragma unroll 1
    for (int f = 0; f < a.nfields; ++f) {
        const int t = opaque(tid);
        const int kind = a.kind[f];
        const int knot = a.knot0 + f;
        if (kind == FK_KNOT) {
            // EXACT spline: f_i = rho^a L_i(k_F), written to buf first
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const int idx = t + q * NTP;
                if (idx >= PAIRS) continue;
                const int i1 = idx / M, n = idx % M;
                cpx<T> xq;
                if constexpr (STX) xq = xs[idx];
                else xq = in[idx];
                const T xv[2] = {xq.x, xq.y};
                T o[2];
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const T v = xv[c];
                    const T rho = a.in_is_phi ? v * v : (v > T(0) ? v : T(0));
                    const T lu = rho > T(0) ? d_log2(rho) : neg_inf<T>();
                    int j;
                    T t;
                    bool inside;
                    knot_bracket_kf(kf_from_log2(lu), a.knots, j, t, inside);
                    const T L = a.knots.nk == 1 ? T(1)
                                                : (j == knot ? T(1) - t
                                                             : (j + 1 == knot ? t : T(0)));
                    o[c] = L == T(0) ? T(0) : L * d_exp2(T(a.alpha) * lu);
                }
                buf[n * A + i1] = {o[0], o[1]};
            }
            lds_sync();
            // axis 2: half-length complex transforms of the N1 rows
            lds_fft<T, M, false, N1, NTP, A, 1>(buf, twM, t);
        } else {
            // rho, phi or rho^beta at the points 2n, 2n + 1 of row i1 into
            // element n (computing them in the first FFT stage instead puts the
            // transcendentals on the fewer threads that hold butterflies:
            // measured slower), then the axis-2 half-length transforms
            // (the field kind and the input kind are uniform: each pair is
            // compiled separately so that a point computes only its own field)
            const bool b56 = a.beta == 5.0 / 6.0;
            auto fill = [&](auto kd, auto ph) {
                constexpr int K = decltype(kd)::value;
                constexpr bool P = decltype(ph)::value;
                auto field = [&](T v) -> T {
                    if constexpr (K == FK_RAW) return v;
                    else if constexpr (K == FK_RHO) return P ? v * v : v;
                    // (a negative density is counted by the prologue and
                    // fails the evaluation: no clamp here)
                    else if constexpr (K == FK_PHI) return P ? v : d_sqrt_fast(v);
                    else if constexpr (sizeof(T) == 8) {
                        // FK_RHOB; FP64 with beta = 5/6: rho^(5/6) = rho rho^(-1/6)
                        const T r = P ? v * v : v;
                        return b56 ? r * rsixth(r) : d_exp2(T(a.beta) * d_log2(r));
                    } else return d_exp2(T(a.beta) * d_log2(P ? v * v : v));   // FK_RHOB; log2(0) = -inf
                };
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const unsigned idx = (unsigned)(t + q * NTP);
                    if (idx >= (unsigned)PAIRS) continue;
                    const unsigned i1 = idx / (unsigned)M, n = idx % (unsigned)M;
                    cpx<T> xq;
                    if constexpr (STX) xq = xs[idx];
                    else xq = in[idx];
                    buf[n * A + i1] = {field(xq.x), field(xq.y)};
                }
            };
            using std::integral_constant;
            using std::true_type;
            using std::false_type;
            if (a.in_is_phi) {
                if (kind == FK_RHO) fill(integral_constant<int, FK_RHO>(), true_type());
                else if (kind == FK_PHI) fill(integral_constant<int, FK_PHI>(), true_type());
                else if (kind == FK_RHOB) fill(integral_constant<int, FK_RHOB>(), true_type());
                else fill(integral_constant<int, FK_RAW>(), true_type());
            } else {
                if (kind == FK_RHO) fill(integral_constant<int, FK_RHO>(), false_type());
                else if (kind == FK_PHI) fill(integral_constant<int, FK_PHI>(), false_type());
                else if (kind == FK_RHOB) fill(integral_constant<int, FK_RHOB>(), false_type());
                else fill(integral_constant<int, FK_RAW>(), false_type());
            }
            lds_sync();
            lds_fft<T, M, false, N1, NTP, A, 1>(buf, twM, t);
        }
        (void)knots;
        // axis 1 over the M + 1 columns: the first stage unpacks element i1
        // of column k of the r2c half spectrum from Z[k] and Z[M-k] of row
        // i1 (Z has period M; X[0] and X[M] are real), the last stage writes
        // it straight to out[i1 * (M + 1) + k]
        cpx<T> *out = (cpx<T> *)a.out + f * a.out_fstride + (long long)b * g.Nh +
                      (long long)i0 * N1 * (M + 1);
        const BufRes ro = buf_res(out, (unsigned)(N1 * (M + 1)) * S);
        lds_fft_io<T, N1, false, M + 1, NTP, 1, A>(
            buf, tw1, t,
            [&](unsigned n, unsigned p) {
                const unsigned k = p == (unsigned)M ? 0u : p;
                const unsigned km = k == 0 ? 0u : M - k;
                cpx<T> x = r2c_unpack(buf[k * A + n], buf[km * A + n], twN[p]);
                if (k == 0) x.y = T(0);
                return x;
            },
            [&](unsigned nb, unsigned dn, unsigned p, cpx<T> v) {
                bst(ro, (nb * (M + 1) + p) * S, dn * (unsigned)(M + 1) * S, v);
            });
    }
}

// Inverse of one field's (i0, batch) plane into buf: axis-1 c2c of the
// M + 1 columns, c2r pack, axis-2 transforms; element (i1, n) of the result
// (f[2n] + i f[2n+1] of row i1) is at buf[n * A + i1].
template <typename T, int N1, int M, int NTP>
__device__ __forceinline__ void plane_inverse(cpx<T> *buf, const cpx<T> *spec,
                                              const cpx<T> *tw1,
                                              const cpx<T> *twM,
                                              const cpx<T> *twN, int tid)
{
    constexpr int A = plane_A<N1>();
    constexpr unsigned S = sizeof(cpx<T>);
    tid = opaque(tid);
    // axis 1: the first stage reads column k (element i1) straight from the
    // spectrum, spec[i1 * (M + 1) + k]
    const BufRes rs = buf_res(spec, (unsigned)(N1 * (M + 1)) * S);
    lds_fft_src<T, N1, true, M + 1, NTP, 1, A>(
        buf, tw1, tid, [&](unsigned nb, unsigned dn, unsigned p) {
            return bld<cpx<T>>(rs, (nb * (M + 1) + p) * S, dn * (unsigned)(M + 1) * S);
        });
    // axis 2: the first stage forms element n of row i1 of the half-length
    // input by the c2r pack Z[n] = (X[n] + conj X[M-n]) + i (X[n] - conj
    // X[M-n]) conj(W^n) (imaginary parts of X[0] and X[M] dropped).  A lane
    // holds n = nb + dn for dn = 0, NB, .., DNMAX (NB = M / R, R the first
    // radix): X[M - n] is addressed from the lane's lowest row, M - nb - DNMAX
    // (>= 1), so that every offset is a positive constant.
    constexpr Plan pm = make_plan(M, sizeof(T) == 4);
    constexpr unsigned DNMAX = (unsigned)((pm.r[0] - 1) * (M / pm.r[0]));
    lds_fft_src<T, M, true, N1, NTP, A, 1>(buf, twM, tid, [&](unsigned nb, unsigned dn, unsigned p) {
        const unsigned n = nb + dn;
        cpx<T> xk = buf[n * A + p];
        // the base is kept opaque (folded back into M - n, every element
        // would cost a subtraction and a multiply-add); the same asm on the
        // same operands is formed once for all dn
        unsigned lo = ((unsigned)M - nb - DNMAX) * A + p;
        asm("" : "+v"(lo));
        cpx<T> xm = buf[lo + (DNMAX - dn) * A];
        if (dn == 0 && nb == 0) {
            xk.y = T(0);
            xm.y = T(0);
        }
        return c2r_pack(xk, xm, twN[n]);
    });
}

// As plane_inverse with the field's spectrum plane already in LDS (pre,
// element (i1, k) at pre[i1 * (M + 1) + k]); next() is called once the
// axis-1 transform has read pre (after a barrier), so that it can start the
// copy of the next plane into it.
template <typename T, int N1, int M, int NTP, class NEXT>
__device__ __forceinline__ void plane_inverse_pre(cpx<T> *buf, const cpx<T> *pre,
                                                  const cpx<T> *tw1, const cpx<T> *twM,
                                                  const cpx<T> *twN, int tid, const NEXT &next)
{
    constexpr int A = plane_A<N1>();
    tid = opaque(tid);
    lds_copy_wait();   // this wave's part of pre; lds_fft_src starts with a barrier
    lds_fft_src<T, N1, true, M + 1, NTP, 1, A>(
        buf, tw1, tid, [&](unsigned n, unsigned p) { return pre[n * (M + 1) + p]; });
    next();
    constexpr Plan pm = make_plan(M, sizeof(T) == 4);
    constexpr unsigned DNMAX = (unsigned)((pm.r[0] - 1) * (M / pm.r[0]));
    lds_fft_src<T, M, true, N1, NTP, A, 1>(buf, twM, tid, [&](unsigned nb, unsigned dn, unsigned p) {
        const unsigned n = nb + dn;
        cpx<T> xk = buf[n * A + p];
        unsigned lo = ((unsigned)M - nb - DNMAX) * A + p;
        asm("" : "+v"(lo));
        cpx<T> xm = buf[lo + (DNMAX - dn) * A];
        if (dn == 0 && nb == 0) {
            xk.y = T(0);
            xm.y = T(0);
        }
        return c2r_pack(xk, xm, twN[n]);
    });
}

template <typename T, int N1, int M, int MODE, int CF>
__global__ __launch_bounds__((plane_NT<N1, M>()), (plane_minw<T>())) void k_plane_inv(RowInvArgs a, Geom g)
{
    constexpr int NTP = plane_NT<N1, M>();
    constexpr int A = plane_A<N1>();
    constexpr int PAIRS = N1 * M;
    constexpr int PER = (PAIRS + NTP - 1) / NTP;
    __shared__ cpx<T> buf[(M + 1) * A];
    constexpr bool STX = plane_stage_x<T>();
    // the staged input plane; with a fixed term set (PRE) the same array
    // first takes each field's spectrum plane, copied in while the previous
    // field is transformed, and then the input plane
    constexpr bool PRE = STX && CF != 0 && MODE == EP_COMBINE;
    __shared__ cpx<T> xsbuf[STX ? N1 * (M + 1) : 1];
    __shared__ cpx<T> tws[N1 + 2 * M + 1];
    __shared__ double red[5 * NTP / 64];
    const int tid = threadIdx.x;
    const int i0 = blockIdx.x, b = blockIdx.y;
    stage_plane_twiddles<T, N1, M, NTP>(tws, a.tw1, a.twM, a.twN, tid);
    lds_sync();
    const cpx<T> *tw1 = tws;
    const cpx<T> *twM = tws + N1;
    const cpx<T> *twN = tws + N1 + M;
    const long long plane_off = (long long)i0 * N1 * (M + 1);
    auto spec_of = [&](int f) {
        return (const cpx<T> *)a.spec + f * a.spec_fstride + (long long)b * g.Nh + plane_off;
    };
    const long long real_off = (long long)b * g.N + (long long)i0 * N1 * g.n2;
    auto at = [&](int t, int q) {
        const int idx = t + q * NTP;
        return (idx % M) * A + idx / M;
    };

    if constexpr (MODE == EP_STORE) {
#pragma unroll 1
        for (int f = 0; f < a.nfields; ++f) {
            const int t = opaque(tid);
            plane_inverse<T, N1, M, NTP>(buf, spec_of(f), tw1, twM, twN, t);
            cpx<T> *out = (cpx<T> *)((T *)a.out + (long long)f * a.nbatch * g.N + real_off);
#pragma unroll
            for (int q = 0; q < PER; ++q)
                if (t + q * NTP < PAIRS) out[t + q * NTP] = buf[at(t, q)];
            lds_sync();
        }
        return;
    }
    else {

    const cpx<T> *in = (const cpx<T> *)((const T *)a.in + real_off);
    constexpr unsigned S = sizeof(cpx<T>);
    // pair q of thread t is element t + q NTP of the plane: byte offset t S
    // per lane plus the constant q NTP S
    const BufRes rin = buf_res(in, PAIRS * S);
    cpx<T> xin[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q)
        xin[q] = tid + q * NTP < PAIRS ? bld<cpx<T>>(rin, (unsigned)tid * S, (unsigned)(q * NTP) * S)
                                       : cpx<T>{T(0), T(0)};

    if constexpr (MODE == EP_KNOTS) {
        bool acc_init = a.acc_init != 0;
        if (a.kneed) {
            const int klo = a.kneed[2 * b], khi = a.kneed[2 * b + 1];
            if (a.knot0 > khi || a.knot0 + a.nfields - 1 < klo) return;
            acc_init = a.knot0 <= klo;
        }
        int jj[PER][2];
        T tt[PER][2];
        cpx<T> v1[PER], v2[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const T vv[2] = {xin[q].x, xin[q].y};
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const T rho = a.in_is_phi ? vv[c] * vv[c] : (vv[c] > T(0) ? vv[c] : T(0));
                const T lu = rho > T(0) ? d_log2(rho) : neg_inf<T>();
                bool inside;
                knot_bracket_kf(kf_from_log2(lu), a.knots, jj[q][c], tt[q][c], inside);
            }
            v1[q] = {T(0), T(0)};
            v2[q] = {T(0), T(0)};
        }
        const int nk = a.knots.nk;
#pragma unroll 1
        for (int f = 0; f < a.nfields; ++f) {
            const int t = opaque(tid);
            const int i = a.knot0 + f;
            bool need = false;
#pragma unroll
            for (int q = 0; q < PER; ++q)
                need |= t + q * NTP < PAIRS &&
                        (nk == 1 || jj[q][0] == i || jj[q][0] + 1 == i || jj[q][1] == i ||
                         jj[q][1] + 1 == i);
            if (!__syncthreads_or(need)) continue;
            plane_inverse<T, N1, M, NTP>(buf, spec_of(f), tw1, twM, twN, t);
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                if (t + q * NTP >= PAIRS) continue;
                const cpx<T> z = buf[at(t, q)];
                knot_interp(jj[q], tt[q], i, nk, a.exact, z, v1[q], v2[q]);
            }
            lds_sync();
        }
        if (a.exact) {
#pragma unroll
            for (int q = 0; q < PER; ++q) knot_slope_scale(a.knots, jj[q], v2[q]);
        }
        cpx<T> *acc1 = (cpx<T> *)((T *)a.acc1 + real_off);
        cpx<T> *acc2 = a.exact ? (cpx<T> *)((T *)a.acc2 + real_off) : nullptr;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = tid + q * NTP;
            if (idx >= PAIRS) continue;
            acc1[idx] = acc_init ? v1[q] : cadd(v1[q], acc1[idx]);
            if (acc2) acc2[idx] = acc_init ? v2[q] : cadd(v2[q], acc2[idx]);
        }
        return;
    }
    else {

    // EP_COMBINE.  The fields come back from reciprocal space one at a time;
    // a thread keeps the raw values of all but the last in registers (at
    // most two fields: WT and the EXACT spline field are exclusive) and
    // forms v and g once, after the last inverse, so that the per-point
    // powers of rho are evaluated once.  The input plane is kept in LDS (xs).
    cpx<T> *xs = (cpx<T> *)xsbuf;
    constexpr unsigned PLANE_BYTES = (unsigned)(N1 * (M + 1)) * S;
    // the input plane is copied into LDS asynchronously when 16-byte aligned
    const bool xasync = PRE && (((size_t)in) & 15) == 0;
    if constexpr (STX && !PRE) {
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if (tid + q * NTP < PAIRS) xs[tid + q * NTP] = xin[q];
    }
    if constexpr (PRE)
        lds_copy_async<NTP>(xs, spec_of(a.fld_hext), PLANE_BYTES, tid);
    lds_sync();
    const cpx<T> *acc1 = a.spline ? (const cpx<T> *)((const T *)a.acc1 + real_off) : nullptr;
    const cpx<T> *acc2 = (a.spline && a.exact) ? (const cpx<T> *)((const T *)a.acc2 + real_off)
                                                : nullptr;
    cpx<T> *vout = a.v_out ? (cpx<T> *)((T *)a.v_out + real_off) : nullptr;
    cpx<T> *gout = a.g_out ? (cpx<T> *)((T *)a.g_out + real_off) : nullptr;
    const CombineConst<T> cc = combine_const<T>(a);
    double sums[combine_nsum<CF>()] = {};   // rho^a Phi, g phi, g^2, phi^2 (, rho eps_xc)
    // fields in the order H+ext, vW, WT | EXACT-A (the present ones); WT and
    // A are exclusive and come last, so only H+ext and vW are ever held
    cpx<T> fh[PER], fv[PER];
    if constexpr (CF != 0) {
        // fixed term set: H+ext and vW are always present (the host picks a
        // fixed set only then), the nonlocal field when NLF.  The transforms
        // are unrolled, so the held fields need no per-field selects, and
        // the input kind (phi or rho) is compiled into the point loop.
        constexpr bool NLF = (CF & (CB_WT | CB_A)) != 0;
        // LDS slot of pair q of thread t after the inverse: element (i1, n)
        // at n * A + i1
        auto uat = [&](int t, int q) {
            const unsigned idx = (unsigned)(t + q * NTP);
            return (idx % (unsigned)M) * (unsigned)A + idx / (unsigned)M;
        };
        auto hold = [&](cpx<T> (&f)[PER], int t) {
#pragma unroll
            for (int q = 0; q < PER; ++q)
                if (t + q * NTP < PAIRS) f[q] = buf[uat(t, q)];
        };
        const int fld_nl = (CF & CB_WT) ? a.fld_wt : a.fld_a;
        // PRE: the next plane (a spectrum, or the input plane after the
        // last) streams into xs while this field's axis-2 transforms run
        auto copy_x = [&]() {
            if (xasync) lds_copy_async<NTP>(xs, in, (unsigned)PAIRS * S, opaque(tid));
        };
        auto inverse = [&](int fld, int t, auto next) {
            if constexpr (PRE) plane_inverse_pre<T, N1, M, NTP>(buf, xs, tw1, twM, twN, t, next);
            else plane_inverse<T, N1, M, NTP>(buf, spec_of(fld), tw1, twM, twN, t);
        };
        {
            const int t = opaque(tid);
            inverse(a.fld_hext, t, [&]() {
                lds_copy_async<NTP>(xs, spec_of(a.fld_vw), PLANE_BYTES, opaque(tid));
            });
            hold(fh, t);
            lds_sync();
        }
        {
            const int t = opaque(tid);
            inverse(a.fld_vw, t, [&]() {
                if constexpr (NLF) lds_copy_async<NTP>(xs, spec_of(fld_nl), PLANE_BYTES, opaque(tid));
                else copy_x();
            });
            if constexpr (NLF) {
                hold(fv, t);
                lds_sync();
            }
        }
        if constexpr (NLF) {
            const int t = opaque(tid);
            inverse(fld_nl, t, copy_x);
        }
        if constexpr (PRE) {
            lds_copy_wait();
            lds_sync();
        }
        const BufRes ra1 = buf_res(acc1, PAIRS * S), ra2 = buf_res(acc2, PAIRS * S);
        const BufRes rvo = buf_res(vout, PAIRS * S), rgo = buf_res(gout, PAIRS * S);
        auto points = [&](auto ph) {
            constexpr int PH = decltype(ph)::value;
            const int t = opaque(tid);
            const unsigned vo_ = (unsigned)t * S;
            T ts[combine_nsum<CF>()] = {};   // a thread's few points, summed in T
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const unsigned idx = (unsigned)(t + q * NTP);
                if (idx >= (unsigned)PAIRS) continue;
                const unsigned so = (unsigned)(q * NTP) * S;
                cpx<T> s1 = {T(0), T(0)}, s2 = {T(0), T(0)};
                if (acc1) s1 = bld<cpx<T>>(ra1, vo_, so);
                if (acc2) s2 = bld<cpx<T>>(ra2, vo_, so);
                cpx<T> xq;
                if constexpr (PRE) xq = xasync ? xs[idx] : bld<cpx<T>>(rin, vo_, so);
                else if constexpr (STX) xq = xs[idx];
                else xq = bld<cpx<T>>(rin, vo_, so);
                const cpx<T> zb = buf[uat(t, q)];
                const cpx<T> zh = fh[q];
                const cpx<T> zv = NLF ? fv[q] : zb;
                const cpx<T> zl = NLF ? zb : cpx<T>{T(0), T(0)};
                cpx<T> vo, go;
                combine_point<T, CF, PH, T>(a, cc, xq.x, zh.x, zv.x, zl.x, s1.x, s2.x, vo.x, go.x,
                                            ts);
                combine_point<T, CF, PH, T>(a, cc, xq.y, zh.y, zv.y, zl.y, s1.y, s2.y, vo.y, go.y,
                                            ts);
                if (vout) bst(rvo, vo_, so, vo);
                if (gout) bst(rgo, vo_, so, go);
            }
#pragma unroll
            for (int k = 0; k < combine_nsum<CF>(); ++k) sums[k] = (double)ts[k];
        };
        if (a.in_is_phi) points(std::integral_constant<int, 1>());
        else points(std::integral_constant<int, 0>());
    } else {
        // the von Weizsaecker term may arrive in real space (general combine
        // only: the host picks CF = 0 for it)
        const bool vwf = a.vw_field != nullptr;
        const int all[4] = {a.fld_hext, vwf ? -1 : a.fld_vw, a.fld_wt, a.fld_a};
        int last = -1;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (all[k] >= 0) last = k;
#pragma unroll
        for (int q = 0; q < PER; ++q) fh[q] = fv[q] = {T(0), T(0)};
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
            if (all[k] < 0) continue;
            const int t = opaque(tid);
            plane_inverse<T, N1, M, NTP>(buf, spec_of(all[k]), tw1, twM, twN, t);
            if (k == last) break;   // the last field stays in buf
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                if (t + q * NTP >= PAIRS) continue;
                const cpx<T> z = buf[at(t, q)];
                if (k == 0) fh[q] = z;
                else fv[q] = z;
            }
            lds_sync();
        }
        const int t = opaque(tid);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int idx = t + q * NTP;
            if (idx >= PAIRS) continue;
            cpx<T> s1 = {T(0), T(0)}, s2 = {T(0), T(0)};
            if (acc1) s1 = acc1[idx];
            if (acc2) s2 = acc2[idx];
            cpx<T> xq;
            if constexpr (STX) xq = xs[idx];
            else xq = in[idx];
            const cpx<T> zl = last >= 0 ? buf[at(t, q)] : cpx<T>{T(0), T(0)};
            const cpx<T> zh = last == 0 ? zl : fh[q];
            cpx<T> zv = last == 1 ? zl : fv[q];
            if (vwf) zv = ((const cpx<T> *)((const T *)a.vw_field + real_off))[idx];
            cpx<T> vo, go;
            combine_point<T, CF>(a, cc, xq.x, zh.x, zv.x, zl.x, s1.x, s2.x, vo.x, go.x, sums);
            combine_point<T, CF>(a, cc, xq.y, zh.y, zv.y, zl.y, s1.y, s2.y, vo.y, go.y, sums);
            if (vout) vout[idx] = vo;
            if (gout) gout[idx] = go;
        }
    }
    if constexpr (combine_nsum<CF>() * NTP * sizeof(double) <= sizeof(buf))
        block_sums_lds<NTP, combine_nsum<CF>()>(sums, (double *)buf, red, tid);
    else
        block_sums<NTP, combine_nsum<CF>()>(sums, red, tid);
    if (tid == 0) {
        part_ptr(a.part, b, SL_NL, a.pstride)[i0] = sums[0];
        part_ptr(a.part, b, SL_GPHI, a.pstride)[i0] = sums[1];
        part_ptr(a.part, b, SL_GG, a.pstride)[i0] = sums[2];
        part_ptr(a.part, b, SL_PHIPHI, a.pstride)[i0] = sums[3];
        if constexpr (combine_nsum<CF>() == 5)
            part_ptr(a.part, b, SL_XC, a.pstride)[i0] = sums[combine_nsum<CF>() - 1];
    }
    }
    }
}

#define OFDFT_PLANES(X) \
    X(16, 8) X(24, 12) X(32, 16) X(48, 24) X(54, 27) X(64, 32) X(72, 36) X(96, 48) \
    X(108, 54) X(128, 64)

template <typename T, int N1, int M>
hipError_t plane_fwd_go(const Geom &g, int nbatch, const RowFwdArgs &a, int &nblocks, hipStream_t s)
{
    if constexpr (!plane_fits<T, N1, M>()) {
        return hipErrorInvalidValue;
    } else {
        nblocks = g.n0;
        if (a.partials && nblocks > a.pstride) return hipErrorInvalidValue;
        if (a.nfields < 0 || a.nfields > MAXKB) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_plane_fwd<T, N1, M>), dim3(g.n0, nbatch), dim3(plane_NT<N1, M>()),
                           0, s, a, g);
        return hipGetLastError();
    }
}

template <typename T, int N1, int M>
hipError_t plane_inv_go(const Geom &g, const RowInvArgs &a, int &nblocks, hipStream_t s)
{
    if constexpr (!plane_fits<T, N1, M>()) {
        return hipErrorInvalidValue;
    } else {
        nblocks = g.n0;
        if (a.mode == EP_COMBINE && nblocks > a.pstride) return hipErrorInvalidValue;
        const dim3 grid(g.n0, a.nbatch), block(plane_NT<N1, M>());
        if (a.mode == EP_STORE)
            hipLaunchKernelGGL((k_plane_inv<T, N1, M, EP_STORE, 0>), grid, block, 0, s, a, g);
        else if (a.mode == EP_KNOTS)
            hipLaunchKernelGGL((k_plane_inv<T, N1, M, EP_KNOTS, 0>), grid, block, 0, s, a, g);
        else if (a.cf == CF_LOCAL)
            hipLaunchKernelGGL((k_plane_inv<T, N1, M, EP_COMBINE, CF_LOCAL>), grid, block, 0, s, a, g);
        else if (a.cf == CF_WT)
            hipLaunchKernelGGL((k_plane_inv<T, N1, M, EP_COMBINE, CF_WT>), grid, block, 0, s, a, g);
        else if (a.cf == CF_S3S4)
            hipLaunchKernelGGL((k_plane_inv<T, N1, M, EP_COMBINE, CF_S3S4>), grid, block, 0, s, a, g);
        else if (a.cf == CF_EXACT)
            hipLaunchKernelGGL((k_plane_inv<T, N1, M, EP_COMBINE, CF_EXACT>), grid, block, 0, s, a, g);
        else if (a.cf == (CF_LOCAL | CB_XC))
            hipLaunchKernelGGL((k_plane_inv<T, N1, M, EP_COMBINE, CF_LOCAL | CB_XC>), grid, block, 0, s, a, g);
        else if (a.cf == (CF_WT | CB_XC))
            hipLaunchKernelGGL((k_plane_inv<T, N1, M, EP_COMBINE, CF_WT | CB_XC>), grid, block, 0, s, a, g);
        else if (a.cf == (CF_S3S4 | CB_XC))
            hipLaunchKernelGGL((k_plane_inv<T, N1, M, EP_COMBINE, CF_S3S4 | CB_XC>), grid, block, 0, s, a, g);
        else if (a.cf == (CF_EXACT | CB_XC))
            hipLaunchKernelGGL((k_plane_inv<T, N1, M, EP_COMBINE, CF_EXACT | CB_XC>), grid, block, 0, s, a, g);
        else
            hipLaunchKernelGGL((k_plane_inv<T, N1, M, EP_COMBINE, 0>), grid, block, 0, s, a, g);
        return hipGetLastError();
    }
}

#define OFDFT_PLANE_CASE_SUP(N1, M) if (n1 == N1 && m == M) return plane_fits<PT, N1, M>();
#define OFDFT_PLANE_CASE_F(N1, M) if (g.n1 == N1 && g.m == M) return plane_fwd_go<PT, N1, M>(g, nbatch, a, nb, s);
#define OFDFT_PLANE_CASE_I(N1, M) if (g.n1 == N1 && g.m == M) return plane_inv_go<PT, N1, M>(g, a, nb, s);
#define OFDFT_INSTANTIATE_PLANES()                                                              \
    template <> bool plane_supported<PT>(int n1, int m)                                         \
    {                                                                                           \
        OFDFT_PLANES(OFDFT_PLANE_CASE_SUP)                                                      \
        return false;                                                                           \
    }                                                                                           \
    template <> hipError_t launch_plane_fwd<PT>(const Geom &g, int nbatch, const RowFwdArgs &a, \
                                                int &nb, hipStream_t s)                         \
    {                                                                                           \
        OFDFT_PLANES(OFDFT_PLANE_CASE_F)                                                        \
        return hipErrorInvalidValue;                                                            \
    }                                                                                           \
    template <> hipError_t launch_plane_inv<PT>(const Geom &g, const RowInvArgs &a, int &nb,    \
                                                hipStream_t s)                                  \
    {                                                                                           \
        OFDFT_PLANES(OFDFT_PLANE_CASE_I)                                                        \
        return hipErrorInvalidValue;                                                            \
    }

// ================================================================ launchers
#define OFDFT_LENGTHS(X) \
    X(2) X(3) X(4) X(6) X(8) X(9) X(12) X(16) X(18) X(24) X(27) X(32) X(36) X(48) X(54) \
    X(64) X(72) X(81) X(96) X(108) X(128) X(144) X(162) X(192) X(216) X(256) X(288) X(384) \
    X(512) X(1024)

template <typename T, int M>
hipError_t row_fwd_go(const Geom &g, int nbatch, const RowFwdArgs &a, int &nblocks, hipStream_t s)
{
    constexpr int P = row_P<T, M>();
    const long long nrows = (long long)g.n0 * g.n1;
    nblocks = (int)((nrows + P - 1) / P);
    if (a.partials && nblocks > a.pstride) return hipErrorInvalidValue;
    if (a.nfields < 0 || a.nfields > MAXKB) return hipErrorInvalidValue;
    dim3 grid(nblocks, nbatch);
    hipLaunchKernelGGL((k_row_fwd<T, M>), grid, dim3(NT), 0, s, a, g);
    return hipGetLastError();
}

template <typename T, int M, int CF = 0>
hipError_t row_inv_go(const Geom &g, const RowInvArgs &a, int &nblocks, hipStream_t s)
{
    constexpr int P = row_P<T, M>();
    const long long nrows = (long long)g.n0 * g.n1;
    nblocks = (int)((nrows + P - 1) / P);
    if (a.mode == EP_COMBINE && nblocks > a.pstride) return hipErrorInvalidValue;
    dim3 grid(nblocks, a.nbatch);
    if (CF != 0 || a.mode == EP_COMBINE)
        hipLaunchKernelGGL((k_row_inv<T, M, CF, EP_COMBINE>), grid, dim3(NT), 0, s, a, g);
    else if (a.mode == EP_KNOTS && a.exact)
        hipLaunchKernelGGL((k_row_inv<T, M, CB_SPL | CB_EXACT, EP_KNOTS>), grid, dim3(NT), 0, s, a, g);
    else if (a.mode == EP_KNOTS)
        hipLaunchKernelGGL((k_row_inv<T, M, CB_SPL, EP_KNOTS>), grid, dim3(NT), 0, s, a, g);
    else
        hipLaunchKernelGGL((k_row_inv<T, M, 0, EP_STORE>), grid, dim3(NT), 0, s, a, g);
    return hipGetLastError();
}

template <typename T, int M>
hipError_t row_combine_fixed_go(const Geom &g, const RowInvArgs &a, int &nblocks, hipStream_t s)
{
    if (a.mode != EP_COMBINE) return hipErrorNotSupported;
    switch (a.cf) {
    case CF_LOCAL: return row_inv_go<T, M, CF_LOCAL>(g, a, nblocks, s);
    case CF_WT: return row_inv_go<T, M, CF_WT>(g, a, nblocks, s);
    case CF_S3S4: return row_inv_go<T, M, CF_S3S4>(g, a, nblocks, s);
    case CF_EXACT: return row_inv_go<T, M, CF_EXACT>(g, a, nblocks, s);
    case CF_LOCAL | CB_XC: return row_inv_go<T, M, CF_LOCAL | CB_XC>(g, a, nblocks, s);
    case CF_WT | CB_XC: return row_inv_go<T, M, CF_WT | CB_XC>(g, a, nblocks, s);
    case CF_S3S4 | CB_XC: return row_inv_go<T, M, CF_S3S4 | CB_XC>(g, a, nblocks, s);
    case CF_EXACT | CB_XC: return row_inv_go<T, M, CF_EXACT | CB_XC>(g, a, nblocks, s);
    default: return hipErrorNotSupported;
    }
}

// Column lengths whose reciprocal-space passes offer the autotuner two more
// launch shapes (FP32): half the columns per block (more, smaller blocks)
// and the reversed radix order (plan_variant).
template <typename T, int L> constexpr int col_variant_mask()
{
    if constexpr (sizeof(T) != 4 || !(L == 64 || L == 96 || L == 128 || L == 192 || L == 256)) {
        return 0;
    } else {
        int m = 0;
        if (col_P<T, L>() / 2 >= 4) m |= 1;
        if (plan_reversible(L, true)) m |= 2;
        return m;
    }
}
template <typename T, int L> constexpr int col_tile_of(int variant)
{
    return (variant & col_variant_mask<T, L>() & 1) ? col_P<T, L>() / 2 : col_P<T, L>();
}

// the reciprocal-space (non-plain) column pass with tile P and plan variant PV
template <typename T, int L, int P, int PV>
hipError_t col_go_tile(int nfb, const ColArgs &a, bool plain, bool has_part, int &nblocks,
                       hipStream_t s)
{
    nblocks = (int)((a.ncols + P - 1) / P);
    if (has_part && nblocks > a.pstride) return hipErrorInvalidValue;
    // a block takes a tile of the same field for COL_GROUP densities where
    // that still leaves at least COL_MIN_BLOCKS blocks (not for multi-cell
    // batches, whose densities have tables of their own)
    constexpr bool grp_ok = L * P / col_NT<T, L, P>() <= 8;
    ColArgs ag = a;
    ag.nbb = 1;
    const int nfields = nfb / (a.nbatch > 0 ? a.nbatch : 1);
    if constexpr (grp_ok && col_grouped<T, L>()) {
        if (!a.ct && !plain && a.nbatch > 1 && a.nbb > 1) {
            const int want = a.nbb < COL_GROUP ? a.nbb : COL_GROUP;
            int nbb = want < a.nbatch ? want : a.nbatch;
            while (nbb > 1 &&
                   (long long)nblocks * nfields * ((a.nbatch + nbb - 1) / nbb) < COL_MIN_BLOCKS)
                nbb /= 2;
            ag.nbb = nbb;
        }
    }
    const int nfg = nfields * ((a.nbatch + ag.nbb - 1) / ag.nbb);
    const long long total = (long long)nblocks * nfg;
    if (total > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)total), block(col_NT<T, L, P>());
    if (a.ct && !plain) {
        if constexpr (PV == 0 && P == col_P<T, L>())
            hipLaunchKernelGGL((k_col<T, L, P, true>), grid, block, 0, s, ag, nfg, nblocks);
        else
            return hipErrorInvalidValue;   // multi-cell batches take the default shape
    } else if (ag.nbb > 1) {
        if constexpr (grp_ok && col_grouped<T, L>())
            hipLaunchKernelGGL((k_col<T, L, P, false, true, PV>), grid, block, 0, s, ag, nfg,
                               nblocks);
    } else {
        hipLaunchKernelGGL((k_col<T, L, P, false, false, PV>), grid, block, 0, s, ag, nfg, nblocks);
    }
    return hipGetLastError();
}

template <typename T, int L>
hipError_t col_go(int nfb, const ColArgs &a, int &nblocks, hipStream_t s)
{
    constexpr int P = col_P<T, L>();
    constexpr int PP = col_P_plain<T, L>();
    bool has_part = false, plain = true;
    for (int f = 0; f < MAXKB; ++f) {
        has_part |= (a.op[f] == GO_HEXT || a.op[f] == GO_VW);
        plain &= a.op[f] == GO_NONE;
    }
    if constexpr (PP != P) {
        if (plain) {
            nblocks = (int)((a.ncols + PP - 1) / PP);
            const long long total = (long long)nblocks * nfb;
            if (total > 0x7fffffffLL) return hipErrorInvalidValue;
            hipLaunchKernelGGL((k_col<T, L, PP>), dim3((unsigned)total), dim3(col_NT<T, L, PP>()),
                               0, s, a, nfb,
                               nblocks);
            return hipGetLastError();
        }
    }
    constexpr int VM = col_variant_mask<T, L>();
    if constexpr (VM != 0) {
        const int v = (plain || a.ct) ? 0 : (a.variant & VM);
        if constexpr ((VM & 1) != 0)
            if (v == 1) return col_go_tile<T, L, P / 2, 0>(nfb, a, plain, has_part, nblocks, s);
        if constexpr ((VM & 2) != 0)
            if (v == 2) return col_go_tile<T, L, P, 1>(nfb, a, plain, has_part, nblocks, s);
        if constexpr (VM == 3)
            if (v == 3) return col_go_tile<T, L, P / 2, 1>(nfb, a, plain, has_part, nblocks, s);
    }
    return col_go_tile<T, L, P, 0>(nfb, a, plain, has_part, nblocks, s);
}

template <typename T, int L>
hipError_t knot_inv_go(const KnotArgs &a, hipStream_t s)
{
    constexpr int P = knot_P<T, L>();
    dim3 grid((unsigned)((a.ncols + P - 1) / P), a.nbatch);
    hipLaunchKernelGGL((k_knot_inv<T, L>), grid, dim3(knot_NT<T, L>()), 0, s, a);
    return hipGetLastError();
}

template <typename T, int L>
hipError_t knot_acc_go(const KnotArgs &a, hipStream_t s)
{
    constexpr int P = knot_P<T, L>();
    dim3 grid((unsigned)((a.ncols + P - 1) / P), a.nbatch);
    hipLaunchKernelGGL((k_knot_acc<T, L>), grid, dim3(knot_NT<T, L>()), 0, s, a);
    return hipGetLastError();
}

// row lengths with fixed-term-set combine kernels (grids whose planes do not
// fit in LDS: the larger serving cells, the slab and the 10^6-atom cell)
#define OFDFT_ROWC_LENGTHS(X) \
    X(48) X(64) X(72) X(96) X(108) X(128) X(144) X(192) X(216) X(256) X(288) X(384) X(512)

#define OFDFT_INSTANTIATE_ROW(T)                                                               \
    template <> hipError_t launch_row_fwd<T>(const Geom &g, int nbatch, const RowFwdArgs &a,   \
                                             int &nb, hipStream_t s)                           \
    {                                                                                          \
        switch (g.m) {                                                                         \
            OFDFT_LENGTHS(OFDFT_CASE_ROWF_##T)                                                 \
        default: return hipErrorInvalidValue;                                                  \
        }                                                                                      \
    }                                                                                          \
    template <> hipError_t launch_row_inv<T>(const Geom &g, const RowInvArgs &a, int &nb,      \
                                             hipStream_t s)                                    \
    {                                                                                          \
        if (a.mode == EP_COMBINE && a.cf != 0) {                                               \
            const hipError_t e = launch_row_combine_fixed<T>(g, a, nb, s);                     \
            if (e != hipErrorNotSupported) return e;                                           \
        }                                                                                      \
        switch (g.m) {                                                                         \
            OFDFT_LENGTHS(OFDFT_CASE_ROWI_##T)                                                 \
        default: return hipErrorInvalidValue;                                                  \
        }                                                                                      \
    }                                                                                          \
    template <> int row_blocks<T>(const Geom &g)                                               \
    {                                                                                          \
        switch (g.m) {                                                                         \
            OFDFT_LENGTHS(OFDFT_CASE_RB_##T)                                                   \
        default: return 0;                                                                     \
        }                                                                                      \
    }

#define OFDFT_INSTANTIATE_ROW_FIXED(T)                                                         \
    template <> hipError_t launch_row_combine_fixed<T>(const Geom &g, const RowInvArgs &a,     \
                                                       int &nb, hipStream_t s)                 \
    {                                                                                          \
        switch (g.m) {                                                                         \
            OFDFT_ROWC_LENGTHS(OFDFT_CASE_ROWC_##T)                                            \
        default: return hipErrorNotSupported;                                                  \
        }                                                                                      \
    }

#define OFDFT_INSTANTIATE_COL(T)                                                               \
    template <> hipError_t launch_col<T>(int L, int nfb, const ColArgs &a, int &nb,            \
                                         hipStream_t s)                                        \
    {                                                                                          \
        switch (L) {                                                                           \
            OFDFT_LENGTHS(OFDFT_CASE_COL_##T)                                                  \
        default: return hipErrorInvalidValue;                                                  \
        }                                                                                      \
    }                                                                                          \
    template <> hipError_t launch_knot_inv<T>(const KnotArgs &a, hipStream_t s)                \
    {                                                                                          \
        switch (a.g.n0) {                                                                      \
            OFDFT_LENGTHS(OFDFT_CASE_KI_##T)                                                   \
        default: return hipErrorInvalidValue;                                                  \
        }                                                                                      \
    }                                                                                          \
    template <> hipError_t launch_knot_acc<T>(const KnotArgs &a, hipStream_t s)                \
    {                                                                                          \
        switch (a.g.n0) {                                                                      \
            OFDFT_LENGTHS(OFDFT_CASE_KA_##T)                                                   \
        default: return hipErrorInvalidValue;                                                  \
        }                                                                                      \
    }                                                                                          \
    template <> int col_blocks<T>(int L, long long ncols, int variant)                         \
    {                                                                                          \
        switch (L) {                                                                           \
            OFDFT_LENGTHS(OFDFT_CASE_CB_##T)                                                   \
        default: return 0;                                                                     \
        }                                                                                      \
    }                                                                                          \
    template <> int col_variants<T>(int L)                                                     \
    {                                                                                          \
        switch (L) {                                                                           \
            OFDFT_LENGTHS(OFDFT_CASE_CV_##T)                                                   \
        default: return 0;                                                                     \
        }                                                                                      \
    }

#define OFDFT_CASE_ROWF_float(L) case L: return row_fwd_go<float, L>(g, nbatch, a, nb, s);
#define OFDFT_CASE_ROWF_double(L) case L: return row_fwd_go<double, L>(g, nbatch, a, nb, s);
#define OFDFT_CASE_ROWI_float(L) case L: return row_inv_go<float, L>(g, a, nb, s);
#define OFDFT_CASE_ROWI_double(L) case L: return row_inv_go<double, L>(g, a, nb, s);
#define OFDFT_CASE_ROWC_float(L) case L: return row_combine_fixed_go<float, L>(g, a, nb, s);
#define OFDFT_CASE_ROWC_double(L) case L: return row_combine_fixed_go<double, L>(g, a, nb, s);
#define OFDFT_CASE_COL_float(L) case L: return col_go<float, L>(nfb, a, nb, s);
#define OFDFT_CASE_COL_double(L) case L: return col_go<double, L>(nfb, a, nb, s);
#define OFDFT_CASE_KI_float(L) case L: return knot_inv_go<float, L>(a, s);
#define OFDFT_CASE_KI_double(L) case L: return knot_inv_go<double, L>(a, s);
#define OFDFT_CASE_KA_float(L) case L: return knot_acc_go<float, L>(a, s);
#define OFDFT_CASE_KA_double(L) case L: return knot_acc_go<double, L>(a, s);
#define OFDFT_CASE_RB_float(L) case L: return (int)(((long long)g.n0 * g.n1 + row_P<float, L>() - 1) / row_P<float, L>());
#define OFDFT_CASE_RB_double(L) case L: return (int)(((long long)g.n0 * g.n1 + row_P<double, L>() - 1) / row_P<double, L>());
#define OFDFT_CASE_CB_float(L) case L: return (int)((ncols + col_tile_of<float, L>(variant) - 1) / col_tile_of<float, L>(variant));
#define OFDFT_CASE_CB_double(L) case L: return (int)((ncols + col_tile_of<double, L>(variant) - 1) / col_tile_of<double, L>(variant));
#define OFDFT_CASE_CV_float(L) case L: return col_variant_mask<float, L>();
#define OFDFT_CASE_CV_double(L) case L: return col_variant_mask<double, L>();

}  // namespace ofdft
