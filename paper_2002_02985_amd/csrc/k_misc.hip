// Non-FFT kernels: fixed-order FP64 reductions, the ionic structure factor
// and local pseudopotential v_ext(G), electron-ion forces, and the vector
// operations of the density optimiser.
#include "kernels_impl.hpp"

namespace ofdft {

static const int SUPPORTED[] = {2,  3,  4,  6,  8,   9,   12,  16,  18,  24,  27,  32,  36,  48,  54,
                                64, 72, 81, 96, 108, 128, 144, 162, 192, 216, 256, 288, 384, 512, 1024};

bool length_supported(int L)
{
    for (int v : SUPPORTED)
        if (v == L) return true;
    return false;
}

// ---------------------------------------------------------------- finalize
__global__ __launch_bounds__(NT) void k_finalize(const double *part, int pstride, SlotCounts count,
                                                 double *sums)
{
    __shared__ double red[NT];
    const int s = blockIdx.x, b = blockIdx.y, tid = threadIdx.x;
    const double *p = part + ((long long)b * NSLOT + s) * pstride;
    const int n = count.n[s];
    double acc = 0.0;
    for (int i = tid; i < n; i += NT) acc += p[i];
    acc = block_sum<NT>(acc, red, tid);
    if (tid == 0) sums[b * NSLOT + s] = acc;
}

hipError_t launch_finalize(const double *part, int pstride, const SlotCounts &count, int nbatch,
                           double *sums, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize, dim3(NSLOT, nbatch), dim3(NT), 0, s, part, pstride, count,
                       sums);
    return hipGetLastError();
}

// ---------------------------------------------------------------- knot range
template <typename T>
__global__ __launch_bounds__(NT) void k_knot_range_part(long long N, const T *in, int in_is_phi,
                                                        double *part)
{
    __shared__ double red[2 * NT / 64];
    const int b = blockIdx.y, tid = threadIdx.x;
    const T *x = in + (long long)b * N;
    double lo = 1e300, hi = -1e300;
    for (long long i = (long long)blockIdx.x * NT + tid; i < N; i += (long long)gridDim.x * NT) {
        const T v = x[i];
        const T rho = in_is_phi ? v * v : (v > T(0) ? v : T(0));
        lo = fmin(lo, (double)rho);
        hi = fmax(hi, (double)rho);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    constexpr int NW = NT / 64;
    if ((tid & 63) == 0) {
        red[tid >> 6] = lo;
        red[NW + (tid >> 6)] = hi;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < NW; ++w) {
            lo = fmin(lo, red[w]);
            hi = fmax(hi, red[NW + w]);
        }
        part[((long long)b * 2) * KR_BLOCKS + blockIdx.x] = lo;
        part[((long long)b * 2 + 1) * KR_BLOCKS + blockIdx.x] = hi;
    }
}

template <typename T>
__device__ int knot_bracket_of_rho(T rho, const Knots &kn)
{
    const T lu = rho > T(0) ? d_log2(rho) : neg_inf<T>();
    int j;
    T t;
    bool inside;
    knot_bracket_kf(kf_from_log2(lu), kn, j, t, inside);
    return j;
}

template <typename T>
__global__ __launch_bounds__(64) void k_knot_range_final(const double *part, Knots kn, int *kneed)
{
    const int b = blockIdx.x, tid = threadIdx.x;
    double lo = 1e300, hi = -1e300;
    for (int i = tid; i < KR_BLOCKS; i += 64) {
        lo = fmin(lo, part[((long long)b * 2) * KR_BLOCKS + i]);
        hi = fmax(hi, part[((long long)b * 2 + 1) * KR_BLOCKS + i]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
    }
    if (tid == 0) {
        int k0 = 0, k1 = kn.nk - 1;
        if (kn.nk > 1 && lo <= hi) {
            // the extremes are values of the field type, bracketed as the grid
            // points are; knots j .. j + 1 of each bracket, one more each side
            const int jl = knot_bracket_of_rho<T>(T(lo), kn);
            const int jh = knot_bracket_of_rho<T>(T(hi), kn);
            k0 = jl - 1 < 0 ? 0 : jl - 1;
            k1 = jh + 2 > kn.nk - 1 ? kn.nk - 1 : jh + 2;
        }
        kneed[2 * b] = k0;
        kneed[2 * b + 1] = k1;
    }
}

template <typename T>
hipError_t launch_knot_range(long long N, int nbatch, const void *in, int in_is_phi,
                             const Knots &kn, double *part, int *kneed, hipStream_t s)
{
    hipLaunchKernelGGL((k_knot_range_part<T>), dim3(KR_BLOCKS, nbatch), dim3(NT), 0, s, N,
                       (const T *)in, in_is_phi, part);
    hipLaunchKernelGGL((k_knot_range_final<T>), dim3(nbatch), dim3(64), 0, s, part, kn, kneed);
    return hipGetLastError();
}
template hipError_t launch_knot_range<float>(long long, int, const void *, int, const Knots &,
                                             double *, int *, hipStream_t);
template hipError_t launch_knot_range<double>(long long, int, const void *, int, const Knots &,
                                              double *, int *, hipStream_t);

// ---------------------------------------------------------------- G tables
// tab[e] = 1/G^2 (0 at G = 0), tab[Nh + e] = G^2,
// tab[2 Nh + e] = C_WT K(|G| / (2 kf)) for half-spectrum point e (K = G_NL for
// Wang-Teter, the MGP-family kernel otherwise), in FP64.
template <typename T>
__global__ __launch_bounds__(NT) void k_gtab(Geom g, double kf, NlKern kern, T *tab)
{
    const long long e = (long long)blockIdx.x * NT + threadIdx.x;
    if (e >= g.Nh) return;
    const int k2 = (int)(e % g.n2h);
    const long long row = e / g.n2h;
    const int i1 = (int)(row % g.n1), i0 = (int)(row / g.n1);
    const int m2 = (k2 == g.m) ? -g.m : k2;
    const double G2 = gvec2<double>(g, freq(i0, g.n0), freq(i1, g.n1), m2);
    tab[e] = T(G2 > 0.0 ? 1.0 / G2 : 0.0);
    tab[g.Nh + e] = T(G2);
    tab[2 * g.Nh + e] = T(C_WT_D * nl_kernel_dev<double>(sqrt(G2) / (2.0 * kf), kern));
}

template <typename T>
hipError_t launch_gtab(const Geom &g, double kf_wt, const NlKern &kern, void *gtab, hipStream_t s)
{
    const long long nb = (g.Nh + NT - 1) / NT;
    hipLaunchKernelGGL((k_gtab<T>), dim3((unsigned)nb), dim3(NT), 0, s, g, kf_wt, kern, (T *)gtab);
    return hipGetLastError();
}
template hipError_t launch_gtab<float>(const Geom &, double, const NlKern &, void *, hipStream_t);
template hipError_t launch_gtab<double>(const Geom &, double, const NlKern &, void *, hipStream_t);

// ---------------------------------------------------------------- v_ext(G)
// v_ext(G) = (1/V) sum_s v_s(|G|) sum_{a in s} e^{-i G.R_a}; the phase is the
// product of per-axis tables ph_d[a][i] = exp(-2 pi i m_d(i) s_{a,d}) (s the
// fractional coordinates), built in FP64 with exact argument reduction.
// One block per (i0, i1) row of the half spectrum; atoms are grouped by species.
template <typename T>
__global__ __launch_bounds__(NT) void k_vext(Geom g, int natoms, const int *spec_off,
                                             int nspecies, const double *ph0, const double *ph1,
                                             const double *ph2, const double *Z,
                                             const double *rc, double inv_vol, cpx<T> *vext)
{
    const int row = blockIdx.x;
    const int i0 = row / g.n1, i1 = row % g.n1;
    const int m0 = freq(i0, g.n0), m1 = freq(i1, g.n1);
    for (int k2 = threadIdx.x; k2 < g.n2h; k2 += NT) {
        const int m2 = (k2 == g.m) ? -g.m : k2;
        const double G2 = gvec2<double>(g, m0, m1, m2);
        double vr = 0.0, vi = 0.0;
        for (int s = 0; s < nspecies; ++s) {
            double sr = 0.0, si = 0.0;
            for (int a = spec_off[s]; a < spec_off[s + 1]; ++a) {
                const double *p0 = ph0 + 2 * ((long long)a * g.n0 + i0);
                const double *p1 = ph1 + 2 * ((long long)a * g.n1 + i1);
                const double *p2 = ph2 + 2 * ((long long)a * g.n2h + k2);
                const double ar = p0[0] * p1[0] - p0[1] * p1[1];
                const double ai = p0[0] * p1[1] + p0[1] * p1[0];
                sr += ar * p2[0] - ai * p2[1];
                si += ar * p2[1] + ai * p2[0];
            }
            const double z = Z[s], r = rc[s];
            const double vs = G2 > 0.0 ? -4.0 * PI_D * z * exp(-G2 * r * r * 0.25) / G2
                                       : PI_D * z * r * r;
            vr += vs * sr;
            vi += vs * si;
        }
        vext[(long long)row * g.n2h + k2] = {T(vr * inv_vol), T(vi * inv_vol)};
    }
}

template <typename T>
hipError_t launch_vext(const Geom &g, int natoms, const int *spec_off, int nspecies,
                       const double *ph0, const double *ph1, const double *ph2, const double *Z,
                       const double *rc, double volume, void *vext, hipStream_t s)
{
    (void)natoms;
    hipLaunchKernelGGL((k_vext<T>), dim3(g.n0 * g.n1), dim3(NT), 0, s, g, natoms, spec_off,
                       nspecies, ph0, ph1, ph2, Z, rc, 1.0 / volume, (cpx<T> *)vext);
    return hipGetLastError();
}
template hipError_t launch_vext<float>(const Geom &, int, const int *, int, const double *,
                                       const double *, const double *, const double *,
                                       const double *, double, void *, hipStream_t);
template hipError_t launch_vext<double>(const Geom &, int, const int *, int, const double *,
                                        const double *, const double *, const double *,
                                        const double *, double, void *, hipStream_t);

// ---------------------------------------------------------------- forces
// F_a = sum_half c(m2) G v_{s(a)}(|G|) Im[e^{i G.R_a} rho(G)], the exact
// derivative -d/dR_a of int v_ext rho = V sum_half c Re[conj(v_ext(G)) rho(G)].
// One block per atom; its phase tables are staged in LDS.
constexpr int FORCE_MAXTAB = 2 * 1024 + 513;

template <typename T>
__global__ __launch_bounds__(NT) void k_forces(Geom g, const int *atom_species,
                                               const double *ph0, const double *ph1,
                                               const double *ph2, const double *Z,
                                               const double *rc, const cpx<T> *rho_g,
                                               double *f_out)
{
    __shared__ double tab[2 * FORCE_MAXTAB];
    __shared__ double red[NT];
    const int a = blockIdx.x, tid = threadIdx.x;
    const int ntab = g.n0 + g.n1 + g.n2h;
    for (int i = tid; i < g.n0; i += NT) {
        tab[2 * i] = ph0[2 * ((long long)a * g.n0 + i)];
        tab[2 * i + 1] = ph0[2 * ((long long)a * g.n0 + i) + 1];
    }
    for (int i = tid; i < g.n1; i += NT) {
        tab[2 * (g.n0 + i)] = ph1[2 * ((long long)a * g.n1 + i)];
        tab[2 * (g.n0 + i) + 1] = ph1[2 * ((long long)a * g.n1 + i) + 1];
    }
    for (int i = tid; i < g.n2h; i += NT) {
        tab[2 * (g.n0 + g.n1 + i)] = ph2[2 * ((long long)a * g.n2h + i)];
        tab[2 * (g.n0 + g.n1 + i) + 1] = ph2[2 * ((long long)a * g.n2h + i) + 1];
    }
    (void)ntab;
    __syncthreads();
    const int s = atom_species[a];
    const double z = Z[s], r = rc[s];
    double fx = 0.0, fy = 0.0, fz = 0.0;
    for (long long e = tid; e < g.Nh; e += NT) {
        const int k2 = (int)(e % g.n2h);
        const long long row = e / g.n2h;
        const int i1 = (int)(row % g.n1), i0 = (int)(row / g.n1);
        const int m0 = freq(i0, g.n0), m1 = freq(i1, g.n1);
        const int m2 = (k2 == g.m) ? -g.m : k2;
        const double gx = m0 * g.b[0][0] + m1 * g.b[1][0] + m2 * g.b[2][0];
        const double gy = m0 * g.b[0][1] + m1 * g.b[1][1] + m2 * g.b[2][1];
        const double gz = m0 * g.b[0][2] + m1 * g.b[1][2] + m2 * g.b[2][2];
        const double G2 = gx * gx + gy * gy + gz * gz;
        if (G2 == 0.0) continue;
        const double *p0 = tab + 2 * i0;
        const double *p1 = tab + 2 * (g.n0 + i1);
        const double *p2 = tab + 2 * (g.n0 + g.n1 + k2);
        // tables hold exp(-i G.R); the force needs exp(+i G.R) = conj
        const double ar = p0[0] * p1[0] - p0[1] * p1[1];
        const double ai = p0[0] * p1[1] + p0[1] * p1[0];
        const double er = ar * p2[0] - ai * p2[1];
        const double ei = -(ar * p2[1] + ai * p2[0]);
        const cpx<T> rg = rho_g[e];
        const double im = er * (double)rg.y + ei * (double)rg.x;
        const double vs = -4.0 * PI_D * z * exp(-G2 * r * r * 0.25) / G2;
        const double w = (k2 == 0 || k2 == g.m) ? 1.0 : 2.0;
        const double sc = w * vs * im;
        fx += sc * gx;
        fy += sc * gy;
        fz += sc * gz;
    }
    fx = block_sum<NT>(fx, red, tid);
    fy = block_sum<NT>(fy, red, tid);
    fz = block_sum<NT>(fz, red, tid);
    if (tid == 0) {
        f_out[3 * a + 0] = fx;
        f_out[3 * a + 1] = fy;
        f_out[3 * a + 2] = fz;
    }
}

template <typename T>
hipError_t launch_forces(const Geom &g, int natoms, const int *atom_species, const double *ph0,
                         const double *ph1, const double *ph2, const double *Z, const double *rc,
                         const void *rho_g, double *f_out, hipStream_t s)
{
    if (g.n0 + g.n1 + g.n2h > FORCE_MAXTAB) return hipErrorInvalidValue;
    if (natoms <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_forces<T>), dim3(natoms), dim3(NT), 0, s, g, atom_species, ph0, ph1, ph2,
                       Z, rc, (const cpx<T> *)rho_g, f_out);
    return hipGetLastError();
}
template hipError_t launch_forces<float>(const Geom &, int, const int *, const double *,
                                         const double *, const double *, const double *,
                                         const double *, const void *, double *, hipStream_t);
template hipError_t launch_forces<double>(const Geom &, int, const int *, const double *,
                                          const double *, const double *, const double *,
                                          const double *, const void *, double *, hipStream_t);

// ---------------------------------------------------------------- vectors
constexpr int DOT_ITEMS = 8;

int dots_blocks(long long n) { return (int)((n + (long long)NT * DOT_ITEMS - 1) / (NT * DOT_ITEMS)); }

template <typename T>
__global__ __launch_bounds__(NT) void k_dots(long long n, int nd, const T *x0, const T *y0,
                                             const T *x1, const T *y1, const T *x2, const T *y2,
                                             const T *x3, const T *y3, double *part, int pstride)
{
    __shared__ double red[NT];
    const int tid = threadIdx.x;
    const long long base = (long long)blockIdx.x * NT * DOT_ITEMS;
    const T *xs[4] = {x0, x1, x2, x3};
    const T *ys[4] = {y0, y1, y2, y3};
    for (int d = 0; d < nd; ++d) {
        double acc = 0.0;
        for (int it = 0; it < DOT_ITEMS; ++it) {
            const long long i = base + (long long)it * NT + tid;
            if (i < n) acc += (double)xs[d][i] * (double)ys[d][i];
        }
        acc = block_sum<NT>(acc, red, tid);
        if (tid == 0) part[(long long)(SL_AUX0 + d) * pstride + blockIdx.x] = acc;
    }
}

template <typename T>
hipError_t launch_dots(long long n, int nd, const void *x0, const void *y0, const void *x1,
                       const void *y1, const void *x2, const void *y2, const void *x3,
                       const void *y3, double *part, int pstride, int &nblocks, hipStream_t s)
{
    nblocks = dots_blocks(n);
    if (nblocks > pstride || nd < 1 || nd > 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_dots<T>), dim3(nblocks), dim3(NT), 0, s, n, nd, (const T *)x0,
                       (const T *)y0, (const T *)x1, (const T *)y1, (const T *)x2, (const T *)y2,
                       (const T *)x3, (const T *)y3, part, pstride);
    return hipGetLastError();
}
template hipError_t launch_dots<float>(long long, int, const void *, const void *, const void *,
                                       const void *, const void *, const void *, const void *,
                                       const void *, double *, int, int &, hipStream_t);
template hipError_t launch_dots<double>(long long, int, const void *, const void *, const void *,
                                        const void *, const void *, const void *, const void *,
                                        const void *, double *, int, int &, hipStream_t);

template <typename T>
__global__ __launch_bounds__(NT) void k_lincomb(long long n, T *z, double a, const T *x, double b,
                                                const T *y)
{
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    if (i < n) z[i] = T(a * (double)x[i] + (y ? b * (double)y[i] : 0.0));
}

template <typename T>
hipError_t launch_lincomb(long long n, void *z, double a, const void *x, double b, const void *y,
                          hipStream_t s)
{
    const long long nb = (n + NT - 1) / NT;
    hipLaunchKernelGGL((k_lincomb<T>), dim3((unsigned)nb), dim3(NT), 0, s, n, (T *)z, a,
                       (const T *)x, b, (const T *)y);
    return hipGetLastError();
}
template hipError_t launch_lincomb<float>(long long, void *, double, const void *, double,
                                          const void *, hipStream_t);
template hipError_t launch_lincomb<double>(long long, void *, double, const void *, double,
                                           const void *, hipStream_t);

template <typename T>
__global__ __launch_bounds__(NT) void k_pointwise(long long n, int op, T *z, const T *x)
{
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const T v = x[i];
    z[i] = op == PW_SQRT ? (v > T(0) ? sqrt(v) : T(0)) : v * v;
}

template <typename T>
hipError_t launch_pointwise(long long n, int op, void *z, const void *x, hipStream_t s)
{
    const long long nb = (n + NT - 1) / NT;
    hipLaunchKernelGGL((k_pointwise<T>), dim3((unsigned)nb), dim3(NT), 0, s, n, op, (T *)z,
                       (const T *)x);
    return hipGetLastError();
}
template hipError_t launch_pointwise<float>(long long, int, void *, const void *, hipStream_t);
template hipError_t launch_pointwise<double>(long long, int, void *, const void *, hipStream_t);

// ---------------------------------------------------------------- interpolation
// Fourier interpolation onto a grid at least as fine on every axis (the
// multi-step optimisation of the section "Density optimization strategies"):
// coefficient f(G) of the destination is the source's for the frequencies
// strictly inside the source band, half the source's Nyquist coefficient at
// each of +-n_s/2 (the band-limited cosine that the Nyquist samples
// represent), and zero beyond; an axis of equal size is copied as it is.
// Full axes 0 and 1: frequency m of the destination -> source index and
// weight; returns false when the source has no such frequency.
__device__ __forceinline__ bool interp_axis(int m, int ns, int nd, int &is, double &w)
{
    w = 1.0;
    if (nd == ns) {
        is = m < 0 ? m + ns : m;
        return true;
    }
    if (ns % 2 == 0 && (m == ns / 2 || m == -ns / 2)) {
        is = ns / 2;   // the source Nyquist frequency -ns/2 sits at index ns/2
        w = 0.5;
        return true;
    }
    if (2 * m >= ns || -2 * m >= ns) return false;
    is = m < 0 ? m + ns : m;
    return true;
}

// Half axis 2 (k >= 0 stored): source index k and weight.
__device__ __forceinline__ bool interp_half(int k, int ns, int nd, double &w)
{
    w = 1.0;
    if (nd == ns) return true;
    if (ns % 2 == 0 && 2 * k == ns) {
        w = 0.5;
        return true;
    }
    return 2 * k < ns;
}

template <typename T>
__global__ __launch_bounds__(NT) void k_interp_spec(Geom gs, Geom gd, const cpx<T> *src,
                                                    cpx<T> *dst)
{
    const long long e = (long long)blockIdx.x * NT + threadIdx.x;
    if (e >= gd.Nh) return;
    const int k2 = (int)(e % gd.n2h);
    const long long row = e / gd.n2h;
    const int i1 = (int)(row % gd.n1), i0 = (int)(row / gd.n1);
    int s0, s1;
    double w0, w1, w2;
    cpx<T> v = {T(0), T(0)};
    if (interp_axis(freq(i0, gd.n0), gs.n0, gd.n0, s0, w0) &&
        interp_axis(freq(i1, gd.n1), gs.n1, gd.n1, s1, w1) && interp_half(k2, gs.n2, gd.n2, w2)) {
        const cpx<T> x = src[((long long)s0 * gs.n1 + s1) * gs.n2h + k2];
        const T w = T(w0 * w1 * w2);
        v = {w * x.x, w * x.y};
    }
    dst[e] = v;
}

template <typename T>
hipError_t launch_interp_spec(const Geom &gs, const Geom &gd, const void *src, void *dst,
                              hipStream_t s)
{
    const long long nb = (gd.Nh + NT - 1) / NT;
    hipLaunchKernelGGL((k_interp_spec<T>), dim3((unsigned)nb), dim3(NT), 0, s, gs, gd,
                       (const cpx<T> *)src, (cpx<T> *)dst);
    return hipGetLastError();
}
template hipError_t launch_interp_spec<float>(const Geom &, const Geom &, const void *, void *,
                                              hipStream_t);
template hipError_t launch_interp_spec<double>(const Geom &, const Geom &, const void *, void *,
                                               hipStream_t);

}  // namespace ofdft
