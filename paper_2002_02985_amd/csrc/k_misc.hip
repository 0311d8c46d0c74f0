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
// One pass over each density for its smallest and largest rho: 16-byte
// loads, KR_U of them in flight per thread (when N is a multiple of the
// vector width, so that every density starts aligned), the extremes taken in
// the field type (exact) and widened once.
template <typename T> struct Vec16;
template <> struct Vec16<float> {
    using type = float4;
    static constexpr int n = 4;
};
template <> struct Vec16<double> {
    using type = double2;
    static constexpr int n = 2;
};
constexpr int KR_U = 4;
// With BR (the S3S4 interpolation's knots), each point's bracket is also
// taken exactly as the interpolation takes it (rho -> log2 -> k_F -> knot
// segment, knots in T from LDS), and its smallest and largest reduced.
template <typename T, bool BR>
__global__ __launch_bounds__(NT) void k_knot_range_part(long long N, const T *in, int in_is_phi,
                                                        Knots kn, double *part)
{
    using V = typename Vec16<T>::type;
    constexpr int VN = Vec16<T>::n;
    __shared__ double red[4 * NT / 64];
    __shared__ T knl[BR ? MAXKNOTS : 1];
    const int b = blockIdx.y, tid = threadIdx.x;
    const T *x = in + (long long)b * N;
    if constexpr (BR) {
        if (tid < kn.nk) knl[tid] = T(kn.k[tid]);   // nk <= MAXKNOTS <= NT
        __syncthreads();
    }
    T tlo = __builtin_huge_valf(), thi = -__builtin_huge_valf();
    int jlo = 1 << 30, jhi = -1;
    auto upd = [&](T v) {
        const T rho = in_is_phi ? v * v : (v > T(0) ? v : T(0));
        tlo = fmin(tlo, rho);
        thi = fmax(thi, rho);
        if constexpr (BR) {
            const T lu = rho > T(0) ? d_log2(rho) : neg_inf<T>();
            int j;
            T t;
            bool inside;
            knot_bracket_tab(kf_from_log2(lu), kn.nk, kn.log_spacing, kn.inv_span, knl, j, t,
                             inside);
            jlo = j < jlo ? j : jlo;
            jhi = j > jhi ? j : jhi;
        }
    };
    const long long stride = (long long)gridDim.x * NT;
    const long long nv = N % VN == 0 ? N / VN : 0;
    const V *xv = (const V *)x;
    long long i = (long long)blockIdx.x * NT + tid;
    for (; i + (KR_U - 1) * stride < nv; i += KR_U * stride) {
        V a[KR_U];
#pragma unroll
        for (int u = 0; u < KR_U; ++u) a[u] = xv[i + u * stride];
#pragma unroll
        for (int u = 0; u < KR_U; ++u) {
            const T *e = (const T *)&a[u];
#pragma unroll
            for (int c = 0; c < VN; ++c) upd(e[c]);
        }
    }
    for (; i < nv; i += stride) {
        const V a = xv[i];
        const T *e = (const T *)&a;
#pragma unroll
        for (int c = 0; c < VN; ++c) upd(e[c]);
    }
    for (long long k = nv * VN + (long long)blockIdx.x * NT + tid; k < N; k += stride) upd(x[k]);
    double lo = fmin(1e300, (double)tlo), hi = fmax(-1e300, (double)thi);
    double dj0 = (double)jlo, dj1 = (double)jhi;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
        dj0 = fmin(dj0, __shfl_xor(dj0, off, 64));
        dj1 = fmax(dj1, __shfl_xor(dj1, off, 64));
    }
    constexpr int NW = NT / 64;
    if ((tid & 63) == 0) {
        red[tid >> 6] = lo;
        red[NW + (tid >> 6)] = hi;
        red[2 * NW + (tid >> 6)] = dj0;
        red[3 * NW + (tid >> 6)] = dj1;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < NW; ++w) {
            lo = fmin(lo, red[w]);
            hi = fmax(hi, red[NW + w]);
            dj0 = fmin(dj0, red[2 * NW + w]);
            dj1 = fmax(dj1, red[3 * NW + w]);
        }
        part[((long long)b * KR_SLOTS) * KR_BLOCKS + blockIdx.x] = lo;
        part[((long long)b * KR_SLOTS + 1) * KR_BLOCKS + blockIdx.x] = hi;
        part[((long long)b * KR_SLOTS + 2) * KR_BLOCKS + blockIdx.x] = dj0;
        part[((long long)b * KR_SLOTS + 3) * KR_BLOCKS + blockIdx.x] = dj1;
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
__global__ __launch_bounds__(64) void k_knot_range_final(const double *part, int nblk, Knots kn,
                                                         int exact_brackets, int *kneed)
{
    const int b = blockIdx.x, tid = threadIdx.x;
    double lo = 1e300, hi = -1e300, dj0 = 1e300, dj1 = -1e300;
    for (int i = tid; i < nblk; i += 64) {
        lo = fmin(lo, part[((long long)b * KR_SLOTS) * KR_BLOCKS + i]);
        hi = fmax(hi, part[((long long)b * KR_SLOTS + 1) * KR_BLOCKS + i]);
        dj0 = fmin(dj0, part[((long long)b * KR_SLOTS + 2) * KR_BLOCKS + i]);
        dj1 = fmax(dj1, part[((long long)b * KR_SLOTS + 3) * KR_BLOCKS + i]);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        lo = fmin(lo, __shfl_xor(lo, off, 64));
        hi = fmax(hi, __shfl_xor(hi, off, 64));
        dj0 = fmin(dj0, __shfl_xor(dj0, off, 64));
        dj1 = fmax(dj1, __shfl_xor(dj1, off, 64));
    }
    if (tid == 0) {
        int k0 = 0, k1 = kn.nk - 1;
        if (kn.nk > 1 && lo <= hi) {
            if (exact_brackets) {
                // every point's bracket j: its hat functions are knots j, j + 1
                const int jl = (int)dj0, jh = (int)dj1;
                k0 = jl;
                k1 = jh + 1 > kn.nk - 1 ? kn.nk - 1 : jh + 1;
            } else {
                // the extremes are values of the field type, bracketed as the
                // grid points are; knots j .. j + 1 of each bracket, one more
                // each side (a pass that brackets by another formula, the FP64
                // EXACT forward fields, may differ by one near a knot)
                const int jl = knot_bracket_of_rho<T>(T(lo), kn);
                const int jh = knot_bracket_of_rho<T>(T(hi), kn);
                k0 = jl - 1 < 0 ? 0 : jl - 1;
                k1 = jh + 2 > kn.nk - 1 ? kn.nk - 1 : jh + 2;
            }
        }
        kneed[2 * b] = k0;
        kneed[2 * b + 1] = k1;
    }
}

template <typename T>
hipError_t launch_knot_range(long long N, int nbatch, const void *in, int in_is_phi,
                             const Knots &kn, int exact_brackets, double *part, int *kneed,
                             hipStream_t s)
{
    // blocks: one KR_U-vector sweep each, at most KR_BLOCKS
    const long long per = (long long)NT * Vec16<T>::n * KR_U;
    const int nblk = (int)std::max(1LL, std::min((long long)KR_BLOCKS, (N + per - 1) / per));
    if (exact_brackets)
        hipLaunchKernelGGL((k_knot_range_part<T, true>), dim3(nblk, nbatch), dim3(NT), 0, s, N,
                           (const T *)in, in_is_phi, kn, part);
    else
        hipLaunchKernelGGL((k_knot_range_part<T, false>), dim3(nblk, nbatch), dim3(NT), 0, s, N,
                           (const T *)in, in_is_phi, kn, part);
    hipLaunchKernelGGL((k_knot_range_final<T>), dim3(nbatch), dim3(64), 0, s, part, nblk, kn,
                       exact_brackets, kneed);
    return hipGetLastError();
}
template hipError_t launch_knot_range<float>(long long, int, const void *, int, const Knots &, int,
                                             double *, int *, hipStream_t);
template hipError_t launch_knot_range<double>(long long, int, const void *, int, const Knots &, int,
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
// product of per-axis tables ph_d[a][i] = exp(-2 pi i m_d(i) s_d) (s the
// fractional coordinates), built in FP64 with exact argument reduction.
// A lane takes VS consecutive k2 of one (i0, i1) row (a segment) and sums
// each species' structure factor at its points, the phase of an atom
// advanced along k2 by one complex multiplication per point (times
// ph2[a][1]); the negative Nyquist point, which breaks the progression, takes
// its table entry.  Atoms are grouped by species.
constexpr int VS = 8;
template <typename T>
__global__ __launch_bounds__(NT) void k_vext(Geom g, int natoms, const int *spec_off,
                                             int nspecies, const double *ph0, const double *ph1,
                                             const double *ph2, const double *Z,
                                             const double *rc, double inv_vol, long long nseg,
                                             int segs_row, cpx<T> *vext)
{
    (void)natoms;
    const long long sg = (long long)blockIdx.x * NT + threadIdx.x;
    if (sg >= nseg) return;
    const long long row = sg / segs_row;
    const int k0 = (int)(sg % segs_row) * VS;
    const int cnt = min(VS, g.n2h - k0);
    const int i1 = (int)(row % g.n1), i0 = (int)(row / g.n1);
    const int m0 = freq(i0, g.n0), m1 = freq(i1, g.n1);
    const bool nyq_even = g.m > 0 && 2 * g.m == g.n2;
    const int kn = (nyq_even && k0 + cnt - 1 == g.m) ? cnt - 1 : -1;
    double vr[VS], vi[VS];
#pragma unroll
    for (int j = 0; j < VS; ++j) vr[j] = vi[j] = 0.0;
    for (int s = 0; s < nspecies; ++s) {
        double sr[VS], si[VS];
#pragma unroll
        for (int j = 0; j < VS; ++j) sr[j] = si[j] = 0.0;
        double snr = 0.0, sni = 0.0;   // the Nyquist point
        for (int a = spec_off[s]; a < spec_off[s + 1]; ++a) {
            const double *p0 = ph0 + 2 * ((long long)a * g.n0 + i0);
            const double *p1 = ph1 + 2 * ((long long)a * g.n1 + i1);
            const double *p2 = ph2 + 2 * ((long long)a * g.n2h);   // uniform
            const double qr = p0[0] * p1[0] - p0[1] * p1[1];
            const double qi = p0[0] * p1[1] + p0[1] * p1[0];
            const double dr = p2[2], di = p2[3];
            double tr = qr * p2[2 * k0] - qi * p2[2 * k0 + 1];
            double ti = qr * p2[2 * k0 + 1] + qi * p2[2 * k0];
#pragma unroll
            for (int j = 0; j < VS; ++j) {
                sr[j] += tr;
                si[j] += ti;
                const double t2 = tr * dr - ti * di;
                ti = tr * di + ti * dr;
                tr = t2;
            }
            const int mq = g.m > 0 ? g.m : 0;
            snr += qr * p2[2 * mq] - qi * p2[2 * mq + 1];
            sni += qr * p2[2 * mq + 1] + qi * p2[2 * mq];
        }
        const double z = Z[s], r = rc[s];
#pragma unroll
        for (int j = 0; j < VS; ++j) {
            const bool nq = j == kn;
            const int m2 = nq ? -g.m : k0 + j;
            const double G2 = gvec2<double>(g, m0, m1, m2);
            const double vs = G2 > 0.0 ? -4.0 * PI_D * z * exp(-G2 * r * r * 0.25) / G2
                                       : PI_D * z * r * r;
            vr[j] += vs * (nq ? snr : sr[j]);
            vi[j] += vs * (nq ? sni : si[j]);
        }
    }
    cpx<T> *out = vext + row * g.n2h + k0;
#pragma unroll
    for (int j = 0; j < VS; ++j)
        if (j < cnt) out[j] = {T(vr[j] * inv_vol), T(vi[j] * inv_vol)};
}

template <typename T>
hipError_t launch_vext(const Geom &g, int natoms, const int *spec_off, int nspecies,
                       const double *ph0, const double *ph1, const double *ph2, const double *Z,
                       const double *rc, double volume, void *vext, hipStream_t s)
{
    const int segs_row = (g.n2h + VS - 1) / VS;
    const long long nseg = (long long)g.n0 * g.n1 * segs_row;
    hipLaunchKernelGGL((k_vext<T>), dim3((unsigned)((nseg + NT - 1) / NT)), dim3(NT), 0, s, g,
                       natoms, spec_off, nspecies, ph0, ph1, ph2, Z, rc, 1.0 / volume, nseg,
                       segs_row, (cpx<T> *)vext);
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
//
// A lane takes FS consecutive k2 of one (i0, i1) row of the half spectrum
// (a segment).  For each species it forms w(G) = c(m2) v_s(|G|) rho(G) of its
// points once; for each atom of a chunk of at most FATOMS it sums
// im = Im[e^{i G.R_a} w(G)] over the segment, the phase advanced along k2 by
// one complex multiplication per point (e^{-i G.R} = ph0 ph1 ph2, times
// ph2[a][1] per step; the negative Nyquist point, which breaks the
// progression, from its table entry).  G is linear along the segment,
// G = G_0 + j b_2, so the lane keeps S0 = sum im_j and S1 = sum j im_j and
// its force is G_0 S0 + b_2 S1.  Wave sums of each atom's force go to LDS;
// a block's partial forces go to part[block][atom][3], and k_forces_sum adds
// them in block order (deterministic).
constexpr int FS = 8;
constexpr int FATOMS = 512;
constexpr int FBLOCKS = 1024;

template <typename T>
__global__ __launch_bounds__(NT) void k_forces_part(Geom g, int a0, int a1, const int *spec_off,
                                                    int nspecies, const double *ph0,
                                                    const double *ph1, const double *ph2,
                                                    const double *Z, const double *rc,
                                                    const cpx<T> *rho_g, long long nseg,
                                                    int segs_row, double *part)
{
    constexpr int NW = NT / 64;
    __shared__ double acc[FATOMS * 3 * NW];
    const int tid = threadIdx.x, wv = tid >> 6;
    const int na = a1 - a0;
    for (int i = tid; i < na * 3 * NW; i += NT) acc[i] = 0.0;
    __syncthreads();
    const bool nyq_even = g.m > 0 && 2 * g.m == g.n2;   // the last k2 is -m
    for (long long sg0 = (long long)blockIdx.x * NT; sg0 < nseg; sg0 += (long long)gridDim.x * NT) {
        const long long sg = sg0 + tid;
        const bool live = sg < nseg;
        const long long row = live ? sg / segs_row : 0;
        const int k0 = live ? (int)(sg % segs_row) * FS : 0;
        const int cnt = live ? min(FS, g.n2h - k0) : 0;
        const int i1 = (int)(row % g.n1), i0 = (int)(row / g.n1);
        const int m0 = freq(i0, g.n0), m1 = freq(i1, g.n1);
        // the segment's points: k2 = k0 + j; the Nyquist point (if any) apart
        const int kn = (nyq_even && k0 + cnt - 1 == g.m) ? cnt - 1 : -1;
        const double G0x = m0 * g.b[0][0] + m1 * g.b[1][0] + k0 * g.b[2][0];
        const double G0y = m0 * g.b[0][1] + m1 * g.b[1][1] + k0 * g.b[2][1];
        const double G0z = m0 * g.b[0][2] + m1 * g.b[1][2] + k0 * g.b[2][2];
        const double GNx = m0 * g.b[0][0] + m1 * g.b[1][0] - g.m * g.b[2][0];
        const double GNy = m0 * g.b[0][1] + m1 * g.b[1][1] - g.m * g.b[2][1];
        const double GNz = m0 * g.b[0][2] + m1 * g.b[1][2] - g.m * g.b[2][2];
        const cpx<T> *rrow = rho_g + row * g.n2h + k0;
        for (int s = 0; s < nspecies; ++s) {
            const int lo = max(spec_off[s], a0), hi = min(spec_off[s + 1], a1);
            if (lo >= hi) continue;   // uniform
            const double z = Z[s], r2 = rc[s] * rc[s] * 0.25;
            // w(G) of the segment's points (0 past the row's end and at
            // G = 0); the Nyquist point's w apart (wn), 0 in the progression.
            // Along the segment G^2 = G0^2 + 2 j G0.b2 + j^2 b2^2, so the form
            // factor exp(-r2 G^2) = E0 A^j B^(j^2) advances by C_j = A B^(2j+1)
            // (three exponentials per segment; every factor is at most
            // exp(2 r2 |G0| |b2|), and terms below e^-700 round to 0)
            const double b2x = g.b[2][0], b2y = g.b[2][1], b2z = g.b[2][2];
            const double G00 = G0x * G0x + G0y * G0y + G0z * G0z;
            const double gb = G0x * b2x + G0y * b2y + G0z * b2z;
            const double bb = b2x * b2x + b2y * b2y + b2z * b2z;
            const double Bq = exp(-r2 * bb);
            double E = exp(-r2 * G00), C = exp(-2.0 * r2 * gb) * Bq;
            const double B2 = Bq * Bq, K = -4.0 * PI_D * z;
            double wr[FS], wi[FS];
#pragma unroll
            for (int j = 0; j < FS; ++j) {
                const int k2 = k0 + j;
                const double G2 = G00 + (double)j * (2.0 * gb + (double)j * bb);
                const bool on = j < cnt && j != kn && G2 > 0.0;
                const double c = (k2 == 0 || k2 == g.m) ? 1.0 : 2.0;
                const double w = on ? c * K * E / G2 : 0.0;
                double rx = 0.0, ry = 0.0;
                if (j < cnt) {
                    const cpx<T> rg = rrow[j];
                    rx = (double)rg.x;
                    ry = (double)rg.y;
                }
                wr[j] = w * rx;
                wi[j] = w * ry;
                E *= C;
                C *= B2;
                // one point at a time: interleaving the points' divisions
                // costs registers, not time
                __builtin_amdgcn_sched_barrier(0);
            }
            double wnr = 0.0, wni = 0.0;
            if (kn >= 0) {
                const double GN2 = GNx * GNx + GNy * GNy + GNz * GNz;
                const double w = GN2 > 0.0 ? K * exp(-r2 * GN2) / GN2 : 0.0;   // c = 1
                const cpx<T> rg = rrow[kn];
                wnr = w * (double)rg.x;
                wni = w * (double)rg.y;
            }
            for (int a = lo; a < hi; ++a) {
                double fx = 0.0, fy = 0.0, fz = 0.0;
                if (live) {
                    const double *p0 = ph0 + 2 * ((long long)a * g.n0 + i0);
                    const double *p1 = ph1 + 2 * ((long long)a * g.n1 + i1);
                    const double *p2 = ph2 + 2 * ((long long)a * g.n2h);   // uniform
                    const double qr = p0[0] * p1[0] - p0[1] * p1[1];
                    const double qi = p0[0] * p1[1] + p0[1] * p1[0];
                    const double dr = p2[2], di = p2[3];   // e^{-i b_2.R_a}
                    double tr = qr * p2[2 * k0] - qi * p2[2 * k0 + 1];
                    double ti = qr * p2[2 * k0 + 1] + qi * p2[2 * k0];
                    double s0 = 0.0, s1 = 0.0;
#pragma unroll
                    for (int j = 0; j < FS; ++j) {
                        // Im[conj(t) w] with t = e^{-i G.R}
                        const double im = tr * wi[j] - ti * wr[j];
                        s0 += im;
                        s1 += (double)j * im;
                        const double t2 = tr * dr - ti * di;
                        ti = tr * di + ti * dr;
                        tr = t2;
                    }
                    // the Nyquist point (wn = 0 on lanes without one)
                    const int mq = g.m > 0 ? g.m : 0;
                    const double nr = qr * p2[2 * mq] - qi * p2[2 * mq + 1];
                    const double ni = qr * p2[2 * mq + 1] + qi * p2[2 * mq];
                    const double imn = nr * wni - ni * wnr;
                    fx = G0x * s0 + g.b[2][0] * s1 + GNx * imn;
                    fy = G0y * s0 + g.b[2][1] * s1 + GNy * imn;
                    fz = G0z * s0 + g.b[2][2] * s1 + GNz * imn;
                }
                fx = wave_sum_to_last(fx);
                fy = wave_sum_to_last(fy);
                fz = wave_sum_to_last(fz);
                if ((tid & 63) == 63) {
                    double *o = acc + ((a - a0) * 3) * NW + wv;
                    o[0] += fx;
                    o[NW] += fy;
                    o[2 * NW] += fz;
                }
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < na * 3; i += NT) {
        double v = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) v += acc[i * NW + w];
        part[(long long)blockIdx.x * na * 3 + i] = v;
    }
}

// 16 lanes per force component: lane l adds blocks l, l + 16, .. in order,
// then the 16 sums are added by a fixed butterfly (deterministic)
constexpr int FSUM = 16;
__global__ __launch_bounds__(NT) void k_forces_sum(int na, int nblk, const double *part,
                                                   double *f_out)
{
    const int l = threadIdx.x % FSUM;
    const int i = (int)((blockIdx.x * NT + threadIdx.x) / FSUM);
    const bool ok = i < na * 3;
    double v = 0.0;
    if (ok)
        for (int b = l; b < nblk; b += FSUM) v += part[(long long)b * na * 3 + i];
#pragma unroll
    for (int off = FSUM / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, FSUM);
    if (ok && l == 0) f_out[i] = v;
}

// blocks of the partial-force kernel and the doubles of its partial table
long long forces_blocks(const Geom &g)
{
    const long long nseg = (long long)g.n0 * g.n1 * ((g.n2h + FS - 1) / FS);
    const long long nb = (nseg + NT - 1) / NT;
    return nb < FBLOCKS ? nb : FBLOCKS;
}
long long forces_part_doubles(const Geom &g, int natoms)
{
    return forces_blocks(g) * (long long)(natoms < FATOMS ? natoms : FATOMS) * 3;
}

template <typename T>
hipError_t launch_forces(const Geom &g, int natoms, const int *spec_off, int nspecies,
                         const double *ph0, const double *ph1, const double *ph2, const double *Z,
                         const double *rc, const void *rho_g, double *part, double *f_out,
                         hipStream_t s)
{
    if (natoms <= 0) return hipSuccess;
    const int segs_row = (g.n2h + FS - 1) / FS;
    const long long nseg = (long long)g.n0 * g.n1 * segs_row;
    const int nblk = (int)forces_blocks(g);
    for (int a0 = 0; a0 < natoms; a0 += FATOMS) {
        const int a1 = a0 + FATOMS < natoms ? a0 + FATOMS : natoms;
        hipLaunchKernelGGL((k_forces_part<T>), dim3(nblk), dim3(NT), 0, s, g, a0, a1, spec_off,
                           nspecies, ph0, ph1, ph2, Z, rc, (const cpx<T> *)rho_g, nseg, segs_row,
                           part);
        const int n3 = (a1 - a0) * 3;
        hipLaunchKernelGGL(k_forces_sum, dim3((n3 * FSUM + NT - 1) / NT), dim3(NT), 0, s, a1 - a0,
                           nblk, (const double *)part, f_out + 3 * (long long)a0);
    }
    return hipGetLastError();
}
template hipError_t launch_forces<float>(const Geom &, int, const int *, int, const double *,
                                         const double *, const double *, const double *,
                                         const double *, const void *, double *, double *,
                                         hipStream_t);
template hipError_t launch_forces<double>(const Geom &, int, const int *, int, const double *,
                                          const double *, const double *, const double *,
                                          const double *, const void *, double *, double *,
                                          hipStream_t);

// ---------------------------------------------------------------- vectors
constexpr int DOT_ITEMS = 8;

int dots_blocks(long long n) { return (int)((n + (long long)NT * DOT_ITEMS - 1) / (NT * DOT_ITEMS)); }

// Up to four dot products over the same index range, each block adding its
// NT * DOT_ITEMS elements; with AL (16-byte aligned vectors, n a multiple of
// the group) every load takes 16 bytes.  All products go through one
// block reduction.
template <typename T, bool AL>
__global__ __launch_bounds__(NT) void k_dots(long long n, int nd, const T *x0, const T *y0,
                                             const T *x1, const T *y1, const T *x2, const T *y2,
                                             const T *x3, const T *y3, double *part, int pstride)
{
    __shared__ double red[NT];
    const int tid = threadIdx.x;
    const long long base = (long long)blockIdx.x * NT * DOT_ITEMS;
    const T *xs[4] = {x0, x1, x2, x3};
    const T *ys[4] = {y0, y1, y2, y3};
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if constexpr (AL) {
        constexpr int E = 16 / sizeof(T);
        struct alignas(16) V { T v[E]; };
        static_assert(DOT_ITEMS % E == 0, "whole groups");
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            if (d >= nd) break;
            for (int it = 0; it < DOT_ITEMS / E; ++it) {
                const long long g = base / E + (long long)it * NT + tid;
                if (g * E < n) {
                    const V xv = ((const V *)xs[d])[g], yv = ((const V *)ys[d])[g];
#pragma unroll
                    for (int k = 0; k < E; ++k) acc[d] += (double)xv.v[k] * (double)yv.v[k];
                }
            }
        }
    } else {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            if (d >= nd) break;
            for (int it = 0; it < DOT_ITEMS; ++it) {
                const long long i = base + (long long)it * NT + tid;
                if (i < n) acc[d] += (double)xs[d][i] * (double)ys[d][i];
            }
        }
    }
    block_sums<NT, 4>(acc, red, tid);
    if (tid == 0)
        for (int d = 0; d < nd; ++d) part[(long long)(SL_AUX0 + d) * pstride + blockIdx.x] = acc[d];
}

template <typename T>
hipError_t launch_dots(long long n, int nd, const void *x0, const void *y0, const void *x1,
                       const void *y1, const void *x2, const void *y2, const void *x3,
                       const void *y3, double *part, int pstride, int &nblocks, hipStream_t s)
{
    nblocks = dots_blocks(n);
    if (nblocks > pstride || nd < 1 || nd > 4) return hipErrorInvalidValue;
    constexpr int E = 16 / sizeof(T);
    const bool al = n % E == 0 &&
                    ((size_t)x0 | (size_t)y0 | (size_t)x1 | (size_t)y1 | (size_t)x2 | (size_t)y2 |
                     (size_t)x3 | (size_t)y3) % 16 == 0;
    if (al)
        hipLaunchKernelGGL((k_dots<T, true>), dim3(nblocks), dim3(NT), 0, s, n, nd, (const T *)x0,
                           (const T *)y0, (const T *)x1, (const T *)y1, (const T *)x2,
                           (const T *)y2, (const T *)x3, (const T *)y3, part, pstride);
    else
        hipLaunchKernelGGL((k_dots<T, false>), dim3(nblocks), dim3(NT), 0, s, n, nd, (const T *)x0,
                           (const T *)y0, (const T *)x1, (const T *)y1, (const T *)x2,
                           (const T *)y2, (const T *)x3, (const T *)y3, part, pstride);
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

// 16 bytes per thread (4 floats or 2 doubles) for 16-byte aligned vectors
// whose length is a multiple of the group; the same arithmetic per element
template <typename T>
__global__ __launch_bounds__(NT) void k_lincomb16(long long ng, T *z, double a, const T *x,
                                                  double b, const T *y)
{
    constexpr int E = 16 / sizeof(T);
    struct alignas(16) V { T v[E]; };
    const long long i = (long long)blockIdx.x * NT + threadIdx.x;
    if (i >= ng) return;
    const V xv = ((const V *)x)[i];
    V yv{};
    if (y) yv = ((const V *)y)[i];
    V zv;
#pragma unroll
    for (int k = 0; k < E; ++k) zv.v[k] = T(a * (double)xv.v[k] + (y ? b * (double)yv.v[k] : 0.0));
    ((V *)z)[i] = zv;
}

template <typename T>
hipError_t launch_lincomb(long long n, void *z, double a, const void *x, double b, const void *y,
                          hipStream_t s)
{
    constexpr int E = 16 / sizeof(T);
    const bool al = n % E == 0 && ((size_t)z | (size_t)x | (size_t)y) % 16 == 0;
    if (al) {
        const long long ng = n / E, nb = (ng + NT - 1) / NT;
        hipLaunchKernelGGL((k_lincomb16<T>), dim3((unsigned)nb), dim3(NT), 0, s, ng, (T *)z, a,
                           (const T *)x, b, (const T *)y);
        return hipGetLastError();
    }
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
