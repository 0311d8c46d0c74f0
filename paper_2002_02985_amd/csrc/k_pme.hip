// Smooth particle-mesh Ewald structure factor (Essmann et al. 1995), the
// paper's method for the ionic structure factor of large cells (Sections
// "OFDFT software background" and "Leveraging existing techniques").  Each
// species' atoms are spread onto the grid with order-P cardinal B-splines,
// the charge grid goes through the grid's forward transform, and a last pass
// multiplies by the exponential-spline factors b(m) and forms that species'
// share of v_ext(G) and of the Ewald reciprocal sum.
//
// The spread accumulates in 64-bit fixed point (PME_FIX_BITS fractional
// bits) with integer atomics: the sum is exact, so the charge grid does not
// depend on the order in which atoms land, and the set-up is reproducible.
#include "kernels_impl.hpp"

namespace ofdft {

namespace {
constexpr double PME_FIX = (double)(1ull << PME_FIX_BITS);
constexpr int PME_FINISH_BLOCKS = 4096;
}

// One thread per (atom, j0, j1): axis-0 and axis-1 weights for its pair of
// offsets, the P axis-2 points in a loop.  Atom a with scaled coordinate
// u = n s touches k = floor(u) - j (mod n), j = 0 .. P-1, with weight
// M_P(u - floor(u) + j).
template <int P>
__global__ __launch_bounds__(NT) void k_pme_spread(Geom g, int a_beg, int natoms,
                                                   const double *frac, unsigned long long *q)
{
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t >= (long long)natoms * (P * P)) return;
    const int a = a_beg + (int)(t / (P * P));
    const int j0 = (int)((t / P) % P), j1 = (int)(t % P);
    const int n[3] = {g.n0, g.n1, g.n2};
    int base[3];
    double sel[2], w2[P];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double u = frac[3LL * a + d] * n[d];
        int b = (int)floor(u);
        const double tt = u - b;
        if (b >= n[d]) b -= n[d];     // s rounded up to 1
        if (b < 0) b += n[d];
        base[d] = b;
        double w[P];
        bspline_fill<P>(tt, w);
        if (d == 2) {
#pragma unroll
            for (int j = 0; j < P; ++j) w2[j] = w[j];
        } else {
            // the weight at this thread's offset, selected without a
            // dynamically indexed array
            const int jd = d == 0 ? j0 : j1;
            double x = 0.0;
#pragma unroll
            for (int j = 0; j < P; ++j) x = (j == jd) ? w[j] : x;
            sel[d] = x;
        }
    }
    int k0 = base[0] - j0, k1 = base[1] - j1;
    if (k0 < 0) k0 += n[0];
    if (k1 < 0) k1 += n[1];
    const double w01 = sel[0] * sel[1];
    unsigned long long *row = q + ((long long)k0 * n[1] + k1) * n[2];
#pragma unroll
    for (int j2 = 0; j2 < P; ++j2) {
        int k2 = base[2] - j2;
        if (k2 < 0) k2 += n[2];
        atomicAdd(row + k2, __double2ull_rn(w01 * w2[j2] * PME_FIX));
    }
}

template <typename T>
__global__ __launch_bounds__(NT) void k_pme_to_real(long long n, const unsigned long long *q,
                                                    T *out)
{
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n;
         i += (long long)gridDim.x * NT) {
        const double v = (double)q[i] * (1.0 / PME_FIX);
        out[i] = T(v);   // may alias q (T = double): same thread, read before write
    }
}

// S(G) = N b0(m0) b1(m1) b2(m2) F(G) with F the normalised forward transform
// of the charge grid and b the (conjugated) exponential-spline factors in bt
// (n0 + n1 + n2h entries); v_ext += v_s(|G|) S / V; Z S accumulated in qbuf
// across species, and after the last one the Ewald reciprocal partial
// c exp(-G^2/(4 a^2)) / G^2 |sum_s Z_s S_s|^2 for 0 < G^2 <= gcut^2.
template <typename T>
__global__ __launch_bounds__(NT) void k_pme_finish(Geom g, const cpx<T> *F, const double2 *bt,
                                                   double z, double rcs, double inv_vol,
                                                   double ew_a, double ew_gcut2, int first,
                                                   int last, cpx<T> *vext, double2 *qbuf,
                                                   double *ew_part)
{
    __shared__ double red[NT / 64];
    const int tid = threadIdx.x;
    const double scale = (double)g.N;
    double ew = 0.0;
    for (long long e = (long long)blockIdx.x * NT + tid; e < g.Nh;
         e += (long long)gridDim.x * NT) {
        const int k2 = (int)(e % g.n2h);
        const long long r = e / g.n2h;
        const int i1 = (int)(r % g.n1), i0 = (int)(r / g.n1);
        const double2 b0 = bt[i0], b1 = bt[g.n0 + i1], b2 = bt[g.n0 + g.n1 + k2];
        const double br = b0.x * b1.x - b0.y * b1.y, bi = b0.x * b1.y + b0.y * b1.x;
        const double cr = br * b2.x - bi * b2.y, ci = br * b2.y + bi * b2.x;
        const double fr = (double)F[e].x * scale, fi = (double)F[e].y * scale;
        const double sr = cr * fr - ci * fi, si = cr * fi + ci * fr;
        const int m2 = (k2 == g.m) ? -g.m : k2;
        const double G2 = gvec2<double>(g, freq(i0, g.n0), freq(i1, g.n1), m2);
        const double vs = G2 > 0.0 ? -4.0 * PI_D * z * exp(-G2 * rcs * rcs * 0.25) / G2
                                   : PI_D * z * rcs * rcs;
        double vr = vs * sr * inv_vol, vi = vs * si * inv_vol;
        if (!first) {
            vr += (double)vext[e].x;
            vi += (double)vext[e].y;
        }
        vext[e] = {T(vr), T(vi)};
        double qr = z * sr, qi = z * si;
        if (!first) {
            qr += qbuf[e].x;
            qi += qbuf[e].y;
        }
        if (!last) {
            qbuf[e] = {qr, qi};
        } else if (G2 > 0.0 && G2 <= ew_gcut2) {
            const double c = (k2 == 0 || k2 == g.m) ? 1.0 : 2.0;
            ew += c * exp(-G2 / (4.0 * ew_a * ew_a)) / G2 * (qr * qr + qi * qi);
        }
    }
    ew = block_sum<NT>(ew, red, tid);
    if (tid == 0) ew_part[blockIdx.x] = ew;
}

int pme_finish_blocks(const Geom &g)
{
    const long long need = (g.Nh + NT - 1) / NT;
    return (int)(need < PME_FINISH_BLOCKS ? need : PME_FINISH_BLOCKS);
}

template <int P>
static hipError_t spread_p(const Geom &g, int a_beg, int natoms, const double *frac,
                           unsigned long long *q, hipStream_t s)
{
    const long long nt = (long long)natoms * P * P;
    hipLaunchKernelGGL((k_pme_spread<P>), dim3((unsigned)((nt + NT - 1) / NT)), dim3(NT), 0, s,
                       g, a_beg, natoms, frac, q);
    return hipGetLastError();
}

hipError_t launch_pme_spread(const Geom &g, int order, int a_beg, int natoms, const double *frac,
                             unsigned long long *q, hipStream_t s)
{
    if (natoms <= 0) return hipSuccess;
    if (order > g.n0 || order > g.n1 || order > g.n2) return hipErrorInvalidValue;
    if ((long long)natoms * order * order / NT >= (1ll << 31)) return hipErrorInvalidValue;
    switch (order) {
    case 4: return spread_p<4>(g, a_beg, natoms, frac, q, s);
    case 6: return spread_p<6>(g, a_beg, natoms, frac, q, s);
    case 8: return spread_p<8>(g, a_beg, natoms, frac, q, s);
    case 10: return spread_p<10>(g, a_beg, natoms, frac, q, s);
    case 12: return spread_p<12>(g, a_beg, natoms, frac, q, s);
    case 14: return spread_p<14>(g, a_beg, natoms, frac, q, s);
    case 16: return spread_p<16>(g, a_beg, natoms, frac, q, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t launch_pme_to_real(const Geom &g, const unsigned long long *q, void *out, hipStream_t s)
{
    const long long nb = (g.N + NT - 1) / NT;
    hipLaunchKernelGGL((k_pme_to_real<T>), dim3((unsigned)(nb < 65536 ? nb : 65536)), dim3(NT), 0,
                       s, g.N, q, (T *)out);
    return hipGetLastError();
}
template hipError_t launch_pme_to_real<float>(const Geom &, const unsigned long long *, void *,
                                              hipStream_t);
template hipError_t launch_pme_to_real<double>(const Geom &, const unsigned long long *, void *,
                                               hipStream_t);

template <typename T>
hipError_t launch_pme_finish(const Geom &g, const void *F, const double2 *bt, double z, double rc,
                             double volume, double ew_a, double ew_gcut2, int first, int last,
                             void *vext, void *qbuf, double *ew_part, hipStream_t s)
{
    if (!last && !qbuf) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_pme_finish<T>), dim3((unsigned)pme_finish_blocks(g)), dim3(NT), 0, s, g,
                       (const cpx<T> *)F, bt, z, rc, 1.0 / volume, ew_a, ew_gcut2, first, last,
                       (cpx<T> *)vext, (double2 *)qbuf, ew_part);
    return hipGetLastError();
}
template hipError_t launch_pme_finish<float>(const Geom &, const void *, const double2 *, double,
                                             double, double, double, double, int, int, void *,
                                             void *, double *, hipStream_t);
template hipError_t launch_pme_finish<double>(const Geom &, const void *, const double2 *, double,
                                              double, double, double, double, int, int, void *,
                                              void *, double *, hipStream_t);

}  // namespace ofdft
