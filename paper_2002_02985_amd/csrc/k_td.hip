// Real-time TD-OFDFT (Section "Time-Dependent OFDFT"): pointwise kernels of
// the Crank-Nicolson propagation of the collective orbital psi.  Complex
// vectors are stored split, the N real parts followed by the N imaginary
// parts, so that the pair goes through the real-to-complex transforms as a
// batch of two fields.
#include "kernels_impl.hpp"

namespace ofdft {

namespace {
constexpr int TD_BLOCKS = 2048;     // grid-stride launches
}

// rho = wa |a|^2 + wb |b|^2 (b may be null)
template <typename T>
__global__ __launch_bounds__(NT) void k_td_density(long long n, const T *a, double wa, const T *b,
                                                   double wb, T *rho)
{
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n;
         i += (long long)gridDim.x * NT) {
        const double ar = a[i], ai = a[n + i];
        double r = wa * (ar * ar + ai * ai);
        if (b) {
            const double br = b[i], bi = b[n + i];
            r += wb * (br * br + bi * bi);
        }
        rho[i] = T(r);
    }
}

// Cartesian position of grid point (i0, i1, i2): sum_d (i_d / n_d) a_d
__device__ __forceinline__ void td_position(const Geom &g, const double *lat, long long i,
                                            double (&r)[3])
{
    const int i2 = (int)(i % g.n2);
    const long long q = i / g.n2;
    const int i1 = (int)(q % g.n1), i0 = (int)(q / g.n1);
    const double f0 = (double)i0 / g.n0, f1 = (double)i1 / g.n1, f2 = (double)i2 / g.n2;
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = f0 * lat[c] + f1 * lat[3 + c] + f2 * lat[6 + c];
}

// per-block partial sums of rho x, rho y, rho z (part[3 * block + c])
template <typename T>
__global__ __launch_bounds__(NT) void k_td_dipole(Geom g, TdLattice L, const T *rho, double *part)
{
    __shared__ double red[NT / 64];
    const int tid = threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    for (long long i = (long long)blockIdx.x * NT + tid; i < g.N;
         i += (long long)gridDim.x * NT) {
        double r[3];
        td_position(g, L.a, i, r);
        const double w = (double)rho[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] += r[c] * w;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double s = block_sum<NT>(acc[c], red, tid);
        if (tid == 0) part[3 * blockIdx.x + c] = s;
    }
}

// psi = sqrt(rho) exp(-i k.r)
template <typename T>
__global__ __launch_bounds__(NT) void k_td_kick(Geom g, TdLattice L, double k0, double k1,
                                                double k2, const T *rho, T *psi)
{
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < g.N;
         i += (long long)gridDim.x * NT) {
        double r[3];
        td_position(g, L.a, i, r);
        const double ph = k0 * r[0] + k1 * r[1] + k2 * r[2];
        double sn, cs;
        sincos(ph, &sn, &cs);
        const double a = sqrt(fmax((double)rho[i], 0.0));
        psi[i] = T(a * cs);
        psi[g.N + i] = T(-a * sn);
    }
}

// A diagonal operator c(G) of the complex field on the half spectra A, B of
// its real and imaginary parts (psi = a + i b): with c = cr + i ci even in G,
// the result's parts have spectra cr A - ci B and ci A + cr B.  With
// q = tau h, h = G^2 / 2: TD_KIN c = h (the kinetic operator), TD_K
// c = 1 + i q, TD_KINV c = 1 / (1 + i q).  On the self-conjugate planes
// (k2 = 0 and n2/2) the inverse real transform keeps the Hermitian part, so
// a point and its partner ((n0 - i0) % n0, (n1 - i1) % n1) act with the mean
// of their two h (different for the aliased Nyquist frequencies of a skewed
// cell): h is taken as that mean there, which keeps c even and makes TD_KINV
// the exact inverse of TD_K.
template <typename T>
__global__ __launch_bounds__(NT) void k_td_spectral(Geom g, cpx<T> *spec, const T *g2,
                                                    double tau, int mode)
{
    const long long nh = g.Nh;
    for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < nh;
         e += (long long)gridDim.x * NT) {
        double h = 0.5 * (double)g2[e];
        const int k2 = (int)(e % g.n2h);
        if (k2 == 0 || k2 == g.m) {
            const long long r = e / g.n2h;
            const int i1 = (int)(r % g.n1), i0 = (int)(r / g.n1);
            const int p0 = i0 == 0 ? 0 : g.n0 - i0, p1 = i1 == 0 ? 0 : g.n1 - i1;
            const long long ep = ((long long)p0 * g.n1 + p1) * g.n2h + k2;
            h = 0.5 * (h + 0.5 * (double)g2[ep]);
        }
        double cr, ci;
        if (mode == TD_KIN) {
            cr = h;
            ci = 0.0;
        } else if (mode == TD_K) {
            cr = 1.0;
            ci = tau * h;
        } else {
            const double q = tau * h, d = 1.0 / (1.0 + q * q);
            cr = d;
            ci = -q * d;
        }
        const cpx<T> A = spec[e], B = spec[nh + e];
        const double ar = A.x, ai = A.y, br = B.x, bi = B.y;
        spec[e] = {T(cr * ar - ci * br), T(cr * ai - ci * bi)};
        spec[nh + e] = {T(ci * ar + cr * br), T(ci * ai + cr * bi)};
    }
}

// out = x + i tau (Tx + v x), Tx the kinetic part already applied
template <typename T>
__global__ __launch_bounds__(NT) void k_td_apply(long long n, const T *x, const T *tx, const T *v,
                                                 double tau, T *out)
{
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n;
         i += (long long)gridDim.x * NT) {
        const double xr = x[i], xi = x[n + i], vv = v[i];
        const double hr = (double)tx[i] + vv * xr, hi = (double)tx[n + i] + vv * xi;
        out[i] = T(xr - tau * hi);
        out[n + i] = T(xi + tau * hr);
    }
}

// out = z + i tau v u (the right-preconditioned operator with u = K^-1 z)
template <typename T>
__global__ __launch_bounds__(NT) void k_td_pc_apply(long long n, const T *z, const T *u,
                                                    const T *v, double tau, T *out)
{
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n;
         i += (long long)gridDim.x * NT) {
        const double vv = v[i], ur = u[i], ui = u[n + i];
        const double zr = z[i], zi = z[n + i];
        out[i] = T(zr - tau * vv * ui);
        out[n + i] = T(zi + tau * vv * ur);
    }
}

// z = a x + b y + c w with complex coefficients (y, w may be null; z may
// alias any of them: each element is read before it is written)
template <typename T>
__global__ __launch_bounds__(NT) void k_td_zlincomb(long long n, T *z, double ar, double ai,
                                                    const T *x, double br, double bi, const T *y,
                                                    double cr, double ci, const T *w)
{
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n;
         i += (long long)gridDim.x * NT) {
        const double xr = x[i], xi = x[n + i];
        double zr = ar * xr - ai * xi, zi = ar * xi + ai * xr;
        if (y) {
            const double yr = y[i], yi = y[n + i];
            zr += br * yr - bi * yi;
            zi += br * yi + bi * yr;
        }
        if (w) {
            const double wr = w[i], wi = w[n + i];
            zr += cr * wr - ci * wi;
            zi += cr * wi + ci * wr;
        }
        z[i] = T(zr);
        z[n + i] = T(zi);
    }
}

static unsigned td_grid(long long n)
{
    const long long nb = (n + NT - 1) / NT;
    return (unsigned)(nb < TD_BLOCKS ? nb : TD_BLOCKS);
}

int td_dipole_blocks(const Geom &g) { return (int)td_grid(g.N); }

template <typename T>
hipError_t launch_td_density(long long n, const void *a, double wa, const void *b, double wb,
                             void *rho, hipStream_t s)
{
    hipLaunchKernelGGL((k_td_density<T>), dim3(td_grid(n)), dim3(NT), 0, s, n, (const T *)a, wa,
                       (const T *)b, wb, (T *)rho);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_td_dipole(const Geom &g, const TdLattice &L, const void *rho, double *part,
                            hipStream_t s)
{
    hipLaunchKernelGGL((k_td_dipole<T>), dim3(td_grid(g.N)), dim3(NT), 0, s, g, L,
                       (const T *)rho, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_td_kick(const Geom &g, const TdLattice &L, const double k[3], const void *rho,
                          void *psi, hipStream_t s)
{
    hipLaunchKernelGGL((k_td_kick<T>), dim3(td_grid(g.N)), dim3(NT), 0, s, g, L, k[0], k[1], k[2],
                       (const T *)rho, (T *)psi);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_td_spectral(const Geom &g, void *spec, const void *g2, double tau, int mode,
                              hipStream_t s)
{
    if (mode != TD_KIN && mode != TD_K && mode != TD_KINV) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_td_spectral<T>), dim3(td_grid(g.Nh)), dim3(NT), 0, s, g,
                       (cpx<T> *)spec, (const T *)g2, tau, mode);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_td_pc_apply(long long n, const void *z, const void *u, const void *v,
                              double tau, void *out, hipStream_t s)
{
    hipLaunchKernelGGL((k_td_pc_apply<T>), dim3(td_grid(n)), dim3(NT), 0, s, n, (const T *)z,
                       (const T *)u, (const T *)v, tau, (T *)out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_td_apply(long long n, const void *x, const void *tx, const void *v, double tau,
                           void *out, hipStream_t s)
{
    hipLaunchKernelGGL((k_td_apply<T>), dim3(td_grid(n)), dim3(NT), 0, s, n, (const T *)x,
                       (const T *)tx, (const T *)v, tau, (T *)out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_td_zlincomb(long long n, void *z, const double a[2], const void *x,
                              const double b[2], const void *y, const double c[2], const void *w,
                              hipStream_t s)
{
    hipLaunchKernelGGL((k_td_zlincomb<T>), dim3(td_grid(n)), dim3(NT), 0, s, n, (T *)z, a[0], a[1],
                       (const T *)x, b[0], b[1], (const T *)y, c[0], c[1], (const T *)w);
    return hipGetLastError();
}

// ---------------------------------------------------------------- device-side BiCGSTAB
int td_dot_blocks(long long n) { return (int)td_grid(n); }

template <typename T>
__global__ __launch_bounds__(NT) void k_td_cdots(long long n, const T *a, const T *b, const T *c,
                                                 const T *d, double *part, int rows)
{
    __shared__ double red[4 * NT / 64];
    const int tid = threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long i = (long long)blockIdx.x * NT + tid; i < n; i += (long long)gridDim.x * NT) {
        const double ar = a[i], ai = a[n + i], br = b[i], bi = b[n + i];
        v[0] += ar * br + ai * bi;
        v[1] += ar * bi - ai * br;
        if (c) {
            const double cr = c[i], ci = c[n + i], dr = d[i], di = d[n + i];
            v[2] += cr * dr + ci * di;
            v[3] += cr * di - ci * dr;
        }
    }
    block_sums<NT, 4>(v, red, tid);
    if (tid == 0)
        for (int k = 0; k < rows; ++k) part[(long long)k * gridDim.x + blockIdx.x] = v[k];
}

template <typename T>
hipError_t launch_td_cdots(long long n, const void *a, const void *b, const void *c,
                           const void *d, double *part, hipStream_t s)
{
    hipLaunchKernelGGL((k_td_cdots<T>), dim3(td_grid(n)), dim3(NT), 0, s, n, (const T *)a,
                       (const T *)b, (const T *)c, (const T *)d, part, c ? 4 : 2);
    return hipGetLastError();
}

namespace {
struct zc {
    double r, i;
};
__device__ __forceinline__ zc zmul(zc a, zc b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__device__ __forceinline__ zc zdiv(zc a, zc b)
{
    const double d = b.r * b.r + b.i * b.i;
    return {(a.r * b.r + a.i * b.i) / d, (a.i * b.r - a.r * b.i) / d};
}
__device__ __forceinline__ zc zget(const double *sc, int k) { return {sc[k], sc[k + 1]}; }
__device__ __forceinline__ void zput(double *sc, int k, zc v)
{
    sc[k] = v.r;
    sc[k + 1] = v.i;
}
}  // namespace

// one block: the dot products in fixed order, then the step's scalars
__global__ __launch_bounds__(NT) void k_td_scalars(int step, int nblk, const double *part,
                                                   double *sc)
{
    __shared__ double red[4 * NT / 64];
    const int tid = threadIdx.x;
    const int rows = (step == TD_STEP_INIT || step == TD_STEP_OMEGA) ? 4 : 2;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < rows; ++k)
        for (int i = tid; i < nblk; i += NT) v[k] += part[(long long)k * nblk + i];
    block_sums<NT, 4>(v, red, tid);
    if (tid != 0) return;
    const zc d0 = {v[0], v[1]}, d1 = {v[2], v[3]};
    if (step == TD_STEP_INIT) {
        const double bnorm = sqrt(fmax(d0.r, 1e-300));
        sc[TS_BNORM] = bnorm;
        sc[TS_RES] = sqrt(fmax(d1.r, 0.0)) / bnorm;
        sc[TS_DONE] = sc[TS_RES] > sc[TS_TOL] && sc[TS_MAXIT] > 0 ? 0.0 : 1.0;
        sc[TS_IT] = 0.0;
        zput(sc, TS_RHOP, {1.0, 0.0});
        zput(sc, TS_ALPHA, {1.0, 0.0});
        zput(sc, TS_OMEGA, {1.0, 0.0});
        return;
    }
    if (sc[TS_DONE] != 0.0) return;
    if (step == TD_STEP_RHO) {
        sc[TS_IT] += 1.0;
        if (d0.r == 0.0 && d0.i == 0.0) {   // breakdown: stop with the current iterate
            sc[TS_DONE] = 1.0;
            return;
        }
        zput(sc, TS_RHO, d0);
        const zc beta = zmul(zdiv(d0, zget(sc, TS_RHOP)), zdiv(zget(sc, TS_ALPHA), zget(sc, TS_OMEGA)));
        const zc bw = zmul(beta, zget(sc, TS_OMEGA));
        zput(sc, TS_CP, {1.0, 0.0});
        zput(sc, TS_CP + 2, beta);
        zput(sc, TS_CP + 4, {-bw.r, -bw.i});
    } else if (step == TD_STEP_RV) {
        if (d0.r == 0.0 && d0.i == 0.0) {
            sc[TS_DONE] = 1.0;
            return;
        }
        const zc alpha = zdiv(zget(sc, TS_RHO), d0);
        zput(sc, TS_ALPHA, alpha);
        zput(sc, TS_CS, {1.0, 0.0});
        zput(sc, TS_CS + 2, {-alpha.r, -alpha.i});
    } else if (step == TD_STEP_OMEGA) {
        // d0 = <t,s>, d1 = <t,t> (real)
        const zc omega = d1.r > 0.0 ? zc{d0.r / d1.r, d0.i / d1.r} : zc{0.0, 0.0};
        zput(sc, TS_OMEGA, omega);
        zput(sc, TS_CY, {1.0, 0.0});
        zput(sc, TS_CY + 2, zget(sc, TS_ALPHA));
        zput(sc, TS_CY + 4, omega);
        zput(sc, TS_CR, {1.0, 0.0});
        zput(sc, TS_CR + 2, {-omega.r, -omega.i});
    } else {   // TD_STEP_RR
        sc[TS_RES] = sqrt(fmax(d0.r, 0.0)) / sc[TS_BNORM];
        const zc om = zget(sc, TS_OMEGA);
        if (sc[TS_RES] <= sc[TS_TOL] || (om.r == 0.0 && om.i == 0.0) || sc[TS_IT] >= sc[TS_MAXIT])
            sc[TS_DONE] = 1.0;
        zput(sc, TS_RHOP, zget(sc, TS_RHO));
    }
}

hipError_t launch_td_scalars(int step, long long n, const double *part, double *sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_td_scalars, dim3(1), dim3(NT), 0, s, step, (int)td_grid(n), part, sc);
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(NT) void k_td_zlincomb_dev(long long n, T *z, const double *sc,
                                                        int coef, const T *x, const T *y,
                                                        const T *w)
{
    if (sc[TS_DONE] != 0.0) return;
    const double ar = sc[coef], ai = sc[coef + 1];
    const double br = y ? sc[coef + 2] : 0.0, bi = y ? sc[coef + 3] : 0.0;
    const double cr = w ? sc[coef + 4] : 0.0, ci = w ? sc[coef + 5] : 0.0;
    for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n;
         i += (long long)gridDim.x * NT) {
        const double xr = x[i], xi = x[n + i];
        double zr = ar * xr - ai * xi, zi = ar * xi + ai * xr;
        if (y) {
            const double yr = y[i], yi = y[n + i];
            zr += br * yr - bi * yi;
            zi += br * yi + bi * yr;
        }
        if (w) {
            const double wr = w[i], wi = w[n + i];
            zr += cr * wr - ci * wi;
            zi += cr * wi + ci * wr;
        }
        z[i] = T(zr);
        z[n + i] = T(zi);
    }
}

template <typename T>
hipError_t launch_td_zlincomb_dev(long long n, void *z, const double *sc, int coef, const void *x,
                                  const void *y, const void *w, hipStream_t s)
{
    hipLaunchKernelGGL((k_td_zlincomb_dev<T>), dim3(td_grid(n)), dim3(NT), 0, s, n, (T *)z, sc,
                       coef, (const T *)x, (const T *)y, (const T *)w);
    return hipGetLastError();
}

#define OFDFT_TD_INSTANTIATE(T)                                                                   \
    template hipError_t launch_td_cdots<T>(long long, const void *, const void *, const void *,   \
                                           const void *, double *, hipStream_t);                  \
    template hipError_t launch_td_zlincomb_dev<T>(long long, void *, const double *, int,         \
                                                  const void *, const void *, const void *,       \
                                                  hipStream_t);                                   \
    template hipError_t launch_td_density<T>(long long, const void *, double, const void *,      \
                                             double, void *, hipStream_t);                        \
    template hipError_t launch_td_dipole<T>(const Geom &, const TdLattice &, const void *,        \
                                            double *, hipStream_t);                               \
    template hipError_t launch_td_kick<T>(const Geom &, const TdLattice &, const double *,        \
                                          const void *, void *, hipStream_t);                     \
    template hipError_t launch_td_spectral<T>(const Geom &, void *, const void *, double, int,     \
                                              hipStream_t);                                       \
    template hipError_t launch_td_pc_apply<T>(long long, const void *, const void *, const void *, \
                                              double, void *, hipStream_t);                       \
    template hipError_t launch_td_apply<T>(long long, const void *, const void *, const void *,   \
                                           double, void *, hipStream_t);                          \
    template hipError_t launch_td_zlincomb<T>(long long, void *, const double *, const void *,    \
                                              const double *, const void *, const double *,       \
                                              const void *, hipStream_t);
OFDFT_TD_INSTANTIATE(float)
OFDFT_TD_INSTANTIATE(double)

}  // namespace ofdft
