// Ionic set-up kernels, all FP64: the per-axis structure-factor phase tables
// and the Ewald energy and forces of the point ions (the constant E_ion of
// the total energy, and the ion-ion part of the forces).
#include "kernels_impl.hpp"

namespace ofdft {

// ---------------------------------------------------------------- phases
// One thread per (atom, table entry).  The product m s is reduced to
// [-1/2, 1/2] exactly before the sine and cosine.
__global__ __launch_bounds__(NT) void k_phases(Geom g, int natoms, const double *frac,
                                               double *ph0, double *ph1, double *ph2)
{
    const int ntab = g.n0 + g.n1 + g.n2h;
    const long long idx = (long long)blockIdx.x * NT + threadIdx.x;
    if (idx >= (long long)natoms * ntab) return;
    const int a = (int)(idx / ntab);
    int i = (int)(idx % ntab);
    int d, n;
    double *tab;
    if (i < g.n0) {
        d = 0;
        n = g.n0;
        tab = ph0;
    } else if (i < g.n0 + g.n1) {
        d = 1;
        i -= g.n0;
        n = g.n1;
        tab = ph1;
    } else {
        d = 2;
        i -= g.n0 + g.n1;
        n = g.n2h;
        tab = ph2;
    }
    const int m = (d == 2) ? ((i == g.m) ? -g.m : i) : freq(i, n);
    double x = (double)m * frac[3 * a + d];
    x -= rint(x);
    double sn, cs;
    sincospi(-2.0 * x, &sn, &cs);
    tab[2 * ((long long)a * n + i)] = cs;
    tab[2 * ((long long)a * n + i) + 1] = sn;
}

hipError_t launch_phases(const Geom &g, int natoms, const double *frac, double *ph0, double *ph1,
                         double *ph2, hipStream_t s)
{
    if (natoms <= 0) return hipSuccess;
    const long long n = (long long)natoms * (g.n0 + g.n1 + g.n2h);
    hipLaunchKernelGGL(k_phases, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, g, natoms,
                       frac, ph0, ph1, ph2);
    return hipGetLastError();
}

// ---------------------------------------------------------------- Ewald
__device__ __forceinline__ void ewald_gvec(const EwaldGeom &e, long long t, double (&G)[3],
                                           double &g2)
{
    const int w1 = 2 * e.gmax[1] + 1, w2 = 2 * e.gmax[2] + 1;
    const int k = (int)(t % w2) - e.gmax[2];
    const long long r = t / w2;
    const int j = (int)(r % w1) - e.gmax[1];
    const int i = (int)(r / w1) - e.gmax[0];
#pragma unroll
    for (int c = 0; c < 3; ++c) G[c] = i * e.b[0][c] + j * e.b[1][c] + k * e.b[2][c];
    g2 = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
    if (i == 0 && j == 0 && k == 0) g2 = 0.0;
}

// S(G) = sum_a q_a exp(i G.R_a), one thread per point of the integer box,
// atoms summed in order
__global__ __launch_bounds__(NT) void k_ewald_sf(EwaldGeom e, int natoms, const double *pos,
                                                 const double *q, double *sf)
{
    const long long t = (long long)blockIdx.x * NT + threadIdx.x;
    if (t >= ewald_gbox_count(e)) return;
    double G[3], g2;
    ewald_gvec(e, t, G, g2);
    double sr = 0.0, si = 0.0;
    if (g2 > 0.0 && g2 <= e.gcut2) {
        for (int a = 0; a < natoms; ++a) {
            double sn, cs;
            sincos(G[0] * pos[3 * a] + G[1] * pos[3 * a + 1] + G[2] * pos[3 * a + 2], &sn, &cs);
            sr += q[a] * cs;
            si += q[a] * sn;
        }
    }
    sf[2 * t] = sr;
    sf[2 * t + 1] = si;
}

// One block per atom i: real-space pairs (j, image) with r < rcut, and the
// reciprocal sum over G of Re/Im[exp(i G.R_i) conj S(G)].
__global__ __launch_bounds__(NT) void k_ewald_atoms(EwaldGeom e, int natoms, const double *pos,
                                                    const double *q, const double *sf,
                                                    double *e_atom, double *f)
{
    __shared__ double red[4 * NT / 64];
    const int i = blockIdx.x, tid = threadIdx.x;
    const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2], qi = q[i];
    const int w1 = 2 * e.nmax[1] + 1, w2 = 2 * e.nmax[2] + 1;
    const long long nimg = ewald_image_count(e);
    const double a = e.a;
    const double two_a_sqrtpi = 2.0 * a / sqrt(PI_D);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};   // energy, fx, fy, fz
    for (long long p = tid; p < (long long)natoms * nimg; p += NT) {
        const int j = (int)(p / nimg);
        const long long l = p % nimg;
        const int kk = (int)(l % w2) - e.nmax[2];
        const long long r1 = l / w2;
        const int jj = (int)(r1 % w1) - e.nmax[1];
        const int ii = (int)(r1 / w1) - e.nmax[0];
        const double dx = xi - pos[3 * j] - (ii * e.lat[0][0] + jj * e.lat[1][0] + kk * e.lat[2][0]);
        const double dy = yi - pos[3 * j + 1] - (ii * e.lat[0][1] + jj * e.lat[1][1] + kk * e.lat[2][1]);
        const double dz = zi - pos[3 * j + 2] - (ii * e.lat[0][2] + jj * e.lat[1][2] + kk * e.lat[2][2]);
        const double r2 = dx * dx + dy * dy + dz * dz;
        if (r2 < 1e-20 || r2 > e.rcut2) continue;
        const double r = sqrt(r2);
        const double ec = erfc(a * r);
        const double qq = qi * q[j];
        acc[0] += 0.5 * qq * ec / r;
        const double mag = qq * (ec / r2 + two_a_sqrtpi * exp(-a * a * r2) / r) / r;
        acc[1] += mag * dx;
        acc[2] += mag * dy;
        acc[3] += mag * dz;
    }
    const long long nbox = ewald_gbox_count(e);
    const double pre = 2.0 * PI_D / e.volume;
    for (long long t = tid; t < nbox; t += NT) {
        double G[3], g2;
        ewald_gvec(e, t, G, g2);
        if (!(g2 > 0.0 && g2 <= e.gcut2)) continue;
        double sn, cs;
        sincos(G[0] * xi + G[1] * yi + G[2] * zi, &sn, &cs);
        const double sr = sf[2 * t], si = sf[2 * t + 1];
        const double w = exp(-g2 / (4.0 * a * a)) / g2;
        acc[0] += pre * w * qi * (cs * sr + sn * si);
        const double fm = 2.0 * pre * w * qi * (sn * sr - cs * si);
        acc[1] += fm * G[0];
        acc[2] += fm * G[1];
        acc[3] += fm * G[2];
    }
    block_sums<NT, 4>(acc, red, tid);
    if (tid == 0) {
        e_atom[i] = acc[0];
        if (f) {
            f[3 * i] = acc[1];
            f[3 * i + 1] = acc[2];
            f[3 * i + 2] = acc[3];
        }
    }
}

hipError_t launch_ewald(const EwaldGeom &e, int natoms, const double *pos, const double *q,
                        double *sf, double *e_atom, double *f, hipStream_t s)
{
    if (natoms <= 0) return hipSuccess;
    const long long nbox = ewald_gbox_count(e);
    hipLaunchKernelGGL(k_ewald_sf, dim3((unsigned)((nbox + NT - 1) / NT)), dim3(NT), 0, s, e, natoms,
                       pos, q, sf);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_ewald_atoms, dim3(natoms), dim3(NT), 0, s, e, natoms, pos, q, sf, e_atom, f);
    return hipGetLastError();
}

}  // namespace ofdft
