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

// S(G) = sum_a q_a exp(i G.R_a) over the integer box of reciprocal vectors,
// and w(G) = exp(-G^2 / 4a^2) / G^2 (0 at G = 0 and beyond the cut-off,
// where S is 0 too): sf[2t], sf[2t + 1] = S, sf[2 nbox + t] = w.  A thread
// takes EW_K consecutive k of one (i, j) row; per atom it evaluates one sine
// and cosine and advances the phase along k by exp(i b_2.R) (one complex
// multiplication per point); atoms are summed in order.
constexpr int EW_K = 8;
__global__ __launch_bounds__(NT) void k_ewald_sf(EwaldGeom e, int natoms, const double *pos,
                                                 const double *q, double *sf)
{
    const int w0 = 2 * e.gmax[0] + 1, w1 = 2 * e.gmax[1] + 1, w2 = 2 * e.gmax[2] + 1;
    const int segs = (w2 + EW_K - 1) / EW_K;
    const long long sg = (long long)blockIdx.x * NT + threadIdx.x;
    if (sg >= (long long)w0 * w1 * segs) return;
    const int row = (int)(sg / segs), k0 = (int)(sg % segs) * EW_K;
    const int i = row / w1 - e.gmax[0], j = row % w1 - e.gmax[1];
    const int cnt = min(EW_K, w2 - k0);
    const long long nbox = ewald_gbox_count(e);
    double G0[3], B2[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        G0[c] = i * e.b[0][c] + j * e.b[1][c] + (k0 - e.gmax[2]) * e.b[2][c];
        B2[c] = e.b[2][c];
    }
    double sr[EW_K], si[EW_K];
    bool on[EW_K];
#pragma unroll
    for (int kk = 0; kk < EW_K; ++kk) {
        sr[kk] = si[kk] = 0.0;
        const double gx = G0[0] + kk * B2[0], gy = G0[1] + kk * B2[1], gz = G0[2] + kk * B2[2];
        const double g2 = gx * gx + gy * gy + gz * gz;
        const bool zero = i == 0 && j == 0 && k0 + kk == e.gmax[2];
        on[kk] = kk < cnt && !zero && g2 > 0.0 && g2 <= e.gcut2;
        if (kk < cnt)
            sf[2 * nbox + (long long)row * w2 + k0 + kk] =
                on[kk] ? exp(-g2 / (4.0 * e.a * e.a)) / g2 : 0.0;
    }
    for (int a = 0; a < natoms; ++a) {
        const double x = pos[3 * a], y = pos[3 * a + 1], z = pos[3 * a + 2], qa = q[a];
        double tr, ti, dr, di;
        sincos(G0[0] * x + G0[1] * y + G0[2] * z, &ti, &tr);
        sincos(B2[0] * x + B2[1] * y + B2[2] * z, &di, &dr);
#pragma unroll
        for (int kk = 0; kk < EW_K; ++kk) {
            sr[kk] += qa * tr;
            si[kk] += qa * ti;
            const double t2 = tr * dr - ti * di;
            ti = tr * di + ti * dr;
            tr = t2;
        }
    }
#pragma unroll
    for (int kk = 0; kk < EW_K; ++kk) {
        if (kk >= cnt) continue;
        const long long t = (long long)row * w2 + k0 + kk;
        sf[2 * t] = on[kk] ? sr[kk] : 0.0;
        sf[2 * t + 1] = on[kk] ? si[kk] : 0.0;
    }
}

// One block per atom i: real-space pairs (j, image) with r < rcut, and the
// reciprocal sum over G of Re/Im[exp(i G.R_i) conj S(G)] w(G), a thread
// taking whole (i, j) rows of the box with the phase advanced along k (G is
// linear along a row, so the force needs two running sums per row).
__global__ __launch_bounds__(NT) void k_ewald_atoms(EwaldGeom e, int natoms, const double *pos,
                                                    const double *q, const double *sf,
                                                    double *e_atom, double *f)
{
    __shared__ double red[4 * NT / 64];
    const int i = blockIdx.x, tid = threadIdx.x;
    const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2], qi = q[i];
    const double a = e.a;
    const double two_a_sqrtpi = 2.0 * a / sqrt(PI_D);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};   // energy, fx, fy, fz
    // real space: for atom j the displacement d = R_i - R_j has fractional
    // coordinates f_c = b_c.d / 2 pi; an image d - sum_c n_c a_c lies within
    // rcut only if |f_c - n_c| <= rcut |b_c| / 2 pi, so each j visits the
    // few n in those ranges (inside e.nmax) instead of the whole image box
    const double rcut = sqrt(e.rcut2);
    double rcf[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        rcf[c] = rcut * sqrt(e.b[c][0] * e.b[c][0] + e.b[c][1] * e.b[c][1] + e.b[c][2] * e.b[c][2]) /
                 (2.0 * PI_D);
    for (int j = tid; j < natoms; j += NT) {
        const double d0x = xi - pos[3 * j], d0y = yi - pos[3 * j + 1], d0z = zi - pos[3 * j + 2];
        int lo[3], hi[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double fc = (e.b[c][0] * d0x + e.b[c][1] * d0y + e.b[c][2] * d0z) / (2.0 * PI_D);
            lo[c] = max((int)ceil(fc - rcf[c]), -e.nmax[c]);
            hi[c] = min((int)floor(fc + rcf[c]), e.nmax[c]);
        }
        const double qq = qi * q[j];
        for (int ii = lo[0]; ii <= hi[0]; ++ii)
            for (int jj = lo[1]; jj <= hi[1]; ++jj)
                for (int kk = lo[2]; kk <= hi[2]; ++kk) {
                    const double dx = d0x - (ii * e.lat[0][0] + jj * e.lat[1][0] + kk * e.lat[2][0]);
                    const double dy = d0y - (ii * e.lat[0][1] + jj * e.lat[1][1] + kk * e.lat[2][1]);
                    const double dz = d0z - (ii * e.lat[0][2] + jj * e.lat[1][2] + kk * e.lat[2][2]);
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 < 1e-20 || r2 > e.rcut2) continue;
                    const double r = sqrt(r2);
                    const double ec = erfc(a * r);
                    acc[0] += 0.5 * qq * ec / r;
                    const double mag = qq * (ec / r2 + two_a_sqrtpi * exp(-a * a * r2) / r) / r;
                    acc[1] += mag * dx;
                    acc[2] += mag * dy;
                    acc[3] += mag * dz;
                }
    }
    const int g0 = 2 * e.gmax[0] + 1, g1 = 2 * e.gmax[1] + 1, g2w = 2 * e.gmax[2] + 1;
    const long long nbox = ewald_gbox_count(e);
    const double pre = 2.0 * PI_D / e.volume;
    const double *wg = sf + 2 * nbox;
    double dr, di;   // exp(i b_2.R_i)
    sincos(e.b[2][0] * xi + e.b[2][1] * yi + e.b[2][2] * zi, &di, &dr);
    for (int row = tid; row < g0 * g1; row += NT) {
        const int gi = row / g1 - e.gmax[0], gj = row % g1 - e.gmax[1];
        double Gs[3];
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Gs[c] = gi * e.b[0][c] + gj * e.b[1][c] - e.gmax[2] * e.b[2][c];
        double tr, ti;
        sincos(Gs[0] * xi + Gs[1] * yi + Gs[2] * zi, &ti, &tr);
        double en = 0.0, f0 = 0.0, f1 = 0.0;
        const long long t0 = (long long)row * g2w;
        for (int k = 0; k < g2w; ++k) {
            const double w = wg[t0 + k];
            const double sr = sf[2 * (t0 + k)], si = sf[2 * (t0 + k) + 1];
            en += w * (tr * sr + ti * si);
            const double fm = w * (ti * sr - tr * si);
            f0 += fm;
            f1 += (double)k * fm;
            const double t2 = tr * dr - ti * di;
            ti = tr * di + ti * dr;
            tr = t2;
        }
        acc[0] += pre * qi * en;
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[1 + c] += 2.0 * pre * qi * (Gs[c] * f0 + e.b[2][c] * f1);
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
    const long long nseg = (long long)(2 * e.gmax[0] + 1) * (2 * e.gmax[1] + 1) *
                           ((2 * e.gmax[2] + 1 + EW_K - 1) / EW_K);
    hipLaunchKernelGGL(k_ewald_sf, dim3((unsigned)((nseg + NT - 1) / NT)), dim3(NT), 0, s, e,
                       natoms, pos, q, sf);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_ewald_atoms, dim3(natoms), dim3(NT), 0, s, e, natoms, pos, q, sf, e_atom, f);
    return hipGetLastError();
}


// ---------------------------------------------------------------- large cells
// Tiled direct sum of the structure factor for many atoms, without per-atom
// phase tables: a block owns SF_TM1 x SF_TM2 half-spectrum points of one
// axis-0 plane and walks the atoms (species-sorted fractional coordinates)
// in chunks staged in LDS.  For each atom the chunk stage holds
//   p[r] = exp(-2 pi i (m0 s0 + m1_r s1))  for the block's SF_TM1 rows,
//   e[q] = exp(-2 pi i m2_q s2)            for the first point of each group,
//   w    = exp(-2 pi i s2)                 (the step along k2),
// and a thread accumulates S(G) = sum_a p e w^j for its 2 rows x 4 points,
// FP64 throughout.  The output is v_ext(G) = (1/V) sum_s v_s(|G|) S_s(G) and,
// per block, the Ewald reciprocal-space energy sum_G c(k2) E(G) |sum_s Z_s S_s|^2
// over G^2 <= gcut2 with E(G) = exp(-G^2 / 4a^2) / G^2.
constexpr int SF_NT = 256;
constexpr int SF_TG = 16;              // groups of 4 consecutive k2 per row
constexpr int SF_TM2 = 4 * SF_TG;      // 64 points along k2
constexpr int SF_TM1 = 2 * (SF_NT / SF_TG);   // 32 rows (two per thread)
constexpr int SF_CH = 32;              // atoms per LDS chunk

__device__ __forceinline__ double frac_phase(int m, double s)
{
    double x = (double)m * s;
    return x - rint(x);
}

// one atom's contribution to the thread's 2 x 4 points; NYQ: one of the
// four is the Nyquist plane k2 = n2/2, whose m2 = -n2/2 makes its phase the
// conjugate of the recurrence's
template <bool NYQ>
__device__ __forceinline__ void sf_accumulate(double (&sr)[2][4], double (&si)[2][4], double2 p0,
                                              double2 p1, double2 e, double2 w, const double *nyq)
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const double ex = e.x, ey = NYQ ? nyq[k] * e.y : e.y;
        sr[0][k] = fma(p0.x, ex, fma(-p0.y, ey, sr[0][k]));
        si[0][k] = fma(p0.x, ey, fma(p0.y, ex, si[0][k]));
        sr[1][k] = fma(p1.x, ex, fma(-p1.y, ey, sr[1][k]));
        si[1][k] = fma(p1.x, ey, fma(p1.y, ex, si[1][k]));
        if (k < 3) e = {fma(e.x, w.x, -e.y * w.y), fma(e.x, w.y, e.y * w.x)};
    }
}

template <typename T>
__global__ __launch_bounds__(SF_NT, 4) void k_sf_tiled(Geom g, const int *spec_off, int nspecies,
                                                    const double *frac, const double *Z,
                                                    const double *rc, double inv_vol,
                                                    double ew_a, double ew_gcut2, cpx<T> *vext,
                                                    double2 *qbuf, double *ew_part)
{
    __shared__ double2 sp[SF_CH][SF_TM1];
    __shared__ double2 se[SF_CH][SF_TG];
    __shared__ double2 sw[SF_CH];
    __shared__ double red[SF_NT / 64];
    const int tid = threadIdx.x;
    const int ntx = (g.n2h + SF_TM2 - 1) / SF_TM2;
    const int nty = (g.n1 + SF_TM1 - 1) / SF_TM1;
    const long long blk = blockIdx.x;
    const int tx = (int)(blk % ntx);
    const int ty = (int)((blk / ntx) % nty);
    const int i0 = (int)(blk / ((long long)ntx * nty));
    const int m0 = freq(i0, g.n0);
    const int r = tid / SF_TG, grp = tid % SF_TG;
    const int k2b = tx * SF_TM2 + 4 * grp;          // first k2 of this thread
    const bool tile_nyq = tx * SF_TM2 <= g.m && g.m < (tx + 1) * SF_TM2;   // block-uniform
    double nyq[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) nyq[k] = (k2b + k == g.m) ? -1.0 : 1.0;

    double ew = 0.0;
    for (int sidx = 0; sidx < nspecies; ++sidx) {
        double sr[2][4] = {}, si[2][4] = {};
        const int a_beg = spec_off[sidx], a_end = spec_off[sidx + 1];
        for (int c0 = a_beg; c0 < a_end; c0 += SF_CH) {
            const int nc = min(SF_CH, a_end - c0);
            __syncthreads();
            // stage the chunk: row phases, group starts and k2 steps
            for (int e = tid; e < SF_CH * SF_TM1; e += SF_NT) {
                const int a = e / SF_TM1, rr = e % SF_TM1;
                double2 v = {0.0, 0.0};
                const int i1 = ty * SF_TM1 + rr;
                if (a < nc && i1 < g.n1) {
                    const double *f = frac + 3 * (long long)(c0 + a);
                    const double x = frac_phase(m0, f[0]) + frac_phase(freq(i1, g.n1), f[1]);
                    sincospi(-2.0 * x, &v.y, &v.x);
                }
                sp[a][rr] = v;
            }
            for (int e = tid; e < SF_CH * SF_TG; e += SF_NT) {
                const int a = e / SF_TG, q = e % SF_TG;
                double2 v = {0.0, 0.0};
                if (a < nc) {
                    const double s2 = frac[3 * (long long)(c0 + a) + 2];
                    sincospi(-2.0 * frac_phase(tx * SF_TM2 + 4 * q, s2), &v.y, &v.x);
                }
                se[a][q] = v;
            }
            if (tid < SF_CH) {
                double2 v = {0.0, 0.0};
                if (tid < nc) sincospi(-2.0 * frac[3 * (long long)(c0 + tid) + 2], &v.y, &v.x);
                sw[tid] = v;
            }
            __syncthreads();
            if (tile_nyq) {
#pragma unroll 2
                for (int a = 0; a < nc; ++a)
                    sf_accumulate<true>(sr, si, sp[a][r], sp[a][r + SF_TM1 / 2], se[a][grp], sw[a],
                                        nyq);
            } else {
#pragma unroll 2
                for (int a = 0; a < nc; ++a)
                    sf_accumulate<false>(sr, si, sp[a][r], sp[a][r + SF_TM1 / 2], se[a][grp],
                                         sw[a], nyq);
            }
        }
        // this species' share of v_ext(G), and of the ionic charge's S(G)
        const double z = Z[sidx], rcs = rc[sidx];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i1 = ty * SF_TM1 + r + h * (SF_TM1 / 2);
            if (i1 >= g.n1) continue;
            const int m1 = freq(i1, g.n1);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int k2 = k2b + k;
                if (k2 >= g.n2h) continue;
                const int m2 = (k2 == g.m) ? -g.m : k2;
                const double G2 = gvec2<double>(g, m0, m1, m2);
                const double vs = G2 > 0.0 ? -4.0 * PI_D * z * exp(-G2 * rcs * rcs * 0.25) / G2
                                           : PI_D * z * rcs * rcs;
                cpx<T> *dst = vext + ((long long)i0 * g.n1 + i1) * g.n2h + k2;
                double vr = vs * sr[h][k] * inv_vol, vi = vs * si[h][k] * inv_vol;
                if (sidx > 0) {
                    vr += (double)dst->x;
                    vi += (double)dst->y;
                }
                *dst = {T(vr), T(vi)};
                // ionic charge structure factor sum_s Z_s S_s: carried in qbuf
                // between species, its Ewald term taken after the last one
                const long long e = ((long long)i0 * g.n1 + i1) * g.n2h + k2;
                double qr = z * sr[h][k], qi = z * si[h][k];
                if (sidx > 0) {
                    qr += qbuf[e].x;
                    qi += qbuf[e].y;
                }
                if (sidx + 1 < nspecies) {
                    qbuf[e] = {qr, qi};
                } else if (G2 > 0.0 && G2 <= ew_gcut2) {
                    const double c = (k2 == 0 || k2 == g.m) ? 1.0 : 2.0;
                    ew += c * exp(-G2 / (4.0 * ew_a * ew_a)) / G2 * (qr * qr + qi * qi);
                }
            }
        }
    }
    ew = block_sum<SF_NT>(ew, red, tid);
    if (tid == 0 && ew_part) ew_part[blk] = ew;
}

long long sf_tiled_blocks(const Geom &g)
{
    return (long long)g.n0 * ((g.n1 + SF_TM1 - 1) / SF_TM1) * ((g.n2h + SF_TM2 - 1) / SF_TM2);
}

template <typename T>
hipError_t launch_sf_tiled(const Geom &g, const int *spec_off, int nspecies, const double *frac,
                           const double *Z, const double *rc, double volume, double ew_a,
                           double ew_gcut2, void *vext, void *qbuf, double *ew_part,
                           hipStream_t s)
{
    if (nspecies > 1 && !qbuf) return hipErrorInvalidValue;
    const long long nb = sf_tiled_blocks(g);
    hipLaunchKernelGGL((k_sf_tiled<T>), dim3((unsigned)nb), dim3(SF_NT), 0, s, g, spec_off,
                       nspecies, frac, Z, rc, 1.0 / volume, ew_a, ew_gcut2, (cpx<T> *)vext,
                       (double2 *)qbuf, ew_part);
    return hipGetLastError();
}
template hipError_t launch_sf_tiled<float>(const Geom &, const int *, int, const double *,
                                           const double *, const double *, double, double, double,
                                           void *, void *, double *, hipStream_t);
template hipError_t launch_sf_tiled<double>(const Geom &, const int *, int, const double *,
                                            const double *, const double *, double, double, double,
                                            void *, void *, double *, hipStream_t);

// Real-space Ewald sum over a cell list: the cell is cut into nc[d] >= 3 bins
// per lattice direction, each at least rcut wide across; atom i (thread)
// visits the 27 neighbouring bins with the lattice translation that wrapping
// implies, and sums 1/2 q_i q_j erfc(a r)/r over r < rcut.  Atoms are stored
// bin-sorted (pos, q in that order); e_atom[i] is written in that order.
__global__ __launch_bounds__(NT) void k_ewald_real_cells(EwaldGeom e, int natoms, const double *pos,
                                                         const double *q, const int *bin_start,
                                                         const int *bin_of, int nc0, int nc1,
                                                         int nc2, double *e_atom)
{
    const int i = blockIdx.x * NT + threadIdx.x;
    if (i >= natoms) return;
    const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2], qi = q[i];
    const int bi = bin_of[i];
    const int c2 = bi % nc2, c1 = (bi / nc2) % nc1, c0 = bi / (nc1 * nc2);
    const double a = e.a;
    double acc = 0.0;
    for (int d0 = -1; d0 <= 1; ++d0)
        for (int d1 = -1; d1 <= 1; ++d1)
            for (int d2 = -1; d2 <= 1; ++d2) {
                int b0 = c0 + d0, b1 = c1 + d1, b2 = c2 + d2;
                // the image of the bin: wrap and note the lattice shift
                const int s0 = b0 < 0 ? -1 : (b0 >= nc0 ? 1 : 0);
                const int s1 = b1 < 0 ? -1 : (b1 >= nc1 ? 1 : 0);
                const int s2 = b2 < 0 ? -1 : (b2 >= nc2 ? 1 : 0);
                b0 -= s0 * nc0;
                b1 -= s1 * nc1;
                b2 -= s2 * nc2;
                const double tx = s0 * e.lat[0][0] + s1 * e.lat[1][0] + s2 * e.lat[2][0];
                const double ty = s0 * e.lat[0][1] + s1 * e.lat[1][1] + s2 * e.lat[2][1];
                const double tz = s0 * e.lat[0][2] + s1 * e.lat[1][2] + s2 * e.lat[2][2];
                const int bin = (b0 * nc1 + b1) * nc2 + b2;
                for (int j = bin_start[bin]; j < bin_start[bin + 1]; ++j) {
                    const double dx = xi - pos[3 * j] - tx;
                    const double dy = yi - pos[3 * j + 1] - ty;
                    const double dz = zi - pos[3 * j + 2] - tz;
                    const double r2 = dx * dx + dy * dy + dz * dz;
                    if (r2 < 1e-20 || r2 > e.rcut2) continue;
                    const double rr = sqrt(r2);
                    acc += 0.5 * qi * q[j] * erfc(a * rr) / rr;
                }
            }
    e_atom[i] = acc;
}

hipError_t launch_ewald_real_cells(const EwaldGeom &e, int natoms, const double *pos,
                                   const double *q, const int *bin_start, const int *bin_of,
                                   const int nc[3], double *e_atom, hipStream_t s)
{
    if (natoms <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ewald_real_cells, dim3((natoms + NT - 1) / NT), dim3(NT), 0, s, e, natoms,
                       pos, q, bin_start, bin_of, nc[0], nc[1], nc[2], e_atom);
    return hipGetLastError();
}

}  // namespace ofdft
