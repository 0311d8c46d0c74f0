// Device-side FFT building blocks for gfx950: radix-2/3/4/6/8/12/16 butterflies
// in registers and Stockham autosort stages on pencils staged in LDS.
//
// Every reciprocal-space term of the orbital-free energy (Hartree, the
// von Weizsaecker Laplacian, the nonlocal kernels of eqs. "nl2"/"WT" and the
// per-knot convolutions of step s3) is a 3D FFT round trip; the paper runs
// them through FFTW on one CPU core.  Here a workgroup of NT threads loads P
// pencils of length L into LDS, runs log_R(L) Stockham stages in place
// (all loads of a stage are held in registers across a barrier before the
// stores), and writes them back.  L and the radix sequence are compile-time
// so every index is a constant-divisor operation.
//
// Forward transforms use exp(-2 pi i nk/L), inverse exp(+2 pi i nk/L); no
// scaling is applied.  Twiddles W_L^n come from a table built in FP64 on the
// host and rounded to the field type.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>

namespace ofdft {

// A workgroup barrier for data exchanged through LDS: the wave's LDS
// operations complete (s_waitcnt lgkmcnt(0)) before the barrier, and the
// empty asm statements with a memory clobber keep the compiler from moving
// memory accesses across it.  Global loads, stores and asynchronous LDS
// copies in flight are not waited for (__syncthreads, whose workgroup fence
// also covers global memory and LDS copies, would wait for them).  Every
// barrier of the transforms below exchanges data through LDS alone.
constexpr int WAIT_LGKM0 = 0xC07F;   // s_waitcnt lgkmcnt(0), other counters at their maximum
__device__ __forceinline__ void lds_sync()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

template <typename T>
struct cpx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <typename T, bool INV>
__device__ __forceinline__ cpx<T> mul_mi(cpx<T> a)
{
    if constexpr (INV) return {-a.y, a.x};
    else return {a.y, -a.x};
}

// ---------------------------------------------------------------- plans
struct Plan {
    int n;
    int r[16];
};

// Radices for a length-L transform: the fewest Stockham stages (each stage is
// an LDS round trip and a barrier) over the register butterflies 16, 12, 8,
// 6, 4, 3, 2; among those, the largest smallest radix (4*4 rather than 8*2);
// then larger radices first.  Score = stages * 16 - smallest radix.
// Radix 16 holds 32 values per butterfly: used for FP32 only (in FP64 its
// register footprint costs more than the saved stage).
constexpr int plan_score(int L, int minr, bool r16)
{
    if (L == 1) return -minr;
    int best = 1 << 20;
    const int rs[7] = {16, 12, 8, 6, 4, 3, 2};
    for (int i = r16 ? 0 : 1; i < 7; ++i)
        if (L % rs[i] == 0) {
            const int s = 16 + plan_score(L / rs[i], rs[i] < minr ? rs[i] : minr, r16);
            if (s < best) best = s;
        }
    return best;
}

constexpr Plan make_plan(int L, bool r16 = false)
{
    Plan p{0, {}};
    int m = L, minr = 64;
    const int rs[7] = {16, 12, 8, 6, 4, 3, 2};
    while (m > 1) {
        const int need = plan_score(m, minr, r16);
        int pick = 0;
        for (int i = r16 ? 0 : 1; i < 7 && !pick; ++i)
            if (m % rs[i] == 0 &&
                16 + plan_score(m / rs[i], rs[i] < minr ? rs[i] : minr, r16) == need)
                pick = rs[i];
        if (!pick) break;
        p.r[p.n++] = pick;
        if (pick < minr) minr = pick;
        m /= pick;
    }
    return p;
}

// Plan variants, a choice of the autotuner: 0 is make_plan's order, 1 the
// same radices in reverse order (another Stockham factorisation of the same
// transform: different twiddle strides and LDS access patterns).
constexpr Plan plan_variant(int L, bool r16, int pv)
{
    Plan p = make_plan(L, r16);
    if (pv == 1)
        for (int i = 0; i < p.n / 2; ++i) {
            const int t = p.r[i];
            p.r[i] = p.r[p.n - 1 - i];
            p.r[p.n - 1 - i] = t;
        }
    return p;
}
// whether variant 1 differs from variant 0
constexpr bool plan_reversible(int L, bool r16)
{
    const Plan a = plan_variant(L, r16, 0), b = plan_variant(L, r16, 1);
    for (int i = 0; i < a.n; ++i)
        if (a.r[i] != b.r[i]) return true;
    return false;
}

constexpr bool plan_ok(int L)
{
    // only lengths made of 2s and 3s
    int m = L;
    while (m % 2 == 0) m /= 2;
    while (m % 3 == 0) m /= 3;
    return m == 1 && L >= 2;
}

// ---------------------------------------------------------------- butterflies
template <typename T, int R, bool INV>
__device__ __forceinline__ void dft(cpx<T> *a)
{
    if constexpr (R == 2) {
        cpx<T> t = a[0];
        a[0] = cadd(t, a[1]);
        a[1] = csub(t, a[1]);
    } else if constexpr (R == 3) {
        const T h = T(-0.5);
        const T s = INV ? T(0.86602540378443864676372317075294)
                        : T(-0.86602540378443864676372317075294);
        cpx<T> t = cadd(a[1], a[2]);
        cpx<T> d = csub(a[1], a[2]);
        cpx<T> m = {a[0].x + h * t.x, a[0].y + h * t.y};
        // s * i * d
        cpx<T> sd = {-s * d.y, s * d.x};
        a[0] = cadd(a[0], t);
        a[1] = cadd(m, sd);
        a[2] = csub(m, sd);
    } else if constexpr (R == 4) {
        cpx<T> t0 = cadd(a[0], a[2]);
        cpx<T> t1 = csub(a[0], a[2]);
        cpx<T> t2 = cadd(a[1], a[3]);
        cpx<T> t3 = mul_mi<T, INV>(csub(a[1], a[3]));
        a[0] = cadd(t0, t2);
        a[2] = csub(t0, t2);
        a[1] = cadd(t1, t3);
        a[3] = csub(t1, t3);
    } else if constexpr (R == 6) {
        // prime-factor algorithm, 6 = 2 x 3: no internal twiddles.
        // input n = (3 n1 + 2 n2) mod 6, output k = (3 k1 + 4 k2) mod 6
        cpx<T> y[3][2];
#pragma unroll
        for (int n2 = 0; n2 < 3; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 2; ++n1) y[n2][n1] = a[(3 * n1 + 2 * n2) % 6];
            dft<T, 2, INV>(y[n2]);
        }
#pragma unroll
        for (int k1 = 0; k1 < 2; ++k1) {
            cpx<T> z[3] = {y[0][k1], y[1][k1], y[2][k1]};
            dft<T, 3, INV>(z);
#pragma unroll
            for (int k2 = 0; k2 < 3; ++k2) a[(3 * k1 + 4 * k2) % 6] = z[k2];
        }
    } else if constexpr (R == 12) {
        // prime-factor algorithm, 12 = 4 x 3: no internal twiddles.
        // input n = (3 n1 + 4 n2) mod 12, output k = (9 k1 + 4 k2) mod 12
        cpx<T> y[3][4];
#pragma unroll
        for (int n2 = 0; n2 < 3; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) y[n2][n1] = a[(3 * n1 + 4 * n2) % 12];
            dft<T, 4, INV>(y[n2]);
        }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            cpx<T> z[3] = {y[0][k1], y[1][k1], y[2][k1]};
            dft<T, 3, INV>(z);
#pragma unroll
            for (int k2 = 0; k2 < 3; ++k2) a[(9 * k1 + 4 * k2) % 12] = z[k2];
        }
    } else if constexpr (R == 16) {
        // 16 = 4 x 4 Cooley-Tukey: DFT4 over n1 of x[4 n1 + n2], the twiddle
        // W16^(n2 k1), DFT4 over n2; output k = k1 + 4 k2
        constexpr double C1 = 0.92387953251128675613;   // cos(pi/8)
        constexpr double S1 = 0.38268343236508977173;   // sin(pi/8)
        constexpr double R2 = 0.70710678118654752440;
        cpx<T> y[4][4];
#pragma unroll
        for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
            for (int n1 = 0; n1 < 4; ++n1) y[n2][n1] = a[4 * n1 + n2];
            dft<T, 4, INV>(y[n2]);
        }
#pragma unroll
        for (int n2 = 1; n2 < 4; ++n2)
#pragma unroll
            for (int k1 = 1; k1 < 4; ++k1) {
                const int m = n2 * k1;   // 1..9
                // W16^m = cos(2 pi m/16) -/+ i sin(2 pi m/16)
                const double cr = m == 1 ? C1 : m == 2 ? R2 : m == 3 ? S1 : m == 4 ? 0.0
                                : m == 6 ? -R2 : m == 9 ? -C1 : 0.0;
                const double si = m == 1 ? S1 : m == 2 ? R2 : m == 3 ? C1 : m == 4 ? 1.0
                                : m == 6 ? R2 : m == 9 ? -S1 : 0.0;
                if (m == 4) {
                    y[n2][k1] = mul_mi<T, INV>(y[n2][k1]);
                } else {
                    const cpx<T> w = {T(cr), INV ? T(si) : T(-si)};
                    y[n2][k1] = cmul(y[n2][k1], w);
                }
            }
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            cpx<T> z[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
            dft<T, 4, INV>(z);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = z[k2];
        }
    } else if constexpr (R == 8) {
        const T r2 = T(0.70710678118654752440084436210485);
        cpx<T> e[4] = {a[0], a[2], a[4], a[6]};
        cpx<T> o[4] = {a[1], a[3], a[5], a[7]};
        dft<T, 4, INV>(e);
        dft<T, 4, INV>(o);
        // o[k] *= W8^k (forward W8 = (1 - i)/sqrt2, inverse conjugate)
        cpx<T> o1, o3;
        if constexpr (INV) {
            o1 = {r2 * (o[1].x - o[1].y), r2 * (o[1].x + o[1].y)};
            o3 = {-r2 * (o[3].x + o[3].y), r2 * (o[3].x - o[3].y)};
        } else {
            o1 = {r2 * (o[1].x + o[1].y), r2 * (o[1].y - o[1].x)};
            o3 = {r2 * (o[3].y - o[3].x), -r2 * (o[3].x + o[3].y)};
        }
        cpx<T> o2 = mul_mi<T, INV>(o[2]);
        a[0] = cadd(e[0], o[0]);
        a[4] = csub(e[0], o[0]);
        a[1] = cadd(e[1], o1);
        a[5] = csub(e[1], o1);
        a[2] = cadd(e[2], o2);
        a[6] = csub(e[2], o2);
        a[3] = cadd(e[3], o3);
        a[7] = csub(e[3], o3);
    }
}

// ---------------------------------------------------------------- LDS layout
// Element n of pencil p lives at buf[n * ES + p * PS]; butterflies are
// assigned pencil-fastest.  Column kernels use ES = P, PS = 1 (a tile of P
// adjacent columns); row kernels use ES = P + 1, PS = 1 so that the
// row-ordered global loads, which walk n across lanes, also hit distinct
// banks.  The plane kernels keep one padded buffer with odd A and run their
// row transforms with (ES, PS) = (A, 1) and their column transforms with
// (1, A): consecutive lanes then step by 1 or by the odd A, both free of bank
// conflicts, and no transpose is needed between the two axes.
template <int ES, int PS>
__device__ __forceinline__ int lidx(int n, int p)
{
    return n * ES + p * PS;
}

// One Stockham stage of radix R after NS points have been combined.
// Input element (j + r L/R) of every pencil is twiddled by W_{NS R}^{r (j mod NS)},
// transformed, and stored at (j / NS) NS R + (j mod NS) + s NS.
template <typename T, int L, int R, int NS, bool INV, int P, int NT, int ES, int PS>
__device__ __forceinline__ void stockham_stage(cpx<T> *buf, const cpx<T> *tw,
                                               int tid)
{
    constexpr int NBF = L / R;
    constexpr int TOT = NBF * P;
    constexpr int PER = (TOT + NT - 1) / NT;
    // an opaque copy of the thread index: the index arithmetic of this stage
    // is recomputed here instead of being hoisted out of callers' loops and
    // held in registers across the whole kernel
    asm volatile("" : "+v"(tid));
    // unsigned index arithmetic: divisions by the compile-time P and NS
    // become multiply-high and shifts without sign fix-ups
    const unsigned ut = (unsigned)tid;
    cpx<T> v[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const unsigned b = ut + (unsigned)(q * NT);
        if (TOT % NT == 0 || b < (unsigned)TOT) {
            const unsigned j = b / (unsigned)P;
            const unsigned p = b % (unsigned)P;
            const unsigned a0 = j * (unsigned)ES + p * (unsigned)PS;
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[a0 + (unsigned)(r * NBF * ES)];
        }
    }
    lds_sync();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const unsigned b = ut + (unsigned)(q * NT);
        if (TOT % NT == 0 || b < (unsigned)TOT) {
            const unsigned j = b / (unsigned)P;
            const unsigned p = b % (unsigned)P;
            const unsigned k = j % (unsigned)NS;
            if constexpr (NS > 1) {
                constexpr int STEP = L / (NS * R);
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cpx<T> w = tw[k * (unsigned)(r * STEP)];
                    if constexpr (INV) w.y = -w.y;
                    v[q][r] = cmul(v[q][r], w);
                }
            }
            dft<T, R, INV>(v[q]);
            const unsigned a0 = ((j / (unsigned)NS) * (unsigned)(NS * R) + k) * (unsigned)ES +
                                p * (unsigned)PS;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[a0 + (unsigned)(r * NS * ES)] = v[q][r];
        }
    }
    lds_sync();
}

// The first stage of a transform with its inputs taken from src(n, p)
// (element n of pencil p, read from memory or computed) instead of LDS; the
// outputs go to buf as in stockham_stage.  NS = 1: no twiddles.
// A source src(n, p) takes element n of pencil p.  A source that also takes
// three arguments is called as src(nb, dn, p) with n = nb + dn, where dn is
// the same for every lane (a constant of the unrolled loops): it can form
// one per-lane offset from nb and hand dn to the scalar part of the address.
// Destinations likewise: dst(n, p, v), or dst(nb, dn, p, v).
template <class SRC>
constexpr bool src_split() { return std::is_invocable_v<const SRC &, unsigned, unsigned, unsigned>; }
template <class DST, typename T>
constexpr bool dst_split()
{
    return std::is_invocable_v<const DST &, unsigned, unsigned, unsigned, cpx<T>>;
}

template <typename T, int L, int R, bool INV, int P, int NT, int ES, int PS, class SRC>
__device__ __forceinline__ void stockham_stage_src(cpx<T> *buf, int tid, const SRC &src)
{
    constexpr int NBF = L / R;
    constexpr int TOT = NBF * P;
    constexpr int PER = (TOT + NT - 1) / NT;
    // with NT a multiple of P a lane keeps its pencil across q and its
    // element index moves by the constant q NT / P
    constexpr bool EVEN = NT % P == 0;
    asm volatile("" : "+v"(tid));
    const unsigned ut = (unsigned)tid;
    cpx<T> v[PER][R];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const unsigned b = ut + (unsigned)(q * NT);
        if (TOT % NT == 0 || b < (unsigned)TOT) {
            const unsigned j = b / (unsigned)P;
            const unsigned p = b % (unsigned)P;
            if constexpr (src_split<SRC>()) {
                const unsigned jb = EVEN ? ut / (unsigned)P : j;
                const unsigned pb = EVEN ? ut % (unsigned)P : p;
                const unsigned DQ = EVEN ? (unsigned)(q * (NT / P)) : 0u;
#pragma unroll
                for (int r = 0; r < R; ++r) v[q][r] = src(jb, DQ + (unsigned)(r * NBF), pb);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) v[q][r] = src(j + (unsigned)(r * NBF), p);
            }
        }
    }
    lds_sync();
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const unsigned b = ut + (unsigned)(q * NT);
        if (TOT % NT == 0 || b < (unsigned)TOT) {
            const unsigned j = b / (unsigned)P;
            const unsigned p = b % (unsigned)P;
            dft<T, R, INV>(v[q]);
            const unsigned a0 = j * (unsigned)(R * ES) + p * (unsigned)PS;
#pragma unroll
            for (int r = 0; r < R; ++r) buf[a0 + (unsigned)(r * ES)] = v[q][r];
        }
    }
    lds_sync();
}

// The last stage of a transform (NS R = L) with its outputs handed to
// dst(n, p, value) instead of LDS.
template <typename T, int L, int R, int NS, bool INV, int P, int NT, int ES, int PS, class DST>
__device__ __forceinline__ void stockham_stage_dst(const cpx<T> *buf, const cpx<T> *tw, int tid,
                                                   const DST &dst)
{
    static_assert(NS * R == L, "the last stage");
    constexpr int NBF = L / R;
    constexpr int TOT = NBF * P;
    constexpr int PER = (TOT + NT - 1) / NT;
    asm volatile("" : "+v"(tid));
    const unsigned ut = (unsigned)tid;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const unsigned b = ut + (unsigned)(q * NT);
        if (TOT % NT == 0 || b < (unsigned)TOT) {
            const unsigned j = b / (unsigned)P;   // j < NS
            const unsigned p = b % (unsigned)P;
            const unsigned a0 = j * (unsigned)ES + p * (unsigned)PS;
            cpx<T> v[R];
#pragma unroll
            for (int r = 0; r < R; ++r) v[r] = buf[a0 + (unsigned)(r * NBF * ES)];
            if constexpr (NS > 1) {
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    cpx<T> w = tw[j * (unsigned)r];
                    if constexpr (INV) w.y = -w.y;
                    v[r] = cmul(v[r], w);
                }
            }
            dft<T, R, INV>(v);
            if constexpr (dst_split<DST, T>()) {
                constexpr bool EVEN = NT % P == 0;
                const unsigned jb = EVEN ? ut / (unsigned)P : j;
                const unsigned pb = EVEN ? ut % (unsigned)P : p;
                const unsigned DQ = EVEN ? (unsigned)(q * (NT / P)) : 0u;
#pragma unroll
                for (int r = 0; r < R; ++r) dst(jb, DQ + (unsigned)(r * NS), pb, v[r]);
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) dst(j + (unsigned)(r * NS), p, v[r]);
            }
        }
    }
    lds_sync();
}

template <typename T, int L, bool INV, int P, int NT, int ES, int PS, int S, int NS, int PV = 0>
__device__ __forceinline__ void fft_stages(cpx<T> *buf, const cpx<T> *tw, int tid)
{
    constexpr Plan pl = plan_variant(L, sizeof(T) == 4, PV);
    if constexpr (S < pl.n) {
        constexpr int R = pl.r[S];
        stockham_stage<T, L, R, NS, INV, P, NT, ES, PS>(buf, tw, tid);
        fft_stages<T, L, INV, P, NT, ES, PS, S + 1, NS * R, PV>(buf, tw, tid);
    }
}

// Transform P pencils of length L held in LDS (buf[n * ES + p * PS]), in
// place.  Caller must lds_sync() after filling buf; returns after a
// barrier.
template <typename T, int L, bool INV, int P, int NT, int ES, int PS = 1, int PV = 0>
__device__ __forceinline__ void lds_fft(cpx<T> *buf, const cpx<T> *tw, int tid)
{
    static_assert(plan_ok(L), "FFT length must be 2^a 3^b");
    fft_stages<T, L, INV, P, NT, ES, PS, 0, 1, PV>(buf, tw, tid);
}

// As lds_fft, with the first stage reading element n of pencil p from
// src(n, p) instead of buf (which need not be filled: the call starts with a
// barrier so that earlier readers of buf are done).  Returns after a barrier.
template <typename T, int L, bool INV, int P, int NT, int ES, int PS, int PV = 0, class SRC>
__device__ __forceinline__ void lds_fft_src(cpx<T> *buf, const cpx<T> *tw, int tid, const SRC &src)
{
    static_assert(plan_ok(L), "FFT length must be 2^a 3^b");
    constexpr Plan pl = plan_variant(L, sizeof(T) == 4, PV);
    lds_sync();
    stockham_stage_src<T, L, pl.r[0], INV, P, NT, ES, PS>(buf, tid, src);
    fft_stages<T, L, INV, P, NT, ES, PS, 1, pl.r[0], PV>(buf, tw, tid);
}

// As lds_fft, with the outputs of the last stage handed to dst(n, p, value)
// instead of being written back to buf.  Returns after a barrier.
template <typename T, int L, bool INV, int P, int NT, int ES, int PS, int S, int NS, int PV = 0,
          class DST>
__device__ __forceinline__ void fft_stages_dst(cpx<T> *buf, const cpx<T> *tw, int tid, const DST &dst)
{
    constexpr Plan pl = plan_variant(L, sizeof(T) == 4, PV);
    constexpr int R = pl.r[S];
    if constexpr (S + 1 < pl.n) {
        stockham_stage<T, L, R, NS, INV, P, NT, ES, PS>(buf, tw, tid);
        fft_stages_dst<T, L, INV, P, NT, ES, PS, S + 1, NS * R, PV>(buf, tw, tid, dst);
    } else {
        stockham_stage_dst<T, L, R, NS, INV, P, NT, ES, PS>(buf, tw, tid, dst);
    }
}

template <typename T, int L, bool INV, int P, int NT, int ES, int PS, int PV = 0, class DST>
__device__ __forceinline__ void lds_fft_dst(cpx<T> *buf, const cpx<T> *tw, int tid, const DST &dst)
{
    static_assert(plan_ok(L), "FFT length must be 2^a 3^b");
    fft_stages_dst<T, L, INV, P, NT, ES, PS, 0, 1, PV>(buf, tw, tid, dst);
}

// As lds_fft with both ends outside buf: the first stage reads src(n, p),
// the last stage hands its outputs to dst(n, p, value) (a single-stage
// transform writes buf and then hands every element to dst).  Starts and
// returns with a barrier.
template <typename T, int L, bool INV, int P, int NT, int ES, int PS, int PV = 0, class SRC,
          class DST>
__device__ __forceinline__ void lds_fft_io(cpx<T> *buf, const cpx<T> *tw, int tid, const SRC &src,
                                           const DST &dst)
{
    static_assert(plan_ok(L), "FFT length must be 2^a 3^b");
    constexpr Plan pl = plan_variant(L, sizeof(T) == 4, PV);
    lds_sync();
    stockham_stage_src<T, L, pl.r[0], INV, P, NT, ES, PS>(buf, tid, src);
    if constexpr (pl.n >= 2) {
        fft_stages_dst<T, L, INV, P, NT, ES, PS, 1, pl.r[0], PV>(buf, tw, tid, dst);
    } else {
        for (unsigned o = (unsigned)tid; o < (unsigned)(L * P); o += NT) {
            const unsigned n = o / (unsigned)P, p = o % (unsigned)P;
            if constexpr (dst_split<DST, T>()) dst(n, 0u, p, buf[n * ES + p * PS]);
            else dst(n, p, buf[n * ES + p * PS]);
        }
        lds_sync();
    }
}

// ---------------------------------------------------------------- reductions
// One DPP move of a double (both 32-bit halves with the same control);
// lanes without a source, and rows outside ROWM, read +0.
template <int CTRL, int ROWM>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)bits, CTRL, ROWM, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, ROWM, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum of v over the 64 lanes of a wave, valid in lane 63, in a fixed order:
// running sums over 2, 4, 8 and 16 lanes inside each row of 16 (row_shr),
// then row 0's total added to row 1 and row 2's to row 3 (row_bcast:15),
// then the total of rows 0-1 added to rows 2-3 (row_bcast:31).
__device__ __forceinline__ double wave_sum_to_last(double v)
{
    v += dpp_f64<0x111, 0xf>(v);
    v += dpp_f64<0x112, 0xf>(v);
    v += dpp_f64<0x114, 0xf>(v);
    v += dpp_f64<0x118, 0xf>(v);
    v += dpp_f64<0x142, 0xa>(v);
    v += dpp_f64<0x143, 0xc>(v);
    return v;
}

// Deterministic workgroup sums of K doubles per thread: a fixed DPP tree
// inside each 64-lane wave, then the per-wave results added in wave order by
// thread 0.  The sums are valid in thread 0 only.  red must hold K * NT / 64
// doubles; the call ends with a barrier so red can be reused.
template <int NT, int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double *red, int tid)
{
    static_assert(NT % 64 == 0, "whole waves");
    constexpr int NW = NT / 64;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum_to_last(v[k]);
    if ((tid & 63) == 63) {
#pragma unroll
        for (int k = 0; k < K; ++k) red[k * NW + (tid >> 6)] = v[k];
    }
    lds_sync();
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
#pragma unroll
            for (int w = 0; w < NW; ++w) s += red[k * NW + w];
            v[k] = s;
        }
    }
    lds_sync();
}

// As block_sums, through LDS, for blocks with a free LDS area of K * NT
// doubles (lds; the caller's reads of it must be complete, which the first
// barrier here ensures): every thread stores its K values, then wave k adds
// the NT values of quantity k (each lane NT / 64 of them, in wave order) and
// reduces them with the DPP tree.  Valid in thread 0 only; red holds K
// doubles and is read by thread 0 before any later barrier.
template <int NT, int K>
__device__ __forceinline__ void block_sums_lds(double (&v)[K], double *lds, double *red, int tid)
{
    static_assert(NT % 64 == 0 && K * 64 <= NT, "one wave per quantity");
    constexpr int NW = NT / 64;
    lds_sync();
#pragma unroll
    for (int k = 0; k < K; ++k) lds[k * NT + tid] = v[k];
    lds_sync();
    if (tid < K * 64) {
        const int k = tid >> 6, l = tid & 63;
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += lds[k * NT + w * 64 + l];
        s = wave_sum_to_last(s);
        if (l == 63) red[k] = s;
    }
    lds_sync();
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = red[k];
    }
}

// element i of an array at a block-uniform base, addressed by a 32-bit byte
// offset: the load or store then takes the base from scalar registers and one
// 32-bit offset per lane.  Only for bases whose elements used lie within
// 4 GiB of them (a plane of a field, not a whole field: a half spectrum of
// 1024^3 points in FP32 is 4.3 GB)
template <typename V>
__device__ __forceinline__ V ld32(const V *base, unsigned i)
{
    return *(const V *)((const char *)base + i * (unsigned)sizeof(V));
}
template <typename V>
__device__ __forceinline__ void st32(V *base, unsigned i, V v)
{
    *(V *)((char *)base + i * (unsigned)sizeof(V)) = v;
}

// Loads and stores through a buffer resource over a region of `bytes` bytes
// (under 4 GiB) at `base`: the address is base + soff + voff, with voff a
// 32-bit per-lane byte offset and soff a wave-uniform one, which the
// hardware takes from a scalar register, so that the constant strides
// between a lane's elements cost no vector instruction.  Callers keep every
// access inside the region.
struct BufRes {
    __amdgpu_buffer_rsrc_t r;
};
// word 3 of a gfx9 buffer resource: 32-bit data format, no swizzle
constexpr int BUF_RES_WORD3 = 0x00020000;
__device__ __forceinline__ BufRes buf_res(const void *base, unsigned bytes)
{
    return {__builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                              BUF_RES_WORD3)};
}
typedef unsigned buf_u32x2 __attribute__((vector_size(8)));
typedef unsigned buf_u32x4 __attribute__((vector_size(16)));
template <typename V>
__device__ __forceinline__ V bld(const BufRes &b, unsigned voff, unsigned soff)
{
    static_assert(sizeof(V) == 8 || sizeof(V) == 16, "8- or 16-byte elements");
    if constexpr (sizeof(V) == 8)
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(b.r, voff, soff, 0));
    else
        return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(b.r, voff, soff, 0));
}
// Stores of more than 8 bytes need a wait state before a vector instruction
// overwrites their data registers; for buffer stores the compiler does not
// always leave one (16-byte stores followed at once by a write of their
// first data registers were found in the FP64 kernels, and stored wrong low
// halves now and then), so a 16-byte element is stored as two 8-byte halves.
template <typename V>
__device__ __forceinline__ void bst(const BufRes &b, unsigned voff, unsigned soff, V v)
{
    static_assert(sizeof(V) == 8 || sizeof(V) == 16, "8- or 16-byte elements");
    if constexpr (sizeof(V) == 8) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(buf_u32x2, v), b.r, voff, soff, 0);
    } else {
        const buf_u32x4 w = __builtin_bit_cast(buf_u32x4, v);
        const buf_u32x2 lo = {w[0], w[1]}, hi = {w[2], w[3]};
        __builtin_amdgcn_raw_buffer_store_b64(lo, b.r, voff, soff, 0);
        // (keeps the two halves from being merged back into one store)
        asm volatile("" ::: "memory");
        __builtin_amdgcn_raw_buffer_store_b64(hi, b.r, voff + 8u, soff, 0);
    }
}

// Copy `bytes` (a multiple of 16; both addresses 16-byte aligned) from
// global memory straight into LDS, without registers: the waves of an
// NT-thread block take 1 KB chunks in turn, lane l of a wave moving the 16
// bytes at offset 16 l of its chunk (global_load_lds_dwordx4).  The copy is
// asynchronous: lds_copy_wait() and a barrier come before any read of dst.
template <int NT>
__device__ __forceinline__ void lds_copy_async(void *dst, const void *src, unsigned bytes, int tid)
{
    const unsigned w = (unsigned)tid / 64u, l = (unsigned)tid % 64u;
    const unsigned nchunk = (bytes + 1023u) / 1024u;
    for (unsigned c = w; c < nchunk; c += (unsigned)(NT / 64)) {
        const unsigned off = c * 1024u + l * 16u;
        if (off < bytes)
            __builtin_amdgcn_global_load_lds(
                (const char *)src + off,
                (__attribute__((address_space(3))) char *)((char *)dst + c * 1024u), 16, 0, 0);
    }
}
// waits for this wave's outstanding memory operations (the copies above)
__device__ __forceinline__ void lds_copy_wait() { __builtin_amdgcn_s_waitcnt(0); }

template <int NT>
__device__ __forceinline__ double block_sum(double x, double *red, int tid)
{
    double v[1] = {x};
    block_sums<NT, 1>(v, red, tid);
    return v[0];
}

}  // namespace ofdft
