/*
 * Oracle FFT: a plain, slow, obviously-correct FP64 discrete Fourier transform.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may link or call this
 * file; it exists so that the reference (oracle) implementation of the
 * orbital-free DFT energy has a Fourier transform of its own that shares no
 * code with the GPU path.
 *
 * The paper (Section "Leveraging existing techniques") uses FFTW for the 3D
 * transforms behind every reciprocal-space term.  This is an independent,
 * textbook recursive mixed-radix Cooley-Tukey transform:
 *
 *     X[k] = sum_{j=0}^{n-1} x[j] * exp(sign * 2 pi i j k / n)
 *
 * computed by splitting n = p * m with p the smallest prime factor of n,
 * transforming the p decimated subsequences recursively and recombining with
 * a direct length-p DFT.  Any n >= 1 is accepted; a prime n falls back to the
 * direct O(n^2) sum.  Twiddles are cos/sin of 2 pi (q k mod n) / n in FP64.
 * No normalisation is applied in either direction.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* w[j] = exp(sign * 2 pi i j / n), j = 0..n-1 */
static void twiddle_table(cplx *w, int n, int sign)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int j = 0; j < n; ++j) {
        double a = two_pi * (double)j / (double)n;
        w[j] = cos(a) + (double)sign * sin(a) * I;
    }
}

/*
 * Transform the n elements in[0], in[istride], ... into out[0..n-1].
 * w is the table of the top-level length ntop; W_n^e = w[e * (ntop / n)].
 */
static void dft_rec(const cplx *in, long istride, cplx *out, int n,
                    const cplx *w, int ntop, cplx *scratch)
{
    if (n == 1) {
        out[0] = in[0];
        return;
    }
    int p = smallest_factor(n);
    int m = n / p;
    int wstep = ntop / n;
    if (m == 1) {
        /* prime length: direct sum */
        for (int k = 0; k < n; ++k) {
            cplx acc = 0;
            for (int j = 0; j < n; ++j)
                acc += in[(long)j * istride] * w[(long)((long)j * k % n) * wstep];
            scratch[k] = acc;
        }
        memcpy(out, scratch, sizeof(cplx) * (size_t)n);
        return;
    }
    /* sub-transform q holds x[q], x[q+p], x[q+2p], ... */
    for (int q = 0; q < p; ++q)
        dft_rec(in + (long)q * istride, istride * p, out + (long)q * m, m, w, ntop,
                scratch);
    /* X[k + m s] = sum_q W_n^{q (k + m s)} Y_q[k] */
    for (int k = 0; k < m; ++k) {
        for (int s = 0; s < p; ++s) {
            int kk = k + m * s;
            cplx acc = 0;
            for (int q = 0; q < p; ++q)
                acc += out[(long)q * m + k] * w[(long)((long)q * kk % n) * wstep];
            scratch[kk] = acc;
        }
    }
    memcpy(out, scratch, sizeof(cplx) * (size_t)n);
}

/* In-place 1D transforms of `count` lines of length n; line c starts at
 * data + c * line_step and its elements are `stride` apart. */
static int fft_lines(cplx *data, int n, long stride, long count, long line_step,
                     int sign)
{
    cplx *w = malloc(sizeof(cplx) * (size_t)n);
    cplx *buf = malloc(sizeof(cplx) * (size_t)n);
    cplx *out = malloc(sizeof(cplx) * (size_t)n);
    cplx *scr = malloc(sizeof(cplx) * (size_t)n);
    if (!w || !buf || !out || !scr) {
        free(w); free(buf); free(out); free(scr);
        return -1;
    }
    twiddle_table(w, n, sign);
    for (long c = 0; c < count; ++c) {
        cplx *line = data + c * line_step;
        for (int j = 0; j < n; ++j) buf[j] = line[(long)j * stride];
        dft_rec(buf, 1, out, n, w, n, scr);
        for (int j = 0; j < n; ++j) line[(long)j * stride] = out[j];
    }
    free(w); free(buf); free(out); free(scr);
    return 0;
}

/*
 * Unnormalised in-place 3D transform of a C-ordered n0 x n1 x n2 complex array
 * (index (i0,i1,i2) at i2 + n2*(i1 + n1*i0)).  sign = -1 forward, +1 inverse.
 * Returns 0 on success, -1 on allocation failure.
 */
int oracle_fft3d(double *data_interleaved, int n0, int n1, int n2, int sign)
{
    cplx *a = (cplx *)data_interleaved;
    long s2 = 1, s1 = n2, s0 = (long)n1 * n2;
    /* axis 2: n0*n1 contiguous lines */
    if (fft_lines(a, n2, s2, (long)n0 * n1, s1, sign)) return -1;
    /* axis 1: for each i0, n2 lines of stride n2 */
    for (long i0 = 0; i0 < n0; ++i0)
        if (fft_lines(a + i0 * s0, n1, s1, n2, 1, sign)) return -1;
    /* axis 0: n1*n2 lines of stride n1*n2 */
    if (fft_lines(a, n0, s0, (long)n1 * n2, 1, sign)) return -1;
    return 0;
}

/* Unnormalised in-place 1D transforms along the last axis (for tests). */
int oracle_fft1d_batch(double *data_interleaved, int n, long count, int sign)
{
    return fft_lines((cplx *)data_interleaved, n, 1, count, n, sign);
}
