/*
 * oracle.c -- plain, slow, obviously correct CPU reference for the FX
 * correlator hot path of Roy et al., "A real-time software backend for the
 * GMRT" (arXiv:0910.1517).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the GPU library.
 *
 * Arithmetic is IEEE double precision (FP64) for floating point and int64 for
 * the integer X-engine.  Each function follows one definition of the paper,
 * written out without blocking, fusion or reordering:
 *
 *   integer delay        section 2.1 (block shift) and section 2.3.2
 *                        (read-pointer offset into the overlapped slice)
 *   channelisation       section 2.1 (FX architecture: FFT, then multiply)
 *   FSTC + fringe        Eq. 2 of section 2.1
 *   cross-multiply       section 2.1 (all four polar products per baseline,
 *                        integrated over time)
 *   requantisation       section 4.1 (fixed-point pipeline up to the MAC,
 *                        32-bit products, float long-term accumulation)
 *   MAD statistic        Eq. 3 and Eq. 4 of section 5
 *   array beams          section 2.2 (incoherent and coherent beamformer)
 *   ADC unpacking        sections 2.3.2 and 3.3 (four-input demultiplexing,
 *                        4-bit samples to 8 bits)
 *   voltage blanker      section 5 (Eq. 3 and 4 on voltage blocks, outliers
 *                        replaced by precomputed Gaussian noise, one table
 *                        per signal from Philox4x32-10)
 *
 * Readings where the paper is silent (FFT sign, bins kept, time stamp of a
 * spectrum, sign convention of Eq. 2, requantisation scale, e4m3 format) are
 * the ones listed in the design notes of the repository and are restated at
 * each function below.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC oracle.c
 *        -o liboracle.so -lm
 * (no -ffast-math and no FMA contraction: every operation is the plain IEEE
 * one).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef double complex cplx;

static int is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

/* ------------------------------------------------------------------------ */
/* Discrete Fourier transform, X[k] = sum_n z[n] exp(-2 pi i k n / N).        */
/* Sign negative, no normalisation, rectangular window (section 2.1 leaves    */
/* these open; this is the textbook forward DFT).                             */
/* ------------------------------------------------------------------------ */

/* Direct evaluation of the definition.  The exponent k*n is reduced modulo N
 * in exact integer arithmetic before the libm cos/sin call. */
void orc_dft(const double *zin, double *zout, int64_t n)
{
    for (int64_t k = 0; k < n; ++k) {
        cplx acc = 0;
        for (int64_t j = 0; j < n; ++j) {
            int64_t r = (k * j) % n;
            double a = -2.0 * M_PI * (double)r / (double)n;
            cplx w = cos(a) + I * sin(a);
            acc += (zin[2 * j] + I * zin[2 * j + 1]) * w;
        }
        zout[2 * k] = creal(acc);
        zout[2 * k + 1] = cimag(acc);
    }
}

/* Radix-2 decimation-in-time Cooley-Tukey FFT, in place, same definition as
 * orc_dft.  Textbook form: bit-reversal permutation, then log2(N) stages of
 * butterflies whose twiddles come straight from libm cos/sin. */
static void fft_inplace(cplx *z, int64_t n)
{
    for (int64_t i = 1, j = 0; i < n; ++i) {
        int64_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { cplx t = z[i]; z[i] = z[j]; z[j] = t; }
    }
    for (int64_t len = 2; len <= n; len <<= 1) {
        int64_t half = len >> 1;
        for (int64_t j = 0; j < half; ++j) {
            double a = -2.0 * M_PI * (double)j / (double)len;
            cplx w = cos(a) + I * sin(a);
            for (int64_t i = 0; i < n; i += len) {
                cplx u = z[i + j];
                cplx v = z[i + j + half] * w;
                z[i + j] = u + v;
                z[i + j + half] = u - v;
            }
        }
    }
}

int orc_fft(double *z, int64_t n)
{
    if (!is_pow2(n)) return -1;
    fft_inplace((cplx *)z, n);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* F-engine.                                                                  */
/*                                                                            */
/* Signal s, spectrum m (0-based inside this call, absolute index             */
/* spectrum0 + m):                                                            */
/*   window   w[n] = x[s][m*N + D_s + n],  n = 0..N-1   (integer delay as a   */
/*            read-pointer advance into a row that carries D_pad extra        */
/*            samples, the paper's overlap region)                            */
/*   spectrum X[k] = sum_n w[n] exp(-2 pi i k n / N),  k = 0..N/2-1           */
/*            (DC kept, Nyquist bin dropped)                                  */
/*   phase    theta = 2 pi [ (nu_BB + k fs/N) * f_s/fs                        */
/*                          + sigma * (psi_s + r_s * t_m) ],                  */
/*            t_m = (spectrum0 + m + 1/2) N / fs, the window centre measured  */
/*            from the call's reference epoch (Eq. 2; f_s is the fractional   */
/*            delay in samples, so tau_frac = f_s/fs; psi_s and r_s are the   */
/*            fringe phase in cycles and the fringe rate in Hz, sigma = +-1   */
/*            the sideband sign of Eq. 2)                                     */
/*   output   Y[k] = X[k] * exp(+i theta)                                     */
/*                                                                            */
/* Y layout: [S][T][C][2] doubles, C = N/2.                                   */
/* method 0: radix-2 FFT; method 1: direct DFT.                               */
/* ------------------------------------------------------------------------ */
static double fstc_fringe_phase(int64_t k, int64_t N, double fs, double nu_bb,
                                double f, double psi0, double rate,
                                int sideband, int64_t spectrum)
{
    double nu_k = (double)k * fs / (double)N;
    double t_m = ((double)spectrum + 0.5) * (double)N / fs;
    return 2.0 * M_PI * ((nu_bb + nu_k) * f / fs +
                         (double)sideband * (psi0 + rate * t_m));
}

int orc_fengine(const int8_t *x, int64_t row_stride, int S, int64_t N,
                int64_t T, int64_t spectrum0, const int32_t *D,
                const double *f, const double *psi0, const double *rate,
                double fs, double nu_bb, int sideband, int method, double *Y)
{
    if (!is_pow2(N) || S <= 0 || T < 0) return -1;
    int64_t C = N / 2;
    int bad = 0;
#pragma omp parallel for collapse(2) schedule(static)
    for (int s = 0; s < S; ++s) {
        for (int64_t m = 0; m < T; ++m) {
            cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)N);
            cplx *X = (cplx *)malloc(sizeof(cplx) * (size_t)N);
            if (!w || !X) { bad = 1; free(w); free(X); continue; }
            const int8_t *row = x + (int64_t)s * row_stride;
            for (int64_t n = 0; n < N; ++n)
                w[n] = (double)row[m * N + D[s] + n];
            if (method == 1) {
                orc_dft((const double *)w, (double *)X, N);
            } else {
                memcpy(X, w, sizeof(cplx) * (size_t)N);
                fft_inplace(X, N);
            }
            double *out = Y + (((int64_t)s * T + m) * C) * 2;
            for (int64_t k = 0; k < C; ++k) {
                double th = fstc_fringe_phase(k, N, fs, nu_bb, f[s], psi0[s],
                                              rate[s], sideband, spectrum0 + m);
                cplx y = X[k] * (cos(th) + I * sin(th));
                out[2 * k] = creal(y);
                out[2 * k + 1] = cimag(y);
            }
            free(w);
            free(X);
        }
    }
    return bad ? -2 : 0;
}

/* F-engine with the phase taken from the 1440-step sin/cos table of section  */
/* 2.3.2 (0.25 degree steps).  The phase of Eq. 2 in cycles is formed per     */
/* channel and spectrum as                                                    */
/*   c   = nu_BB f / fs + sigma (psi + r t_m),  t_m = (spectrum + 1/2)(N/fs), */
/*   c  -= floor(c),                                                          */
/*   phi = c + k (f / N),                                                     */
/* each operation rounded on its own in FP64 (the table index is an integer   */
/* decision, so the reading fixes this order), and the table entry is         */
/* j = rint(1440 phi) mod 1440: Y[k] = X[k] exp(2 pi i j / 1440).             */
int orc_fengine_lut(const int8_t *x, int64_t row_stride, int S, int64_t N, int64_t T, int64_t spectrum0,
                    const int32_t *D, const double *f, const double *psi0, const double *rate, double fs,
                    double nu_bb, int sideband, double *Y)
{
    if (!is_pow2(N) || S <= 0 || T < 0) return -1;
    int64_t C = N / 2;
    int bad = 0;
#pragma omp parallel for collapse(2) schedule(static)
    for (int s = 0; s < S; ++s) {
        for (int64_t m = 0; m < T; ++m) {
            cplx *X = (cplx *)malloc(sizeof(cplx) * (size_t)N);
            if (!X) { bad = 1; continue; }
            const int8_t *row = x + (int64_t)s * row_stride;
            for (int64_t n = 0; n < N; ++n) X[n] = (double)row[m * N + D[s] + n];
            fft_inplace(X, N);
            double t_spec = (double)N / fs;
            double tm = ((double)(spectrum0 + m) + 0.5) * t_spec;
            double c = nu_bb * f[s] / fs + (double)sideband * (psi0[s] + rate[s] * tm);
            c -= floor(c);
            double fn = f[s] / (double)N;
            double *out = Y + (((int64_t)s * T + m) * C) * 2;
            for (int64_t k = 0; k < C; ++k) {
                double phi = c + (double)k * fn;
                int64_t j = (int64_t)rint(phi * 1440.0) % 1440;
                double th = 2.0 * M_PI * (double)j / 1440.0;
                cplx y = X[k] * (cos(th) + I * sin(th));
                out[2 * k] = creal(y);
                out[2 * k + 1] = cimag(y);
            }
            free(X);
        }
    }
    return bad ? -2 : 0;
}

/* Same F-engine for a list of channels only, by the direct DFT sum of the
 * definition (used to check sampled outputs of full-size runs).
 * Y layout: [S][T][nk][2]. */
int orc_fengine_channels(const int8_t *x, int64_t row_stride, int S,
                         int64_t N, int64_t T, int64_t spectrum0,
                         const int32_t *D, const double *f, const double *psi0,
                         const double *rate, double fs, double nu_bb,
                         int sideband, const int64_t *kk, int nk, double *Y)
{
    if (!is_pow2(N) || S <= 0 || T < 0 || nk <= 0) return -1;
    for (int i = 0; i < nk; ++i)
        if (kk[i] < 0 || kk[i] >= N / 2) return -1;
    /* exp(-2 pi i r / N) for r = 0..N-1, from libm */
    cplx *tw = (cplx *)malloc(sizeof(cplx) * (size_t)N);
    if (!tw) return -2;
    for (int64_t r = 0; r < N; ++r) {
        double a = -2.0 * M_PI * (double)r / (double)N;
        tw[r] = cos(a) + I * sin(a);
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int s = 0; s < S; ++s) {
        for (int64_t m = 0; m < T; ++m) {
            const int8_t *w = x + (int64_t)s * row_stride + m * N + D[s];
            for (int i = 0; i < nk; ++i) {
                int64_t k = kk[i];
                cplx acc = 0;
                for (int64_t n = 0; n < N; ++n)
                    acc += (double)w[n] * tw[(k * n) % N];
                double th = fstc_fringe_phase(k, N, fs, nu_bb, f[s], psi0[s],
                                              rate[s], sideband, spectrum0 + m);
                cplx y = acc * (cos(th) + I * sin(th));
                double *out = Y + (((int64_t)s * T + m) * nk + i) * 2;
                out[0] = creal(y);
                out[1] = cimag(y);
            }
        }
    }
    free(tw);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* X-engine (section 2.1): for every channel k and every signal pair i <= j   */
/*   V_k[i][j] = sum_m Y_i[m,k] * conj(Y_j[m,k])                              */
/* stored at pair index p = j(j+1)/2 + i.  Autocorrelations (i == j) and the  */
/* cross-polar products are included: with s = 2a + pol this yields RR*, RL*, */
/* LR* and LL* of every baseline.  V is accumulated (+=) so that a caller can */
/* integrate over several calls.                                              */
/* Y layout [S][T][C][2]; V layout [C][P][2].                                 */
/* ------------------------------------------------------------------------ */
void orc_xengine_f64(const double *Y, int S, int64_t T, int64_t C, double *V)
{
    int64_t P = (int64_t)S * (S + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < C; ++k) {
        for (int j = 0; j < S; ++j) {
            for (int i = 0; i <= j; ++i) {
                cplx acc = 0;
                for (int64_t m = 0; m < T; ++m) {
                    const double *yi = Y + (((int64_t)i * T + m) * C + k) * 2;
                    const double *yj = Y + (((int64_t)j * T + m) * C + k) * 2;
                    acc += (yi[0] + I * yi[1]) * (yj[0] - I * yj[1]);
                }
                int64_t p = (int64_t)j * (j + 1) / 2 + i;
                V[(k * P + p) * 2] += creal(acc);
                V[(k * P + p) * 2 + 1] += cimag(acc);
            }
        }
    }
}

/* Integer X-engine: the same triple loop on requantised int8 spectra,
 * accumulated in int64 (exact).  q layout [S][T][C][2]; A layout [C][P][2]. */
void orc_xengine_int(const int8_t *q, int S, int64_t T, int64_t C, int64_t *A)
{
    int64_t P = (int64_t)S * (S + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < C; ++k) {
        for (int j = 0; j < S; ++j) {
            for (int i = 0; i <= j; ++i) {
                int64_t re = 0, im = 0;
                for (int64_t m = 0; m < T; ++m) {
                    const int8_t *a = q + (((int64_t)i * T + m) * C + k) * 2;
                    const int8_t *b = q + (((int64_t)j * T + m) * C + k) * 2;
                    /* (ar + i ai)(br - i bi) */
                    re += (int64_t)a[0] * b[0] + (int64_t)a[1] * b[1];
                    im += (int64_t)a[1] * b[0] - (int64_t)a[0] * b[1];
                }
                int64_t p = (int64_t)j * (j + 1) / 2 + i;
                A[(k * P + p) * 2] += re;
                A[(k * P + p) * 2 + 1] += im;
            }
        }
    }
}

/* The same cross products on 16-bit integer spectra (the 16-bit fixed-point   */
/* data of the real-time pipeline, sections 3.1 and 4.1): every product is    */
/* exact in 32 bits and the sums are int64.                                    */
void orc_xengine_i16(const int16_t *q, int S, int64_t T, int64_t C, int64_t *A)
{
    int64_t P = (int64_t)S * (S + 1) / 2;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < C; ++k) {
        for (int j = 0; j < S; ++j) {
            for (int i = 0; i <= j; ++i) {
                int64_t re = 0, im = 0;
                for (int64_t m = 0; m < T; ++m) {
                    const int16_t *a = q + (((int64_t)i * T + m) * C + k) * 2;
                    const int16_t *b = q + (((int64_t)j * T + m) * C + k) * 2;
                    re += (int64_t)a[0] * b[0] + (int64_t)a[1] * b[1];
                    im += (int64_t)a[1] * b[0] - (int64_t)a[0] * b[1];
                }
                int64_t p = (int64_t)j * (j + 1) / 2 + i;
                A[(k * P + p) * 2] += re;
                A[(k * P + p) * 2 + 1] += im;
            }
        }
    }
}

/* The 1440-step table of section 2.3.2 as the integers the real-time code    */
/* multiplies by (section 4.1: scaled so that a 16-bit spectrum times the      */
/* table keeps its result in the low half of a 32-bit product): Q14,           */
/* w[j] = (rint(2^14 cos(2 pi j / 1440)), rint(2^14 sin(2 pi j / 1440))).        */
void orc_fix16_table(int32_t *w)
{
    for (int j = 0; j < 1440; ++j) {
        double th = 2.0 * M_PI * (double)j / 1440.0;
        w[2 * j] = (int32_t)rint(16384.0 * cos(th));
        w[2 * j + 1] = (int32_t)rint(16384.0 * sin(th));
    }
}

/* floor(v / 2^14) for any sign */
static int64_t floor_div16384(int64_t v) { return v >= 0 ? v / 16384 : -((-v + 16383) / 16384); }
static int64_t sat16(int64_t v) { return v > 32767 ? 32767 : (v < -32767 ? -32767 : v); }
/* the 16-bit code of one component: x / level in FP32 (the precision of the   */
/* spectra the code is taken from), rounded half to even, saturated            */
static int64_t code16(double x, double level)
{
    double r = nearbyint((double)((float)x / (float)level));
    return r > 32767.0 ? 32767 : (r < -32767.0 ? -32767 : (int64_t)r);
}

/* The 16-bit fixed-point spectra of the real-time pipeline (sections 3.1 and  */
/* 4.1), from the unrotated FFT output X [S][T][C][2] (FP64):                  */
/*   q = sat16(round-half-even(X / scale[s][k])) per component: the 16-bit      */
/*       fixed-point FFT output, the level set per signal and channel (the       */
/*       division in FP32, X and scale being FP32 values);                       */
/*   j = the table entry of the Eq. 2 phase, chosen as in orc_fengine_lut;       */
/*   y = sat16(floor((q w_j + 2^13) / 2^14)) per component, q w_j the complex    */
/*       product in integers: the integer fringe stop and FSTC, rounded to the   */
/*       nearest (halves up) rather than truncated.                             */
/* Saturation at +-32767 keeps negation (and conjugation) exact.               */
void orc_fix16_spectra(const double *X, int S, int64_t T, int64_t C, int64_t spectrum0, const double *f,
                       const double *psi0, const double *rate, double fs, double nu_bb, int sideband,
                       const double *scale, int16_t *q16, int16_t *y16)
{
    int32_t w[2 * 1440];
    orc_fix16_table(w);
    int64_t N = 2 * C;
#pragma omp parallel for collapse(2) schedule(static)
    for (int s = 0; s < S; ++s) {
        for (int64_t m = 0; m < T; ++m) {
            double t_spec = (double)N / fs;
            double tm = ((double)(spectrum0 + m) + 0.5) * t_spec;
            double c = nu_bb * f[s] / fs + (double)sideband * (psi0[s] + rate[s] * tm);
            c -= floor(c);
            double fn = f[s] / (double)N;
            for (int64_t k = 0; k < C; ++k) {
                int64_t o = (((int64_t)s * T + m) * C + k) * 2;
                double sc = scale[(int64_t)s * C + k];
                int64_t qr = code16(X[o], sc);
                int64_t qi = code16(X[o + 1], sc);
                double phi = c + (double)k * fn;
                int64_t j = (int64_t)rint(phi * 1440.0) % 1440;
                int64_t wr = w[2 * j], wi = w[2 * j + 1];
                q16[o] = (int16_t)qr;
                q16[o + 1] = (int16_t)qi;
                y16[o] = (int16_t)sat16(floor_div16384(qr * wr - qi * wi + 8192));
                y16[o + 1] = (int16_t)sat16(floor_div16384(qr * wi + qi * wr + 8192));
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Requantisation (section 4.1: fixed point up to the MAC with tuned levels). */
/* sigma[s][k] = sqrt( sum_m |Y_s[m,k]|^2 / (2T) )  -- RMS of one component. */
/* ------------------------------------------------------------------------ */
void orc_sigma(const double *Y, int S, int64_t T, int64_t C, double *sigma)
{
    for (int s = 0; s < S; ++s)
        for (int64_t k = 0; k < C; ++k) {
            double acc = 0;
            for (int64_t m = 0; m < T; ++m) {
                const double *y = Y + (((int64_t)s * T + m) * C + k) * 2;
                acc += y[0] * y[0] + y[1] * y[1];
            }
            sigma[(int64_t)s * C + k] = sqrt(acc / (2.0 * (double)T));
        }
}

/* Round half to even, written out from its definition. */
static double round_half_even(double u)
{
    double fl = floor(u);
    double d = u - fl;
    if (d > 0.5) return fl + 1.0;
    if (d < 0.5) return fl;
    return (fmod(fl, 2.0) == 0.0) ? fl : fl + 1.0;
}

/* q = clamp(rne(Y / scale), -127, +127) for both components; -128 is never
 * produced, so conjugation and negation stay exact.  scale layout [S][C]. */
void orc_quantize_int8(const double *Y, const double *scale, int S, int64_t T,
                       int64_t C, int8_t *q)
{
    for (int s = 0; s < S; ++s)
        for (int64_t m = 0; m < T; ++m)
            for (int64_t k = 0; k < C; ++k)
                for (int c = 0; c < 2; ++c) {
                    int64_t idx = (((int64_t)s * T + m) * C + k) * 2 + c;
                    double u = Y[idx] / scale[(int64_t)s * C + k];
                    double r = round_half_even(u);
                    if (r > 127.0) r = 127.0;
                    if (r < -127.0) r = -127.0;
                    q[idx] = (int8_t)r;
                }
}

/* OCP 8-bit float E4M3 ("e4m3fn"): 1 sign bit, 4 exponent bits (bias 7),
 * 3 mantissa bits, subnormals, no infinities, 0x7F/0xFF are NaN, largest
 * finite magnitude 448. */
double orc_e4m3_decode(uint8_t b)
{
    int sign = b >> 7, e = (b >> 3) & 0xF, mnt = b & 7;
    double v;
    if (e == 0xF && mnt == 7) return NAN;
    if (e == 0) v = ldexp((double)mnt / 8.0, -6);
    else v = ldexp(1.0 + (double)mnt / 8.0, e - 7);
    return sign ? -v : v;
}

/* Round to the nearest finite e4m3 value, ties to the even code, saturating
 * to +-448: a brute-force search over the 127 non-negative finite codes. */
uint8_t orc_e4m3_encode(double v)
{
    double a = fabs(v);
    int best = 0;
    double bestd = INFINITY;
    for (int c = 0; c <= 0x7E; ++c) {
        double d = fabs(orc_e4m3_decode((uint8_t)c) - a);
        if (d < bestd || (d == bestd && (c & 1) == 0 && (best & 1) == 1)) {
            bestd = d;
            best = c;
        }
    }
    if (a > 448.0) best = 0x7E;
    if (best == 0) return 0; /* +0 for both signs */
    return (uint8_t)(best | (v < 0 ? 0x80 : 0));
}

/* FP8 requantisation: b = e4m3(Y / scale8), scale8 = 4 sigma / 448. */
void orc_quantize_fp8(const double *Y, const double *scale, int S, int64_t T,
                      int64_t C, uint8_t *q)
{
#pragma omp parallel for schedule(static)
    for (int s = 0; s < S; ++s)
        for (int64_t m = 0; m < T; ++m)
            for (int64_t k = 0; k < C; ++k)
                for (int c = 0; c < 2; ++c) {
                    int64_t idx = (((int64_t)s * T + m) * C + k) * 2 + c;
                    q[idx] = orc_e4m3_encode(Y[idx] / scale[(int64_t)s * C + k]);
                }
}

/* ------------------------------------------------------------------------ */
/* Integration (section 2.3.2 / 4.1): visibilities of the integer path are    */
/* V = scale_i * scale_j * A, formed and accumulated in floating point.       */
/* scale layout [S][C]; A layout [C][P][2]; V layout [C][P][2] (+=).          */
/* ------------------------------------------------------------------------ */
void orc_scale_visibilities(const double *A, const double *scale, int S,
                            int64_t C, double *V)
{
    int64_t P = (int64_t)S * (S + 1) / 2;
    for (int64_t k = 0; k < C; ++k)
        for (int j = 0; j < S; ++j)
            for (int i = 0; i <= j; ++i) {
                int64_t p = (int64_t)j * (j + 1) / 2 + i;
                double g = scale[(int64_t)i * C + k] * scale[(int64_t)j * C + k];
                V[(k * P + p) * 2] += g * A[(k * P + p) * 2];
                V[(k * P + p) * 2 + 1] += g * A[(k * P + p) * 2 + 1];
            }
}

/* ------------------------------------------------------------------------ */
/* MAD statistic, Eq. 3 and Eq. 4 of section 5.                               */
/* ------------------------------------------------------------------------ */
static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Median of n values; for even n the mean of the two middle values. */
double orc_median(const double *v, int64_t n)
{
    double *t = (double *)malloc(sizeof(double) * (size_t)n);
    memcpy(t, v, sizeof(double) * (size_t)n);
    qsort(t, (size_t)n, sizeof(double), cmp_double);
    double med = (n & 1) ? t[n / 2] : 0.5 * (t[n / 2 - 1] + t[n / 2]);
    free(t);
    return med;
}

/* Eq. 3: MAD = median |x_i - median(x)|.  Eq. 4: flag x_i when
 * |x_i - median(x)| > M * MAD / 0.6745 (strict).  Returns the number flagged
 * and writes flags[i] in {0, 1}; med and mad are returned through pointers. */
int64_t orc_mad_flags(const double *x, int64_t n, double M, uint8_t *flags,
                      double *med_out, double *mad_out)
{
    double med = orc_median(x, n);
    double *dev = (double *)malloc(sizeof(double) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) dev[i] = fabs(x[i] - med);
    double mad = orc_median(dev, n);
    int64_t cnt = 0;
    for (int64_t i = 0; i < n; ++i) {
        flags[i] = dev[i] > M * mad / 0.6745;
        cnt += flags[i];
    }
    free(dev);
    if (med_out) *med_out = med;
    if (mad_out) *mad_out = mad;
    return cnt;
}

/* ------------------------------------------------------------------------ */
/* Flagging on dynamic spectra (section 5: MAD statistic of Eq. 3 / Eq. 4).   */
/*                                                                            */
/* The paper blanks time-domain voltages; on the channelised path the same    */
/* statistic is taken on power tiles of TT spectra x KT channels of one       */
/* signal: per tile, the row statistic (mean power of a spectrum over the     */
/* tile's channels, which exposes broadband bursts) and the column statistic  */
/* (mean power of a channel over the tile's spectra, which exposes persistent */
/* tones) are each thresholded with Eq. 4, and a cell is flagged when its row */
/* or its column is.  power layout [S][T][C]; flags layout [S][T][C] (0/1).   */
/* T must be a multiple of TT and C of KT.                                    */
/* ------------------------------------------------------------------------ */
/* which: 1 the row statistic only, 2 the column statistic only, 3 both.    */
int orc_mad_tile_flags_which(const double *power, int S, int64_t T, int64_t C, int TT,
                             int KT, double M, int which, uint8_t *flags);
int orc_mad_tile_flags(const double *power, int S, int64_t T, int64_t C, int TT,
                       int KT, double M, uint8_t *flags)
{
    return orc_mad_tile_flags_which(power, S, T, C, TT, KT, M, 3, flags);
}

int orc_mad_tile_flags_which(const double *power, int S, int64_t T, int64_t C, int TT,
                             int KT, double M, int which, uint8_t *flags)
{
    if (T % TT || C % KT) return -1;
    double *row = (double *)malloc(sizeof(double) * (size_t)TT);
    double *col = (double *)malloc(sizeof(double) * (size_t)KT);
    uint8_t *rf = (uint8_t *)malloc((size_t)TT);
    uint8_t *cf = (uint8_t *)malloc((size_t)KT);
    for (int s = 0; s < S; ++s)
        for (int64_t m0 = 0; m0 < T; m0 += TT)
            for (int64_t k0 = 0; k0 < C; k0 += KT) {
                for (int r = 0; r < TT; ++r) {
                    double acc = 0;
                    for (int k = 0; k < KT; ++k)
                        acc += power[((int64_t)s * T + m0 + r) * C + k0 + k];
                    row[r] = acc / KT;
                }
                for (int k = 0; k < KT; ++k) {
                    double acc = 0;
                    for (int r = 0; r < TT; ++r)
                        acc += power[((int64_t)s * T + m0 + r) * C + k0 + k];
                    col[k] = acc / TT;
                }
                orc_mad_flags(row, TT, M, rf, NULL, NULL);
                orc_mad_flags(col, KT, M, cf, NULL, NULL);
                for (int r = 0; r < TT; ++r)
                    for (int k = 0; k < KT; ++k)
                        flags[((int64_t)s * T + m0 + r) * C + k0 + k] =
                            (uint8_t)(((which & 1) ? rf[r] : 0) | ((which & 2) ? cf[k] : 0));
            }
    free(row);
    free(col);
    free(rf);
    free(cf);
    return 0;
}

/* Unflagged-product counts: n_ij[k] = sum_m (1 - F_i[m,k]) (1 - F_j[m,k]) for
 * every pair i <= j (p = j(j+1)/2 + i).  flags [S][T][C]; n [C][P] (+=). */
void orc_pair_counts(const uint8_t *flags, int S, int64_t T, int64_t C, int64_t *n)
{
    int64_t P = (int64_t)S * (S + 1) / 2;
    for (int64_t k = 0; k < C; ++k)
        for (int j = 0; j < S; ++j)
            for (int i = 0; i <= j; ++i) {
                int64_t cnt = 0;
                for (int64_t m = 0; m < T; ++m)
                    cnt += (flags[((int64_t)i * T + m) * C + k] == 0) &&
                           (flags[((int64_t)j * T + m) * C + k] == 0);
                n[k * P + (int64_t)j * (j + 1) / 2 + i] += cnt;
            }
}

/* ------------------------------------------------------------------------ */
/* Array beams (section 2.2).  Signal s = 2a + pol.  Per spectrum m, channel k: */
/*   incoherent  I_pol  = sum over s of pol of  w_s |Y_s|^2                  */
/*   coherent    V_b,pol = sum over s of pol of  c_b,s Y_s                    */
/* and the coherent products by mode: 0 |V_0|^2, |V_1|^2; 1 those and Re, Im  */
/* of V_0 conj(V_1); 2 the voltages V_0, V_1 themselves.  Outputs are sums    */
/* over tint consecutive spectra.  Y [S][T][C] complex (re, im); w [S] or     */
/* NULL; c [nb][S] complex; inc [2][T/tint][C] (+=); coh [nb][planes][T/tint] */
/* [C] (+=; complex for mode 2, tint = 1).                                   */
void orc_beamform(const double *Y, int S, int64_t T, int64_t C, const double *w, const double *c, int nb,
                  int mode, int tint, double *inc, double *coh)
{
    int64_t To = T / tint;
    for (int64_t m = 0; m < T; ++m)
        for (int64_t k = 0; k < C; ++k) {
            int64_t o = m / tint;
            if (w && inc)
                for (int s = 0; s < S; ++s) {
                    const double *y = Y + 2 * (((int64_t)s * T + m) * C + k);
                    inc[((int64_t)(s % 2) * To + o) * C + k] += w[s] * (y[0] * y[0] + y[1] * y[1]);
                }
            for (int b = 0; b < nb; ++b) {
                double vr[2] = {0.0, 0.0}, vi[2] = {0.0, 0.0};
                for (int s = 0; s < S; ++s) {
                    const double *y = Y + 2 * (((int64_t)s * T + m) * C + k);
                    const double *cs = c + 2 * ((int64_t)b * S + s);
                    vr[s % 2] += cs[0] * y[0] - cs[1] * y[1];
                    vi[s % 2] += cs[0] * y[1] + cs[1] * y[0];
                }
                if (mode == 2) {
                    for (int p = 0; p < 2; ++p) {
                        double *out = coh + 2 * (((int64_t)(2 * b + p) * T + m) * C + k);
                        out[0] += vr[p];
                        out[1] += vi[p];
                    }
                    continue;
                }
                int np = mode == 1 ? 4 : 2;
                double prod[4];
                prod[0] = vr[0] * vr[0] + vi[0] * vi[0];
                prod[1] = vr[1] * vr[1] + vi[1] * vi[1];
                prod[2] = vr[0] * vr[1] + vi[0] * vi[1]; /* Re V0 conj(V1) */
                prod[3] = vi[0] * vr[1] - vr[0] * vi[1]; /* Im V0 conj(V1) */
                for (int q = 0; q < np; ++q) coh[(((int64_t)b * np + q) * To + o) * C + k] += prod[q];
            }
        }
}

/* ------------------------------------------------------------------------ */
/* ADC input formats (section 2.3.2 and 3.3): each acquisition card digitises */
/* four inputs, either 8-bit (16 MHz mode) or 4-bit (33 MHz mode), and the    */
/* compute nodes demultiplex the four streams and unpack 4-bit samples to     */
/* 8 bits.  Raw stream of a card: time-major, the four inputs of a time       */
/* sample together; 8-bit: byte 4t + i is input i; 4-bit: byte 2t + i/2,      */
/* nibble i mod 2 (low nibble first).  Samples are two's complement, 4-bit    */
/* ones sign-extended to int8 (value kept).  Output row 4 c + i holds input i */
/* of card c.                                                                 */
void orc_adc_unpack(const uint8_t *raw, int64_t raw_stride, int n_cards, int64_t n, int bits, int8_t *x,
                    int64_t row_stride)
{
    for (int c = 0; c < n_cards; ++c)
        for (int64_t t = 0; t < n; ++t)
            for (int i = 0; i < 4; ++i) {
                const uint8_t *r = raw + (int64_t)c * raw_stride;
                int v;
                if (bits == 8) {
                    v = (int8_t)r[4 * t + i];
                } else {
                    int nib = (r[2 * t + i / 2] >> (4 * (i % 2))) & 0xF;
                    v = nib >= 8 ? nib - 16 : nib;
                }
                x[(int64_t)(4 * c + i) * row_stride + t] = (int8_t)v;
            }
}

/* ------------------------------------------------------------------------ */
/* Time-domain MAD voltage blanker (section 5, Eq. 3 and 4).  Per block of B */
/* consecutive samples of one signal: x~ = median, MAD = median |x - x~|; a   */
/* sample with |x - x~| > M MAD / 0.6745 is replaced by a precomputed         */
/* Gaussian noise sample, the tables being independent per signal (so per    */
/* antenna).  The replacement has the block's robust statistics (mean x~,     */
/* sigma = MAD / 0.6745): rint(x~ + sigma z), clamped to the int8 range.  A   */
/* block with MAD = 0 has no scale estimate and is passed unchanged.  Medians */
/* are kept exactly as integers: med2 = 2 x~, mad4 = 4 MAD.                   */
/*                                                                            */
/* Noise table: z[s][j] for j < L is the Irwin-Hall sum of twelve 16-bit      */
/* uniforms (U + 1/2) / 65536 minus 6 (mean 0, variance 1), the uniforms      */
/* being the 16-bit halves of two Philox4x32-10 outputs (Salmon, Moraes,      */
/* Dror and Shaw, SC'11) keyed by the seed at counters (j, 0, s, 0) and       */
/* (j, 0, s, 1): halves low then high of words 0..3 of the first and words    */
/* 0..1 of the second.  Sample p of a row uses z[s][p mod L].                 */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { /* key schedule: Weyl increments between rounds */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

/* entry j of signal s's table row (a multiple of 2^-16 below 6: exact in float) */
float orc_blank_noise_entry(uint64_t seed, int s, int64_t j)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t a[4], b[4];
    uint32_t c0[4] = {(uint32_t)j, (uint32_t)((uint64_t)j >> 32), (uint32_t)s, 0u};
    uint32_t c1[4] = {(uint32_t)j, (uint32_t)((uint64_t)j >> 32), (uint32_t)s, 1u};
    orc_philox4x32_10(c0, key, a);
    orc_philox4x32_10(c1, key, b);
    uint32_t w[6] = {a[0], a[1], a[2], a[3], b[0], b[1]};
    int64_t sum = 0;
    for (int q = 0; q < 6; ++q) sum += (int64_t)(w[q] & 0xFFFFu) + (int64_t)(w[q] >> 16);
    /* sum of (U + 1/2) / 65536 over 12, minus 6 */
    return (float)((double)(sum + 6 - 6 * 65536) / 65536.0);
}

/* table[s * L + j] */
void orc_blank_noise_table(uint64_t seed, int S, int64_t L, float *table)
{
    for (int s = 0; s < S; ++s)
        for (int64_t j = 0; j < L; ++j) table[(int64_t)s * L + j] = orc_blank_noise_entry(seed, s, j);
}

static int cmp_int(const void *a, const void *b)
{
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* 2 x median of v[0 .. n-1] (sorts v): the middle value, or the sum of the two */
/* middle values for even n */
static int median2(int *v, int64_t n)
{
    qsort(v, (size_t)n, sizeof(int), cmp_int);
    return (n & 1) ? 2 * v[n / 2] : v[n / 2 - 1] + v[n / 2];
}

/* x: S rows of n samples, row s at x + s * row_stride; out: same layout (may */
/* be x).  table [S][L] (L a power of two), sample i of a row uses entry      */
/* (sample0 + i) mod L.  counts [S][ceil(n / B)] blanked samples and stats    */
/* [S][ceil(n / B)][2] = (med2, mad4), each optional (NULL).                  */
void orc_mad_blank(const int8_t *x, int64_t row_stride, int S, int64_t n, int64_t B, double M, const float *table,
                   int64_t L, int64_t sample0, int8_t *out, int32_t *counts, int32_t *stats)
{
    int64_t nb = (n + B - 1) / B;
    int *v = (int *)malloc(sizeof(int) * (size_t)B);
    int *d = (int *)malloc(sizeof(int) * (size_t)B);
    for (int s = 0; s < S; ++s)
        for (int64_t b = 0; b < nb; ++b) {
            int64_t i0 = b * B, len = (i0 + B <= n) ? B : n - i0;
            const int8_t *xr = x + (int64_t)s * row_stride + i0;
            int8_t *o = out + (int64_t)s * row_stride + i0;
            for (int64_t i = 0; i < len; ++i) v[i] = xr[i];
            int med2 = median2(v, len);                            /* Eq. 3: x~ */
            for (int64_t i = 0; i < len; ++i) d[i] = abs(2 * (int)xr[i] - med2);
            int mad4 = median2(d, len);                            /* Eq. 3: MAD */
            double mad = (double)mad4 * 0.25;
            double thr = (double)M * mad / 0.6745;                 /* Eq. 4 */
            double sigma = mad / 0.6745;
            int32_t cnt = 0;
            for (int64_t i = 0; i < len; ++i) {
                int xi = xr[i];
                double dev = 0.5 * (double)abs(2 * xi - med2);     /* |x - x~| */
                if (mad4 > 0 && dev > thr) {
                    double z = (double)table[(int64_t)s * L + ((sample0 + i0 + i) & (L - 1))];
                    double r = rint(0.5 * (double)med2 + sigma * z);
                    if (r < -128.0) r = -128.0;
                    if (r > 127.0) r = 127.0;
                    o[i] = (int8_t)r;
                    ++cnt;
                } else {
                    o[i] = (int8_t)xi;
                }
            }
            if (counts) counts[(int64_t)s * nb + b] = cnt;
            if (stats) {
                stats[((int64_t)s * nb + b) * 2] = med2;
                stats[((int64_t)s * nb + b) * 2 + 1] = mad4;
            }
        }
    free(v);
    free(d);
}

/* ------------------------------------------------------------------------ */
/* Learned flagger (an addition to the paper, which only notes that          */
/* better RFI filtering has scope, section 5): 3x3 convolutions with zero     */
/* padding ("same" size), written from the definition of a 2-D               */
/* cross-correlation:                                                         */
/*   y[b][o][r][c] = bias[o] + sum_i sum_{u,v in -1..1}                       */
/*                   w[o][i][u+1][v+1] * x[b][i][r+u][c+v]                     */
/* (x outside the H x W tile is 0).  Layouts: x [B][Cin][H][W],               */
/* w [Cout][Cin][3][3], y [B][Cout][H][W].                                    */
/* ------------------------------------------------------------------------ */
void orc_conv3x3_fwd(const double *x, const double *w, const double *bias, int B, int Cin,
                     int Cout, int H, int W, double *y)
{
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < B; ++b)
        for (int o = 0; o < Cout; ++o)
            for (int r = 0; r < H; ++r)
                for (int c = 0; c < W; ++c) {
                    double acc = bias[o];
                    for (int i = 0; i < Cin; ++i)
                        for (int u = -1; u <= 1; ++u)
                            for (int v = -1; v <= 1; ++v) {
                                int rr = r + u, cc = c + v;
                                if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
                                acc += w[((o * Cin + i) * 3 + u + 1) * 3 + v + 1] *
                                       x[(((int64_t)b * Cin + i) * H + rr) * W + cc];
                            }
                    y[(((int64_t)b * Cout + o) * H + r) * W + c] = acc;
                }
}

/* Gradients of the convolution above from its definition (chain rule):
 *   dx[b][i][r][c] = sum_o sum_{u,v} w[o][i][u+1][v+1] dy[b][o][r-u][c-v]
 *   dw[o][i][u+1][v+1] = sum_{b,r,c} dy[b][o][r][c] x[b][i][r+u][c+v]
 *   dbias[o] = sum_{b,r,c} dy[b][o][r][c]
 * dx may be NULL. */
void orc_conv3x3_bwd(const double *x, const double *w, const double *dy, int B, int Cin,
                     int Cout, int H, int W, double *dx, double *dw, double *dbias)
{
    if (dx) {
#pragma omp parallel for collapse(2) schedule(static)
        for (int b = 0; b < B; ++b)
            for (int i = 0; i < Cin; ++i)
                for (int r = 0; r < H; ++r)
                    for (int c = 0; c < W; ++c) {
                        double acc = 0;
                        for (int o = 0; o < Cout; ++o)
                            for (int u = -1; u <= 1; ++u)
                                for (int v = -1; v <= 1; ++v) {
                                    int rr = r - u, cc = c - v;
                                    if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
                                    acc += w[((o * Cin + i) * 3 + u + 1) * 3 + v + 1] *
                                           dy[(((int64_t)b * Cout + o) * H + rr) * W + cc];
                                }
                        dx[(((int64_t)b * Cin + i) * H + r) * W + c] = acc;
                    }
    }
#pragma omp parallel for collapse(2) schedule(static)
    for (int o = 0; o < Cout; ++o)
        for (int i = 0; i < Cin; ++i)
            for (int u = -1; u <= 1; ++u)
                for (int v = -1; v <= 1; ++v) {
                    double acc = 0;
                    for (int b = 0; b < B; ++b)
                        for (int r = 0; r < H; ++r)
                            for (int c = 0; c < W; ++c) {
                                int rr = r + u, cc = c + v;
                                if (rr < 0 || rr >= H || cc < 0 || cc >= W) continue;
                                acc += dy[(((int64_t)b * Cout + o) * H + r) * W + c] *
                                       x[(((int64_t)b * Cin + i) * H + rr) * W + cc];
                            }
                    dw[((o * Cin + i) * 3 + u + 1) * 3 + v + 1] = acc;
                }
    for (int o = 0; o < Cout; ++o) {
        double acc = 0;
        for (int b = 0; b < B; ++b)
            for (int r = 0; r < H; ++r)
                for (int c = 0; c < W; ++c) acc += dy[(((int64_t)b * Cout + o) * H + r) * W + c];
        dbias[o] = acc;
    }
}
