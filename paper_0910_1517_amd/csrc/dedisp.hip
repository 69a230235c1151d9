// Coherent dedispersion of phased-array voltages (section 4.3).
//
// The coherent beam's voltages of each polarisation, channel k of spectrum m
// (V[m][k], k = 0..C-1, upper sideband, channel k at sky frequency
// nu0 + k fs/N, N = 2C), become the broadband complex series
//     z[m C + n] = sum_k V[m][k] exp(+2 pi i k n / C)
// (the inverse FFT of each spectrum; a complex baseband signal at fs/2).  Its
// transform over the whole block of L = T C samples is multiplied by the
// inverse of the cold-plasma transfer function referenced to nu0,
//     exp(-2 pi i K DM f^2 / (nu0^2 (nu0 + f))),  f = q fs / (2L),
// (Hankins and Rickett 1975; group delay K DM (nu^-2 - nu0^-2)), transformed
// back (divided by L), detected and summed over the polarisations and over
// n_int samples.  The transform is circular: the first sweep across the band
// (K DM (nu0^-2 - (nu0 + fs/2)^-2) fs/2 samples) wraps around, so a caller
// streams blocks that overlap by that much, as it does for the integer delays.
//
// One LDS kernel does all the transforms: W instances of an R-point DFT
// (radix-4 Stockham stages in LDS, one radix-2 stage for odd log2 R, natural
// order in and out, twiddles from an LDS table), loaded from and stored to
// the instance's elements; a tile holds 4096 points.  The per-spectrum inverse DFT is
// that kernel with R = C.  The long transform is a sequence of passes of a
// decimation-in-frequency decomposition: pass j splits blocks of Bp samples
// into R_j strided sub-sequences (stride s = Bp / R_j), takes their R_j-point
// DFTs and multiplies output k of column b by exp(-2 pi i b k / Bp).  A small
// radix goes first and then radix 256, so the stride is either >= the tile
// width (a tile is 4096 / R adjacent columns: rows of at least 128 bytes) or
// 1 (a tile is contiguous).  The result is in digit-reversed order; the chirp kernel maps
// each position to its frequency, and the inverse passes (the mirror image:
// conjugate twiddle, then the inverse DFT, in reverse order) restore time
// order.  All passes run in place: a workgroup reads its whole tile into LDS
// before it writes it back.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "corr_internal.h"

namespace {

constexpr int kDdThreads = 256;
constexpr double kDmConst = 4.148808e15;  // Hz^2 s / (pc cm^-3): delay = K DM / nu^2
constexpr int kDdMaxPasses = 8;

struct DdPasses {
    int n;                     // number of passes of the long transform
    int lr[kDdMaxPasses];      // log2 radix of each pass, in forward order
};

// Instances per workgroup: a 4096-point tile up to R = 4096, one instance
// above.  (Every pass with R < 4096 has stride 1 or >= 4096 / R.)
template <int LOGR>
constexpr int dd_w() { return LOGR >= 12 ? 1 : (1 << (12 - LOGR)); }
// R <= 4096: twiddles exp(dir 2 pi i t / R), t < R, from an LDS table
template <int LOGR>
constexpr bool dd_table() { return LOGR <= 12; }

// W instances of an R-point DFT.  Instance i = tile * W + w covers block
// beta = i / s, column b = i mod s; its point a is element beta Bp + a s + b.
// dir = -1: forward (exp(-2 pi i ...)), +1: inverse (exp(+...), unscaled).
// twid: forward, multiply output k by exp(-2 pi i b k / Bp) after the DFT;
// inverse, multiply input k by exp(+2 pi i b k / Bp) before it.
template <int LOGR>
__global__ __launch_bounds__(kDdThreads) void dd_fft_kernel(const float2 *in, float2 *out, int64_t L, int64_t Bp,
                                                            int dir, int twid) {
    constexpr int R = 1 << LOGR, W = dd_w<LOGR>(), RP = R + 1;
    extern __shared__ float2 dd_lds[];
    float2 *A = dd_lds, *B = dd_lds + W * RP, *tw = dd_lds + 2 * W * RP;
    const int tid = threadIdx.x;
    const int64_t s = Bp >> LOGR;
    const int64_t tile = blockIdx.x;
    const int64_t pol_off = (int64_t)blockIdx.y * L;
    const float2 *src = in + pol_off;
    float2 *dst = out + pol_off;
    const float sgn = (float)dir;

    // element (w, a) of the tile <-> global index.  With s > 1, W divides s
    // (both powers of two, s >= W), so the tile's W instances are adjacent
    // columns b0 + w of one block beta.
    const int64_t i0 = tile * W;
    const int64_t beta = s == 1 ? 0 : i0 / s, b0 = s == 1 ? 0 : i0 - beta * s;
    const int64_t base = s == 1 ? i0 * R : beta * Bp + b0;
    auto gidx = [&](int w, int a) -> int64_t {
        return s == 1 ? base + (int64_t)w * R + a : base + (int64_t)a * s + w;
    };
    auto colb = [&](int w) -> int64_t { return s == 1 ? 0 : b0 + w; };
    // exp(dir 2 pi i t / R)
    auto rot = [&](int t) -> float2 {
        if constexpr (dd_table<LOGR>()) {
            return tw[t & (R - 1)];
        } else {
            float sn, cs;
            sincospif(sgn * 2.0f * (float)(t & (R - 1)) / (float)R, &sn, &cs);
            return make_float2(cs, sn);
        }
    };
    if constexpr (dd_table<LOGR>()) {
        for (int t = tid; t < R; t += kDdThreads) {
            float sn, cs;
            sincospif(sgn * 2.0f * (float)t / (float)R, &sn, &cs);
            tw[t] = make_float2(cs, sn);
        }
    }

    // load (coalesced: s == 1 -> contiguous, else rows of W adjacent columns)
    for (int e = tid; e < W * R; e += kDdThreads) {
        int w, a;
        if (s == 1) { w = e >> LOGR; a = e & (R - 1); }
        else { w = e % W; a = e / W; }
        float2 v = src[gidx(w, a)];
        if (twid && dir > 0) {  // inverse: conjugate twiddle of input k = a first
            const int64_t bk = colb(w) * a;  // < s R = Bp
            float sn, cs;
            sincospif(2.0f * (float)((double)bk / (double)Bp), &sn, &cs);
            v = make_float2(v.x * cs - v.y * sn, v.x * sn + v.y * cs);
        }
        A[w * RP + a] = v;
    }
    __syncthreads();

    // Stockham stages (natural order in and out): one radix-2 stage when
    // log2 R is odd, then radix 4.  A radix-P stage with span ns reads
    // v_q = in[j + q R/P] (j < R/P), rotates v_q by exp(dir 2 pi i q k / (P ns)),
    // k = j mod ns, takes the P-point DFT V_r and writes
    // out[(j / ns) P ns + k + r ns] = V_r.
    float2 *X = A, *Y = B;
    if constexpr (LOGR & 1) {
        for (int e = tid; e < W * (R / 2); e += kDdThreads) {
            const int w = e / (R / 2), j = e % (R / 2);
            const float2 a = X[w * RP + j], b = X[w * RP + j + R / 2];
            Y[w * RP + 2 * j] = make_float2(a.x + b.x, a.y + b.y);
            Y[w * RP + 2 * j + 1] = make_float2(a.x - b.x, a.y - b.y);
        }
        __syncthreads();
        float2 *t = X;
        X = Y;
        Y = t;
    }
    if constexpr (LOGR >= 2) {
        constexpr int Q = R / 4;
#pragma unroll 1
        for (int lns = LOGR & 1; lns < LOGR; lns += 2) {  // span ns = 2^lns
            const int ns = 1 << lns;
            const int lstep = LOGR - 2 - lns;  // exp(dir 2 pi i k / (4 ns)) = rot(k << lstep)
            for (int e = tid; e < W * Q; e += kDdThreads) {
                const int w = e / Q, j = e % Q;
                const int k = j & (ns - 1);
                const float2 *x = X + w * RP;
                float2 v0 = x[j], v1 = x[j + Q], v2 = x[j + 2 * Q], v3 = x[j + 3 * Q];
                if (lns > 0) {
                    const int t = k << lstep;
                    const float2 w1 = rot(t), w2 = rot(2 * t), w3 = rot(3 * t);
                    v1 = make_float2(v1.x * w1.x - v1.y * w1.y, v1.x * w1.y + v1.y * w1.x);
                    v2 = make_float2(v2.x * w2.x - v2.y * w2.y, v2.x * w2.y + v2.y * w2.x);
                    v3 = make_float2(v3.x * w3.x - v3.y * w3.y, v3.x * w3.y + v3.y * w3.x);
                }
                // 4-point DFT with exp(dir 2 pi i q r / 4) = (dir i)^(q r)
                const float2 s02 = make_float2(v0.x + v2.x, v0.y + v2.y), d02 = make_float2(v0.x - v2.x, v0.y - v2.y);
                const float2 s13 = make_float2(v1.x + v3.x, v1.y + v3.y), d13 = make_float2(v1.x - v3.x, v1.y - v3.y);
                const float2 jd13 = make_float2(-sgn * d13.y, sgn * d13.x);  // (dir i) (v1 - v3)
                float2 *y = Y + w * RP + ((j >> lns) << (lns + 2)) + k;
                y[0] = make_float2(s02.x + s13.x, s02.y + s13.y);
                y[ns] = make_float2(d02.x + jd13.x, d02.y + jd13.y);
                y[2 * ns] = make_float2(s02.x - s13.x, s02.y - s13.y);
                y[3 * ns] = make_float2(d02.x - jd13.x, d02.y - jd13.y);
            }
            __syncthreads();
            float2 *t = X;
            X = Y;
            Y = t;
        }
    }

    // store (forward: twiddle of output k = a last)
    for (int e = tid; e < W * R; e += kDdThreads) {
        int w, a;
        if (s == 1) { w = e >> LOGR; a = e & (R - 1); }
        else { w = e % W; a = e / W; }
        float2 v = X[w * RP + a];
        if (twid && dir < 0) {
            const int64_t bk = colb(w) * a;  // < s R = Bp
            float sn, cs;
            sincospif(-2.0f * (float)((double)bk / (double)Bp), &sn, &cs);
            v = make_float2(v.x * cs - v.y * sn, v.x * sn + v.y * cs);
        }
        dst[gidx(w, a)] = v;
    }
}

// Inverse dispersion transfer function at every position of the forward
// transform's digit-reversed order, with the 1/L of the inverse transform.
__global__ __launch_bounds__(256) void dd_chirp_kernel(float2 *z, int64_t L, int lgL, DdPasses ps, double df,
                                                       double nu0, double kdm) {
    const int64_t P = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (P >= L) return;
    // position -> frequency index: digits of the passes, first pass least significant
    int64_t k = 0, rem = P;
    int sh = lgL, mult = 0;
    for (int j = 0; j < ps.n; ++j) {
        sh -= ps.lr[j];
        const int64_t digit = rem >> sh;
        rem &= ((int64_t)1 << sh) - 1;
        k += digit << mult;
        mult += ps.lr[j];
    }
    const double f = (double)k * df;
    double c = kdm * f * f / (nu0 * nu0 * (nu0 + f));
    c -= floor(c);
    float sn, cs;
    sincospif(-2.0f * (float)c, &sn, &cs);
    const float inv = 1.0f / (float)L;
    const int64_t off = (int64_t)blockIdx.y * L + P;
    const float2 v = z[off];
    z[off] = make_float2(inv * (v.x * cs - v.y * sn), inv * (v.x * sn + v.y * cs));
}

// I[j] = sum over polarisations and the n_int samples of bin j of |z|^2.
__global__ __launch_bounds__(256) void dd_detect_kernel(const float2 *z, int npol, int64_t L, int n_int,
                                                        float *out) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= L / n_int) return;
    float acc = 0.f;
    for (int p = 0; p < npol; ++p) {
        const float2 *r = z + (int64_t)p * L + j * n_int;
        for (int i = 0; i < n_int; ++i) acc += r[i].x * r[i].x + r[i].y * r[i].y;
    }
    out[j] = acc;
}

template <int LOGR>
hipError_t dd_fft(const float2 *in, float2 *out, int npol, int64_t L, int64_t Bp, int dir, int twid,
                  hipStream_t st) {
    constexpr int R = 1 << LOGR, W = dd_w<LOGR>();
    const size_t lds = sizeof(float2) * (2 * W * (R + 1) + (dd_table<LOGR>() ? R : 0));
    static bool attr = false;  // per process: raise the dynamic LDS limit once
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void *)dd_fft_kernel<LOGR>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    const dim3 grid((unsigned)(L / ((int64_t)R * W)), (unsigned)npol);
    hipLaunchKernelGGL(dd_fft_kernel<LOGR>, grid, dim3(kDdThreads), lds, st, in, out, L, Bp, dir, twid);
    return hipGetLastError();
}

hipError_t dd_fft_any(int lr, const float2 *in, float2 *out, int npol, int64_t L, int64_t Bp, int dir, int twid,
                      hipStream_t st) {
    switch (lr) {
    case 1: return dd_fft<1>(in, out, npol, L, Bp, dir, twid, st);
    case 2: return dd_fft<2>(in, out, npol, L, Bp, dir, twid, st);
    case 3: return dd_fft<3>(in, out, npol, L, Bp, dir, twid, st);
    case 4: return dd_fft<4>(in, out, npol, L, Bp, dir, twid, st);
    case 5: return dd_fft<5>(in, out, npol, L, Bp, dir, twid, st);
    case 6: return dd_fft<6>(in, out, npol, L, Bp, dir, twid, st);
    case 7: return dd_fft<7>(in, out, npol, L, Bp, dir, twid, st);
    case 8: return dd_fft<8>(in, out, npol, L, Bp, dir, twid, st);
    case 9: return dd_fft<9>(in, out, npol, L, Bp, dir, twid, st);
    case 10: return dd_fft<10>(in, out, npol, L, Bp, dir, twid, st);
    case 11: return dd_fft<11>(in, out, npol, L, Bp, dir, twid, st);
    case 12: return dd_fft<12>(in, out, npol, L, Bp, dir, twid, st);
    case 13: return dd_fft<13>(in, out, npol, L, Bp, dir, twid, st);
    default: return hipErrorInvalidValue;
    }
}

thread_local char g_dd_err[512];

corr_status dd_fail(corr_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_dd_err, sizeof(g_dd_err), fmt, ap);
    va_end(ap);
    return st;
}

int ilog2(int64_t v) {
    int r = 0;
    while (((int64_t)1 << r) < v) ++r;
    return r;
}

}  // namespace

extern "C" {

size_t corr_dedisperse_workspace_bytes(int32_t npol, int64_t T, int32_t C) {
    if (npol < 1 || T < 1 || C < 1) return 0;
    return sizeof(float) * 2 * (size_t)npol * (size_t)T * (size_t)C;
}

corr_status corr_dedisperse(const float *d_v, int32_t npol, int64_t T, int32_t C, double sample_rate, double nu0,
                            double dm, int32_t n_int, float *d_work, float *d_out, void *stream) {
    g_dd_err[0] = 0;
    if (!d_v || !d_work || !d_out) return dd_fail(CORR_ERR_NULL, "d_v, d_work and d_out are required");
    if (((uintptr_t)d_v & 7) || ((uintptr_t)d_work & 7) || ((uintptr_t)d_out & 3))
        return dd_fail(CORR_ERR_ALIGN, "d_v and d_work 8-byte, d_out 4-byte alignment");
    if (npol < 1 || npol > 2) return dd_fail(CORR_ERR_INVALID, "npol=%d must be 1 or 2", npol);
    if (C < 16 || C > 8192 || (C & (C - 1))) return dd_fail(CORR_ERR_INVALID, "C=%d must be a power of two in [16, 8192]", C);
    if (T < 1 || (T & (T - 1))) return dd_fail(CORR_ERR_INVALID, "T=%lld must be a power of two", (long long)T);
    const int64_t L = T * (int64_t)C;
    if (L < 4096 || L > ((int64_t)1 << 28))
        return dd_fail(CORR_ERR_INVALID, "T*C=%lld outside [4096, 2^28]", (long long)L);
    if (n_int < 1 || (n_int & (n_int - 1)) || n_int > L)
        return dd_fail(CORR_ERR_INVALID, "n_int=%d must be a power of two <= T*C", n_int);
    if (!(sample_rate > 0) || !std::isfinite(sample_rate) || !(nu0 > 0) || !std::isfinite(nu0) || !(dm >= 0) ||
        !std::isfinite(dm))
        return dd_fail(CORR_ERR_INVALID, "sample_rate and nu0 must be finite and > 0, dm finite and >= 0");
    if ((const void *)d_v == (const void *)d_work) return dd_fail(CORR_ERR_INVALID, "d_v and d_work must differ");
    hipStream_t st = (hipStream_t)stream;
    const float2 *v = reinterpret_cast<const float2 *>(d_v);
    float2 *z = reinterpret_cast<float2 *>(d_work);
    // 1. broadband series: inverse C-point DFT of every spectrum
    hipError_t e = dd_fft_any(ilog2(C), v, z, npol, L, C, +1, 0, st);
    // 2. forward transform over the block: a small radix first, then radix 256
    const int lgL = ilog2(L);
    DdPasses ps{};
    if (lgL % 8) ps.lr[ps.n++] = lgL % 8;
    for (int i = 0; i < lgL / 8; ++i) ps.lr[ps.n++] = 8;
    int64_t Bp = L;
    int64_t bps[kDdMaxPasses];
    for (int j = 0; j < ps.n && e == hipSuccess; ++j) {
        bps[j] = Bp;
        e = dd_fft_any(ps.lr[j], z, z, npol, L, Bp, -1, 1, st);
        Bp >>= ps.lr[j];
    }
    // 3. inverse dispersion transfer function (and 1/L)
    if (e == hipSuccess) {
        hipLaunchKernelGGL(dd_chirp_kernel, dim3((unsigned)((L + 255) / 256), (unsigned)npol), dim3(256), 0, st, z, L,
                           lgL, ps, sample_rate / (2.0 * (double)L), nu0, kDmConst * dm);
        e = hipGetLastError();
    }
    // 4. inverse transform, passes in reverse order
    for (int j = ps.n - 1; j >= 0 && e == hipSuccess; --j) e = dd_fft_any(ps.lr[j], z, z, npol, L, bps[j], +1, 1, st);
    // 5. detection, both polarisations, n_int samples per output
    if (e == hipSuccess) {
        const int64_t nout = L / n_int;
        hipLaunchKernelGGL(dd_detect_kernel, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, st, z, npol, L, n_int,
                           d_out);
        e = hipGetLastError();
    }
    return e == hipSuccess ? CORR_OK : dd_fail(CORR_ERR_DEVICE, "dedispersion launch: %s", hipGetErrorString(e));
}

const char *corr_dedisperse_last_error(void) { return g_dd_err; }

}  // extern "C"
