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
// One kernel does all the transforms: a workgroup of 256 threads takes W
// instances of an R-point DFT (a tile of max(4096, R) points), each thread
// 16 (32 at R = 8192) points in registers.  The DFT is a Stockham sequence of
// radix-16 stages (a radix-2/4/8 stage first when log2 R is not a multiple of
// 4), each an in-register DFT after a twiddle; stages exchange points through
// one LDS buffer (one pad per 16 points), the first reads global memory and
// the last writes it.  The per-spectrum inverse DFT is that kernel with
// R = C.  The long transform is a sequence of passes of a
// decimation-in-frequency decomposition: pass j splits blocks of Bp samples
// into R_j strided sub-sequences (stride s = Bp / R_j), takes their R_j-point
// DFTs and multiplies output k of column b by exp(-2 pi i b k / Bp).  A small
// radix goes first and then radix 256, so the stride is either >= the tile
// width (a tile is 4096 / R adjacent columns: rows of at least 128 bytes) or
// 1 (a tile is contiguous).  The result is in digit-reversed order.  The last
// forward pass (blocks of 256, contiguous) also multiplies each position by
// the transfer function at its frequency and takes the inverse DFT of the
// same tile; the remaining inverse passes (the mirror image: conjugate
// twiddle, then the inverse DFT, in reverse order) restore time order.  All
// passes run in place: a workgroup reads its whole tile before it writes it
// back.

#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <type_traits>

#include "corr_internal.h"

namespace {

constexpr int kDdThreads = 256;
constexpr double kDmConst = 4.148808e15;  // Hz^2 s / (pc cm^-3): delay = K DM / nu^2
constexpr int kDdMaxPasses = 8;
// corr_dedisperse_noalloc: complex samples of its device scratch array (32 MiB)
// and the devices it keeps that array's address for
constexpr int64_t kDdScratchSamples = (int64_t)1 << 22;
constexpr int kDdMaxDevices = 64;

struct DdPasses {
    int n;                     // number of passes of the long transform
    int lr[kDdMaxPasses];      // log2 radix of each pass, in forward order
};

// Shape of one R-point transform kernel: a tile of max(4096, R) points
// (W instances), 256 threads, NPT points per thread in registers.  Stages:
// radix 2^LREM first when log2 R is not a multiple of 4, then radix 16.
template <int LOGR>
struct DdShape {
    static constexpr int R = 1 << LOGR;
    static constexpr int TILE = R > 4096 ? R : 4096;
    static constexpr int W = TILE / R;
    static constexpr int NPT = TILE / kDdThreads;
    static constexpr int LREM = LOGR % 4;
    static constexpr int NST = LOGR / 4 + (LREM ? 1 : 0);
    static constexpr int RP = R + R / 16 + 1;  // LDS row pitch (float2): one pad per 16, plus one
    static constexpr size_t lds_bytes = NST > 1 ? sizeof(float2) * W * RP : 0;
};

// radix and log2 span (ns = 2^LNS: product of the earlier radices) of stage ST
template <int LOGR, int ST>
struct DdStage {
    static constexpr int LREM = DdShape<LOGR>::LREM;
    static constexpr int LP = (ST == 0 && LREM) ? LREM : 4;
    static constexpr int P = 1 << LP;
    static constexpr int LNS = ST == 0 ? 0 : (LREM ? LREM : 4) + 4 * (ST - 1);
    static constexpr int Q = (1 << LOGR) / P;  // butterflies per instance
    static constexpr int NB = DdShape<LOGR>::NPT / P;  // butterflies per thread
};

__device__ inline float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// (SG i) a
template <int SG>
__device__ inline float2 cjmul(float2 a) { return SG > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x); }
__device__ inline float2 cis_turns(float t) {  // exp(2 pi i t)
    float sn, cs;
    sincospif(2.0f * t, &sn, &cs);
    return make_float2(cs, sn);
}

// In-register P-point DFT, X_r = sum_q x_q exp(SG 2 pi i q r / P), natural
// order in and out.  P = 8 and 16 are 2 x 4 and 4 x 4 (index n = n1 + m n2,
// k = k2 + 4 k1, inner twiddle exp(SG 2 pi i n1 k2 / P)).
template <int SG>
__device__ inline void dft4(float2 &x0, float2 &x1, float2 &x2, float2 &x3) {
    const float2 s02 = cadd(x0, x2), d02 = csub(x0, x2), s13 = cadd(x1, x3), j13 = cjmul<SG>(csub(x1, x3));
    x0 = cadd(s02, s13);
    x1 = cadd(d02, j13);
    x2 = csub(s02, s13);
    x3 = csub(d02, j13);
}
template <int P, int SG>
__device__ inline void dft(float2 *x) {
    if constexpr (P == 2) {
        const float2 a = x[0], b = x[1];
        x[0] = cadd(a, b);
        x[1] = csub(a, b);
    } else if constexpr (P == 4) {
        dft4<SG>(x[0], x[1], x[2], x[3]);
    } else if constexpr (P == 8) {
        constexpr float h = 0.70710678118654752f;  // cos(pi/4)
        dft4<SG>(x[0], x[2], x[4], x[6]);
        dft4<SG>(x[1], x[3], x[5], x[7]);
        // y1[k2] *= exp(SG 2 pi i k2 / 8)
        x[3] = cmul(x[3], make_float2(h, SG * h));
        x[5] = cjmul<SG>(x[5]);
        x[7] = cmul(x[7], make_float2(-h, SG * h));
        float2 y[8];
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            y[k2] = cadd(x[2 * k2], x[2 * k2 + 1]);
            y[k2 + 4] = csub(x[2 * k2], x[2 * k2 + 1]);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = y[k];
    } else {
        static_assert(P == 16, "radix 2, 4, 8 or 16");
        constexpr float c1 = 0.92387953251128676f, s1 = 0.38268343236508977f, h = 0.70710678118654752f;
        // y_{n1}[k2] = DFT4 over n2 of x[n1 + 4 n2], held in x[n1 + 4 k2]
#pragma unroll
        for (int n1 = 0; n1 < 4; ++n1) dft4<SG>(x[n1], x[n1 + 4], x[n1 + 8], x[n1 + 12]);
        // twiddles exp(SG 2 pi i m / 16), m = n1 k2
        x[5] = cmul(x[5], make_float2(c1, SG * s1));     // m = 1
        x[9] = cmul(x[9], make_float2(h, SG * h));       // 2
        x[13] = cmul(x[13], make_float2(s1, SG * c1));   // 3
        x[6] = cmul(x[6], make_float2(h, SG * h));       // 2
        x[10] = cjmul<SG>(x[10]);                        // 4
        x[14] = cmul(x[14], make_float2(-h, SG * h));    // 6
        x[7] = cmul(x[7], make_float2(s1, SG * c1));     // 3
        x[11] = cmul(x[11], make_float2(-h, SG * h));    // 6
        x[15] = cmul(x[15], make_float2(-c1, -SG * s1)); // 9
        // X[k2 + 4 k1] = DFT4 over n1 of x[n1 + 4 k2]
        float2 y[16];
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) {
            float2 a = x[4 * k2], b = x[4 * k2 + 1], c = x[4 * k2 + 2], d = x[4 * k2 + 3];
            dft4<SG>(a, b, c, d);
            y[k2] = a;
            y[k2 + 4] = b;
            y[k2 + 8] = c;
            y[k2 + 12] = d;
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) x[k] = y[k];
    }
}

// LDS position of point a of instance w: one pad per 16 points
__device__ inline int dd_pad(int w, int a, int rp) { return w * rp + a + (a >> 4); }

// The inverse dispersion transfer function with the 1/L of the inverse
// transform, at frequency index k (f = k df).  Position P of the forward
// transform's digit-reversed order holds frequency index: the digits of the
// passes, the first pass's least significant.
struct DdChirp {
    DdPasses ps;
    int lgL;
    double df, nu0, kdm_nu0sq;  // kdm_nu0sq = K DM / nu0^2
    float inv_l;
};
__device__ inline int64_t dd_freq_index(const DdChirp &c, int64_t P) {
    int64_t k = 0, rem = P;
    int sh = c.lgL, mult = 0;
    for (int j = 0; j < c.ps.n; ++j) {
        sh -= c.ps.lr[j];
        const int64_t digit = rem >> sh;
        rem &= ((int64_t)1 << sh) - 1;
        k += digit << mult;
        mult += c.ps.lr[j];
    }
    return k;
}
__device__ inline float2 dd_chirp_at(const DdChirp &c, int64_t k) {
    const double f = (double)k * c.df;
    double ph = c.kdm_nu0sq * f * f / (c.nu0 + f);
    ph -= floor(ph);
    const float2 e = cis_turns(-(float)ph);
    return make_float2(c.inv_l * e.x, c.inv_l * e.y);
}

// One thread's butterflies in a stage: butterfly i is b = tid + 256 i, at
// instance w, index j < Q.  Contiguous instances (s == 1) put j fastest
// across the lanes, strided ones put w (adjacent columns) fastest, so that
// the global loads and stores of the first and last stages are coalesced.
template <int LOGR, int ST>
__device__ inline void dd_bf(int i, bool contig, int &w, int &j) {
    using S = DdStage<LOGR, ST>;
    const int b = threadIdx.x + kDdThreads * i;
    if (contig) {
        w = b / S::Q;
        j = b % S::Q;
    } else {
        w = b % DdShape<LOGR>::W;
        j = b / DdShape<LOGR>::W;
    }
}

// stage ST on registers: twiddle exp(SG 2 pi i q k / (P ns)), k = j mod ns, then the P-point DFT
template <int LOGR, int ST, int SG>
__device__ inline void dd_stage(float2 *v, bool contig) {
    using S = DdStage<LOGR, ST>;
#pragma unroll
    for (int i = 0; i < S::NB; ++i) {
        float2 *x = v + i * S::P;
        if constexpr (S::LNS > 0) {
            static_assert(S::P == 16, "twiddled stages are radix 16");
            int w, j;
            dd_bf<LOGR, ST>(i, contig, w, j);
            const int k = j & ((1 << S::LNS) - 1);
            const float t = (float)(SG * k) * (1.0f / (float)(16 << S::LNS));  // exact
            const float2 w1 = cis_turns(t), w4 = cis_turns(4.0f * t);
            const float2 w2 = cmul(w1, w1), w3 = cmul(w2, w1), w8 = cmul(w4, w4), w12 = cmul(w8, w4);
            const float2 lo[4] = {make_float2(1.f, 0.f), w1, w2, w3};
            const float2 hi[4] = {make_float2(1.f, 0.f), w4, w8, w12};
#pragma unroll
            for (int q = 1; q < 16; ++q) {
                const float2 tw = (q & 3) == 0 ? hi[q >> 2] : (q >> 2) == 0 ? lo[q & 3] : cmul(hi[q >> 2], lo[q & 3]);
                x[q] = cmul(x[q], tw);
            }
        }
        dft<S::P, SG>(x);
    }
}

template <int LOGR, int ST>
__device__ inline void dd_read_lds(float2 *v, const float2 *X, bool contig) {
    using S = DdStage<LOGR, ST>;
#pragma unroll
    for (int i = 0; i < S::NB; ++i) {
        int w, j;
        dd_bf<LOGR, ST>(i, contig, w, j);
#pragma unroll
        for (int q = 0; q < S::P; ++q) v[i * S::P + q] = X[dd_pad(w, j + q * S::Q, DdShape<LOGR>::RP)];
    }
}

// Stockham write: output r of butterfly (w, j) goes to (j / ns) P ns + k + r ns
template <int LOGR, int ST>
__device__ inline void dd_write_lds(const float2 *v, float2 *X, bool contig) {
    using S = DdStage<LOGR, ST>;
#pragma unroll
    for (int i = 0; i < S::NB; ++i) {
        int w, j;
        dd_bf<LOGR, ST>(i, contig, w, j);
        const int o = ((j >> S::LNS) << (S::LNS + S::LP)) + (j & ((1 << S::LNS) - 1));
#pragma unroll
        for (int r = 0; r < S::P; ++r) X[dd_pad(w, o + (r << S::LNS), DdShape<LOGR>::RP)] = v[i * S::P + r];
    }
}

// exp(SG 2 pi i (base + r m) / Bp) for r < P, with base, m integers: three
// sincos and products (at most two per factor)
template <int P, int SG>
__device__ inline void dd_ramp(int64_t base, int64_t m, int64_t Bp, float inv_bp, float2 *t) {
    const int64_t msk = Bp - 1;
    const float2 u = cis_turns((float)SG * (float)(base & msk) * inv_bp);
    const float2 m1 = cis_turns((float)SG * (float)(m & msk) * inv_bp);
    const float2 m4 = cis_turns((float)SG * (float)((4 * m) & msk) * inv_bp);
    const float2 m2 = cmul(m1, m1), m3 = cmul(m2, m1), m8 = cmul(m4, m4), m12 = cmul(m8, m4);
    const float2 lo[4] = {u, cmul(u, m1), cmul(u, m2), cmul(u, m3)};
    const float2 hi[4] = {make_float2(1.f, 0.f), m4, m8, m12};
#pragma unroll
    for (int r = 0; r < P; ++r) t[r] = (r >> 2) == 0 ? lo[r & 3] : cmul(hi[r >> 2], lo[r & 3]);
}

// W instances of an R-point DFT per workgroup.  Instance i = tile W + w
// covers block beta = i / s, column b = i mod s (s = Bp / R); its point a is
// element beta Bp + a s + b.
// MODE 0, forward (exp(-2 pi i ...)): the DFT, then output k of column b
//   times exp(-2 pi i b k / Bp).
// MODE 1, inverse (exp(+...), unscaled): input k times exp(+2 pi i b k / Bp),
//   then the DFT.
// MODE 2 (R = Bp = 256): the forward DFT, the dispersion chirp and 1/L at the
//   forward transform's position, then the inverse DFT, on one tile.
template <int LOGR, int MODE>
__global__ __launch_bounds__(kDdThreads) void dd_fft_kernel(const float2 *in, float2 *out, int64_t L, int64_t Bp,
                                                            DdChirp ch) {
    using Sh = DdShape<LOGR>;
    constexpr int R = Sh::R, W = Sh::W, NST = Sh::NST, LAST = NST - 1;
    using S0 = DdStage<LOGR, 0>;
    using SL = DdStage<LOGR, LAST>;
    static_assert(MODE != 2 || (LOGR == 8 && S0::P == SL::P), "fused pass: radix 16 x 16");
    constexpr int SG0 = MODE == 1 ? 1 : -1;
    extern __shared__ float2 dd_lds[];
    const int64_t s = Bp >> LOGR;
    const bool contig = s == 1;
    const int64_t i0 = (int64_t)blockIdx.x * W;
    const int64_t beta = contig ? 0 : i0 / s, b0 = contig ? 0 : i0 - beta * s;
    const int64_t base = contig ? i0 * R : beta * Bp + b0;
    const int64_t pol_off = (int64_t)blockIdx.y * L;
    const float2 *src = in + pol_off;
    float2 *dst = out + pol_off;
    const float inv_bp = 1.0f / (float)Bp;  // Bp is a power of two
    auto gidx = [&](int w, int a) -> int64_t {
        return contig ? base + (int64_t)w * R + a : base + (int64_t)a * s + w;
    };

    float2 v[Sh::NPT];
    // stage 0 inputs from global memory (inverse: the conjugate pass twiddle)
#pragma unroll
    for (int i = 0; i < S0::NB; ++i) {
        int w, j;
        dd_bf<LOGR, 0>(i, contig, w, j);
#pragma unroll
        for (int q = 0; q < S0::P; ++q) v[i * S0::P + q] = src[gidx(w, j + q * S0::Q)];
        if (MODE == 1 && !contig) {
            float2 t[S0::P];
            dd_ramp<S0::P, 1>((b0 + w) * j, (b0 + w) * S0::Q, Bp, inv_bp, t);
#pragma unroll
            for (int q = 0; q < S0::P; ++q) v[i * S0::P + q] = cmul(v[i * S0::P + q], t[q]);
        }
    }
    auto run = [&](auto sg_tag) {
        constexpr int SG = decltype(sg_tag)::value;
        dd_stage<LOGR, 0, SG>(v, contig);
        if constexpr (NST > 1) {
            dd_write_lds<LOGR, 0>(v, dd_lds, contig);
            __syncthreads();
            if constexpr (NST > 2) {
                dd_read_lds<LOGR, 1>(v, dd_lds, contig);
                dd_stage<LOGR, 1, SG>(v, contig);
                __syncthreads();
                dd_write_lds<LOGR, 1>(v, dd_lds, contig);
                __syncthreads();
            }
            if constexpr (NST > 3) {
                dd_read_lds<LOGR, 2>(v, dd_lds, contig);
                dd_stage<LOGR, 2, SG>(v, contig);
                __syncthreads();
                dd_write_lds<LOGR, 2>(v, dd_lds, contig);
                __syncthreads();
            }
            static_assert(NST <= 4, "at most four stages (R <= 2^13)");
            dd_read_lds<LOGR, LAST>(v, dd_lds, contig);
            dd_stage<LOGR, LAST, SG>(v, contig);
        }
    };
    run(std::integral_constant<int, SG0>{});
    if constexpr (MODE == 2) {
        // chirp at the forward transform's positions (this pass's digit, the
        // point index within the instance, is the frequency index's most
        // significant), then the inverse on the same registers
#pragma unroll
        for (int i = 0; i < SL::NB; ++i) {
            int w, j;
            dd_bf<LOGR, LAST>(i, contig, w, j);
            const int64_t k0 = dd_freq_index(ch, gidx(w, 0));
#pragma unroll
            for (int r = 0; r < SL::P; ++r)
                v[i * SL::P + r] =
                    cmul(v[i * SL::P + r], dd_chirp_at(ch, k0 + ((int64_t)(j + r * SL::Q) << (ch.lgL - LOGR))));
        }
        __syncthreads();  // the forward's last LDS reads are done
        run(std::integral_constant<int, 1>{});
    }
    // last stage outputs to global memory (forward: the pass twiddle)
#pragma unroll
    for (int i = 0; i < SL::NB; ++i) {
        int w, j;
        dd_bf<LOGR, LAST>(i, contig, w, j);
        if (MODE == 0 && !contig) {
            float2 t[SL::P];
            dd_ramp<SL::P, -1>((b0 + w) * j, (b0 + w) * SL::Q, Bp, inv_bp, t);
#pragma unroll
            for (int r = 0; r < SL::P; ++r) v[i * SL::P + r] = cmul(v[i * SL::P + r], t[r]);
        }
#pragma unroll
        for (int r = 0; r < SL::P; ++r) dst[gidx(w, j + r * SL::Q)] = v[i * SL::P + r];
    }
}

// I[j] = sum over polarisations and the n_int samples of bin j of |z|^2.
// G = min(n_int, 64) adjacent lanes share a bin (lane l sums samples l, l + G,
// ...), so a wave reads 64 consecutive samples at a time, then a butterfly
// reduction over the G lanes.
__global__ __launch_bounds__(256) void dd_detect_kernel(const float2 *z, int npol, int64_t L, int n_int, int lg_g,
                                                        float *out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int G = 1 << lg_g;
    const int64_t j = t >> lg_g;
    const int l = (int)(t & (G - 1));
    const bool live = j < L / n_int;
    float acc = 0.f;
    if (live) {
        for (int p = 0; p < npol; ++p) {
            const float2 *r = z + (int64_t)p * L + j * n_int;
#pragma unroll 4
            for (int i = l; i < n_int; i += G) acc += r[i].x * r[i].x + r[i].y * r[i].y;
        }
    }
    for (int m = G >> 1; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if (live && l == 0) out[j] = acc;
}

template <int LOGR, int MODE>
hipError_t dd_fft(const float2 *in, float2 *out, int npol, int64_t L, int64_t Bp, const DdChirp &ch, hipStream_t st) {
    using Sh = DdShape<LOGR>;
    if constexpr (Sh::lds_bytes > 65536) {  // above the default dynamic LDS limit (R = 8192 only)
        // set on every call: no process-wide state, right for whichever device is current
        hipError_t e = hipFuncSetAttribute((const void *)dd_fft_kernel<LOGR, MODE>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)Sh::lds_bytes);
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)(L / Sh::TILE), (unsigned)npol);
    hipLaunchKernelGGL((dd_fft_kernel<LOGR, MODE>), grid, dim3(kDdThreads), Sh::lds_bytes, st, in, out, L, Bp, ch);
    return hipGetLastError();
}

template <int MODE>
hipError_t dd_fft_mode(int lr, const float2 *in, float2 *out, int npol, int64_t L, int64_t Bp, const DdChirp &ch,
                       hipStream_t st) {
    switch (lr) {
    case 1: return dd_fft<1, MODE>(in, out, npol, L, Bp, ch, st);
    case 2: return dd_fft<2, MODE>(in, out, npol, L, Bp, ch, st);
    case 3: return dd_fft<3, MODE>(in, out, npol, L, Bp, ch, st);
    case 4: return dd_fft<4, MODE>(in, out, npol, L, Bp, ch, st);
    case 5: return dd_fft<5, MODE>(in, out, npol, L, Bp, ch, st);
    case 6: return dd_fft<6, MODE>(in, out, npol, L, Bp, ch, st);
    case 7: return dd_fft<7, MODE>(in, out, npol, L, Bp, ch, st);
    case 8: return dd_fft<8, MODE>(in, out, npol, L, Bp, ch, st);
    case 9: return dd_fft<9, MODE>(in, out, npol, L, Bp, ch, st);
    case 10: return dd_fft<10, MODE>(in, out, npol, L, Bp, ch, st);
    case 11: return dd_fft<11, MODE>(in, out, npol, L, Bp, ch, st);
    case 12: return dd_fft<12, MODE>(in, out, npol, L, Bp, ch, st);
    case 13: return dd_fft<13, MODE>(in, out, npol, L, Bp, ch, st);
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

// Argument checks shared by both entry points (everything but the work buffer).
static corr_status dd_check(const float *d_v, int32_t npol, int64_t T, int32_t C, double sample_rate, double nu0,
                            double dm, int32_t n_int, float *d_out) {
    if (!d_v || !d_out) return dd_fail(CORR_ERR_NULL, "d_v and d_out are required");
    if (((uintptr_t)d_v & 7) || ((uintptr_t)d_out & 3)) return dd_fail(CORR_ERR_ALIGN, "d_v 8-byte, d_out 4-byte alignment");
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
    return CORR_OK;
}

// The transforms and the detection on a work buffer z of npol T C complex samples.
static corr_status dd_run(const float *d_v, int32_t npol, int64_t T, int32_t C, double sample_rate, double nu0,
                          double dm, int32_t n_int, float2 *z, float *d_out, hipStream_t st) {
    const int64_t L = T * (int64_t)C;
    const float2 *v = reinterpret_cast<const float2 *>(d_v);
    // 1. broadband series: inverse C-point DFT of every spectrum
    const int lgL = ilog2(L);
    DdChirp ch{};
    if (lgL % 8) ch.ps.lr[ch.ps.n++] = lgL % 8;
    for (int i = 0; i < lgL / 8; ++i) ch.ps.lr[ch.ps.n++] = 8;
    ch.lgL = lgL;
    ch.df = sample_rate / (2.0 * (double)L);
    ch.nu0 = nu0;
    ch.kdm_nu0sq = kDmConst * dm / (nu0 * nu0);
    ch.inv_l = 1.0f / (float)L;
    hipError_t e = dd_fft_mode<1>(ilog2(C), v, z, npol, L, C, ch, st);
    // 2. forward transform over the block: a small radix first, then radix
    // 256; the last pass (blocks of 256) also applies the inverse dispersion
    // transfer function and starts the inverse transform: 3. the inverse
    // passes, in reverse order
    const DdPasses &ps = ch.ps;
    int64_t Bp = L;
    int64_t bps[kDdMaxPasses];
    for (int j = 0; j < ps.n - 1 && e == hipSuccess; ++j) {
        bps[j] = Bp;
        e = dd_fft_mode<0>(ps.lr[j], z, z, npol, L, Bp, ch, st);
        Bp >>= ps.lr[j];
    }
    if (e == hipSuccess) e = dd_fft<8, 2>(z, z, npol, L, Bp, ch, st);  // Bp == 256 here
    for (int j = ps.n - 2; j >= 0 && e == hipSuccess; --j) e = dd_fft_mode<1>(ps.lr[j], z, z, npol, L, bps[j], ch, st);
    // 5. detection, both polarisations, n_int samples per output
    if (e == hipSuccess) {
        const int lg_g = ilog2(n_int < 64 ? n_int : 64);
        const int64_t nthr = (L / n_int) << lg_g;
        hipLaunchKernelGGL(dd_detect_kernel, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, st, z, npol, L, n_int,
                           lg_g, d_out);
        e = hipGetLastError();
    }
    return e == hipSuccess ? CORR_OK : dd_fail(CORR_ERR_DEVICE, "dedispersion launch: %s", hipGetErrorString(e));
}

// Work buffer of corr_dedisperse_noalloc: a file-scope device array, one copy on
// every GPU the library runs on, held until the process ends.  Host code reaches
// each device's copy only through the address hipGetSymbolAddress returns there.
static __device__ __align__(256) float2 dd_scratch[kDdScratchSamples];
static std::mutex g_dd_scratch_mu;
static float2 *g_dd_scratch_at[kDdMaxDevices];

// This device's address of dd_scratch (looked up once per device, with it current).
static corr_status dd_scratch_ptr(float2 **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return dd_fail(CORR_ERR_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kDdMaxDevices) return dd_fail(CORR_ERR_UNSUPPORTED, "device %d beyond %d", dev, kDdMaxDevices);
    std::lock_guard<std::mutex> lock(g_dd_scratch_mu);
    if (!g_dd_scratch_at[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(dd_scratch));
        if (e != hipSuccess || !p)
            return dd_fail(CORR_ERR_DEVICE, "hipGetSymbolAddress(dd_scratch): %s", hipGetErrorString(e));
        g_dd_scratch_at[dev] = static_cast<float2 *>(p);
    }
    *out = g_dd_scratch_at[dev];
    return CORR_OK;
}

extern "C" {

size_t corr_dedisperse_workspace_bytes(int32_t npol, int64_t T, int32_t C) {
    if (npol < 1 || T < 1 || C < 1) return 0;
    return sizeof(float) * 2 * (size_t)npol * (size_t)T * (size_t)C;
}

corr_status corr_dedisperse(const float *d_v, int32_t npol, int64_t T, int32_t C, double sample_rate, double nu0,
                            double dm, int32_t n_int, float *d_work, float *d_out, void *stream) {
    g_dd_err[0] = 0;
    if (!d_work) return dd_fail(CORR_ERR_NULL, "d_v, d_work and d_out are required");
    if ((uintptr_t)d_work & 7) return dd_fail(CORR_ERR_ALIGN, "d_v and d_work 8-byte, d_out 4-byte alignment");
    corr_status cs = dd_check(d_v, npol, T, C, sample_rate, nu0, dm, n_int, d_out);
    if (cs != CORR_OK) return cs;
    if ((const void *)d_v == (const void *)d_work) return dd_fail(CORR_ERR_INVALID, "d_v and d_work must differ");
    return dd_run(d_v, npol, T, C, sample_rate, nu0, dm, n_int, reinterpret_cast<float2 *>(d_work), d_out,
                  (hipStream_t)stream);
}

corr_status corr_dedisperse_noalloc(const float *d_v, int32_t npol, int64_t T, int32_t C, double sample_rate,
                                    double nu0, double dm, int32_t n_int, float *d_out, void *stream) {
    g_dd_err[0] = 0;
    corr_status cs = dd_check(d_v, npol, T, C, sample_rate, nu0, dm, n_int, d_out);
    if (cs != CORR_OK) return cs;
    if ((int64_t)npol * T * (int64_t)C > kDdScratchSamples)
        return dd_fail(CORR_ERR_INVALID, "npol*T*C=%lld exceeds the no-allocation limit of %lld samples",
                       (long long)((int64_t)npol * T * (int64_t)C), (long long)kDdScratchSamples);
    float2 *z = nullptr;
    if ((cs = dd_scratch_ptr(&z)) != CORR_OK) return cs;
    return dd_run(d_v, npol, T, C, sample_rate, nu0, dm, n_int, z, d_out, (hipStream_t)stream);
}

const char *corr_dedisperse_last_error(void) { return g_dd_err; }

}  // extern "C"
