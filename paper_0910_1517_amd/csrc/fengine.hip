// fengine.hip -- F-engine of the FX correlator for gfx950.
//
// One workgroup owns one signal s and 16*FPAR consecutive spectra; FPAR
// independent thread groups of L = M/8 threads (M = N/2) each transform 16
// spectra, one at a time:
//
//  1. integer delay (section 2.1, block shift; section 2.3.2, read-pointer
//     offset into the overlapped slice): the window m of signal s is the N
//     bytes at m*N + D_s of its row.  Each thread fetches 16 consecutive bytes
//     with aligned dword loads and a byte funnel shift, so the global reads
//     are coalesced whatever D_s is, and stages them in LDS.
//  2. real-to-complex FFT (section 2.1; section 3.1 uses a real FFT): the N
//     real samples are packed as M complex points z[n] = x[2n] + i x[2n+1] and
//     transformed by a Stockham autosort FFT, radix-8 passes plus one radix-4
//     or radix-2 pass, every thread holding 8 points in registers and the
//     passes exchanging through LDS (ping-pong buffers, one barrier per pass;
//     one pad element per 16 keeps the passes free of bank conflicts).
//     The half-length trick X[k] = E[k] + W_N^k O[k] recovers channels
//     k = 0..M-1 (DC kept, Nyquist dropped).  Twiddles are FP32 values rounded
//     from FP64, read per pass from a contiguous table [k][r] (L1-resident).
//  3. FSTC and fringe stop (Eq. 2): Y[k] = X[k] exp(2 pi i (k f/N + c_m)),
//     c_m = nu_BB f/fs + sideband (psi0 + rate t_m) reduced mod 1 in FP64 once
//     per spectrum; the per-channel ramp exp(2 pi i k f / N) is computed once
//     per workgroup.  Table mode (the paper's 1440-step sin/cos look-up table,
//     section 2.3.2): the phase k f/N + c_m is formed in FP64 per channel and
//     spectrum and rounded to the nearest of 1440 steps, whose FP32 cos and sin
//     replace the direct evaluation.
//  4. requantisation (section 4.1's fixed point up to the MAC): int8
//     clamp(rne(Y/scale), +-127) or OCP e4m3 RNE satfinite; FP32 keeps Y.
//  5. corner turn: a thread owns channels k = t + L*j (j = 0..7) of every
//     spectrum it transforms, so it gathers a whole X-layout chunk per channel
//     in registers (8 spectra of int8/e4m3 re+im, or 2 complex64: 16 bytes).
//     The X layout keeps the chunks of 8 consecutive channels of one signal
//     together, so the 8 lanes holding them write one full 128-byte line.
//
// Calibration mode (scale COMPUTE) runs steps 1-2 and sums |X|^2 per channel
// (the phase rotation does not change it) into per-workgroup partials.
#include <cmath>

#include "corr_internal.h"

namespace corr {
namespace {

template <int LOGM>
struct FCfg {
    static constexpr int M = 1 << LOGM;
    static constexpr int N = 2 * M;
    static constexpr int L = M / 8;                        // threads per transform
    static constexpr int FPAR = (L >= 256) ? 1 : 256 / L;  // transforms in flight
    static constexpr int WG = L * FPAR;
    static constexpr int NPASS8 = LOGM / 3;
    static constexpr int RLAST = 1 << (LOGM % 3);          // 1 = no extra pass
    static constexpr int NPASS = NPASS8 + (RLAST > 1 ? 1 : 0);
    static constexpr int NBUF = (LOGM >= 13) ? 1 : 2;      // ping-pong if it fits
    static constexpr int PADM = M + (M >> 4);
};

// One pad element every 16 float2: with it the contiguous reads and the strided
// radix-8 writes of every pass hit distinct banks (except a 2-way conflict on
// the writes of the pass with P = 8).  For any c that is a multiple of 16,
// padi(j + c) = padi(j) + c + c/16, so every LDS access below is a per-thread
// base plus a compile-time offset.
__device__ __forceinline__ constexpr int padi(int j) { return j + (j >> 4); }
__device__ __forceinline__ constexpr int padc(int c) { return c + c / 16; }  // c % 16 == 0

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // * (-i)

constexpr float kRsqrt2 = 0.70710678118654752440f;

// 4-point DFT, forward sign, outputs in natural order.
__device__ __forceinline__ void dft4(float2 &u0, float2 &u1, float2 &u2, float2 &u3) {
    float2 s0 = cadd(u0, u2), d0 = csub(u0, u2);
    float2 s1 = cadd(u1, u3), d1 = mul_mi(csub(u1, u3));
    u0 = cadd(s0, s1);
    u2 = csub(s0, s1);
    u1 = cadd(d0, d1);
    u3 = csub(d0, d1);
}

// 8-point DFT, forward sign: one radix-2 stage with W_8^r, then two 4-point DFTs
// (even outputs from the sums, odd outputs from the twiddled differences).
__device__ __forceinline__ void dft8(float2 *v) {
    float2 a0 = cadd(v[0], v[4]), b0 = csub(v[0], v[4]);
    float2 a1 = cadd(v[1], v[5]), b1 = csub(v[1], v[5]);
    float2 a2 = cadd(v[2], v[6]), b2 = csub(v[2], v[6]);
    float2 a3 = cadd(v[3], v[7]), b3 = csub(v[3], v[7]);
    b1 = make_float2((b1.x + b1.y) * kRsqrt2, (b1.y - b1.x) * kRsqrt2);   // * W_8^1
    b2 = mul_mi(b2);                                                        // * W_8^2
    b3 = make_float2((b3.y - b3.x) * kRsqrt2, -(b3.x + b3.y) * kRsqrt2);  // * W_8^3
    dft4(a0, a1, a2, a3);
    dft4(b0, b1, b2, b3);
    v[0] = a0; v[1] = b0; v[2] = a1; v[3] = b1;
    v[4] = a2; v[5] = b2; v[6] = a3; v[7] = b3;
}

template <int R>
__device__ __forceinline__ void dftR(float2 *v) {
    if constexpr (R == 8) {
        dft8(v);
    } else if constexpr (R == 4) {
        dft4(v[0], v[1], v[2], v[3]);
    } else {
        float2 a = v[0];
        v[0] = cadd(a, v[1]);
        v[1] = csub(a, v[1]);
    }
}

// Radix of pass ps and offset of its twiddle block: passes 1..ps-1 precede it.
constexpr int pass_radix(int logm, int ps) { return ps < logm / 3 ? 8 : (1 << (logm % 3)); }
constexpr int twiddle_offset(int logm, int ps) {
    int o = 0;
    for (int q = 1; q < ps; ++q) o += (1 << (3 * q)) * pass_radix(logm, q);
    return o;
}

template <int LOGM, int PS>
struct Pass {
    using C = FCfg<LOGM>;
    static constexpr int R = (PS < C::NPASS8) ? 8 : C::RLAST;
    static constexpr int P = 1 << (3 * PS);  // size of the sub-transforms already done
    static constexpr int NB = 8 / R;         // butterflies per thread
    // offset (float2) of this pass's twiddle block [P][R] in the table
    static constexpr int TOFF = twiddle_offset(LOGM, PS);
};

// Radix-R Stockham pass PS >= 1: butterfly i reads src[i + r M/R], applies
// W_{P R}^{r k} (k = i mod P), transforms, and writes dst[(i - k) R + k + q P].
// The twiddles of butterfly k are the contiguous entries [k][0..R) of this
// pass's block of the FP32 table (entry 0 is 1 and unused).
template <int LOGM, int PS>
__device__ __forceinline__ void fft_pass(const float2 *src, float2 *dst, const float2 *__restrict__ twp, int t) {
    using Ps = Pass<LOGM, PS>;
    using C = FCfg<LOGM>;
    constexpr int R = Ps::R, P = Ps::P, NB = Ps::NB, M = C::M, L = C::L;
    float2 v[8];
    const float2 *s0 = src + padi(t);
#pragma unroll
    for (int u = 0; u < NB; ++u) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[u * R + r] = s0[padc(L * u + r * (M / R))];
    }
    if constexpr (C::NBUF == 1) __syncthreads();  // single buffer: all reads before any write
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int k = (t + L * u) & (P - 1);
        const float4 *tw4 = reinterpret_cast<const float4 *>(twp + Ps::TOFF + k * R);
        float2 w[8];
#pragma unroll
        for (int h = 0; h < R / 2; ++h) {
            const float4 q = tw4[h];
            w[2 * h] = make_float2(q.x, q.y);
            w[2 * h + 1] = make_float2(q.z, q.w);
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[u * R + r] = cmul(v[u * R + r], w[r]);
        dftR<R>(&v[u * R]);
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int i = t + L * u;
        const int k = i & (P - 1);
        const int j = (i - k) * R + k;
        if constexpr (P >= 16) {
            float2 *d0 = dst + padi(j);
#pragma unroll
            for (int q = 0; q < R; ++q) d0[padc(q * P)] = v[u * R + q];
        } else if constexpr (P == 8) {
            // j = 64 a + b (b < 8): padi(j + 8 q) = 68 a + b + 8 q + (q >> 1)
            float2 *d0 = dst + (j + ((j >> 6) << 2));
#pragma unroll
            for (int q = 0; q < R; ++q) d0[8 * q + (q >> 1)] = v[u * R + q];
        } else {
#pragma unroll
            for (int q = 0; q < R; ++q) dst[padi(j + q * P)] = v[u * R + q];
        }
    }
}

template <int LOGM, int PS>
__device__ __forceinline__ void fft_passes(float2 *b0, float2 *b1, const float2 *__restrict__ tw, int t) {
    if constexpr (PS < FCfg<LOGM>::NPASS) {
        __syncthreads();
        if constexpr (FCfg<LOGM>::NBUF == 2) {
            if constexpr (PS & 1) fft_pass<LOGM, PS>(b0, b1, tw, t);
            else fft_pass<LOGM, PS>(b1, b0, tw, t);
        } else {
            fft_pass<LOGM, PS>(b0, b0, tw, t);
        }
        fft_passes<LOGM, PS + 1>(b0, b1, tw, t);
    }
}

// Buffer holding the final pass's output (natural order).
template <int LOGM>
__device__ __forceinline__ float2 *result_buffer(float2 *b0, float2 *b1) {
    if constexpr (FCfg<LOGM>::NBUF == 1) return b0;
    else return ((FCfg<LOGM>::NPASS - 1) & 1) ? b1 : b0;
}

// Logical workgroup id with consecutive ids on the same XCD (hardware hands
// workgroups to the 8 XCDs round-robin), so that the chunks of neighbouring
// signals, which are adjacent in the X layout, meet in one L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    const int q = nb >> 3, rem = nb & 7;
    const int x = bid & 7, i = bid >> 3;
    return x * q + min(x, rem) + i;
}

// An opaque zero: added to table indices inside the spectrum loop it keeps the
// compiler from hoisting the loop-invariant table loads out of the loop (which
// would pin them in registers for the whole kernel), while the pointer keeps
// its global address space.
__device__ __forceinline__ int opaque_zero() {
    int z = 0;
    asm volatile("" : "+s"(z));
    return z;
}

// Phase of the 1440-step table (section 2.3.2): the cycles of spectrum m,
// c = nu_BB f / fs + sideband (psi0 + rate t_m), t_m = (m + 1/2) N / fs,
// reduced mod 1, each operation rounded on its own (the table index is an
// integer decision, so the arithmetic is pinned down).
__device__ inline double lut_spectrum_phase(double c_bb, int sideband, double psi0, double rate, int64_t m,
                                            double t_spec) {
#pragma clang fp contract(off)
    const double tm = ((double)m + 0.5) * t_spec;
    double c = c_bb + (double)sideband * (psi0 + rate * tm);
    return c - floor(c);
}
// table entry of channel phase c + k f / N: nearest of the 1440 steps
__device__ inline int lut_index(double c, double kfn) {
#pragma clang fp contract(off)
    const int i = (int)rint((c + kfn) * (double)kLutSteps);
    return i % kLutSteps;
}

template <int LOGM, int MODE>
// 4 waves per SIMD: <= 128 VGPRs, which the kernel meets without scratch.
__global__ void __launch_bounds__(FCfg<LOGM>::WG) __attribute__((amdgpu_waves_per_eu(4, 8)))
fengine_kernel(FLaunch a) {
    using C = FCfg<LOGM>;
    constexpr int BM = MODE & 3;          // 0 FP32, 1 INT8, 2 FP8, 3 calibration
    constexpr bool PL = (MODE & 4) != 0;  // phase from the 1440-step table
    constexpr int M = C::M, N = C::N, L = C::L, FPAR = C::FPAR;
    constexpr int SPB = 16 * FPAR;  // spectra per workgroup
    constexpr int G = (BM == 0) ? kChunk32 : kChunk8;  // spectra per X-layout chunk
    __shared__ __attribute__((aligned(16))) uint32_t lds_in[FPAR][N / 4];
    __shared__ __attribute__((aligned(16))) float2 lds_w[FPAR][C::NBUF][C::PADM];

    const int nblk = (a.T + SPB - 1) / SPB;
    const int lid = xcd_remap(blockIdx.x, a.S * nblk);
    const int s = lid % a.S;
    const int blk = lid / a.S;
    const int u = threadIdx.x / L;  // transform slot
    const int t = threadIdx.x % L;
    const int m0 = blk * SPB + 16 * u;
    const bool active = m0 < a.T;  // T is a multiple of 16

    float2 *b0 = &lds_w[u][0][0];
    float2 *b1 = &lds_w[u][C::NBUF - 1][0];

    // geometry of this signal; out-of-range delays are clamped and reported
    const corr_geom_t g = a.geom[s];
    int D = g.D;
    if (D < 0 || D > a.max_delay) {
        if (threadIdx.x == 0) atomicOr(a.err, 1u);
        D = D < 0 ? 0 : a.max_delay;
    }

    // per-thread channel constants, k_j = t + L j: FSTC ramp exp(2 pi i k f / N)
    // and the inverse requantisation scale
    float2 ramp[8];
    const double fn = (double)g.frac / (double)N;  // table mode: channel k adds k fn cycles
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = t + L * j;
        // the post-process below forms 2 X[k]; the factor 1/2 is folded (exactly)
        // into the ramp
        if constexpr (PL) {
            ramp[j] = make_float2(0.5f, 0.f);
        } else if constexpr (BM != 3) {
            float sn, cs;
            sincospif(2.0f * ((float)k * (g.frac / (float)N)), &sn, &cs);
            ramp[j] = make_float2(0.5f * cs, 0.5f * sn);
        }
        // requantised output: the ramp also carries 1 / scale, so Y arrives scaled
        if constexpr (BM == 1 || BM == 2) {
            const float inv = 1.0f / a.scale[(int64_t)s * M + k];
            ramp[j] = make_float2(ramp[j].x * inv, ramp[j].y * inv);
        }
    }

    const uint32_t *row = reinterpret_cast<const uint32_t *>(a.x + (int64_t)s * a.row_stride);
    uint32_t pw[5];
    auto fetch = [&](int m) {
        const int64_t o = (int64_t)m * N + D + 16 * t;
        const int64_t w = o >> 2;
        pw[0] = row[w];
        pw[1] = row[w + 1];
        pw[2] = row[w + 2];
        pw[3] = row[w + 3];
        pw[4] = (o & 3) ? row[w + 4] : 0u;
    };
    const uint32_t sh = (uint32_t)(D & 3);
    if (active) fetch(m0);
    const double t_spec = (double)N / a.fs;             // seconds per spectrum
    const double c_bb = a.nu_bb * (double)g.frac / a.fs;  // baseband term of the phase, cycles

    // corner-turn staging: one 16-byte chunk per channel
    //   INT8/FP8: dwords {re 0-3, re 4-7, im 0-3, im 4-7}; FP32: 2 complex64
    uint32_t q0[8], q1[8], h0[8], h1[8];
    float2 f0[8];
    float pacc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        q0[j] = q1[j] = h0[j] = h1[j] = 0u;
        pacc[j] = 0.f;
    }

    // The 16 spectra in two chunks of 8.  INT8 / FP8 up to 4096 channels: each
    // chunk as two loops of 4, the copy of the loop body for half hh (a constant
    // after unrolling) putting the codes into the chunk's first (hh = 0, spectra
    // 0..3) or second (hh = 1) pair of words; at 8192 channels and more, where
    // the two copies measured slower, one loop of 8 that copies the first pair
    // aside after its fourth spectrum.  Either way the chunk is stored after its
    // eighth spectrum, outside the loop.
    constexpr int NH = ((BM == 1 || BM == 2) && LOGM <= 11) ? 2 : 1;
#pragma unroll 1
    for (int r8 = 0; r8 < 16; r8 += 8) {
#pragma unroll
    for (int hh = 0; hh < NH; ++hh) {
#pragma unroll 1
    for (int r = r8 + (8 / NH) * hh; r < r8 + (8 / NH) * (hh + 1); ++r) {
        const int m = m0 + r;
        // all in-loop addressing derives from this opaque copy of t, so that it
        // is recomputed per spectrum instead of being hoisted and held live
        const int tt = t + opaque_zero();
        // 1. stage the prefetched window bytes in LDS, then fetch the next one
        __syncthreads();
        if (active) {
            uint4 d;
            d.x = __builtin_amdgcn_alignbyte(pw[1], pw[0], sh);
            d.y = __builtin_amdgcn_alignbyte(pw[2], pw[1], sh);
            d.z = __builtin_amdgcn_alignbyte(pw[3], pw[2], sh);
            d.w = __builtin_amdgcn_alignbyte(pw[4], pw[3], sh);
            *reinterpret_cast<uint4 *>(&lds_in[u][4 * t]) = d;
        }
        __syncthreads();
        // 2a. first radix-8 pass straight from the staged int8 samples
        {
            const int16_t *in16 = reinterpret_cast<const int16_t *>(&lds_in[u][0]);
            float2 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int16_t p = in16[tt + L * q];
                v[q] = make_float2((float)(int8_t)(p & 0xFF), (float)(int8_t)(p >> 8));
            }
            dft8(v);
            // padi(8 t + q) = 8 t + (t >> 1) + q
            float2 *d0 = b0 + (8 * tt + (tt >> 1));
#pragma unroll
            for (int q = 0; q < 8; ++q) d0[q] = v[q];
        }
        // 2b. remaining passes
        fft_passes<LOGM, 1>(b0, b1, a.twp, tt);
        __syncthreads();
        const float2 *Z = result_buffer<LOGM>(b0, b1);
        const float2 *wn = a.wn;

        // 3. phase of this spectrum (FP64 reduction, FP32 sincos; LUT mode:
        //    the reduced cycles c, to which each channel adds k f / N)
        float2 rot = make_float2(1.f, 0.f);
        double c_lut = 0.0;
        if constexpr (PL) {
            c_lut = lut_spectrum_phase(c_bb, a.sideband, g.psi0, g.rate, a.spectrum0 + m, t_spec);
        } else if constexpr (BM != 3) {
            const double tm = ((double)(a.spectrum0 + m) + 0.5) * t_spec;
            double c = c_bb + (double)a.sideband * (g.psi0 + g.rate * tm);
            c -= floor(c);
            float sn, cs;
            sincospif(2.0f * (float)c, &sn, &cs);
            rot = make_float2(cs, sn);
        }
        // byte lane of this spectrum inside its dword of the chunk
        // (v_perm selector: byte 4 = the new value's low byte, bytes 0..3 = the old dword)
        const uint32_t bsel = (0x03020100u & ~(0xFFu << (8 * (r & 3)))) | (0x04u << (8 * (r & 3)));
        // Z[k] and Z[M - k] for k = t + L j: bases plus compile-time offsets
        const float2 *za0 = Z + padi(tt);
        const int nb = -tt + ((-tt) >> 4);  // padi((8 - j) L - t) = padc((8 - j) L) + nb
        const float2 *zb0p = Z + nb;
        const float2 *zbz = (tt == 0) ? Z : (Z + padc(M) + nb);  // j = 0: index (M - t) mod M
        // chunk of spectrum m: 16-byte index g*C*S + ((t/8) S + s) 8 + t%8 + j L S
        const int64_t obase = (int64_t)(m / G) * M * a.S + (((tt >> 3) * a.S + s) << 3) + (tt & 7);
        // the split twiddles are this spectrum's last table loads: fetch the
        // next window only after them, so that waiting for a table load never
        // waits for the window (loads complete in issue order), and the window
        // is not held in registers through the transform
        float2 wv[8], ev[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            wv[j] = wn[tt + L * j];
            // table mode: the table entry nearest each channel's phase, a table load too
            if constexpr (PL) ev[j] = a.lut[lut_index(c_lut, (double)(tt + L * j) * fn)];
        }
        if (active && r < 15) fetch(m + 1);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const float2 za = za0[padc(L * j)];
            const float2 zb0 = (j == 0) ? zbz[0] : zb0p[padc((8 - j) * L)];
            const float2 zb = make_float2(zb0.x, -zb0.y);
            const float2 sm = cadd(za, zb), df = csub(za, zb);
            const float2 w = wv[j];
            // 2 X = (a + b) - i w (a - b)
            float2 X;
            X.x = sm.x + (w.x * df.y + w.y * df.x);
            X.y = sm.y - (w.x * df.x - w.y * df.y);
            if constexpr (BM == 3) {
                pacc[j] += X.x * X.x + X.y * X.y;
            } else {
                if (a.power && active)  // |X|^2 = |2X|^2 / 4 (the phase rotation keeps it)
                    put_power(a, ((int64_t)s * a.T + m) * M + tt + L * j, 0.25f * (X.x * X.x + X.y * X.y));
                // the value; for int8 the value plus 128, formed inside its last products
                float2 Y;
                if constexpr (PL) {  // table entry nearest the channel's phase; ramp = 1/2 (x 1/scale)
                    const float2 e = ev[j];
                    const float2 u = make_float2(X.x * e.x - X.y * e.y, X.x * e.y + X.y * e.x);
                    if constexpr (BM == 1)
                        Y = make_float2(fmaf(ramp[j].x, u.x, 128.0f), fmaf(ramp[j].x, u.y, 128.0f));
                    else
                        Y = make_float2(ramp[j].x * u.x, ramp[j].x * u.y);
                } else if constexpr (BM == 1) {
                    const float2 t = cmul(X, ramp[j]);
                    Y = make_float2(fmaf(t.x, rot.x, fmaf(-t.y, rot.y, 128.0f)),
                                    fmaf(t.x, rot.y, fmaf(t.y, rot.x, 128.0f)));
                } else {
                    Y = cmul(cmul(X, ramp[j]), rot);
                }
                if constexpr (BM == 0) {
                    if (r & 1) {
                        if (active) {
                            float4 *dst = reinterpret_cast<float4 *>(a.spec) + obase + (int64_t)j * L * a.S;
                            *dst = make_float4(f0[j].x, f0[j].y, Y.x, Y.y);
                        }
                    } else {
                        f0[j] = Y;
                    }
                } else {
                    // insert the byte of spectrum r into byte r mod 4 of the chunk's
                    // pair of words for this half (one loop: the second pair, the
                    // first copied aside after spectrum 3 of the chunk)
                    uint32_t &q = (NH == 2 && hh == 0) ? q0[j] : q1[j];
                    uint32_t &h = (NH == 2 && hh == 0) ? h0[j] : h1[j];
                    if constexpr (BM == 1) {
                        q = put_i8_biased(Y.x, r & 3, q);
                        h = put_i8_biased(Y.y, r & 3, h);
                    } else {  // one conversion: real code in byte 0, imaginary in byte 1
                        const uint32_t w = e4m3_pair(Y.x, Y.y);
                        q = __builtin_amdgcn_perm(w, q, bsel);
                        h = __builtin_amdgcn_perm(w, h, bsel + (1u << (8 * (r & 3))));
                    }
                    if (NH == 1 && (r & 7) == 3) {
                        q0[j] = q1[j];
                        h0[j] = h1[j];
                    }
                }
            }
        }
    }
    }
    if constexpr (BM == 1 || BM == 2) {  // the chunk of spectra r8 .. r8 + 7, whole
        if (active) {
            constexpr uint32_t B = BM == 1 ? kI8Bias : 0u;  // int8 bytes carry the bias
            const int64_t ob = (int64_t)((m0 + r8) / G) * M * a.S + (((t >> 3) * a.S + s) << 3) + (t & 7);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                uint4 *dst = reinterpret_cast<uint4 *>(a.spec) + ob + (int64_t)j * L * a.S;
                *dst = make_uint4(q0[j] ^ B, q1[j] ^ B, h0[j] ^ B, h1[j] ^ B);
            }
        }
    }
    }

    if constexpr (BM == 3) {
        if (active) {
            // slot m0/16 of T/16 per signal: the active slots are exactly the first T/16
            float *dst = a.part + ((int64_t)s * (a.T / 16) + (m0 >> 4)) * M;
#pragma unroll
            for (int j = 0; j < 8; ++j) dst[t + L * j] = 0.25f * pacc[j];  // |2X|^2 / 4
        }
    }
}

template <int LOGM>
hipError_t launch_one(int mode, const FLaunch &a, hipStream_t st) {
    using C = FCfg<LOGM>;
    const int spb = 16 * C::FPAR;
    const int nblk = (a.T + spb - 1) / spb;
    const dim3 grid(a.S * nblk), block(C::WG);
    switch (mode) {
    case 0: hipLaunchKernelGGL((fengine_kernel<LOGM, 0>), grid, block, 0, st, a); break;
    case 1: hipLaunchKernelGGL((fengine_kernel<LOGM, 1>), grid, block, 0, st, a); break;
    case 2: hipLaunchKernelGGL((fengine_kernel<LOGM, 2>), grid, block, 0, st, a); break;
    case 3: hipLaunchKernelGGL((fengine_kernel<LOGM, 3>), grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL((fengine_kernel<LOGM, 4>), grid, block, 0, st, a); break;
    case 5: hipLaunchKernelGGL((fengine_kernel<LOGM, 5>), grid, block, 0, st, a); break;
    case 6: hipLaunchKernelGGL((fengine_kernel<LOGM, 6>), grid, block, 0, st, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// sigma^2 = sum of the partials / (2T) in FP64; scale = 4 sigma / qmax (1 if 0).
__global__ void calib_reduce_kernel(const float *part, int S, int C, int nparts, int T, float qmax,
                                    float *scale) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= S * C) return;
    const int s = idx / C, k = idx % C;
    const float *p = part + (int64_t)s * nparts * C + k;
    double acc = 0.0;
    for (int i = 0; i < nparts; ++i) acc += (double)p[(int64_t)i * C];
    const double sig = sqrt(acc / (2.0 * (double)T));
    float sc = (float)(4.0 * sig / (double)qmax);
    scale[idx] = sc > 0.f ? sc : 1.0f;
}

}  // namespace

int fengine_fpar(int log2m) {
    switch (log2m) {
    case 8: return FCfg<8>::FPAR;
    case 9: return FCfg<9>::FPAR;
    case 10: return FCfg<10>::FPAR;
    case 11: return FCfg<11>::FPAR;
    case 12: return FCfg<12>::FPAR;
    case 13: return FCfg<13>::FPAR;
    default: return 0;
    }
}

int fengine_spectra_per_block(int log2m) { return 16 * fengine_fpar(log2m); }

// Twiddles of passes 1..NPASS-1 in the order of Pass<>::TOFF: for each pass the
// block [k < P][r < R] of W_{P R}^{r k} = exp(-2 pi i r k / (P R)), computed in
// FP64 and rounded once to FP32.  With out == nullptr only the count is returned.
void fengine_twiddle_table(int log2m, float2 *out, size_t *count) {
    const int npass8 = log2m / 3, rlast = 1 << (log2m % 3);
    const int npass = npass8 + (rlast > 1 ? 1 : 0);
    size_t n = 0;
    for (int ps = 1; ps < npass; ++ps) {
        const int R = ps < npass8 ? 8 : rlast;
        const int P = 1 << (3 * ps);
        for (int k = 0; k < P; ++k)
            for (int r = 0; r < R; ++r, ++n)
                if (out) {
                    const double a = -2.0 * M_PI * (double)r * (double)k / ((double)P * (double)R);
                    out[n] = make_float2((float)std::cos(a), (float)std::sin(a));
                }
    }
    *count = n;
}

hipError_t launch_fengine(int log2m, int mode, const FLaunch &a, hipStream_t st) {
    switch (log2m) {
    case 8: return launch_one<8>(mode, a, st);
    case 9: return launch_one<9>(mode, a, st);
    case 10: return launch_one<10>(mode, a, st);
    case 11: return launch_one<11>(mode, a, st);
    case 12: return launch_one<12>(mode, a, st);
    case 13: return launch_one<13>(mode, a, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_calib_reduce(const float *part, int S, int C, int nparts, int T, int precision,
                               float *scale, hipStream_t st) {
    const float qmax = (precision == CORR_FP8_E4M3) ? 448.0f : 127.0f;
    const int n = S * C;
    hipLaunchKernelGGL(calib_reduce_kernel, dim3((n + 255) / 256), dim3(256), 0, st, part, S, C, nparts,
                       T, qmax, scale);
    return hipGetLastError();
}

}  // namespace corr
