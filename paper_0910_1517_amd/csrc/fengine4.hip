// fengine4.hip -- F-engine of the FX correlator for gfx950: the real FFT as a
// four-step transform whose first step runs on the matrix cores.
//
// The window of N = 64 N1 real samples of spectrum m of signal s starts at
// sample m N + D_s of its row (integer delay by read-pointer advance: section
// 2.1, block shift; section 2.3.2, read-pointer offset into the overlapped
// slice).  Writing n = n1 + N1 n2 (n1 < N1, n2 < 64) and k = k2 + 64 k1,
//   X[k] = sum_n1 W_N^(n1 k2) A[n1][k2] W_N1^(n1 k1),
//   A[n1][k2] = sum_n2 x[n1 + N1 n2] W_64^(n2 k2)                        (*)
// (W_n = exp(-2 pi i / n)).  The samples are real, so A[n1][64 - k2] is the
// conjugate of A[n1][k2] and X[N - k] of X[k]: the 64 real rows of (*) --
// cos and -sin of k2 = 1..31 and cos of k2 = 0 and 32 -- hold all of it, and
// every channel k < N/2 (section 2.1's spectral channels, DC kept, Nyquist
// dropped) comes from one of 32 columns:
//   column k2 = 1..31:  X[k2 + 64 k1] for k1 < N1/2 and, as conjugates,
//                       X[(64 - k2) + 64 (N1 - 1 - k1)] for k1 >= N1/2;
//   column 0:           the two real rows k2 = 0 and 32 together are the
//                       2 N1-point real sequence y[c] = sum over n = c mod 2 N1
//                       of x[n] (y[n1] = (A0 + A32)/2, y[n1 + N1] = (A0 - A32)/2),
//                       whose real DFT gives the channels k = 32 j, j < N1.  It
//                       is transformed as u[j] = y[2j] + i y[2j + 1] and
//                       unfolded with 2 Y[j] = (U[j] + U*[N1 - j])
//                       - i W_2N1^j (U[j] - U*[N1 - j]).
//
// Steps per spectrum (a workgroup owns one signal and 32 FPAR consecutive
// spectra, FPAR windows in flight):
//  1. the window's int8 bytes are staged in LDS (16-byte aligned loads with a
//     byte funnel shift, prefetched one spectrum ahead);
//  2. (*) on the matrix cores: each wave computes one 32 x 32 tile of the
//     64-row result with v_mfma_f32_32x32x16_f16.  int8 samples are exact in
//     FP16 and each twiddle is the sum of two FP16 numbers (its nearest FP16 and
//     the nearest FP16 of the remainder, ~22 bits), so the two products of a
//     pair of MFMAs are exact and the FP32 sums carry only FP32 rounding.  A
//     lane's operand -- 8 consecutive n2 of one n1 -- comes from the staged
//     bytes with one transposing LDS read (ds_read_b64_tr_b8: eight 16-byte
//     rows given as 8-byte halves by lane pairs, lane c receiving byte column c);
//  3. the four-step twiddle W_N^(n1 k2) (FP32 table) is applied as the tiles
//     are written to LDS, one column per k2;
//  4. the N1-point transforms of the 32 columns: Stockham radix-8 passes (plus
//     one radix-2 or radix-4 pass) through LDS; the last pass keeps its
//     outputs in registers;
//  5. FSTC and fringe stop (Eq. 2): Y[k] = X[k] exp(2 pi i (k f / N + c_m)),
//     the per-channel ramp computed once per workgroup, c_m = nu_BB f / fs +
//     sideband (psi0 + rate t_m) reduced mod 1 in FP64 once per spectrum and
//     workgroup (table mode, the 1440-step sin/cos table of section 2.3.2,
//     runs on the LDS-radix kernel);
//  6. requantisation (section 4.1's fixed point ahead of the MAC) and the
//     corner turn: a thread owns the same channels in every spectrum and
//     gathers a whole 16-byte X-layout chunk per channel (8 spectra of int8 or
//     e4m3 re + im, or 2 complex64) before storing it.
// Calibration mode (scale COMPUTE) sums |X|^2 per channel instead of steps 5-6.
#include <cmath>
#include <type_traits>

#include "corr_internal.h"

namespace corr {
namespace {

typedef _Float16 f4_half8 __attribute__((ext_vector_type(8)));
typedef float f4_float16 __attribute__((ext_vector_type(16)));
typedef int f4_int2 __attribute__((ext_vector_type(2)));
typedef unsigned f4_uint4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) f4_int2 lds_int2;
typedef short f4_short4 __attribute__((ext_vector_type(4)));
typedef short f4_short8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) f4_short4 lds_short4;

template <int LOGM>
struct F4Cfg {
    static constexpr int M = 1 << LOGM;     // channels
    static constexpr int N = 2 * M;         // real samples per window
    static constexpr int N1 = N / 64;       // length of the column transforms
    static constexpr int LOGN1 = LOGM - 5;
    static constexpr int L = M / 8;         // threads per window (4 N1)
    static constexpr int FPAR = (L >= 256) ? 1 : 256 / L;
    static constexpr int WG = L * FPAR;     // 256, 512 or 1024
    static constexpr int J = WG / 32;       // threads per column (over all windows)
    static constexpr int BPC = N1 / 8;      // radix-8 butterflies per column
    static constexpr int NP8 = LOGN1 / 3;
    static constexpr int RLAST = 1 << (LOGN1 % 3);
    static constexpr int NPASS = NP8 + (RLAST > 1 ? 1 : 0);
    // column stride (float2) of the padded columns (one pad per 8 elements, see
    // padi): chosen so that the 8 columns a wave's pass reads and writes touch
    // 64 distinct banks
    static constexpr int CS = N1 == 8 ? 10 : N1 == 16 ? 18 : N1 == 32 ? 36 : N1 == 64 ? 72 : N1 == 128 ? 152 : 296;
    static constexpr int NBUF = 1;          // column passes run in place
    static constexpr int AP = 72;           // LDS row pitch (FP16) of the DFT-64 rows
    static constexpr int NSPEC = WG / 4;    // channels of column 0 per iteration (FPAR N1)
    static constexpr int SPS = 32;          // spectra per window slot
};

// entries of the column-pass twiddle table: P R per pass 1..NPASS-1
constexpr int twb_count(int logn) {
    int n = 0;
    const int np8 = logn / 3, rl = 1 << (logn % 3), np = np8 + (rl > 1 ? 1 : 0);
    for (int ps = 1; ps < np; ++ps) n += (1 << (3 * ps)) * (ps < np8 ? 8 : rl);
    return n;
}

// padded position of element j of a column: one pad per 8 elements, which with
// the column strides above keeps the Stockham reads (consecutive elements) and
// writes (elements 8 apart) of a wave free of LDS bank conflicts
__device__ __forceinline__ constexpr int padi(int j) { return j + (j >> 3); }

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // * (-i)

constexpr float kRsqrt2 = 0.70710678118654752440f;

__device__ __forceinline__ void dft4(float2 &u0, float2 &u1, float2 &u2, float2 &u3) {
    float2 s0 = cadd(u0, u2), d0 = csub(u0, u2);
    float2 s1 = cadd(u1, u3), d1 = mul_mi(csub(u1, u3));
    u0 = cadd(s0, s1);
    u2 = csub(s0, s1);
    u1 = cadd(d0, d1);
    u3 = csub(d0, d1);
}

// 8-point DFT (forward sign), natural output order.  The odd half takes
// b1 W8, b2 W8^2 = -i b2 and b3 W8^3 (W8 = (1 - i) / sqrt 2); the 1 / sqrt 2
// of b1 and b3 is applied once, to their sum and difference, inside the last
// additions (fused multiply-adds).
__device__ __forceinline__ void dft8(float2 *v) {
    float2 a0 = cadd(v[0], v[4]), b0 = csub(v[0], v[4]);
    float2 a1 = cadd(v[1], v[5]), b1 = csub(v[1], v[5]);
    float2 a2 = cadd(v[2], v[6]), b2 = csub(v[2], v[6]);
    float2 a3 = cadd(v[3], v[7]), b3 = csub(v[3], v[7]);
    dft4(a0, a1, a2, a3);
    const float2 B1 = make_float2(b1.x + b1.y, b1.y - b1.x);     // b1 (1 - i)
    const float2 B3 = make_float2(b3.y - b3.x, -(b3.x + b3.y));  // b3 (-1 - i)
    const float2 s0 = cadd(b0, mul_mi(b2)), d0 = csub(b0, mul_mi(b2));
    const float2 S = cadd(B1, B3), D = mul_mi(csub(B1, B3));
    v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
    v[1] = make_float2(fmaf(kRsqrt2, S.x, s0.x), fmaf(kRsqrt2, S.y, s0.y));
    v[5] = make_float2(fmaf(-kRsqrt2, S.x, s0.x), fmaf(-kRsqrt2, S.y, s0.y));
    v[3] = make_float2(fmaf(kRsqrt2, D.x, d0.x), fmaf(kRsqrt2, D.y, d0.y));
    v[7] = make_float2(fmaf(-kRsqrt2, D.x, d0.x), fmaf(-kRsqrt2, D.y, d0.y));
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

constexpr int pass_radix(int logn, int ps) { return ps < logn / 3 ? 8 : (1 << (logn % 3)); }
// LDS pitch (float2) of a butterfly's twiddle row [k][0..R): a radix-8 row is
// read as 4 float4 by lanes whose k differ, and at 64 bytes per row the lanes
// of k and k + 4 met in one bank; 80 bytes spreads the 8 rows over all banks
constexpr int tw_pitch(int r) { return r == 8 ? 10 : r; }
constexpr int twiddle_offset(int logn, int ps) {  // in the LDS copy
    int o = 0;
    for (int q = 1; q < ps; ++q) o += (1 << (3 * q)) * tw_pitch(pass_radix(logn, q));
    return o;
}
constexpr int twl_count(int logn) {
    int n = 0;
    const int np8 = logn / 3, rl = 1 << (logn % 3), np = np8 + (rl > 1 ? 1 : 0);
    for (int ps = 1; ps < np; ++ps) n += (1 << (3 * ps)) * tw_pitch(ps < np8 ? 8 : rl);
    return n;
}

// One radix-R Stockham pass PS over a column of N1 points: butterfly i reads
// src[i + r N1/R], multiplies by W_(P R)^(r k) (k = i mod P; the contiguous
// table entries [k][r] of this pass), transforms and writes dst[(i - k) R + k +
// q P].  The last pass returns its outputs, k1 = i + q N1/R, in v.
template <int LOGM, int PS>
__device__ __forceinline__ void col_pass(const float2 *src, float2 *dst, const float2 *twp, int b,
                                         float2 (&v)[8]) {
    using C = F4Cfg<LOGM>;
    constexpr int R = pass_radix(C::LOGN1, PS);
    constexpr int P = 1 << (3 * PS);
    constexpr int NB = 8 / R;
    constexpr int N1 = C::N1, BPC = C::BPC;
    constexpr bool LAST = PS == C::NPASS - 1;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
#pragma unroll
        for (int r = 0; r < R; ++r) v[u * R + r] = src[padi(b + BPC * u + r * (N1 / R))];
    }
    if constexpr (C::NBUF == 1 && !LAST) __syncthreads();  // in place: every read before any write
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        if constexpr (PS > 0) {
            const int k = (b + BPC * u) & (P - 1);
            const float4 *tw4 = reinterpret_cast<const float4 *>(twp + twiddle_offset(C::LOGN1, PS) + k * tw_pitch(R));
            float2 w[8];
#pragma unroll
            for (int hh = 0; hh < R / 2; ++hh) {
                const float4 q = tw4[hh];
                w[2 * hh] = make_float2(q.x, q.y);
                w[2 * hh + 1] = make_float2(q.z, q.w);
            }
#pragma unroll
            for (int r = 1; r < R; ++r) v[u * R + r] = cmul(v[u * R + r], w[r]);
        }
        dftR<R>(&v[u * R]);
    }
    if constexpr (!LAST) {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int i = b + BPC * u;
            const int k = i & (P - 1);
            const int j = (i - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) dst[padi(j + q * P)] = v[u * R + q];
        }
    }
}

template <int LOGM, int PS>
__device__ __forceinline__ void col_passes(float2 *b0, float2 *b1, const float2 *twp, int colo, int b,
                                           float2 (&v)[8]) {
    using C = F4Cfg<LOGM>;
    if constexpr (PS < C::NPASS) {
        if (PS > 0) __syncthreads();
        float2 *src = (C::NBUF == 1 || (PS & 1) == 0) ? b0 : b1;
        float2 *dst = (C::NBUF == 1 || (PS & 1) == 1) ? b0 : b1;
        col_pass<LOGM, PS>(src + colo, dst + colo, twp, b, v);
        col_passes<LOGM, PS + 1>(b0, b1, twp, colo, b, v);
    }
}

// Consecutive logical ids on one XCD (workgroups are dealt to the 8 XCDs in
// turn), so that neighbouring signals' chunks meet in one L2.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
    const int q = nb >> 3, rem = nb & 7;
    const int x = bid & 7, i = bid >> 3;
    return x * q + min(x, rem) + i;
}

// One output channel of a thread: its ramp (x 1/scale), its corner-turn staging
// and, in calibration mode, its |X|^2 sum.  INT8/FP8 stage a chunk -- the re and
// im bytes of 8 spectra -- and store it when complete.
struct Chan {
    float2 ramp;
    uint32_t q, h;    // INT8/FP8: re and im bytes of the spectra 4j..4j+3 in progress
    uint32_t q0, h0;  // INT8/FP8: those of the first four spectra of the chunk
    float2 f0;      // FP32: the even spectrum of the pair
    float pacc;
};

// Phase, requantisation and corner turn of channel k's value X in spectrum r of
// the slot; chunk is the channel's 16-byte X-layout chunk of this spectrum group.
// INT8 / FP8: the codes go into byte r mod 4 of a pair of words.  H = 0 or 1
// (the caller knows which half of the chunk spectrum r is in): the first
// (spectra 0..3 of the chunk) or second (4..7) pair, the chunk stored whole by
// the caller after its eighth spectrum.  H = -1: the pair in progress, copied
// aside after the fourth spectrum and the chunk stored here after the eighth.
template <int BM, int H>
__device__ __forceinline__ void emit(Chan &c, float2 X, float2 rot, int r, uint32_t bsel, bool active, uint4 *chunk) {
    if constexpr (BM == 3) {
        c.pacc += X.x * X.x + X.y * X.y;
        return;
    } else if constexpr (BM == 0) {
        const float2 Y = cmul(cmul(X, c.ramp), rot);
        if (r & 1) {
            if (active) *reinterpret_cast<float4 *>(chunk) = make_float4(c.f0.x, c.f0.y, Y.x, Y.y);
        } else {
            c.f0 = Y;
        }
    } else {
        uint32_t &q = H == 0 ? c.q0 : c.q, &h = H == 0 ? c.h0 : c.h;
        if constexpr (BM == 1) {
            // int8: the codes plus 128 (formed inside the last products); the chunk's
            // store takes the 128 off
            const float2 t = cmul(X, c.ramp);
            q = put_i8_biased(fmaf(t.x, rot.x, fmaf(-t.y, rot.y, 128.0f)), r & 3, q);
            h = put_i8_biased(fmaf(t.x, rot.y, fmaf(t.y, rot.x, 128.0f)), r & 3, h);
        } else {  // e4m3
            const float2 Y = cmul(cmul(X, c.ramp), rot);
            const uint32_t w = e4m3_pair(Y.x, Y.y);
            q = __builtin_amdgcn_perm(w, q, bsel);
            h = __builtin_amdgcn_perm(w, h, bsel + (1u << (8 * (r & 3))));
        }
        if constexpr (H < 0) {
            // a chunk's two halves are stored together (a half written four spectra
            // before the other leaves L2 twice)
            if ((r & 7) == 3) {
                c.q0 = c.q;
                c.h0 = c.h;
            } else if ((r & 7) == 7 && active) {
                constexpr uint32_t B = BM == 1 ? kI8Bias : 0u;
                *chunk = make_uint4(c.q0 ^ B, c.q ^ B, c.h0 ^ B, c.h ^ B);
            }
        }
    }
}

template <int LOGM, int MODE>
__global__ void __launch_bounds__(F4Cfg<LOGM>::WG) __attribute__((amdgpu_waves_per_eu(3))) fengine4_kernel(FLaunch a) {
    using C = F4Cfg<LOGM>;
    constexpr int BM = MODE & 3;  // 0 FP32, 1 INT8, 2 FP8, 3 calibration
    // power cells: 0 none, 1 FP32 |X|^2, 2 FP16 |X|^2 / N^2 -- a template choice, so that a
    // launch without power output carries none of its registers
    constexpr int PW = MODE >> 2;
    auto store_power = [&](int64_t i, float p) {
        if constexpr (PW == 1) reinterpret_cast<float *>(a.power)[i] = p;
        if constexpr (PW == 2) reinterpret_cast<_Float16 *>(a.power)[i] = (_Float16)(p * a.power_scale);
    };
    constexpr int M = C::M, N = C::N, N1 = C::N1, L = C::L, FPAR = C::FPAR, WG = C::WG;
    constexpr int SPS = C::SPS, SPB = SPS * FPAR;
    constexpr int G = (BM == 0) ? kChunk32 : kChunk8;
    constexpr int RL = C::RLAST == 1 ? 8 : C::RLAST;  // radix of the last column pass
    constexpr int NBL = 8 / RL;                       // its butterflies per thread
    // The window: at 2048 channels converted to FP16 once, as it is staged (rows of
    // N1 samples at a pitch of N1 + 32 halves, so that the 8 rows a 16-bit
    // transposing read pass touches fall on distinct banks), single-buffered (its
    // last reader, stage A of the previous spectrum, is behind that spectrum's
    // barriers); otherwise as bytes, double-buffered, converted after the
    // transposing byte reads.
    constexpr bool H16 = LOGM == 11;
    constexpr int XP = N1 + 32;
    __shared__ __attribute__((aligned(16))) uint32_t lds_x[H16 ? 1 : 2][FPAR][H16 ? 4 : N / 4];
    __shared__ __attribute__((aligned(16))) _Float16 lds_xh[H16 ? FPAR : 1][H16 ? (N / N1) * XP : 8];
    __shared__ __attribute__((aligned(16))) float2 lds_tw[twl_count(C::LOGN1) > 0 ? twl_count(C::LOGN1) : 1];
    __shared__ __attribute__((aligned(16))) float2 lds_b[C::NBUF][FPAR * 32 * C::CS];
    __shared__ __attribute__((aligned(16))) uint16_t lds_a[2][64 * C::AP];  // FP16 rows (hi, lo)
    __shared__ __attribute__((aligned(16))) float2 lds_u[FPAR * N1];  // column 0 outputs
    __shared__ float2 lds_rot[SPB];

    const int tid = threadIdx.x;
    const int nblk = (a.T + SPB - 1) / SPB;
    const int lid = xcd_remap(blockIdx.x, a.S * nblk);
    const int s = lid % a.S;
    const int blk = lid / a.S;
    const int mblk = blk * SPB;  // first spectrum of the workgroup

    // geometry; out-of-range delays are clamped and reported
    const corr_geom_t g = a.geom[s];
    int D = g.D;
    if (D < 0 || D > a.max_delay) {
        if (tid == 0) atomicOr(a.err, 1u);
        D = D < 0 ? 0 : a.max_delay;
    }
    const double t_spec = (double)N / a.fs;
    const double c_bb = a.nu_bb * (double)g.frac / a.fs;

    // per-spectrum phase of the whole workgroup, once: FP64 reduction, FP32 sincos
    if (tid < SPB) {
        const int64_t m = a.spectrum0 + mblk + tid;
        if constexpr (BM != 3) {
            const double tm = ((double)m + 0.5) * t_spec;
            double c = c_bb + (double)a.sideband * (g.psi0 + g.rate * tm);
            c -= floor(c);
            float sn, cs;
            sincospif(2.0f * (float)c, &sn, &cs);
            lds_rot[tid] = make_float2(cs, sn);
        }
    }

    // ---- stage-A (matrix core) lane constants: this wave's 32 x 32 tile
    const int wv = tid >> 6, ln = tid & 63;
    const int mt = wv & 1, nt = wv >> 1, hh = ln >> 5;
    const int acol = 32 * nt + (ln & 31);    // column of the tile: window slot and n1
    const int au = acol / N1, an1 = acol % N1;
    // the DFT-64 rows (FP16 hi and lo) into LDS with a padded row pitch
    for (int i = tid; i < 2 * 64 * 8; i += WG) {
        const int hl = i >> 9, row = (i >> 3) & 63, c8 = i & 7;
        *reinterpret_cast<uint4 *>(&lds_a[hl][row * C::AP + 8 * c8]) =
            reinterpret_cast<const uint4 *>(a.afrag)[(hl * 64 * 64 + row * 64) / 8 + c8];
    }
    const int a_off = (32 * mt + (ln & 31)) * C::AP + 8 * hh;  // this lane's A fragment, K-tile 0
    for (int i = tid; i < twb_count(C::LOGN1); i += WG) {  // table entry i -> its padded LDS place
        int q = 1, off = 0;
        for (;;) {
            const int n = (1 << (3 * q)) * pass_radix(C::LOGN1, q);
            if (i < off + n) break;
            off += n;
            ++q;
        }
        const int R = pass_radix(C::LOGN1, q), l = i - off;
        lds_tw[twiddle_offset(C::LOGN1, q) + (l / R) * tw_pitch(R) + l % R] = a.twb[i];
    }
    // transposing-read address of this lane: its 16-lane group holds 8 rows (n2)
    // of 16 consecutive columns, each row given as two 8-byte halves
    const int tr_i = ln & 15, tr_g = ln >> 4;
    const int tr_c0 = 32 * nt + 16 * (tr_g & 1) + 8 * (tr_i & 1);
    const int tr_off = (tr_c0 / N1) * N + (tr_c0 % N1) + N1 * (8 * (tr_g >> 1) + (tr_i >> 1));
    // 16-bit transposing read (FP16 window): in each 16-lane group, lane 4 q + c gives
    // the address of row (K) q, columns 4 c .. 4 c + 3 of the group's 16, and lane i
    // receives column i of the 4 rows; group g takes columns 16 (g mod 2) + 32 nt
    // and rows 8 (g / 2) (the lane's K half)
    const int t16_off = (8 * (tr_g >> 1) + (tr_i >> 2)) * (N1 + 32) + 32 * nt + 16 * (tr_g & 1) + 4 * (tr_i & 3);
    // four-step twiddles W_N^(n1 p) of this lane's column and its 8 rows p
    float2 tws[8];
#pragma unroll
    for (int v = 0; v < 16; v += 2) {
        const int p = 16 * mt + 4 * (v >> 2) + 2 * hh + ((v & 3) >> 1);
        tws[v >> 1] = a.tw4[p * N1 + an1];
    }

    // ---- column-transform thread mapping: column p, butterfly b of window slot bu.
    // The wave that holds column 0 (its outputs, their unfolding and the channels
    // they give) issues more per spectrum than the other three, and wave w of a
    // workgroup runs on one SIMD: that wave is wave wz, varied across workgroups
    // so that the extra share falls on every SIMD alike.  ctid numbers the
    // threads from wave wz on.
    static_assert(WG == 256, "four waves per workgroup");
    const int wz = (int)(((uint32_t)blockIdx.x * 0x9E3779B1u) >> 30);
    const int ctid = (tid - 64 * wz) & (WG - 1);
    const int cp = ctid / C::J;
    const int cj = ctid % C::J;
    const int bu = cj / C::BPC, bb = cj % C::BPC;
    const int colo = (bu * 32 + cp) * C::CS;
    const int nspec_u = ctid / N1, nspec_j = ctid % N1;  // column-0 channel 32 j (ctid < NSPEC)

    // ---- output channels of this thread: 8 from column cp (none for cp = 0),
    // plus channel 32 j of column 0 for ctid < NSPEC
    auto chan = [&](int o) -> int {
        const int u = o / RL, q = o % RL;
        const int k1 = bb + C::BPC * u + q * (N1 / RL);
        return q < RL / 2 ? cp + 64 * k1 : N - cp - 64 * k1;
    };
    const int ch_s = 32 * nspec_j;
    Chan ch[9];
#pragma unroll
    for (int o = 0; o < 9; ++o) {
        Chan &c = ch[o];
        c.q = c.h = c.q0 = c.h0 = 0u;
        c.f0 = make_float2(0.f, 0.f);
        c.pacc = 0.f;
        const int k = o == 8 ? (ctid < C::NSPEC ? ch_s : 0) : (cp == 0 ? 0 : chan(o));
        // column 0 unfolds 2 X, so its ramp carries the factor 1/2 (exact)
        const float hf = o == 8 ? 0.5f : 1.0f;
        if constexpr (BM == 3) {
            c.ramp = make_float2(hf, 0.f);
        } else {
            float sn, cs;
            sincospif(2.0f * ((float)k * (g.frac / (float)N)), &sn, &cs);
            c.ramp = make_float2(hf * cs, hf * sn);
        }
        if constexpr (BM == 1 || BM == 2) {
            const float inv = 1.0f / a.scale[(int64_t)s * M + k];
            c.ramp = make_float2(c.ramp.x * inv, c.ramp.y * inv);
        }
    }
    const float2 wsp = a.wsp[nspec_j];  // W_2N1^j of the column-0 unfolding

    // ---- window fetch: thread t of slot t / L loads bytes 16 (t mod L) .. + 15
    const int fu = tid / L, ft = tid % L;
    const int m_f0 = mblk + SPS * fu;  // first spectrum of this thread's fetch slot
    const bool f_active = m_f0 < a.T;  // T is a multiple of 32
    const uint32_t *row = reinterpret_cast<const uint32_t *>(a.x + (int64_t)s * a.row_stride);
    const uint32_t sh = (uint32_t)(D & 3);
    uint32_t pw[5];
    auto fetch = [&](int m) {
        const int64_t o = (int64_t)m * N + D + 16 * ft;
        const int64_t w = o >> 2;
        pw[0] = row[w];
        pw[1] = row[w + 1];
        pw[2] = row[w + 2];
        pw[3] = row[w + 3];
        pw[4] = (o & 3) ? row[w + 4] : 0u;
    };
    if (f_active) fetch(m_f0);

    float2 *lb0 = &lds_b[0][0];
    float2 *lb1 = &lds_b[C::NBUF - 1][0];
    // spectra of the thread's column slot and of its column-0 channel
    const int m_c0 = mblk + SPS * bu, m_s0 = mblk + SPS * nspec_u;
    const bool c_active = m_c0 < a.T, s_active = m_s0 < a.T;
    // chunk index of channel k (16-byte units) within a spectrum group
    auto chunk_base = [&](int k) -> uint32_t {
        return (uint32_t)((((k >> 3) * a.S + s) << 3) + (k & 7));
    };

    // one spectrum r of the slot; H: the half of the INT8 / FP8 chunk it fills
    auto spectrum = [&](const int r, auto hsel) __attribute__((always_inline)) {
        constexpr int H = decltype(hsel)::value;
        // 1. stage the window bytes (buffer r mod 2: its last reader, stage A two
        //    spectra back, is behind the barriers of the previous spectrum), then
        //    fetch the next window
        // int8 -> FP16, exactly: b ^ 0x80 is b + 128 (0..255); under the byte 0x64 it
        // forms the FP16 number 1024 + b + 128, and one packed subtraction of 1152
        // leaves b (all integers below 2048 are FP16 numbers).  The subtraction is
        // written on the whole vector: written per FP16 pair, this compiler merged
        // the four byte selections into one.
        auto to_half8 = [](uint32_t w0, uint32_t w1) -> f4_half8 {
            const uint32_t x0 = w0 ^ 0x80808080u, x1 = w1 ^ 0x80808080u;
            f4_uint4 hb;
            hb[0] = __builtin_amdgcn_perm(0x64646464u, x0, 0x04010400u);
            hb[1] = __builtin_amdgcn_perm(0x64646464u, x0, 0x04030402u);
            hb[2] = __builtin_amdgcn_perm(0x64646464u, x1, 0x04010400u);
            hb[3] = __builtin_amdgcn_perm(0x64646464u, x1, 0x04030402u);
            return __builtin_bit_cast(f4_half8, hb) - (f4_half8)((_Float16)1152.0f);
        };
        if (f_active) {
            uint4 d;
            d.x = __builtin_amdgcn_alignbyte(pw[1], pw[0], sh);
            d.y = __builtin_amdgcn_alignbyte(pw[2], pw[1], sh);
            d.z = __builtin_amdgcn_alignbyte(pw[3], pw[2], sh);
            d.w = __builtin_amdgcn_alignbyte(pw[4], pw[3], sh);
            if constexpr (H16) {  // samples 16 ft .. 16 ft + 15: one row, 16 columns
                const int n = 16 * ft;
                _Float16 *dst = &lds_xh[fu][(n / N1) * XP + n % N1];
                *reinterpret_cast<f4_half8 *>(dst) = to_half8(d.x, d.y);
                *reinterpret_cast<f4_half8 *>(dst + 8) = to_half8(d.z, d.w);
            } else {
                *reinterpret_cast<uint4 *>(&lds_x[r & 1][fu][4 * ft]) = d;
            }
        }
        if (f_active && r + 1 < SPS) fetch(m_f0 + r + 1);
        __syncthreads();
        // 2. (*) on the matrix cores: hi and lo twiddle halves into one FP32 sum
        f4_float16 acc = {};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            f4_half8 bf;
            if constexpr (H16) {
                // two 16-bit transposing reads: rows (K) 0..3 and 4..7 of the lane's column
                const _Float16 *xb = &lds_xh[0][0] + t16_off + 16 * XP * kt;
                const f4_short4 k0 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_short4 *)xb);
                const f4_short4 k1 = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_short4 *)(xb + 4 * XP));
                bf = __builtin_bit_cast(f4_half8, __builtin_shufflevector(k0, k1, 0, 1, 2, 3, 4, 5, 6, 7));
            } else {
                const int8_t *lds_xb = reinterpret_cast<const int8_t *>(&lds_x[r & 1][0][0]);
                const f4_int2 raw = __builtin_amdgcn_ds_read_tr8_b64_v2i32(
                    (lds_int2 *)(lds_xb + tr_off + 16 * N1 * kt));
                bf = to_half8((uint32_t)raw[0], (uint32_t)raw[1]);
            }
            const f4_half8 alo = *reinterpret_cast<const f4_half8 *>(&lds_a[1][a_off + 16 * kt]);
            const f4_half8 ahi = *reinterpret_cast<const f4_half8 *>(&lds_a[0][a_off + 16 * kt]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(alo, bf, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(ahi, bf, acc, 0, 0, 0);
        }
        // 3. four-step twiddle, one LDS column per k2; rows k2 = 0 and 32 (column 0)
        //    become the folded real sequence y packed as u[j] = y[2j] + i y[2j + 1]
#pragma unroll
        for (int v = 0; v < 16; v += 2) {
            const int p = 16 * mt + 4 * (v >> 2) + 2 * hh + ((v & 3) >> 1);
            const float2 A = make_float2(acc[v], acc[v + 1]);
            if (v == 0 && mt == 0 && hh == 0) {
                float *u0 = reinterpret_cast<float *>(lb0 + (au * 32) * C::CS);
                const float y0 = 0.5f * (A.x + A.y), y1 = 0.5f * (A.x - A.y);
                u0[2 * padi(an1 >> 1) + (an1 & 1)] = y0;
                u0[2 * padi((an1 >> 1) + N1 / 2) + (an1 & 1)] = y1;
            } else {
                lb0[(au * 32 + p) * C::CS + padi(an1)] = cmul(A, tws[v >> 1]);
            }
        }
        // 4. the 32 column transforms
        __syncthreads();
        float2 z[8];
        col_passes<LOGM, 0>(lb0, lb1, lds_tw, colo, bb, z);
        if (cp == 0) {
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const int u = o / RL, q = o % RL;
                lds_u[bu * N1 + bb + C::BPC * u + q * (N1 / RL)] = z[o];
            }
        }
        // 5-6. phase, requantisation and corner turn of every channel
        const int mc = m_c0 + r;
        const float2 rot_c = lds_rot[SPS * bu + r];
        const uint32_t bsel = (0x03020100u & ~(0xFFu << (8 * (r & 3)))) | (0x04u << (8 * (r & 3)));
        uint4 *gbase_c = reinterpret_cast<uint4 *>(a.spec) + (int64_t)(mc / G) * M * a.S;
        if (cp != 0) {
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                const int q = o % RL;
                const int k = chan(o);
                const float2 X = q < RL / 2 ? z[o] : make_float2(z[o].x, -z[o].y);
                if (PW && c_active) store_power(((int64_t)s * a.T + mc) * M + k, X.x * X.x + X.y * X.y);
                emit<BM, H>(ch[o], X, rot_c, r, bsel, c_active, gbase_c + chunk_base(k));
            }
        }
        // column 0's outputs are written by threads ctid < J and unfolded by threads
        // ctid < NSPEC, both in wave wz, where the wave's own LDS order suffices
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (ctid < C::NSPEC) {
            const int ms = m_s0 + r;
            const float2 U = lds_u[nspec_u * N1 + nspec_j];
            const float2 V = lds_u[nspec_u * N1 + ((N1 - nspec_j) & (N1 - 1))];
            const float2 sm = make_float2(U.x + V.x, U.y - V.y), df = make_float2(U.x - V.x, U.y + V.y);
            // 2 X = (U + V*) - i W (U - V*)
            float2 X;
            X.x = fmaf(wsp.x, df.y, fmaf(wsp.y, df.x, sm.x));
            X.y = fmaf(-wsp.x, df.x, fmaf(wsp.y, df.y, sm.y));
            const float2 rot_s = lds_rot[SPS * nspec_u + r];
            uint4 *gbase_s = reinterpret_cast<uint4 *>(a.spec) + (int64_t)(ms / G) * M * a.S;
            // column 0 unfolds 2 X: power and the calibration sum take |X|^2 = |2 X|^2 / 4
            if constexpr (BM != 3) {
                if (PW && s_active) store_power(((int64_t)s * a.T + ms) * M + ch_s, 0.25f * (X.x * X.x + X.y * X.y));
                emit<BM, H>(ch[8], X, rot_s, r, bsel, s_active, gbase_s + chunk_base(ch_s));
            } else {
                ch[8].pacc += 0.25f * (X.x * X.x + X.y * X.y);
            }
        }
    };
    if constexpr ((BM == 1 || BM == 2) && PW == 0) {
        // spectra in chunks of 8: the first 4 fill one pair of words, the next 4
        // the other (which pair is a constant of each loop), then every chunk is
        // stored whole.  (With power cells the copy of the loop body for each
        // half does not fit the registers; those launches keep one loop.)
        constexpr uint32_t B = BM == 1 ? kI8Bias : 0u;
#pragma unroll 1
        for (int r8 = 0; r8 < SPS; r8 += 8) {
#pragma unroll 1
            for (int r = r8; r < r8 + 4; ++r) spectrum(r, std::integral_constant<int, 0>{});
#pragma unroll 1
            for (int r = r8 + 4; r < r8 + 8; ++r) spectrum(r, std::integral_constant<int, 1>{});
            if (cp != 0 && c_active) {
                uint4 *gb = reinterpret_cast<uint4 *>(a.spec) + (int64_t)((m_c0 + r8) / G) * M * a.S;
#pragma unroll
                for (int o = 0; o < 8; ++o)
                    gb[chunk_base(chan(o))] = make_uint4(ch[o].q0 ^ B, ch[o].q ^ B, ch[o].h0 ^ B, ch[o].h ^ B);
            }
            if (ctid < C::NSPEC && s_active) {
                uint4 *gb = reinterpret_cast<uint4 *>(a.spec) + (int64_t)((m_s0 + r8) / G) * M * a.S;
                gb[chunk_base(ch_s)] = make_uint4(ch[8].q0 ^ B, ch[8].q ^ B, ch[8].h0 ^ B, ch[8].h ^ B);
            }
        }
    } else {
#pragma unroll 1
        for (int r = 0; r < SPS; ++r) spectrum(r, std::integral_constant<int, -1>{});
    }

    if constexpr (BM == 3) {
        // partial sums per channel over this slot's 32 spectra: slots of 16 spectra in the
        // partial layout [S][T/16][C] -- the first holds the sum, the second zero
        if (c_active && cp != 0) {
            float *dst = a.part + ((int64_t)s * (a.T / 16) + (m_c0 >> 4)) * M;
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                dst[chan(o)] = ch[o].pacc;
                dst[M + chan(o)] = 0.f;
            }
        }
        if (ctid < C::NSPEC && s_active) {
            float *dst = a.part + ((int64_t)s * (a.T / 16) + (m_s0 >> 4)) * M;
            dst[ch_s] = ch[8].pacc;
            dst[M + ch_s] = 0.f;
        }
    }
}

template <int LOGM>
hipError_t launch4_one(int mode, const FLaunch &a, hipStream_t st) {
    using C = F4Cfg<LOGM>;
    const int spb = C::SPS * C::FPAR;
    const int nblk = (a.T + spb - 1) / spb;
    const dim3 grid(a.S * nblk), block(C::WG);
    const int pw = (mode == 3 || !a.power) ? 0 : (a.power_f16 ? 2 : 1);
    switch (mode | (pw << 2)) {
#define F4_CASE(m) \
    case m: hipLaunchKernelGGL((fengine4_kernel<LOGM, m>), grid, block, 0, st, a); break;
    F4_CASE(0) F4_CASE(1) F4_CASE(2) F4_CASE(3)     // no power cells
    F4_CASE(4) F4_CASE(5) F4_CASE(6)                // FP32 power
    F4_CASE(8) F4_CASE(9) F4_CASE(10)               // FP16 power
#undef F4_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

// Host tables of the four-step F-engine (FP64, rounded once):
//   afrag  [2][64][64] FP16 (hi, then lo): row 2p + d, column n2 of (*): p = 0 ->
//          (1, (-1)^n2); p >= 1 -> (cos, -sin)(2 pi n2 p / 64), hi the nearest
//          FP16, lo the nearest FP16 of the remainder
//   tw4    [32][N1] float2: W_N^(n1 p)
//   twb    Stockham twiddles of the N1-point column transforms (passes 1..)
//   wsp    [N1] float2: W_2N1^j of the column-0 unfolding
void fengine4_tables(int log2m, uint16_t *afrag, float2 *tw4, float2 *twb, size_t *ntwb, float2 *wsp) {
    const int N = 2 << log2m, N1 = N / 64, logn1 = log2m - 5;
    if (afrag) {
        for (int r = 0; r < 64; ++r)
            for (int n2 = 0; n2 < 64; ++n2) {
                const int p = r >> 1, d = r & 1;
                double w;
                if (p == 0) w = d == 0 ? 1.0 : ((n2 & 1) ? -1.0 : 1.0);
                else w = d == 0 ? std::cos(2.0 * M_PI * n2 * p / 64.0) : -std::sin(2.0 * M_PI * n2 * p / 64.0);
                const _Float16 hi = (_Float16)w;
                const _Float16 lo = (_Float16)(w - (double)hi);
                afrag[r * 64 + n2] = __builtin_bit_cast(uint16_t, hi);
                afrag[64 * 64 + r * 64 + n2] = __builtin_bit_cast(uint16_t, lo);
            }
    }
    if (tw4)
        for (int p = 0; p < 32; ++p)
            for (int n1 = 0; n1 < N1; ++n1) {
                const double b = -2.0 * M_PI * (double)n1 * (double)p / (double)N;
                tw4[p * N1 + n1] = make_float2((float)std::cos(b), (float)std::sin(b));
            }
    // per-pass Stockham twiddles of the column transforms: [pass][k][r] of W_(P R)^(r k)
    const int npass8 = logn1 / 3, rlast = 1 << (logn1 % 3);
    const int npass = npass8 + (rlast > 1 ? 1 : 0);
    size_t n = 0;
    for (int ps = 1; ps < npass; ++ps) {
        const int R = ps < npass8 ? 8 : rlast;
        const int P = 1 << (3 * ps);
        for (int k = 0; k < P; ++k)
            for (int r = 0; r < R; ++r, ++n)
                if (twb) {
                    const double b = -2.0 * M_PI * (double)r * (double)k / ((double)P * (double)R);
                    twb[n] = make_float2((float)std::cos(b), (float)std::sin(b));
                }
    }
    if (ntwb) *ntwb = n;
    if (wsp)
        for (int j = 0; j < N1; ++j) {
            const double b = -M_PI * (double)j / (double)N1;
            wsp[j] = make_float2((float)std::cos(b), (float)std::sin(b));
        }
}

int fengine4_spectra_per_block(int log2m) {
    switch (log2m) {
    case 8: return F4Cfg<8>::SPS * F4Cfg<8>::FPAR;
    case 10: return F4Cfg<10>::SPS * F4Cfg<10>::FPAR;
    case 11: return F4Cfg<11>::SPS * F4Cfg<11>::FPAR;
    default: return 0;
    }
}

hipError_t launch_fengine4(int log2m, int mode, const FLaunch &a, hipStream_t st) {
    switch (log2m) {
    case 8: return launch4_one<8>(mode, a, st);
    case 10: return launch4_one<10>(mode, a, st);
    case 11: return launch4_one<11>(mode, a, st);
    default: return hipErrorInvalidValue;  // the other lengths run on the LDS-radix kernel
    }
}

}  // namespace corr
