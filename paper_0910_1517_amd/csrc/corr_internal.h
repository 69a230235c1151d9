// corr_internal.h -- declarations shared by the translation units of libcorr
// (host API, F-engine, X-engine, integrator).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/corr.h"

namespace corr {

// Geometry as the kernels read it (same bytes as corr_geom_t).
static_assert(sizeof(corr_geom_t) == 24, "corr_geom_t must stay 24 bytes");

// Largest signal count the X-engine tiles handle (two 32-signal MFMA tiles).
constexpr int kMaxSignals = 64;
// Spectra per 16-byte X-layout chunk: 8 for the 8-bit precisions, 2 for FP32.
constexpr int kChunk8 = 8;
constexpr int kChunk32 = 2;
// MAD flagging tiles: spectra x channels.
constexpr int kFlagTileSpectra = 64;
constexpr int kFlagTileChannels = 256;
// int32 accumulator bound: 2 * 127^2 * T <= 2^31 - 1.
constexpr int64_t kMaxInt8Spectra = 66572;

// Device workspace layout (byte offsets from the bound base pointer).
struct WsLayout {
    size_t twp;       // float2[sum P R] per-pass Stockham twiddles W_{PR}^{rk}, [pass][k][r]
    size_t wn;        // float2[M]   exp(-2 pi i k / N), real-FFT post-process
    size_t pairs;     // uint16[2P]  (i, j) of each pair index
    size_t err;       // uint32[4]   device error words
    size_t part;      // float[S][nblk*fpar][C] calibration partial sums
    size_t lut;       // float2[kLutSteps] cos, sin of 2 pi j / kLutSteps (table mode)
    size_t afrag;     // uint16[2][64][64] FP16 rows of the DFT-64 (four-step F-engine)
    size_t tw4;       // float2[N1][32]    W_N^(n1 k2)
    size_t twb;       // float2[...]       column-pass twiddles
    size_t wsp;       // float2[N1]        W_2N1^j
    size_t w16;       // int2[kLutSteps]   Q14 phase table of the 16-bit fixed-point path
    size_t total;
};

struct FLaunch {
    const int8_t *x;
    int64_t row_stride;
    const corr_geom_t *geom;
    int64_t spectrum0;
    void *spec;
    const float *scale;  // HOLD-mode scales [S][C]
    float *part;         // calibration partials
    void *power;         // optional power output [S][T][C] (nullptr: none)
    int power_f16;       // 0: FP32 |X|^2; 1: FP16 |X|^2 * power_scale
    float power_scale;   // 1 / N^2 (exact) for FP16
    const float2 *twp;
    const float2 *wn;
    uint32_t *err;
    int S;
    int T;
    int max_delay;
    int sideband;
    double fs;
    double nu_bb;
    const float2 *lut;   // phase table (table mode only)
    // four-step F-engine tables (fengine4_tables)
    const uint16_t *afrag;
    const float2 *tw4;
    const float2 *twb;
    const float2 *wsp;
};

// The requantisation encoders shared by both F-engines and corr_requantize
// (section 4.1's fixed point ahead of the MAC, at 8 bits).
//
// OCP e4m3 codes (bias 7, max 448) of two already-scaled values, in bytes 0
// and 1: nearest-even, saturating to +-448, a value that rounds to zero
// encoded as +0 whatever its sign.  The hardware conversion rounds to nearest
// even; the clamp makes it saturate, and flushing |v| <= 2^-10 (half the
// smallest subnormal, a tie that rounds to 0) to +0 keeps it from writing -0.
// NaN leaves the clamp as -448 (code 0xFE); +-inf saturate to +-448.
__device__ __forceinline__ uint32_t e4m3_pair(float a, float b) {
    float ca = fminf(fmaxf(a, -448.f), 448.f), cb = fminf(fmaxf(b, -448.f), 448.f);
    ca = fabsf(ca) <= 0x1p-10f ? 0.f : ca;
    cb = fabsf(cb) <= 0x1p-10f ? 0.f : cb;
    return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(ca, cb, 0, false);
}

// int8 code of an already-scaled value in the low byte: clamp to [-127, 127]
// (integers, so the clamp commutes with rounding), then add 1.5 * 2^23 -- the
// FP32 add rounds to the nearest integer, ties to even, and leaves it in the
// low mantissa bits, whose low byte is the two's-complement code.  NaN leaves
// the clamp as -127.
__device__ __forceinline__ uint32_t quant_i8(float v) {
    const float c = fminf(fmaxf(v, -127.0f), 127.0f);
    return __float_as_uint(c + 12582912.0f);  // only the low byte is used
}

// The F-engines' int8 code, biased: vb is the scaled value plus 128 (formed
// inside the value's last products).  Clamped below at 1 (code -127; NaN too),
// converted with rounding to nearest even and saturation at 255 (code +127)
// into byte sel of w.  The word's bytes are the codes xor 0x80.  Adding 128
// before the rounding moves a result only within 2^-16 of a .5 boundary.
__device__ __forceinline__ uint32_t put_i8_biased(float vb, int sel, uint32_t w) {
    return __builtin_amdgcn_cvt_pk_u8_f32(fmaxf(vb, 1.0f), sel, w);
}
constexpr uint32_t kI8Bias = 0x80808080u;

// One power cell of the F-engine: FP32 |X|^2, or FP16 |X|^2 / N^2 (nearest even).
__device__ __forceinline__ void put_power(const FLaunch &a, int64_t i, float p) {
    if (a.power_f16)
        reinterpret_cast<_Float16 *>(a.power)[i] = (_Float16)(p * a.power_scale);
    else
        reinterpret_cast<float *>(a.power)[i] = p;
}

// Which F-engine serves a launch: the four-step (matrix-core) one at log2 M =
// 8, 10 and 11 outside table mode (launch modes 0-3), the LDS-radix one
// (fengine.hip) otherwise.  The choice is measured: 64 signals of 2^27
// samples, int8 output, ms per call
//   log2 M         8      9      10     11     12
//   four-step    7.99  10.20   9.40   9.64  15.92
//   LDS-radix    9.05   9.28  10.35  10.69  12.12
// (FP32 output: the four-step kernel 2-15% faster at 8-11, 10% slower at 12;
// table mode at 11: 14.7 against 12.0 ms); at 13 the four-step kernel spills
// registers.
constexpr bool use_fengine4(int log2m, int mode) {
    return mode < 4 && (log2m == 8 || log2m == 10 || log2m == 11);
}

// Phase look-up table of section 2.3.2: 1440 steps of 0.25 degrees.
constexpr int kLutSteps = 1440;
// mode: 0 FP32 spectra, 1 INT8, 2 FP8, 3 calibration partial sums; 4..6 = the
// first three with the phase from the table

hipError_t launch_fengine(int log2m, int mode, const FLaunch &a, hipStream_t st);
// geometry of the F-engine launch: spectra handled per workgroup, workgroups per signal
int fengine_spectra_per_block(int log2m);
int fengine_fpar(int log2m);
// per-pass twiddle table of the Stockham passes: W_{P R}^{r k} at [pass][k][r]
void fengine_twiddle_table(int log2m, float2 *out, size_t *count);

// Four-step F-engine (fengine4.hip): the first step, a real DFT-64 of the
// int8 samples, on the FP16 matrix cores.  Tables: afrag 2 x 64 x 64 FP16,
// tw4 N1 x 32, twb the column-pass twiddles (count in *ntwb), wsp N1 (N1 = N/64).
void fengine4_tables(int log2m, uint16_t *afrag, float2 *tw4, float2 *twb, size_t *ntwb, float2 *wsp);
int fengine4_spectra_per_block(int log2m);
hipError_t launch_fengine4(int log2m, int mode, const FLaunch &a, hipStream_t st);

// 16-bit fixed-point numerics (fix16.hip)
void fix16_table(int2 *w);  // rint(2^14 cos, sin) of the kLutSteps phase steps
hipError_t launch_fix16(const void *spec, const corr_geom_t *geom, int64_t spectrum0, const float *scale,
                        const int2 *wtab, int S, int T, int C, double fs, double nu_bb, int sideband, int16_t *q16,
                        int16_t *y16, hipStream_t st);
hipError_t launch_xengine16(const int16_t *y16, int S, int64_t T, int C, const float *scale, int64_t *acc,
                            double *vis, hipStream_t st);

hipError_t launch_calib_reduce(const float *part, int S, int C, int nparts, int T, int precision,
                               float *scale, hipStream_t st);

// keep: bit-packed keep words [C/8][T/32][S][8] whose clear bits are zeroed as the
// spectra are staged (NULL: every cell)
hipError_t launch_xengine(int precision, const void *spec, const uint32_t *keep, void *acc, int S, int C, int T,
                          int splits, hipStream_t st);
// Gated X-engine: accumulator set b (acc_elems elements apart) sums the
// spectra m with gate[m] == b, for b < n_bins.
hipError_t launch_xengine_gated(int precision, const void *spec, const uint8_t *gate, int n_bins, void *acc,
                                int64_t acc_elems, int S, int C, int T, int splits, hipStream_t st);
// Batched int8 X-engine: one entry per correlation; correlation i owns the
// workgroups [first[i], first[i+1]), one per (channel block of 8, split).
constexpr int kMaxBatch = 8;
struct XBatchEntry {
    const void *spec;
    void *acc;
    int S, C, T, splits;
};
struct XBatchArgs {
    XBatchEntry cor[kMaxBatch];
    int first[kMaxBatch + 1];
    int n;
};
hipError_t launch_xengine_batch(const XBatchArgs &a, hipStream_t st);
hipError_t launch_xpack(int precision, const void *in, void *spec, int S, int C, int T,
                        hipStream_t st);
hipError_t launch_requantize(int precision, const float *in, const float *scale, int S, int64_t T, int C,
                             uint8_t *out, hipStream_t st);

hipError_t launch_mad_flag(const void *power, bool f16, int S, int T, int C, float M, uint8_t *flags,
                           hipStream_t st);
hipError_t launch_apply_flags(int precision, const uint8_t *flags, void *spec, uint32_t *keep, int S, int T,
                              int C, hipStream_t st);
hipError_t launch_pair_counts(const uint32_t *keep, int S, int T, int C, int32_t *counts, hipStream_t st);

// Ascending bitonic sort of n (power of two, <= blockDim.x) floats in LDS;
// every thread of the block must call it.
__device__ inline void block_sort(float *v, int n) {
    const int t = threadIdx.x;
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (t < n) {
                const int p = t ^ j;
                if (p > t) {
                    const float a = v[t], b = v[p];
                    const bool up = (t & k) == 0;
                    if ((a > b) == up) {
                        v[t] = b;
                        v[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Ascending bitonic sort of 4 x 64 = 256 floats held by one wave, element
// 4 lane + q in v[q]: exchanges at distance >= 4 go across lanes with
// __shfl_xor, shorter ones stay in registers.  No barriers.
__device__ inline void wave_sort256(float (&v)[4], int lane) {
#pragma unroll
    for (int k = 2; k <= 256; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 4) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float o = __shfl_xor(v[q], j >> 2);
                    const int e = 4 * lane + q;
                    const bool keep_min = ((e & j) == 0) == ((e & k) == 0);
                    v[q] = keep_min ? fminf(v[q], o) : fmaxf(v[q], o);
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q & j) continue;
                    const int e = 4 * lane + q;
                    const float a = v[q], b = v[q ^ j];
                    const bool up = (e & k) == 0;
                    v[q] = up ? fminf(a, b) : fmaxf(a, b);
                    v[q ^ j] = up ? fmaxf(a, b) : fminf(a, b);
                }
            }
        }
    }
}

// Median (mean of the two middle values) of the 256 floats of a wave.
__device__ inline float wave_median256(float (&v)[4], int lane) {
    wave_sort256(v, lane);
    return 0.5f * (__shfl(v[3], 31) + __shfl(v[0], 32));  // sorted elements 127 and 128
}

// Median of |s_i - med| over the 256 values s that wave_median256 sorted into v
// (s[4 lane + q] in v[q]), med their median, without a second sort.  Below the
// median the deviations A[i] = med - s[127 - i] ascend with i, above it
// B[j] = s[128 + j] - med ascend with j (both exactly the FP32 |s - med|), so
// the 128 smallest deviations are A[0 .. p - 1] and B[0 .. 127 - p] for the
// split p = #{i < 128 : B[127 - i] > A[i]} (the comparison holds on a prefix
// of i), and the two middle ones are max(A[p - 1], B[127 - p]) and
// min(A[p], B[128 - p]).  buf: 256 floats of LDS used by this wave alone.
__device__ inline float wave_mad256_sorted(const float (&v)[4], float med, int lane, float *buf) {
    *reinterpret_cast<float4 *>(buf + 4 * lane) = make_float4(v[0], v[1], v[2], v[3]);
    int p = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int i = lane + 64 * h;
        p += __popcll(__ballot(buf[255 - i] - med > med - buf[127 - i]));
    }
    const float inf = __builtin_inff();
    const float a_lo = med - buf[p > 0 ? 128 - p : 0];     // A[p - 1]
    const float b_lo = buf[p < 128 ? 255 - p : 128] - med;  // B[127 - p]
    const float a_hi = med - buf[p < 128 ? 127 - p : 0];   // A[p]
    const float b_hi = buf[p > 0 ? 256 - p : 128] - med;    // B[128 - p]
    const float lo = fmaxf(p > 0 ? a_lo : -inf, p < 128 ? b_lo : -inf);
    const float hi = fminf(p < 128 ? a_hi : inf, p > 0 ? b_hi : inf);
    return 0.5f * (lo + hi);
}

hipError_t launch_beamform(int precision, const void *spec, const float *scale, const float *w, const float *cb,
                           int n_beams, int S, int C, int64_t T, int tint, int mode, float *inc, float *coh,
                           hipStream_t st);
hipError_t launch_integrate(int precision, void *acc, const float *scale, double *state,
                            float *vis, const uint16_t *pairs, int S, int C, int splits,
                            uint32_t flags, hipStream_t st);

// Learned flagger (cnn.hip).  Parameters: flat FP32 vector, layer by layer,
// weights [Cout][Cin][3][3] then biases.
constexpr int kCnnParams = 16 * 9 + 16 + 16 * 16 * 9 + 16 + 16 * 9 + 1;  // 2625
// inference addresses a tile's cells with 32-bit offsets r C + c (r <= 66)
constexpr int kCnnMaxInferChannels = 1 << 22;
constexpr int kCnnPixels = kFlagTileSpectra * kFlagTileChannels;      // 16384 per tile
// per-tile training blocks (8 x 64 pixels) and the widest per-block gradient
constexpr int kCnnBlocksPerTile = 32;
constexpr int kCnnGradEntries = 16 * 16 * 9 + 16;
struct CnnTrainBufs {
    float *x, *y, *z1, *z2, *z3, *d3, *d2, *d1, *part, *grad, *loss;
    double *lpart;
    uint32_t *err;
};
constexpr int kCnnLossBlocks = 1024;
// FP32 training path on n tiles listed in tiles (tile id = (s ntm + mt) ntk + kt)
hipError_t launch_cnn_gather(const float *power, const uint8_t *labels, int S, int64_t T, int C,
                             const int32_t *tiles, int n, const CnnTrainBufs &b, hipStream_t st);
hipError_t launch_cnn_forward(const float *params, int n, const CnnTrainBufs &b, hipStream_t st);
hipError_t launch_cnn_backward(const float *params, int n, const CnnTrainBufs &b, float *grad, float *loss,
                               hipStream_t st);
hipError_t launch_cnn_adam(float *params, float *m, float *v, const float *grad, float lr, float beta1,
                           float beta2, float eps, float c1, float c2, hipStream_t st);
// fused FP16 MFMA inference over every tile of power [S][T][C]
hipError_t launch_cnn_infer(const float *params, const void *power, bool f16, int S, int64_t T, int C,
                            float thr_logit, float guard_m, uint8_t *flags, float *logits, hipStream_t st);

}  // namespace corr
