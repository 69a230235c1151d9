// xengine.hip -- X-engine of the FX correlator on gfx950 matrix cores.
//
// For every channel k the visibility matrix is the Hermitian rank-T update
//   V_k = sum_m y_m y_m^H      (y_m = the S signals' spectra at (m, k))
// over all signal pairs, autocorrelations and cross polarisations included
// (section 2.1: RR*, RL*, LR*, LL* of every baseline; the MAC of sections
// 2.3.2 / 3.4).  With y = r + i q:
//   Re V = r r^T + q q^T        Im V = M - M^T,  M = q r^T
// so each channel needs three real products over the spectra: r r^T and q q^T
// on the upper triangle of 32x32 signal tiles and M on all tiles.  They map
// directly onto 32x32 MFMA tiles whose K dimension is the time axis:
//   INT8   v_mfma_i32_32x32x32_i8   (exact int32 sums)
//   FP8    v_mfma_f32_32x32x16_fp8_fp8 (OCP e4m3, FP32 sums)
//   FP32   v_mfma_f32_32x32x2_f32
// A and B operands are loaded straight from the X layout into registers: lane
// l holds signal 32a + (l mod 32) and the chunks of spectra picked by l / 32;
// since A and B lanes hold the same spectra in the same byte order, the
// product is exact regardless of how the hardware orders K inside a lane.
// X layout: 16-byte chunks indexed [g][k/8][s][k mod 8] (g = chunk of spectra),
// so the chunks of 8 consecutive channels of one signal form one 128-byte
// line.  A workgroup of 8 waves owns 8 consecutive channels and one split of
// the spectra; wave w handles channel 8 kb + w, so the 8 waves together read
// whole lines.  Each wave keeps its accumulator tiles in registers and at the
// end forms Im = M - M^T through LDS and adds its result into
// acc[split][k][p] (sole owner, so no atomics and a fixed order).
#include "corr_internal.h"

namespace corr {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int ntri(int nt) { return nt * (nt + 1) / 2; }
// index of tile pair (a <= b) in the upper triangle
__device__ __forceinline__ constexpr int tri_idx(int a, int b) { return b * (b + 1) / 2 + a; }

// Row of accumulator register r held by lane group lg (32x32 MFMA D layout).
__device__ __forceinline__ int acc_row(int r, int lg) { return 8 * (r >> 2) + 4 * lg + (r & 3); }

// Epilogue shared by all precisions: accR / accM hold sums in ACC type.
template <int NT, typename ACC, typename V16>
__device__ __forceinline__ void x_epilogue(const V16 (&accR)[ntri(NT)], const V16 (&accM)[NT * NT],
                                           ACC *acc_out, int S, int64_t P, ACC (*mlds)[32][33]) {
    const int lane = threadIdx.x & 63, col = lane & 31, lg = lane >> 5;
#pragma unroll
    for (int t = 0; t < NT * NT; ++t)
#pragma unroll
        for (int r = 0; r < 16; ++r) mlds[t][acc_row(r, lg)][col] = accM[t][r];
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NT; ++b)
#pragma unroll
        for (int a = 0; a <= b; ++a) {
            const int J = 32 * b + col;
            if (J >= S) continue;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int i = acc_row(r, lg);
                const int I = 32 * a + i;
                if (I > J) continue;
                const ACC re = accR[tri_idx(a, b)][r];
                const ACC im = mlds[a * NT + b][i][col] - mlds[b * NT + a][col][i];
                const int64_t p = (int64_t)J * (J + 1) / 2 + I;
                ACC *dst = acc_out + 2 * p;
                dst[0] += re;
                dst[1] += im;
            }
        }
}

// Chunk indices of K-step st: lanes 0-31 take chunks 4st and 4st+2, lanes
// 32-63 chunks 4st+1 and 4st+3 (the two lane groups form the K halves).
// INT8/FP8 chunk: 8 real bytes then 8 imaginary bytes; FP32 chunk: 2 complex64.
constexpr int kXWaves = 8;  // channels (waves) per workgroup

// ---------------------------------------------------------------- INT8 ----
template <int NT>
__global__ void __launch_bounds__(64 * kXWaves) xengine_i8_kernel(const uint8_t *__restrict__ spec, int32_t *acc,
                                                          int S, int C, int T, int splits) {
    __shared__ int32_t mlds[kXWaves][NT * NT][32][33];
    const int kb = blockIdx.x, sp = blockIdx.y, wv = threadIdx.x >> 6, c = kXWaves * kb + wv;
    const int lane = threadIdx.x & 63, row = lane & 31, lg = lane >> 5;
    const int ngrp = T / kChunk8;
    const int steps = ngrp / 4 / splits;  // K-steps of 32 spectra for this split
    const int64_t P = (int64_t)S * (S + 1) / 2;
    // chunk (g, s) of channel c at 16-byte index g C S + (kb S + s) 8 + wv
    const v4i *base = reinterpret_cast<const v4i *>(spec) + (int64_t)kb * S * 8 + wv;
    const int64_t gstride = (int64_t)C * S;

    v16i accR[ntri(NT)], accM[NT * NT];
#pragma unroll
    for (int t = 0; t < ntri(NT); ++t) accR[t] = v16i{0};
#pragma unroll
    for (int t = 0; t < NT * NT; ++t) accM[t] = v16i{0};

    bool valid[NT];
#pragma unroll
    for (int a = 0; a < NT; ++a) valid[a] = (32 * a + row) < S;

    auto load = [&](int st, v4i (&c0)[NT], v4i (&c1)[NT]) {
        const int g0 = 4 * (sp * steps + st) + lg;
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            if (valid[a]) {
                c0[a] = base[g0 * gstride + (32 * a + row) * 8];
                c1[a] = base[(g0 + 2) * gstride + (32 * a + row) * 8];
            } else {
                c0[a] = v4i{0};
                c1[a] = v4i{0};
            }
        }
    };

    v4i c0[NT], c1[NT], n0[NT], n1[NT];
    load(0, c0, c1);
    for (int st = 0; st < steps; ++st) {
        if (st + 1 < steps) load(st + 1, n0, n1);
        v4i im[NT], re[NT];  // imaginary / real bytes of both chunks
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            im[a] = v4i{c0[a].z, c0[a].w, c1[a].z, c1[a].w};
            re[a] = v4i{c0[a].x, c0[a].y, c1[a].x, c1[a].y};
        }
#pragma unroll
        for (int b = 0; b < NT; ++b) {
#pragma unroll
            for (int a = 0; a <= b; ++a) {
                v16i &d = accR[tri_idx(a, b)];
                d = __builtin_amdgcn_mfma_i32_32x32x32_i8(c0[a], c0[b], d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_i32_32x32x32_i8(c1[a], c1[b], d, 0, 0, 0);
            }
#pragma unroll
            for (int a = 0; a < NT; ++a)
                accM[a * NT + b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(im[a], re[b], accM[a * NT + b], 0, 0, 0);
        }
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            c0[a] = n0[a];
            c1[a] = n1[a];
        }
    }
    x_epilogue<NT, int32_t>(accR, accM, acc + ((int64_t)sp * C + c) * P * 2, S, P, &mlds[wv][0]);
}

// ----------------------------------------------------------------- FP8 ----
template <int NT>
__global__ void __launch_bounds__(64 * kXWaves) xengine_f8_kernel(const uint8_t *__restrict__ spec, float *acc,
                                                          int S, int C, int T, int splits) {
    __shared__ float mlds[kXWaves][NT * NT][32][33];
    const int kb = blockIdx.x, sp = blockIdx.y, wv = threadIdx.x >> 6, c = kXWaves * kb + wv;
    const int lane = threadIdx.x & 63, row = lane & 31, lg = lane >> 5;
    const int ngrp = T / kChunk8;
    const int steps = ngrp / 4 / splits;
    const int64_t P = (int64_t)S * (S + 1) / 2;
    // chunk (g, s) of channel c at 16-byte index g C S + (kb S + s) 8 + wv
    const v4i *base = reinterpret_cast<const v4i *>(spec) + (int64_t)kb * S * 8 + wv;
    const int64_t gstride = (int64_t)C * S;

    v16f accR[ntri(NT)], accM[NT * NT];
#pragma unroll
    for (int t = 0; t < ntri(NT); ++t) accR[t] = v16f{0.f};
#pragma unroll
    for (int t = 0; t < NT * NT; ++t) accM[t] = v16f{0.f};

    bool valid[NT];
#pragma unroll
    for (int a = 0; a < NT; ++a) valid[a] = (32 * a + row) < S;

    auto load = [&](int st, v4i (&c0)[NT], v4i (&c1)[NT]) {
        const int g0 = 4 * (sp * steps + st) + lg;
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            if (valid[a]) {
                c0[a] = base[g0 * gstride + (32 * a + row) * 8];
                c1[a] = base[(g0 + 2) * gstride + (32 * a + row) * 8];
            } else {
                c0[a] = v4i{0};
                c1[a] = v4i{0};
            }
        }
    };
    auto lo = [](v4i v) { return (long)(((unsigned long)(unsigned)v.y << 32) | (unsigned)v.x); };
    auto hi = [](v4i v) { return (long)(((unsigned long)(unsigned)v.w << 32) | (unsigned)v.z); };

    v4i c0[NT], c1[NT], n0[NT], n1[NT];
    load(0, c0, c1);
    for (int st = 0; st < steps; ++st) {
        if (st + 1 < steps) load(st + 1, n0, n1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            long re[NT], im[NT];
#pragma unroll
            for (int a = 0; a < NT; ++a) {
                re[a] = lo(h ? c1[a] : c0[a]);
                im[a] = hi(h ? c1[a] : c0[a]);
            }
#pragma unroll
            for (int b = 0; b < NT; ++b) {
#pragma unroll
                for (int a = 0; a <= b; ++a) {
                    v16f &d = accR[tri_idx(a, b)];
                    d = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(re[a], re[b], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(im[a], im[b], d, 0, 0, 0);
                }
#pragma unroll
                for (int a = 0; a < NT; ++a)
                    accM[a * NT + b] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(im[a], re[b], accM[a * NT + b], 0, 0, 0);
            }
        }
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            c0[a] = n0[a];
            c1[a] = n1[a];
        }
    }
    x_epilogue<NT, float>(accR, accM, acc + ((int64_t)sp * C + c) * P * 2, S, P, &mlds[wv][0]);
}

// ----------------------------------------------------------------- FP32 ---
template <int NT>
__global__ void __launch_bounds__(64 * kXWaves) xengine_f32_kernel(const float *__restrict__ spec, float *acc,
                                                           int S, int C, int T, int splits) {
    __shared__ float mlds[kXWaves][NT * NT][32][33];
    const int kb = blockIdx.x, sp = blockIdx.y, wv = threadIdx.x >> 6, c = kXWaves * kb + wv;
    const int lane = threadIdx.x & 63, row = lane & 31, lg = lane >> 5;
    const int ngrp = T / kChunk32;
    const int steps = ngrp / 4 / splits;  // K-steps of 8 spectra
    const int64_t P = (int64_t)S * (S + 1) / 2;
    const float4 *base = reinterpret_cast<const float4 *>(spec) + (int64_t)kb * S * 8 + wv;
    const int64_t gstride = (int64_t)C * S;

    v16f accR[ntri(NT)], accM[NT * NT];
#pragma unroll
    for (int t = 0; t < ntri(NT); ++t) accR[t] = v16f{0.f};
#pragma unroll
    for (int t = 0; t < NT * NT; ++t) accM[t] = v16f{0.f};

    bool valid[NT];
#pragma unroll
    for (int a = 0; a < NT; ++a) valid[a] = (32 * a + row) < S;

    auto load = [&](int st, float4 (&c0)[NT], float4 (&c1)[NT]) {
        const int g0 = 4 * (sp * steps + st) + lg;
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            if (valid[a]) {
                c0[a] = base[g0 * gstride + (32 * a + row) * 8];
                c1[a] = base[(g0 + 2) * gstride + (32 * a + row) * 8];
            } else {
                c0[a] = make_float4(0.f, 0.f, 0.f, 0.f);
                c1[a] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
    };

    float4 c0[NT], c1[NT], n0[NT], n1[NT];
    load(0, c0, c1);
    for (int st = 0; st < steps; ++st) {
        if (st + 1 < steps) load(st + 1, n0, n1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {  // spectra (chunk 0: 0, 1; chunk 1: 2, 3)
            float rr[NT], qq[NT];
#pragma unroll
            for (int a = 0; a < NT; ++a) {
                if (q == 0) { rr[a] = c0[a].x; qq[a] = c0[a].y; }
                if (q == 1) { rr[a] = c0[a].z; qq[a] = c0[a].w; }
                if (q == 2) { rr[a] = c1[a].x; qq[a] = c1[a].y; }
                if (q == 3) { rr[a] = c1[a].z; qq[a] = c1[a].w; }
            }
#pragma unroll
            for (int b = 0; b < NT; ++b) {
#pragma unroll
                for (int a = 0; a <= b; ++a) {
                    v16f &d = accR[tri_idx(a, b)];
                    d = __builtin_amdgcn_mfma_f32_32x32x2f32(rr[a], rr[b], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_32x32x2f32(qq[a], qq[b], d, 0, 0, 0);
                }
#pragma unroll
                for (int a = 0; a < NT; ++a)
                    accM[a * NT + b] = __builtin_amdgcn_mfma_f32_32x32x2f32(qq[a], rr[b], accM[a * NT + b], 0, 0, 0);
            }
        }
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            c0[a] = n0[a];
            c1[a] = n1[a];
        }
    }
    x_epilogue<NT, float>(accR, accM, acc + ((int64_t)sp * C + c) * P * 2, S, P, &mlds[wv][0]);
}

// --------------------------------------------------------------- xpack ----
// Corner turn [S][T][C][2] -> X layout; one thread per (k, chunk, s).
template <typename E, int G>
__global__ void xpack_kernel(const E *__restrict__ in, E *out, int S, int C, int T) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ngrp = T / G;
    const int64_t total = (int64_t)C * ngrp * S;
    if (idx >= total) return;
    const int s = (int)(idx % S);
    const int64_t rest = idx / S;
    const int tg = (int)(rest % ngrp);
    const int k = (int)(rest / ngrp);
    // X layout: 16-byte chunk index g C S + ((k / 8) S + s) 8 + k mod 8
    E *dst = out + ((int64_t)tg * C * S + ((int64_t)(k >> 3) * S + s) * 8 + (k & 7)) * (2 * G);
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const E *src = in + (((int64_t)s * T + (int64_t)tg * G + q) * C + k) * 2;
        if (G == kChunk8) {  // planar: G real parts then G imaginary parts
            dst[q] = src[0];
            dst[G + q] = src[1];
        } else {             // interleaved complex
            dst[2 * q] = src[0];
            dst[2 * q + 1] = src[1];
        }
    }
}

}  // namespace

hipError_t launch_xengine(int precision, const void *spec, void *acc, int S, int C, int T, int splits,
                          hipStream_t st) {
    const dim3 grid(C / kXWaves, splits), block(64 * kXWaves);
    const bool two = S > 32;
    switch (precision) {
    case CORR_INT8:
        if (two) hipLaunchKernelGGL(xengine_i8_kernel<2>, grid, block, 0, st, (const uint8_t *)spec, (int32_t *)acc, S, C, T, splits);
        else hipLaunchKernelGGL(xengine_i8_kernel<1>, grid, block, 0, st, (const uint8_t *)spec, (int32_t *)acc, S, C, T, splits);
        break;
    case CORR_FP8_E4M3:
        if (two) hipLaunchKernelGGL(xengine_f8_kernel<2>, grid, block, 0, st, (const uint8_t *)spec, (float *)acc, S, C, T, splits);
        else hipLaunchKernelGGL(xengine_f8_kernel<1>, grid, block, 0, st, (const uint8_t *)spec, (float *)acc, S, C, T, splits);
        break;
    case CORR_FP32:
        if (two) hipLaunchKernelGGL(xengine_f32_kernel<2>, grid, block, 0, st, (const float *)spec, (float *)acc, S, C, T, splits);
        else hipLaunchKernelGGL(xengine_f32_kernel<1>, grid, block, 0, st, (const float *)spec, (float *)acc, S, C, T, splits);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_xpack(int precision, const void *in, void *spec, int S, int C, int T, hipStream_t st) {
    const int G = precision == CORR_FP32 ? kChunk32 : kChunk8;
    const int64_t total = (int64_t)C * (T / G) * S;
    const dim3 grid((unsigned)((total + 255) / 256)), block(256);
    if (precision == CORR_FP32)
        hipLaunchKernelGGL((xpack_kernel<float, kChunk32>), grid, block, 0, st, (const float *)in, (float *)spec, S, C, T);
    else
        hipLaunchKernelGGL((xpack_kernel<uint8_t, kChunk8>), grid, block, 0, st, (const uint8_t *)in, (uint8_t *)spec, S, C, T);
    return hipGetLastError();
}

}  // namespace corr
