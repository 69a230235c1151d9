// B-engine: incoherent and coherent (phased) array beams from the X-layout
// spectra, the beamformer of section 2.2 (two modes: detected intensities added,
// or voltages added and then detected, with the voltage cross products that
// the Stokes parameters need) run on the F-engine output as in section 2.3.2.
//
// Per spectrum m, channel k and polarisation pol (signals s = 2a + pol), with
// Y_s the dequantised spectra:
//   incoherent   I_pol = sum_s w_s |Y_s|^2
//   coherent b   V_b,pol = sum_s c_b,s Y_s   (c complex: gain and antenna phase)
// One thread per channel and 8 consecutive spectra: it walks the S signals of
// its channel (contiguous 16-byte chunks of the X layout, 128-byte lines per 8
// channels), keeps every sum in registers and writes channel-contiguous rows.
// The dequantisation is folded into the weights: w_s scale^2 and c_b,s scale.
#include "corr_internal.h"

namespace corr {
namespace {

constexpr int BK = 256;  // channels per workgroup, one per thread

// The 8 spectra of one chunk group of signal s as raw values (codes for
// INT8 / FP8; the scale is applied through the weights).
template <int PREC>
struct Chunk {
    static constexpr int N = PREC == CORR_FP32 ? 4 : 1;  // 16-byte chunks per 8 spectra
    uint4 v[N];
};

template <int PREC>
__device__ inline void load_chunk(const uint4 *__restrict__ spec, int64_t c0, int64_t gstride, Chunk<PREC> &ch) {
#pragma unroll
    for (int j = 0; j < Chunk<PREC>::N; ++j) ch.v[j] = spec[c0 + j * gstride];
}

template <int PREC>
__device__ inline void decode(const Chunk<PREC> &ch, float (&re)[8], float (&im)[8]) {
    if constexpr (PREC == CORR_FP32) {
        // chunk j: spectra 2j, 2j + 1 as two complex64
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            re[2 * j] = __uint_as_float(ch.v[j].x);
            im[2 * j] = __uint_as_float(ch.v[j].y);
            re[2 * j + 1] = __uint_as_float(ch.v[j].z);
            im[2 * j + 1] = __uint_as_float(ch.v[j].w);
        }
    } else {
        // bytes 0..7: real parts of the 8 spectra, bytes 8..15: imaginary parts
        auto four = [](uint32_t v, float *o) {
            if constexpr (PREC == CORR_INT8) {
#pragma unroll
                for (int i = 0; i < 4; ++i) o[i] = (float)(int8_t)(v >> (8 * i));
            } else {  // OCP e4m3, the encoding the F-engine writes
                o[0] = __builtin_amdgcn_cvt_f32_fp8((int)v, 0);
                o[1] = __builtin_amdgcn_cvt_f32_fp8((int)v, 1);
                o[2] = __builtin_amdgcn_cvt_f32_fp8((int)v, 2);
                o[3] = __builtin_amdgcn_cvt_f32_fp8((int)v, 3);
            }
        };
        four(ch.v[0].x, re);
        four(ch.v[0].y, re + 4);
        four(ch.v[0].z, im);
        four(ch.v[0].w, im + 4);
    }
}

// Sums of outputs over tint = 2^lt consecutive spectra (lt = 0..3): after
// this, x[t] for t a multiple of tint holds the sum of x[t .. t + tint - 1].
__device__ inline void fold_time(float (&x)[8], int lt) {
    const int tint = 1 << lt;
    if (tint >= 2) {
#pragma unroll
        for (int t = 0; t < 8; t += 2) x[t] += x[t + 1];
    }
    if (tint >= 4) {
#pragma unroll
        for (int t = 0; t < 8; t += 4) x[t] += x[t + 2];
    }
    if (tint >= 8) x[0] += x[4];
}

// Rows o = (8 g8 + t) / tint of one plane ([T/tint][C] floats from plane_base).
__device__ inline void store_plane(float *__restrict__ out, int64_t plane_base, float (&x)[8], int g8, int lt,
                                   int64_t C, int k) {
    fold_time(x, lt);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        if ((t & ((1 << lt) - 1)) == 0) {
            const int64_t o = (8 * (int64_t)g8 + t) >> lt;
            out[plane_base + o * C + k] = x[t];
        }
    }
}

template <int PREC, int NB>
__global__ void __launch_bounds__(BK) beam_kernel(const uint4 *__restrict__ spec, const float *__restrict__ scale,
                                                  const float *__restrict__ w, const float *__restrict__ cb, int nb,
                                                  int S, int C, int64_t T, int lt, int mode,
                                                  float *__restrict__ inc, float *__restrict__ coh) {
    const int g8 = blockIdx.x;  // spectra 8 g8 .. 8 g8 + 7
    const int k = blockIdx.y * BK + threadIdx.x;
    // chunk of (signal s, channel k, spectra group g): ((g (C/8) + k/8) S + s) 8 + k mod 8;
    // INT8 / FP8 chunks hold 8 spectra (g = g8), FP32 chunks 2 (g = 4 g8 + j)
    const int64_t cpg = (int64_t)C * S;  // chunks per spectra group
    const int64_t g0 = PREC == CORR_FP32 ? 4 * (int64_t)g8 : (int64_t)g8;
    const int64_t c0 = (g0 * (C / 8) + (k >> 3)) * S * 8 + (k & 7);

    float ire[2][8], vre[NB > 0 ? NB : 1][2][8], vim[NB > 0 ? NB : 1][2][8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        ire[0][t] = ire[1][t] = 0.f;
#pragma unroll
        for (int b = 0; b < NB; ++b) vre[b][0][t] = vre[b][1][t] = vim[b][0][t] = vim[b][1][t] = 0.f;
    }
    const bool do_inc = inc != nullptr;

    // signal s of polarisation POL, dequantisation scale sc: accumulate its 8 spectra
    auto add = [&](const Chunk<PREC> &ch, float sc, int s, auto pol_tag) {
        constexpr int POL = decltype(pol_tag)::value;
        float re[8], im[8];
        decode<PREC>(ch, re, im);
        if (do_inc) {
            const float f = w[s] * sc * sc;
#pragma unroll
            for (int t = 0; t < 8; ++t) ire[POL][t] = fmaf(f, fmaf(im[t], im[t], re[t] * re[t]), ire[POL][t]);
        }
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            if (b >= nb) break;  // NB = 4 also serves three beams
            const float cr = cb[2 * ((int64_t)b * S + s)] * sc, ci = cb[2 * ((int64_t)b * S + s) + 1] * sc;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                vre[b][POL][t] = fmaf(cr, re[t], fmaf(-ci, im[t], vre[b][POL][t]));
                vim[b][POL][t] = fmaf(cr, im[t], fmaf(ci, re[t], vim[b][POL][t]));
            }
        }
    };

    // signals in polarisation pairs (2a, 2a + 1), fetched LA pairs ahead into a
    // ring of LA + 1 pair slots with their scales (the loads in flight keep HBM
    // busy; FP32 chunks are 4x larger); the pair loop runs LA + 1 pairs at a
    // time so every ring slot is a constant.  Every fetch is issued (past the
    // last pair it loads the last pair again, unused), so the compiler sees
    // the same loads in flight at every pair and waits only for the oldest.
    constexpr int LA = PREC == CORR_FP32 ? 1 : 3, R = LA + 1;
    const std::integral_constant<int, 0> p0{};
    const std::integral_constant<int, 1> p1{};
    const int npair = S / 2;
    const uint4 *sp = spec + c0;
    const float *scp = scale + k;
    Chunk<PREC> ring[R][2];
    float rsc[R][2];
    auto fetch = [&](int q, auto slot_tag) {
        constexpr int SL = decltype(slot_tag)::value;
        const int qc = q < npair ? q : npair - 1;
        load_chunk<PREC>(sp, 16 * (int64_t)qc, cpg, ring[SL][0]);
        load_chunk<PREC>(sp, 16 * (int64_t)qc + 8, cpg, ring[SL][1]);
        if constexpr (PREC == CORR_FP32) {
            rsc[SL][0] = rsc[SL][1] = 1.f;
        } else {
            rsc[SL][0] = scp[(int64_t)(2 * qc) * C];
            rsc[SL][1] = scp[(int64_t)(2 * qc + 1) * C];
        }
    };
    if (npair > 0) {
        fetch(0, std::integral_constant<int, 0>{});
        if constexpr (LA > 1) fetch(1, std::integral_constant<int, 1>{});
        if constexpr (LA > 2) fetch(2, std::integral_constant<int, 2>{});
        for (int pr = 0; pr < npair; pr += R) {
            auto one = [&](auto j_tag) {
                constexpr int J = decltype(j_tag)::value;
                const int q = pr + J;
                fetch(q + LA, std::integral_constant<int, (J + LA) % R>{});
                if (q < npair) {
                    add(ring[J][0], rsc[J][0], 2 * q, p0);
                    add(ring[J][1], rsc[J][1], 2 * q + 1, p1);
                }
            };
            one(std::integral_constant<int, 0>{});
            one(std::integral_constant<int, 1>{});
            if constexpr (R > 2) one(std::integral_constant<int, 2>{});
            if constexpr (R > 3) one(std::integral_constant<int, 3>{});
        }
    }
    if (S & 1) {  // last signal: polarisation 0 only
        Chunk<PREC> ch;
        load_chunk<PREC>(spec, c0 + 8 * (S - 1), cpg, ch);
        add(ch, PREC == CORR_FP32 ? 1.f : scale[(int64_t)(S - 1) * C + k], S - 1, p0);
    }

    const int64_t plane = (T >> lt) * C;
    if (do_inc) {
        store_plane(inc, 0, ire[0], g8, lt, C, k);
        store_plane(inc, plane, ire[1], g8, lt, C, k);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        if (b >= nb) break;
        if (mode == CORR_BEAM_VOLTAGE) {  // tint = 1: complex64 planes [2][T][C]
            float2 *cv = reinterpret_cast<float2 *>(coh);
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    cv[((int64_t)(2 * b + p) * T + 8 * (int64_t)g8 + t) * C + k] =
                        make_float2(vre[b][p][t], vim[b][p][t]);
            continue;
        }
        const int np = mode == CORR_BEAM_FULLPOL ? 4 : 2;
        const int64_t pb = (int64_t)b * np * plane;
        float x[8];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
#pragma unroll
            for (int t = 0; t < 8; ++t) x[t] = fmaf(vre[b][p][t], vre[b][p][t], vim[b][p][t] * vim[b][p][t]);
            store_plane(coh, pb + p * plane, x, g8, lt, C, k);
        }
        if (np == 4) {  // V0 conj(V1)
#pragma unroll
            for (int t = 0; t < 8; ++t) x[t] = fmaf(vre[b][0][t], vre[b][1][t], vim[b][0][t] * vim[b][1][t]);
            store_plane(coh, pb + 2 * plane, x, g8, lt, C, k);
#pragma unroll
            for (int t = 0; t < 8; ++t) x[t] = fmaf(vim[b][0][t], vre[b][1][t], -(vre[b][0][t] * vim[b][1][t]));
            store_plane(coh, pb + 3 * plane, x, g8, lt, C, k);
        }
    }
}

template <int PREC>
hipError_t launch_prec(const void *spec, const float *scale, const float *w, const float *cb, int nb, int S, int C,
                       int64_t T, int lt, int mode, float *inc, float *coh, hipStream_t st) {
    const dim3 grid((unsigned)(T / 8), (unsigned)(C / BK)), blk(BK);
    const uint4 *sp = static_cast<const uint4 *>(spec);
    switch (nb) {
    case 0: hipLaunchKernelGGL((beam_kernel<PREC, 0>), grid, blk, 0, st, sp, scale, w, cb, nb, S, C, T, lt, mode, inc, coh); break;
    case 1: hipLaunchKernelGGL((beam_kernel<PREC, 1>), grid, blk, 0, st, sp, scale, w, cb, nb, S, C, T, lt, mode, inc, coh); break;
    case 2: hipLaunchKernelGGL((beam_kernel<PREC, 2>), grid, blk, 0, st, sp, scale, w, cb, nb, S, C, T, lt, mode, inc, coh); break;
    default: hipLaunchKernelGGL((beam_kernel<PREC, 4>), grid, blk, 0, st, sp, scale, w, cb, nb, S, C, T, lt, mode, inc, coh); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_beamform(int precision, const void *spec, const float *scale, const float *w, const float *cb,
                           int n_beams, int S, int C, int64_t T, int tint, int mode, float *inc, float *coh,
                           hipStream_t st) {
    const int lt = tint == 8 ? 3 : tint == 4 ? 2 : tint == 2 ? 1 : 0;
    switch (precision) {  // n_beams 3 runs in the four-beam kernel, which stops after beam 3

    case CORR_FP32: return launch_prec<CORR_FP32>(spec, scale, w, cb, n_beams, S, C, T, lt, mode, inc, coh, st);
    case CORR_INT8: return launch_prec<CORR_INT8>(spec, scale, w, cb, n_beams, S, C, T, lt, mode, inc, coh, st);
    default: return launch_prec<CORR_FP8_E4M3>(spec, scale, w, cb, n_beams, S, C, T, lt, mode, inc, coh, st);
    }
}

}  // namespace corr
