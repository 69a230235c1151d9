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
// the spectra; wave w handles channel 8 kb + w.  The workgroup stages each
// K-step's lines through LDS (below).  Each wave keeps its accumulator tiles in
// registers and at the
// end forms Im = M - M^T through LDS and adds its result into
// acc[split][k][p] (sole owner, so no atomics and a fixed order).
#include <type_traits>

#include "corr_internal.h"

namespace corr {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int ntri(int nt) { return nt * (nt + 1) / 2; }
constexpr int kXcds = 8;  // MI355X: workgroups are dealt to its 8 XCDs in turn

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

// K-step st covers chunks g0..g0+3, g0 = 4 (split offset + st): lanes 0-31
// take chunks g0 and g0+2, lanes 32-63 chunks g0+1 and g0+3 (the two lane
// groups form the K halves).  INT8/FP8 chunk: 8 real bytes then 8 imaginary
// bytes (8 spectra); FP32 chunk: 2 complex64.
//
// Staging: the workgroup's 8 channels x S signals of one chunk form one
// contiguous block of S x 128 bytes; the 512 threads copy the 4 blocks of the
// next K-step with one 16-byte load each per block (fully coalesced) while the
// MFMAs of the current step run, then store them into LDS with a 144-byte row
// pitch per signal so that the per-channel 16-byte operand reads of a wave
// (stride 144 B across lanes) are free of bank conflicts.  Double-buffered;
// the accumulator exchange of the epilogue reuses the same LDS.
constexpr int kXWaves = 8;                  // channels (waves) per workgroup
constexpr int kRowPitch = 144;              // LDS bytes per signal row (8 x 16 + 16)
constexpr int kBlk = kMaxSignals * kRowPitch;  // LDS bytes per staged chunk block

template <int NT>
constexpr int x_lds_bytes() {
    return (2 * 4 * kBlk > kXWaves * NT * NT * 32 * 33 * 4) ? 2 * 4 * kBlk : kXWaves * NT * NT * 32 * 33 * 4;
}

// 0xFF in every byte of w that equals b (exact zero-byte test of w ^ b).
__device__ inline uint32_t eq_bytes(uint32_t w, uint32_t b4) {
    const uint32_t x = w ^ b4;
    const uint32_t z = ~(((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x | 0x7F7F7F7Fu);  // 0x80 in zero bytes
    return (z << 1) - (z >> 7);                                                   // 0x80 -> 0xFF
}

// 4 bits -> 4 bytes of 0x00 / 0xFF
__device__ inline uint32_t keep_bytes(uint32_t b) { return ((b * 0x00204081u) & 0x01010101u) * 0xFFu; }

// Zero the flagged cells of a staged 16-byte chunk: kb8 holds the chunk's keep
// bits (bit i = spectrum i of the chunk kept; 8 spectra for INT8 / FP8, whose
// chunk is 8 real bytes then 8 imaginary bytes, 2 for FP32's two complex64).
template <int PREC>
__device__ __forceinline__ uint4 keep_chunk(uint4 v, uint32_t kb8) {
    if constexpr (PREC == CORR_FP32) {
        if (!(kb8 & 1u)) v.x = v.y = 0u;
        if (!(kb8 & 2u)) v.z = v.w = 0u;
    } else {
        const uint32_t lo = keep_bytes(kb8 & 15u), hi = keep_bytes((kb8 >> 4) & 15u);
        v.x &= lo;
        v.y &= hi;
        v.z &= lo;
        v.w &= hi;
    }
    return v;
}

// One (channel block kb, split sp) of one correlation: PREC is CORR_FP32,
// CORR_INT8 or CORR_FP8_E4M3; ACC float or int32_t; lds holds at least
// x_lds_bytes<NT>() bytes.  GATED: only the spectra m with gate[m] == bin
// are summed (the B operand of every product is masked per spectrum).
// MASKED: the flagged cells (keep bits clear; keep words [C/8][T/32][S][8],
// bit i of word w = spectrum 32 w + i) are zeroed as the chunks are staged,
// which is the product of zeroed spectra without writing them.
template <int NT, int PREC, typename ACC, bool GATED = false, bool MASKED = false>
__device__ __forceinline__ void xengine_block(const uint8_t *__restrict__ spec, ACC *acc, int S, int C, int T,
                                              int splits, int kb, int sp, uint8_t *lds,
                                              const uint8_t *__restrict__ gate = nullptr, int bin = 0,
                                              const uint32_t *__restrict__ keep = nullptr) {
    using V16 = typename std::conditional<PREC == CORR_INT8, v16i, v16f>::type;
    const int wv = threadIdx.x >> 6, c = kXWaves * kb + wv;
    const int lane = threadIdx.x & 63, row = lane & 31, lg = lane >> 5;
    const int G = (PREC == CORR_FP32) ? kChunk32 : kChunk8;
    const int steps = T / G / 4 / splits;
    const int64_t P = (int64_t)S * (S + 1) / 2;
    if (steps < 1) return;  // no K-step (the plan's splits always leave one): nothing to add

    // staging copy: thread i moves bytes [16 i, 16 i + 16) of each block
    const int i = threadIdx.x;
    const bool cp = i < S * 8;
    const int lds_dst = (i >> 3) * kRowPitch + (i & 7) * 16;
    // threads beyond the block load its last 16 bytes and discard them, so
    // every thread issues the same loads (the compiler can then count the
    // loads in flight across steps and wait only for the older set)
    const uint4 *gsrc = reinterpret_cast<const uint4 *>(spec) + (int64_t)kb * S * 8 + (cp ? i : S * 8 - 1);
    const int64_t gstride = (int64_t)C * S;  // 16-byte units between chunks g and g+1
    // keep words of this thread's (channel, signal): a K-step's 4 chunks are 32
    // spectra (one word) for INT8 / FP8 and 8 spectra (one byte) for FP32; the
    // words of the block's S x 8 chunks for one span of 32 spectra are
    // contiguous, in the staging threads' order
    const uint32_t *kw0 = nullptr;
    const int64_t kwstride = (int64_t)S * 8;
    if constexpr (MASKED) kw0 = keep + (int64_t)kb * (T / 32) * kwstride + (cp ? i : S * 8 - 1);
    // two register sets (a, b) alternate between the next two K-steps'
    // chunks, so each load has two steps of MFMA work to land before its LDS
    // store
    uint4 pa0 = make_uint4(0, 0, 0, 0), pa1 = pa0, pa2 = pa0, pa3 = pa0, pb0 = pa0, pb1 = pa0, pb2 = pa0, pb3 = pa0;
    uint32_t pak = 0xFFFFFFFFu, pbk = 0xFFFFFFFFu;  // keep bits of the step each set holds (MASKED)
#define X_GLOAD(st, R)                                                \
    {                                                                 \
        const int64_t s_ = (int64_t)sp * steps + (st);                \
        const uint4 *g_ = gsrc + 4 * s_ * gstride;                    \
        R##0 = g_[0];                                                 \
        R##1 = g_[gstride];                                           \
        R##2 = g_[2 * gstride];                                       \
        R##3 = g_[3 * gstride];                                       \
        if constexpr (MASKED) {                                       \
            if constexpr (PREC == CORR_FP32)                          \
                R##k = kw0[(s_ >> 2) * kwstride] >> (8 * (s_ & 3));   \
            else                                                      \
                R##k = kw0[s_ * kwstride];                            \
        }                                                             \
    }
#define X_LSTORE(buf, R)                                              \
    if (cp) {                                                         \
        uint8_t *l_ = lds + (buf) * 4 * kBlk + lds_dst;               \
        constexpr int SH_ = PREC == CORR_FP32 ? 2 : 8;                \
        if constexpr (MASKED) {                                       \
            R##0 = keep_chunk<PREC>(R##0, R##k);                      \
            R##1 = keep_chunk<PREC>(R##1, R##k >> SH_);               \
            R##2 = keep_chunk<PREC>(R##2, R##k >> (2 * SH_));         \
            R##3 = keep_chunk<PREC>(R##3, R##k >> (3 * SH_));         \
        }                                                             \
        *reinterpret_cast<uint4 *>(l_) = R##0;                        \
        *reinterpret_cast<uint4 *>(l_ + kBlk) = R##1;                 \
        *reinterpret_cast<uint4 *>(l_ + 2 * kBlk) = R##2;             \
        *reinterpret_cast<uint4 *>(l_ + 3 * kBlk) = R##3;             \
    }

    V16 accR[ntri(NT)], accM[NT * NT];
#pragma unroll
    for (int t = 0; t < ntri(NT); ++t) accR[t] = V16{0};
#pragma unroll
    for (int t = 0; t < NT * NT; ++t) accM[t] = V16{0};
    bool valid[NT];
#pragma unroll
    for (int a = 0; a < NT; ++a) valid[a] = (32 * a + row) < S;

    X_GLOAD(0, pa)
    X_LSTORE(0, pa)
    X_GLOAD(steps > 1 ? 1 : 0, pa)
    __syncthreads();
    // K-step st (B = st is odd): set a (even st) or b (odd st) holds step
    // st + 1's chunks, stored to the other LDS buffer at the end; the other
    // set receives step st + 2's
    auto kstep = [&](int st, auto odd) __attribute__((always_inline)) {
        constexpr bool B = decltype(odd)::value;
        const int buf = st & 1;
        // step st + 2's chunks (the last step's again near the end: unused)
        const int nx = st + 2 < steps ? st + 2 : steps - 1;
        if constexpr (B) {
            X_GLOAD(nx, pa)
        } else {
            X_GLOAD(nx, pb)
        }
        v4i c0[NT], c1[NT];
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            const uint8_t *b = lds + (buf * 4 + lg) * kBlk + (32 * a + row) * kRowPitch + wv * 16;
            c0[a] = valid[a] ? *reinterpret_cast<const v4i *>(b) : v4i{0};
            c1[a] = valid[a] ? *reinterpret_cast<const v4i *>(b + 2 * kBlk) : v4i{0};
        }
        // B operands: masked to the gate's spectra when GATED
        v4i b0[NT], b1[NT];
        if constexpr (GATED) {
            // this lane's chunks are g0 + lg and g0 + 2 + lg, g0 = 4 (sp steps + st)
            const int64_t g = 4 * ((int64_t)sp * steps + st) + lg;
            const uint32_t b4 = (uint32_t)bin * 0x01010101u;
            if constexpr (PREC == CORR_FP32) {  // 2 spectra per chunk: one mask word per spectrum
                const uint16_t q0 = *reinterpret_cast<const uint16_t *>(gate + 2 * g);
                const uint16_t q1 = *reinterpret_cast<const uint16_t *>(gate + 2 * (g + 2));
                const int m00 = (q0 & 0xFF) == bin ? -1 : 0, m01 = (q0 >> 8) == bin ? -1 : 0;
                const int m10 = (q1 & 0xFF) == bin ? -1 : 0, m11 = (q1 >> 8) == bin ? -1 : 0;
#pragma unroll
                for (int a = 0; a < NT; ++a) {
                    b0[a] = v4i{c0[a].x & m00, c0[a].y & m00, c0[a].z & m01, c0[a].w & m01};
                    b1[a] = v4i{c1[a].x & m10, c1[a].y & m10, c1[a].z & m11, c1[a].w & m11};
                }
            } else {  // 8 spectra per chunk: real bytes 0-7, imaginary bytes 8-15
                const uint2 q0 = *reinterpret_cast<const uint2 *>(gate + 8 * g);
                const uint2 q1 = *reinterpret_cast<const uint2 *>(gate + 8 * (g + 2));
                const int m0l = (int)eq_bytes(q0.x, b4), m0h = (int)eq_bytes(q0.y, b4);
                const int m1l = (int)eq_bytes(q1.x, b4), m1h = (int)eq_bytes(q1.y, b4);
#pragma unroll
                for (int a = 0; a < NT; ++a) {
                    b0[a] = v4i{c0[a].x & m0l, c0[a].y & m0h, c0[a].z & m0l, c0[a].w & m0h};
                    b1[a] = v4i{c1[a].x & m1l, c1[a].y & m1h, c1[a].z & m1l, c1[a].w & m1h};
                }
            }
        } else {
#pragma unroll
            for (int a = 0; a < NT; ++a) {
                b0[a] = c0[a];
                b1[a] = c1[a];
            }
        }
        if constexpr (PREC == CORR_INT8) {
            v4i im[NT], re[NT];  // imaginary bytes (A side) / real bytes (B side) of both chunks
#pragma unroll
            for (int a = 0; a < NT; ++a) {
                im[a] = v4i{c0[a].z, c0[a].w, c1[a].z, c1[a].w};
                re[a] = v4i{b0[a].x, b0[a].y, b1[a].x, b1[a].y};
            }
#pragma unroll
            for (int b = 0; b < NT; ++b) {
#pragma unroll
                for (int a = 0; a <= b; ++a) {
                    V16 &d = accR[tri_idx(a, b)];
                    d = __builtin_amdgcn_mfma_i32_32x32x32_i8(c0[a], b0[b], d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_i32_32x32x32_i8(c1[a], b1[b], d, 0, 0, 0);
                }
#pragma unroll
                for (int a = 0; a < NT; ++a)
                    accM[a * NT + b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(im[a], re[b], accM[a * NT + b], 0, 0, 0);
            }
        } else if constexpr (PREC == CORR_FP8_E4M3) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                long re[NT], im[NT], reB[NT], imB[NT];  // A side, and the (masked) B side
#pragma unroll
                for (int a = 0; a < NT; ++a) {
                    const v4i v = h ? c1[a] : c0[a];
                    const v4i w = h ? b1[a] : b0[a];
                    re[a] = (long)(((unsigned long)(unsigned)v.y << 32) | (unsigned)v.x);
                    im[a] = (long)(((unsigned long)(unsigned)v.w << 32) | (unsigned)v.z);
                    reB[a] = (long)(((unsigned long)(unsigned)w.y << 32) | (unsigned)w.x);
                    imB[a] = (long)(((unsigned long)(unsigned)w.w << 32) | (unsigned)w.z);
                }
#pragma unroll
                for (int b = 0; b < NT; ++b) {
#pragma unroll
                    for (int a = 0; a <= b; ++a) {
                        V16 &d = accR[tri_idx(a, b)];
                        d = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(re[a], reB[b], d, 0, 0, 0);
                        d = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(im[a], imB[b], d, 0, 0, 0);
                    }
#pragma unroll
                    for (int a = 0; a < NT; ++a)
                        accM[a * NT + b] = __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(im[a], reB[b], accM[a * NT + b], 0, 0, 0);
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {  // spectra (chunk 0: 0, 1; chunk 1: 2, 3)
                float rr[NT], qq[NT], rrB[NT], qqB[NT];  // A side, and the (masked) B side
#pragma unroll
                for (int a = 0; a < NT; ++a) {
                    const v4i v = (q < 2) ? c0[a] : c1[a];
                    const v4i w = (q < 2) ? b0[a] : b1[a];
                    rr[a] = __int_as_float((q & 1) ? v.z : v.x);
                    qq[a] = __int_as_float((q & 1) ? v.w : v.y);
                    rrB[a] = __int_as_float((q & 1) ? w.z : w.x);
                    qqB[a] = __int_as_float((q & 1) ? w.w : w.y);
                }
#pragma unroll
                for (int b = 0; b < NT; ++b) {
#pragma unroll
                    for (int a = 0; a <= b; ++a) {
                        V16 &d = accR[tri_idx(a, b)];
                        d = __builtin_amdgcn_mfma_f32_32x32x2f32(rr[a], rrB[b], d, 0, 0, 0);
                        d = __builtin_amdgcn_mfma_f32_32x32x2f32(qq[a], qqB[b], d, 0, 0, 0);
                    }
#pragma unroll
                    for (int a = 0; a < NT; ++a)
                        accM[a * NT + b] = __builtin_amdgcn_mfma_f32_32x32x2f32(qq[a], rrB[b], accM[a * NT + b], 0, 0, 0);
                }
            }
        }
        if (st + 1 < steps) {
            if constexpr (B) {
                X_LSTORE(buf ^ 1, pb)
            } else {
                X_LSTORE(buf ^ 1, pa)
            }
        }
        __syncthreads();
    };
    int st = 0;
    for (; st + 1 < steps; st += 2) {  // whole pairs, so every loop entry sees the same loads in flight
        kstep(st, std::false_type{});
        kstep(st + 1, std::true_type{});
    }
    if (st < steps) kstep(st, std::false_type{});
#undef X_GLOAD
#undef X_LSTORE
    // the staging buffers are free now: the epilogue's M-tile exchange reuses them
    auto *mlds = reinterpret_cast<ACC(*)[32][33]>(lds + wv * NT * NT * 32 * 33 * 4);
    x_epilogue<NT, ACC>(accR, accM, acc + ((int64_t)sp * C + c) * P * 2, S, P, mlds);
    __syncthreads();  // the LDS may be reused by the next block of a persistent loop
}

template <int NT, int PREC, typename ACC, bool MASKED>
__global__ void __launch_bounds__(64 * kXWaves)
xengine_kernel(const uint8_t *__restrict__ spec, const uint32_t *__restrict__ keep, ACC *acc, int S, int C, int T,
               int splits) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[x_lds_bytes<NT>()];
    xengine_block<NT, PREC, ACC, false, MASKED>(spec, acc, S, C, T, splits, blockIdx.x, blockIdx.y, lds, nullptr, 0,
                                               keep);
}

// Gated correlation: one workgroup per (task, bin), task = (channel block kb,
// split sp); it sums the spectra of gate bin `bin` into accumulator set
// `bin` (acc_elems elements apart).  Every bin reads the same spectra, so the
// bins of one task are given ids 8 apart: workgroups go to the 8 XCDs in
// turn, so those land on the same XCD, run side by side and share its L2
// (the later reads hit).  w -> xcd = w mod 8, j = w / 8, bin = j mod n_bins,
// task = 8 (j / n_bins) + xcd.
template <int NT, int PREC, typename ACC>
__global__ void __launch_bounds__(64 * kXWaves)
xengine_gated_kernel(const uint8_t *__restrict__ spec, const uint8_t *__restrict__ gate, ACC *acc, int64_t acc_elems,
                     int S, int C, int T, int splits, int n_bins) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[x_lds_bytes<NT>()];
    const int w = blockIdx.x, xcd = w & (kXcds - 1), j = w / kXcds;
    const int bin = j % n_bins, task = kXcds * (j / n_bins) + xcd;
    const int nkb = C / kXWaves;
    if (task >= nkb * splits) return;  // padding of the last group of 8 tasks
    xengine_block<NT, PREC, ACC, true>(spec, acc + bin * acc_elems, S, C, T, splits, task % nkb, task / nkb, lds, gate,
                                       bin);
}

// One launch over the tasks of a batch of correlations of different shapes
// (one per sub-array).  The batch table travels by value as the kernel
// argument, so every field is a uniform scalar; workgroup b runs task b: the
// correlation whose task range holds b, then its (channel block, split).  Each
// task runs the body of its sub-array's size, as corr_xengine would: two
// 32-signal tiles above 32 signals, one tile otherwise (the two-tile body on
// a small sub-array issues 7 matrix products per step where 3 suffice).  The
// branch is uniform per workgroup.
__global__ void __launch_bounds__(64 * kXWaves) xengine_batch_kernel(XBatchArgs a) {
    __shared__ __attribute__((aligned(16))) uint8_t lds[x_lds_bytes<2>()];
    const int b = blockIdx.x;
    int i = 0;
    while (i + 1 < a.n && b >= a.first[i + 1]) ++i;
    const XBatchEntry &e = a.cor[i];
    const int local = b - a.first[i];
    const int nkb = e.C / kXWaves;
    if (e.S > 32)
        xengine_block<2, CORR_INT8, int32_t>((const uint8_t *)e.spec, (int32_t *)e.acc, e.S, e.C, e.T, e.splits,
                                             local % nkb, local / nkb, lds);
    else
        xengine_block<1, CORR_INT8, int32_t>((const uint8_t *)e.spec, (int32_t *)e.acc, e.S, e.C, e.T, e.splits,
                                             local % nkb, local / nkb, lds);
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

// Requantisation of FP32 spectra [S][T][C][2] to codes [S][T][C][2] with
// the F-engines' encoders: q = enc(v * (1 / scale[s][k])) per component.  One
// thread per complex value.
template <int PREC>
__global__ void requantize_kernel(const float2 *__restrict__ in, const float *__restrict__ scale, int S, int64_t T,
                                  int C, uint16_t *out) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)S * T * C) return;
    const int k = (int)(idx % C);
    const int s = (int)(idx / ((int64_t)T * C));
    const float inv = 1.0f / scale[(int64_t)s * C + k];
    const float2 v = in[idx];
    if constexpr (PREC == CORR_INT8)
        out[idx] = (uint16_t)((quant_i8(v.x * inv) & 0xFFu) | ((quant_i8(v.y * inv) & 0xFFu) << 8));
    else
        out[idx] = (uint16_t)(e4m3_pair(v.x * inv, v.y * inv) & 0xFFFFu);
}

}  // namespace

hipError_t launch_requantize(int precision, const float *in, const float *scale, int S, int64_t T, int C,
                             uint8_t *out, hipStream_t st) {
    const int64_t n = (int64_t)S * T * C;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (precision == CORR_INT8)
        hipLaunchKernelGGL(requantize_kernel<CORR_INT8>, grid, block, 0, st, reinterpret_cast<const float2 *>(in),
                           scale, S, T, C, reinterpret_cast<uint16_t *>(out));
    else if (precision == CORR_FP8_E4M3)
        hipLaunchKernelGGL(requantize_kernel<CORR_FP8_E4M3>, grid, block, 0, st,
                           reinterpret_cast<const float2 *>(in), scale, S, T, C, reinterpret_cast<uint16_t *>(out));
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_xengine(int precision, const void *spec, const uint32_t *keep, void *acc, int S, int C, int T,
                          int splits, hipStream_t st) {
    const dim3 grid(C / kXWaves, splits), block(64 * kXWaves);
    const uint8_t *sp8 = (const uint8_t *)spec;
    auto go = [&](auto kernel, auto *a) { hipLaunchKernelGGL(kernel, grid, block, 0, st, sp8, keep, a, S, C, T, splits); };
    const bool two = S > 32, m = keep != nullptr;
    int32_t *ai = (int32_t *)acc;
    float *af = (float *)acc;
    switch (precision) {
    case CORR_INT8:
        if (two) m ? go(xengine_kernel<2, CORR_INT8, int32_t, true>, ai) : go(xengine_kernel<2, CORR_INT8, int32_t, false>, ai);
        else m ? go(xengine_kernel<1, CORR_INT8, int32_t, true>, ai) : go(xengine_kernel<1, CORR_INT8, int32_t, false>, ai);
        break;
    case CORR_FP8_E4M3:
        if (two) m ? go(xengine_kernel<2, CORR_FP8_E4M3, float, true>, af) : go(xengine_kernel<2, CORR_FP8_E4M3, float, false>, af);
        else m ? go(xengine_kernel<1, CORR_FP8_E4M3, float, true>, af) : go(xengine_kernel<1, CORR_FP8_E4M3, float, false>, af);
        break;
    case CORR_FP32:
        if (two) m ? go(xengine_kernel<2, CORR_FP32, float, true>, af) : go(xengine_kernel<2, CORR_FP32, float, false>, af);
        else m ? go(xengine_kernel<1, CORR_FP32, float, true>, af) : go(xengine_kernel<1, CORR_FP32, float, false>, af);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_xengine_gated(int precision, const void *spec, const uint8_t *gate, int n_bins, void *acc,
                                int64_t acc_elems, int S, int C, int T, int splits, hipStream_t st) {
    const int tasks = (C / kXWaves) * splits;
    const dim3 grid((unsigned)((tasks + kXcds - 1) / kXcds * kXcds * n_bins)), block(64 * kXWaves);
    const uint8_t *sp8 = (const uint8_t *)spec;
    const bool two = S > 32;
    switch (precision) {
    case CORR_INT8:
        if (two) hipLaunchKernelGGL((xengine_gated_kernel<2, CORR_INT8, int32_t>), grid, block, 0, st, sp8, gate, (int32_t *)acc, acc_elems, S, C, T, splits, n_bins);
        else hipLaunchKernelGGL((xengine_gated_kernel<1, CORR_INT8, int32_t>), grid, block, 0, st, sp8, gate, (int32_t *)acc, acc_elems, S, C, T, splits, n_bins);
        break;
    case CORR_FP8_E4M3:
        if (two) hipLaunchKernelGGL((xengine_gated_kernel<2, CORR_FP8_E4M3, float>), grid, block, 0, st, sp8, gate, (float *)acc, acc_elems, S, C, T, splits, n_bins);
        else hipLaunchKernelGGL((xengine_gated_kernel<1, CORR_FP8_E4M3, float>), grid, block, 0, st, sp8, gate, (float *)acc, acc_elems, S, C, T, splits, n_bins);
        break;
    case CORR_FP32:
        if (two) hipLaunchKernelGGL((xengine_gated_kernel<2, CORR_FP32, float>), grid, block, 0, st, sp8, gate, (float *)acc, acc_elems, S, C, T, splits, n_bins);
        else hipLaunchKernelGGL((xengine_gated_kernel<1, CORR_FP32, float>), grid, block, 0, st, sp8, gate, (float *)acc, acc_elems, S, C, T, splits, n_bins);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_xengine_batch(const XBatchArgs &a, hipStream_t st) {
    if (a.n < 1 || a.n > kMaxBatch) return hipErrorInvalidValue;
    hipLaunchKernelGGL(xengine_batch_kernel, dim3(a.first[a.n]), dim3(64 * kXWaves), 0, st, a);
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
