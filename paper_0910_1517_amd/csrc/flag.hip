// flag.hip -- RFI flagging on the channelised data path.
//
// Section 5 removes outliers with the median absolute deviation (Eq. 3,
// MAD = median |x_i - median(x)|) and the threshold of Eq. 4,
// |x_i - median(x)| > M MAD / 0.6745.  On dynamic spectra the statistic is
// taken per signal on tiles of 64 spectra x 256 channels of power:
//   row statistic    mean power of one spectrum over the tile's 256 channels
//                    (broadband bursts show up here)
//   column statistic mean power of one channel over the tile's 64 spectra
//                    (persistent narrowband tones show up here)
// A cell is flagged when its row or its column exceeds Eq. 4.  Flagged cells
// are zeroed in the X-engine input (or masked as it stages them), and the
// number of unflagged products of every pair, n_ij[k] = sum_m (1 - F_i)(1 - F_j),
// is counted exactly from bit-packed keep masks, as the Gram matrix of the
// keep bits on the int8 matrix cores.
#include "corr_internal.h"

namespace corr {
namespace {

constexpr int TT = kFlagTileSpectra;   // 64
constexpr int KT = kFlagTileChannels;  // 256

// Ascending bitonic sort of 64 floats, one per lane of a wave.
__device__ inline float wave_sort64(float x, int lane) {
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const float o = __shfl_xor(x, j);
            const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
            x = keep_min ? fminf(x, o) : fmaxf(x, o);
        }
    }
    return x;
}


// Median of 64 floats, one per lane; y receives them sorted (element lane).
__device__ inline float wave_median64(float x, int lane, float &y) {
    y = wave_sort64(x, lane);
    return 0.5f * (__shfl(y, 31) + __shfl(y, 32));
}

// Median of |s_i - med| over 64 sorted values (s[lane] in y, med their median)
// without a second sort, as wave_mad256_sorted does for 256: the deviations
// A[i] = med - s[31 - i] and B[j] = s[32 + j] - med ascend, and the 32 smallest
// are A[0 .. p - 1] and B[0 .. 31 - p] for p = #{i < 32 : B[31 - i] > A[i]}.
// buf: 64 floats of LDS used by this wave alone.
__device__ inline float wave_mad64_sorted(float y, float med, int lane, float *buf) {
    buf[lane] = y;
    const int i = lane & 31;
    const bool gt = buf[63 - i] - med > med - buf[31 - i];
    const int p = __popcll(__ballot(lane < 32 && gt));
    const float inf = __builtin_inff();
    const float a_lo = med - buf[p > 0 ? 32 - p : 0];    // A[p - 1]
    const float b_lo = buf[p < 32 ? 63 - p : 32] - med;  // B[31 - p]
    const float a_hi = med - buf[p < 32 ? 31 - p : 0];   // A[p]
    const float b_hi = buf[p > 0 ? 64 - p : 32] - med;   // B[32 - p]
    const float lo = fmaxf(p > 0 ? a_lo : -inf, p < 32 ? b_lo : -inf);
    const float hi = fminf(p < 32 ? a_hi : inf, p > 0 ? b_hi : inf);
    return 0.5f * (lo + hi);
}

// One tile (signal s, spectra m0..m0+63, channels k0..k0+255) per workgroup.
// Eq. 3 / Eq. 4 on the 64 row means and the 256 column means:
// flag[i] = |x_i - med| > M MAD / 0.6745, the median of an even count being
// the mean of the two middle values.  The tile is summed as it is loaded
// (nothing of it is staged): wave w holds rows w + 4 i (i < 16), lane l
// columns 4 l ... 4 l + 3; column sums go through LDS, row sums are reduced
// across the wave.  One wave sorts the row statistic while another sorts the
// column statistic; the MADs come from the sorted values.
template <typename PT>
__global__ void __launch_bounds__(KT) mad_tile_kernel(const PT *__restrict__ power, int S, int T, int C,
                                                      float M, uint8_t *flags) {
    __shared__ float colp[KT / 64][KT];  // column partial sums of each wave's 16 rows
    __shared__ float rowv[TT], colv[KT], rdev[TT], cdev[KT];
    __shared__ float sel[2];  // MAD of the rows, MAD of the columns
    __shared__ __align__(16) float srt[TT + KT];  // sorted row / column statistics
    __shared__ uint8_t rowf[TT];
    __shared__ __align__(16) uint8_t colf[KT];
    const int ntk = C / KT, ntm = T / TT;
    const int b = blockIdx.x;
    const int kt = b % ntk, mt = (b / ntk) % ntm, s = b / (ntk * ntm);
    const int t = threadIdx.x;
    const int64_t tbase = ((int64_t)s * T + (int64_t)mt * TT) * C + (int64_t)kt * KT;  // tile corner
    {
        const int cq = t & 63, r0 = t >> 6;
        float4 v[TT / 4];  // rows r0 + 4 i: 16-byte (FP32) or 8-byte (FP16) loads, all issued first
#pragma unroll
        for (int i = 0; i < TT / 4; ++i) {
            const PT *src = power + tbase + (int64_t)(r0 + 4 * i) * C + 4 * cq;
            if constexpr (sizeof(PT) == 4) {
                v[i] = *reinterpret_cast<const float4 *>(src);
            } else {
                typedef _Float16 h4 __attribute__((ext_vector_type(4)));
                const h4 w = *reinterpret_cast<const h4 *>(src);
                v[i] = make_float4((float)w[0], (float)w[1], (float)w[2], (float)w[3]);
            }
        }
        float4 cs = make_float4(0.f, 0.f, 0.f, 0.f);
        float rp[TT / 4];
#pragma unroll
        for (int i = 0; i < TT / 4; ++i) {
            cs.x += v[i].x;
            cs.y += v[i].y;
            cs.z += v[i].z;
            cs.w += v[i].w;
            rp[i] = (v[i].x + v[i].y) + (v[i].z + v[i].w);
        }
        *reinterpret_cast<float4 *>(&colp[r0][4 * cq]) = cs;
        // row sums: halve the set of rows at each exchange (lane bit 5 keeps rows
        // 8 .. 15 of 16, bit 4 the upper half of the rest, ...), then sum the last
        // one over lane bits 1 and 0; lane l ends with row i = 8 b5 + 4 b4 + 2 b3 + b2
        const int lane = t & 63;
#pragma unroll
        for (int h = 8, bit = 32; h >= 1; h >>= 1, bit >>= 1) {
            const bool up = (lane & bit) != 0;
#pragma unroll
            for (int i = 0; i < h; ++i) {
                const float send = up ? rp[i] : rp[i + h], keep = up ? rp[i + h] : rp[i];
                rp[i] = keep + __shfl_xor(send, bit);
            }
        }
        rp[0] += __shfl_xor(rp[0], 2);
        rp[0] += __shfl_xor(rp[0], 1);
        if ((lane & 3) == 0) {
            const int i = 8 * ((lane >> 5) & 1) + 4 * ((lane >> 4) & 1) + 2 * ((lane >> 3) & 1) + ((lane >> 2) & 1);
            rowv[r0 + 4 * i] = rp[0] / (float)KT;
        }
    }
    __syncthreads();
    colv[t] = (colp[0][t] + colp[1][t] + colp[2][t] + colp[3][t]) / (float)TT;
    __syncthreads();
    // Eq. 3 on the rows (wave 0) and on the columns (wave 1), side by side
    const int lane = t & 63, wv = t >> 6;
    if (wv == 0) {
        const float x = rowv[lane];
        float y;
        const float med = wave_median64(x, lane, y);
        const float d = fabsf(x - med);
        const float mad = wave_mad64_sorted(y, med, lane, srt);
        rdev[lane] = d;
        if (lane == 0) sel[0] = mad;
    } else if (wv == 1) {
        float v[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = colv[4 * lane + q];
        const float med = wave_median256(v, lane);
#pragma unroll
        for (int q = 0; q < 4; ++q) cdev[4 * lane + q] = fabsf(colv[4 * lane + q] - med);
        const float mad = wave_mad256_sorted(v, med, lane, srt + TT);
        if (lane == 0) sel[1] = mad;
    }
    __syncthreads();
    const float madr = sel[0], madc = sel[1];
    colf[t] = cdev[t] > M * madc / 0.6745f;
    if (t < TT) rowf[t] = rdev[t] > M * madr / 0.6745f;
    __syncthreads();
    // 16-byte stores: chunk c = t + 256 j covers row c / 16, columns 16 (c mod 16) .. + 15
#pragma unroll
    for (int j = 0; j < TT * KT / 16 / KT; ++j) {
        const int c = t + KT * j, r = c >> 4, c16 = c & 15;
        const uint32_t rb = rowf[r] * 0x01010101u;
        uint4 f = *reinterpret_cast<const uint4 *>(&colf[16 * c16]);
        f.x |= rb;
        f.y |= rb;
        f.z |= rb;
        f.w |= rb;
        *reinterpret_cast<uint4 *>(flags + tbase + (int64_t)r * C + 16 * c16) = f;
    }
}

// Keep masks and zeroing in one pass.  A workgroup owns 32 spectra (one keep
// word) x 256 channels of one signal.  Thread t builds the keep word of
// channel k0 + t from the 32 flag bytes of that channel (the loads of the
// workgroup's threads are consecutive bytes of a row), writes it to
// keep when keep is given (word (((k / 8) W + w) S + s) 8 + k mod 8: the words of
// 8 consecutive channels of every signal for one span of 32 spectra are
// contiguous, the order in which the X-engine stages its channel blocks); then,
// when spec is given, the workgroup
// zeroes the flagged cells of its X-layout chunks (index
// g C S + (k/8) S 8 + s 8 + k mod 8 in 16-byte units), reading and writing a
// chunk only when one of its cells is flagged.
__device__ inline uint32_t expand4(uint32_t b) {  // 4 bits -> 4 bytes of 0x00 / 0xFF
    return ((b * 0x00204081u) & 0x01010101u) * 0xFFu;
}

template <int G>
__global__ void __launch_bounds__(256) apply_keep_kernel(const uint8_t *__restrict__ flags, uint8_t *spec,
                                                         uint32_t *keep, int S, int T, int C) {
    const int t = threadIdx.x;
    const int nkb = C / 256, W = T / 32;
    const int kblk = blockIdx.x % nkb;
    const int w = (blockIdx.x / nkb) % W;
    const int s = blockIdx.x / (nkb * W);
    const int k = kblk * 256 + t;
    const uint8_t *f = flags + ((int64_t)s * T + (int64_t)w * 32) * C + k;
    uint32_t bits = 0;
#pragma unroll
    for (int i = 0; i < 32; ++i) bits |= (f[(int64_t)i * C] ? 0u : 1u) << i;
    if (keep) keep[(((int64_t)(k >> 3) * W + w) * S + s) * 8 + (k & 7)] = bits;
    if (!spec) return;  // keep words only (the X-engine applies them)
    if (__syncthreads_and(bits == 0xFFFFFFFFu)) return;  // nothing flagged in this block
    uint4 *chunks = reinterpret_cast<uint4 *>(spec);
    constexpr int NG = 32 / G;  // chunks per channel in the block
    // thread t walks chunks (g, channel) with channel = t; consecutive threads
    // touch consecutive chunks of a 128-byte line
#pragma unroll 4
    for (int g = 0; g < NG; ++g) {
        const uint32_t m = (bits >> (G * g)) & ((1u << G) - 1u);
        if (m == (1u << G) - 1u) continue;
        const int64_t gg = (int64_t)w * NG + g;
        uint4 *c = chunks + ((gg * (C / 8) + k / 8) * S + s) * 8 + (k & 7);
        uint4 v = *c;
        if constexpr (G == kChunk8) {  // 8 real bytes (spectra 0..7), then 8 imaginary bytes
            const uint32_t lo = expand4(m & 15u), hi = expand4(m >> 4);
            v.x &= lo;
            v.y &= hi;
            v.z &= lo;
            v.w &= hi;
        } else {  // two complex64
            if (!(m & 1u)) v.x = v.y = 0u;
            if (!(m & 2u)) v.z = v.w = 0u;
        }
        *c = v;
    }
}

// Keep words alone, when no spectra are to be zeroed.  Wave w of a workgroup
// takes signal 4 (block) + w, lane l the 16 channels 16 l ... + 15 of a
// 1024-channel chunk, and one span of 32 spectra: one 16-byte load per
// spectrum row (a wave reads 1 KB of the row), whose flag bytes are reduced to
// their top bits (set when the byte is nonzero) and gathered, 8 rows at a
// time, as bit i of every byte; the 4 gathered words per 4 channels are then
// transposed bytewise into the channels' 32-bit words.  A lane's 16 words are
// two runs of 8 contiguous words in the keep layout (16-byte stores), and the
// 4 waves' runs for the same channels fill whole 128-byte lines.  Needs flags
// 16-byte and keep 16-byte aligned (the caller checks).
__device__ inline uint32_t flagged_bytes(uint32_t v) {  // top bit of each byte: byte != 0
    return (((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v) & 0x80808080u;
}

__device__ inline uint32_t byte_of(uint32_t a, int j) { return (a >> (8 * j)) & 0xFFu; }

__global__ void __launch_bounds__(256) keep_words_kernel(const uint8_t *__restrict__ flags,
                                                         uint32_t *__restrict__ keep, int S, int T, int C) {
    const int nkb = (C + 1023) / 1024, W = T / 32;
    const int kblk = blockIdx.x % nkb;
    const int w = (blockIdx.x / nkb) % W;
    const int s = 4 * (int)(blockIdx.x / (nkb * W)) + (int)(threadIdx.x >> 6);
    const int k = kblk * 1024 + 16 * (int)(threadIdx.x & 63);
    if (k >= C || s >= S) return;
    const uint8_t *f = flags + ((int64_t)s * T + (int64_t)w * 32) * C + k;
    uint32_t a[4][4];  // a[h][g]: byte j = flag bits of spectra 8 g ... 8 g + 7 of channel k + 4 h + j
#pragma unroll
    for (int g = 0; g < 4; ++g) {
#pragma unroll
        for (int h = 0; h < 4; ++h) a[h][g] = 0u;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const uint4 v = *reinterpret_cast<const uint4 *>(f + (int64_t)(8 * g + i) * C);
            a[0][g] |= flagged_bytes(v.x) >> (7 - i);
            a[1][g] |= flagged_bytes(v.y) >> (7 - i);
            a[2][g] |= flagged_bytes(v.z) >> (7 - i);
            a[3][g] |= flagged_bytes(v.w) >> (7 - i);
        }
    }
    uint32_t o[16];
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int j = 0; j < 4; ++j)
            o[4 * h + j] = ~(byte_of(a[h][0], j) | byte_of(a[h][1], j) << 8 | byte_of(a[h][2], j) << 16 |
                             byte_of(a[h][3], j) << 24);
#pragma unroll
    for (int e = 0; e < 2; ++e) {  // channels k + 8 e ... + 7
        uint4 *dst = reinterpret_cast<uint4 *>(keep + ((((int64_t)(k >> 3) + e) * W + w) * S + s) * 8);
        dst[0] = make_uint4(o[8 * e], o[8 * e + 1], o[8 * e + 2], o[8 * e + 3]);
        dst[1] = make_uint4(o[8 * e + 4], o[8 * e + 5], o[8 * e + 6], o[8 * e + 7]);
    }
}

// counts[k][p] += number of spectra where neither signal of pair p = (i, j)
// is flagged: the Gram matrix of the keep bits, G = B B^T with B[s][m] the
// keep bit of signal s in spectrum m (0 or 1), taken on the int8 matrix cores
// (v_mfma_i32_32x32x32_i8: exact int32 sums).  One wave per channel, the 8
// waves of a workgroup on the 8 channels of a channel block, which share every
// 32-byte piece of the keep words.  Lane l holds signals 32 a + (l mod 32)
// (a = 0, 1) and the spectra 16 (l / 32) ... + 15 of each 32-spectrum keep
// word, spread into 16 bytes of 0 / 1; the A and B operands are the same
// registers, so each product pairs the same spectrum of both signals whatever
// order the hardware gives K inside a lane.  Signals at or past S read as
// flagged everywhere.
typedef int v4i_t __attribute__((ext_vector_type(4)));
typedef int v16i_t __attribute__((ext_vector_type(16)));

__device__ inline v4i_t spread16(uint32_t x) {  // bit i of x -> byte i (0 or 1)
    v4i_t r;
#pragma unroll
    for (int d = 0; d < 4; ++d) r[d] = (int)((((x >> (4 * d)) & 15u) * 0x00204081u) & 0x01010101u);
    return r;
}

// The keep words of a channel block are contiguous: spans of 32 spectra, each
// S x 8 words.  The workgroup stages them PKB spans at a time in LDS (16-byte
// loads over all its threads, the next batch in flight during the products)
// at a padded place [span][signal][12] (8 words and a pad of 4).
constexpr int PKB = 8;

__global__ void __launch_bounds__(512) pair_counts_kernel(const uint32_t *__restrict__ keep, int S, int T,
                                                          int32_t *counts) {
    __shared__ __align__(16) uint32_t lk[2][PKB * kMaxSignals * 12];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, col = lane & 31, hf = lane >> 5;
    const int kb = blockIdx.x, k = 8 * kb + wv;
    const int W = T / 32;
    if (W <= 0) return;
    const int64_t P = (int64_t)S * (S + 1) / 2;
    const uint4 *src = reinterpret_cast<const uint4 *>(keep + (int64_t)kb * W * S * 8);
    const int nb = (W + PKB - 1) / PKB, nu = PKB * S * 2;  // batches; 16-byte units per batch (<= 1024)
    uint4 stg[2];
    auto fetch = [&](int b) {  // units past the last span read as zero
        const int nv = min(PKB, W - PKB * b) * S * 2;
        const uint4 *bs = src + (int64_t)b * nu;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int u = tid + 512 * e;
            stg[e] = u < nv ? bs[u] : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    auto put = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int u = tid + 512 * e;
            if (u < nu) {
                const int q = u / (2 * S), r = u - q * 2 * S;
                *reinterpret_cast<uint4 *>(&lk[buf][(q * kMaxSignals + (r >> 1)) * 12 + 4 * (r & 1)]) = stg[e];
            }
        }
    };
    // lanes past S read signal 0's place and mask the word off
    const uint32_t m0 = col < S ? ~0u : 0u, m1 = 32 + col < S ? ~0u : 0u;
    const int o0 = (col < S ? col : 0) * 12 + wv, o1 = (32 + col < S ? 32 + col : 0) * 12 + wv;
    v16i_t g00 = {}, g01 = {}, g11 = {};
    fetch(0);
    put(0);
    __syncthreads();
    for (int b = 0; b < nb; ++b) {
        if (b + 1 < nb) fetch(b + 1);
        const uint32_t *L = lk[b & 1];
#pragma unroll
        for (int q = 0; q < PKB; ++q) {
            const uint32_t x0 = L[q * kMaxSignals * 12 + o0] & m0, x1 = L[q * kMaxSignals * 12 + o1] & m1;
            const v4i_t b0 = spread16(x0 >> (16 * hf)), b1 = spread16(x1 >> (16 * hf));
            g00 = __builtin_amdgcn_mfma_i32_32x32x32_i8(b0, b0, g00, 0, 0, 0);
            g01 = __builtin_amdgcn_mfma_i32_32x32x32_i8(b0, b1, g01, 0, 0, 0);
            g11 = __builtin_amdgcn_mfma_i32_32x32x32_i8(b1, b1, g11, 0, 0, 0);
        }
        // the other buffer was last read in batch b - 1, before the barrier that ended it
        if (b + 1 < nb) put((b + 1) & 1);
        __syncthreads();
    }
    // accumulator r of lane l: row 8 (r / 4) + 4 (l / 32) + r mod 4 (signal i of
    // the A tile), column l mod 32 (signal j of the B tile); pair j (j + 1) / 2 + i
    // All 48 of a lane's counts are read before any is written back (distinct
    // pairs: a read-add-write chain per count would wait out the memory latency
    // 48 times); a lane's slots outside the triangle or past S are left alone.
    int32_t *out = counts + (int64_t)k * P;
    const v16i_t *g[3] = {&g00, &g01, &g11};
    int32_t old[3][16];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int ta = t == 2, j = 32 * (t > 0) + col;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 32 * ta + 8 * (r >> 2) + 4 * hf + (r & 3);
            old[t][r] = (i <= j && j < S) ? out[j * (j + 1) / 2 + i] : 0;
        }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int ta = t == 2, j = 32 * (t > 0) + col;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 32 * ta + 8 * (r >> 2) + 4 * hf + (r & 3);
            if (i <= j && j < S) out[j * (j + 1) / 2 + i] = old[t][r] + (*g[t])[r];
        }
    }
}

}  // namespace

hipError_t launch_mad_flag(const void *power, bool f16, int S, int T, int C, float M, uint8_t *flags,
                           hipStream_t st) {
    const int nb = S * (T / TT) * (C / KT);
    if (f16)
        hipLaunchKernelGGL(mad_tile_kernel<_Float16>, dim3(nb), dim3(KT), 0, st,
                           static_cast<const _Float16 *>(power), S, T, C, M, flags);
    else
        hipLaunchKernelGGL(mad_tile_kernel<float>, dim3(nb), dim3(KT), 0, st, static_cast<const float *>(power), S,
                           T, C, M, flags);
    return hipGetLastError();
}

hipError_t launch_apply_flags(int precision, const uint8_t *flags, void *spec, uint32_t *keep, int S, int T,
                              int C, hipStream_t st) {
    if (!spec && !(reinterpret_cast<uintptr_t>(flags) & 15) && !(reinterpret_cast<uintptr_t>(keep) & 15)) {
        const dim3 grid((unsigned)((int64_t)((S + 3) / 4) * (T / 32) * ((C + 1023) / 1024)));
        hipLaunchKernelGGL(keep_words_kernel, grid, dim3(256), 0, st, flags, keep, S, T, C);
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((int64_t)S * (T / 32) * (C / 256))), block(256);
    if (precision == CORR_FP32)
        hipLaunchKernelGGL((apply_keep_kernel<kChunk32>), grid, block, 0, st, flags, (uint8_t *)spec, keep, S, T, C);
    else
        hipLaunchKernelGGL((apply_keep_kernel<kChunk8>), grid, block, 0, st, flags, (uint8_t *)spec, keep, S, T, C);
    return hipGetLastError();
}

hipError_t launch_pair_counts(const uint32_t *keep, int S, int T, int C, int32_t *counts, hipStream_t st) {
    hipLaunchKernelGGL(pair_counts_kernel, dim3(C / 8), dim3(512), 0, st, keep, S, T, counts);
    return hipGetLastError();
}

}  // namespace corr
