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
// are zeroed in the X-engine input, and the number of unflagged products of
// every pair, n_ij[k] = sum_m (1 - F_i)(1 - F_j), is counted exactly from
// bit-packed keep masks with popcounts.
#include "corr_internal.h"

namespace corr {
namespace {

constexpr int TT = kFlagTileSpectra;   // 64
constexpr int KT = kFlagTileChannels;  // 256

// Eq. 3 / Eq. 4 on n values x[0..n) (x is kept; work is scratch of n floats):
// flag[i] = |x_i - med| > M MAD / 0.6745, median of an even count = mean of
// the two middle values.
__device__ void mad_flags(const float *x, float *work, uint8_t *flag, int n, float M) {
    const int t = threadIdx.x;
    if (t < n) work[t] = x[t];
    __syncthreads();
    block_sort(work, n);
    const float med = 0.5f * (work[n / 2 - 1] + work[n / 2]);
    __syncthreads();
    if (t < n) work[t] = fabsf(x[t] - med);
    __syncthreads();
    block_sort(work, n);
    const float mad = 0.5f * (work[n / 2 - 1] + work[n / 2]);
    if (t < n) flag[t] = fabsf(x[t] - med) > M * mad / 0.6745f;
    __syncthreads();
}

// One tile (signal s, spectra m0..m0+63, channels k0..k0+255) per workgroup.
__global__ void __launch_bounds__(KT) mad_tile_kernel(const float *__restrict__ power, int S, int T, int C,
                                                      float M, uint8_t *flags) {
    __shared__ float tile[TT][KT + 1];
    __shared__ float rowv[TT], colv[KT], work[KT];
    __shared__ uint8_t rowf[TT], colf[KT];
    const int ntk = C / KT, ntm = T / TT;
    const int b = blockIdx.x;
    const int kt = b % ntk, mt = (b / ntk) % ntm, s = b / (ntk * ntm);
    const int t = threadIdx.x;
    const int64_t base = ((int64_t)s * T + (int64_t)mt * TT) * C + (int64_t)kt * KT + t;
    float cs = 0.f;
    for (int r = 0; r < TT; ++r) {
        const float v = power[base + (int64_t)r * C];
        tile[r][t] = v;
        cs += v;
    }
    colv[t] = cs / (float)TT;
    __syncthreads();
    if (t < TT) {
        float rs = 0.f;
        for (int k = 0; k < KT; ++k) rs += tile[t][k];
        rowv[t] = rs / (float)KT;
    }
    __syncthreads();
    mad_flags(rowv, work, rowf, TT, M);
    mad_flags(colv, work, colf, KT, M);
    const uint8_t cf = colf[t];
    for (int r = 0; r < TT; ++r) flags[base + (int64_t)r * C] = rowf[r] | cf;
}

// Keep masks and zeroing in one pass.  A workgroup owns 32 spectra (one keep
// word) x 256 channels of one signal.  Thread t builds the keep word of
// channel k0 + t from the 32 flag bytes of that channel (the loads of the
// workgroup's threads are consecutive bytes of a row), writes it to
// keep[k][s][w] when keep is given; then the workgroup zeroes the flagged cells of its X-layout chunks (index
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
    if (keep) keep[((int64_t)k * S + s) * W + w] = bits;
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

// counts[k][p] += popcount over time of keep_i & keep_j; one channel per
// workgroup, the keep words of all signals staged in LDS 256 words at a time.
__global__ void __launch_bounds__(256) pair_counts_kernel(const uint32_t *__restrict__ keep,
                                                          const uint16_t *__restrict__ pairs, int S, int T,
                                                          int32_t *counts) {
    __shared__ uint32_t kw[kMaxSignals][256 + 1];
    const int k = blockIdx.x;
    const int t = threadIdx.x;
    const int W = T / 32;
    const int P = S * (S + 1) / 2;
    int32_t cnt[9];  // pairs t, t + 256, ... (P <= 2080 < 9 * 256)
#pragma unroll
    for (int q = 0; q < 9; ++q) cnt[q] = 0;
    for (int w0 = 0; w0 < W; w0 += 256) {
        const int nw = min(256, W - w0);
        __syncthreads();
        for (int i = t; i < S * nw; i += 256) {
            const int s = i / nw, w = i % nw;
            kw[s][w] = keep[((int64_t)k * S + s) * W + w0 + w];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int p = t + 256 * q;
            if (p < P) {
                const int i = pairs[2 * p], j = pairs[2 * p + 1];
                int32_t c = 0;
                for (int w = 0; w < nw; ++w) c += __popc(kw[i][w] & kw[j][w]);
                cnt[q] += c;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int p = t + 256 * q;
        if (p < P) counts[(int64_t)k * P + p] += cnt[q];
    }
}

}  // namespace

hipError_t launch_mad_flag(const float *power, int S, int T, int C, float M, uint8_t *flags, hipStream_t st) {
    const int nb = S * (T / TT) * (C / KT);
    hipLaunchKernelGGL(mad_tile_kernel, dim3(nb), dim3(KT), 0, st, power, S, T, C, M, flags);
    return hipGetLastError();
}

hipError_t launch_apply_flags(int precision, const uint8_t *flags, void *spec, uint32_t *keep, int S, int T,
                              int C, hipStream_t st) {
    const dim3 grid((unsigned)((int64_t)S * (T / 32) * (C / 256))), block(256);
    if (precision == CORR_FP32)
        hipLaunchKernelGGL((apply_keep_kernel<kChunk32>), grid, block, 0, st, flags, (uint8_t *)spec, keep, S, T, C);
    else
        hipLaunchKernelGGL((apply_keep_kernel<kChunk8>), grid, block, 0, st, flags, (uint8_t *)spec, keep, S, T, C);
    return hipGetLastError();
}

hipError_t launch_pair_counts(const uint32_t *keep, const uint16_t *pairs, int S, int T, int C, int32_t *counts,
                              hipStream_t st) {
    hipLaunchKernelGGL(pair_counts_kernel, dim3(C), dim3(256), 0, st, keep, pairs, S, T, counts);
    return hipGetLastError();
}

}  // namespace corr
