// Time-domain MAD voltage blanker (section 5, Eq. 3 and 4) and its noise
// table.
//
// The blanker runs on the int8 voltage rows the F-engine reads, before the
// FFT.  Each block of B consecutive samples of one signal gets its median x~
// and MAD = median |x - x~|.  A sample with |x - x~| > M MAD / 0.6745 is
// replaced by rint(x~ + sigma z) clamped to int8, where sigma = MAD / 0.6745
// (the robust estimate of the voltage RMS for normal noise) and z comes from a
// precomputed Gaussian noise table with one row per signal, so the
// replacements of different antennas are independent.  A block with MAD = 0
// has no scale estimate and passes unchanged.
//
// One workgroup per (block, signal).  The block (up to 64 KiB) is loaded once
// into registers and never re-read.  int8 has 256 values, so the median and
// the MAD are exact order statistics of a 256-bin histogram built with LDS
// atomics.  The counters are 32 bits wide, one bin to a word, in 16 copies
// (thread t adds to copy t mod 16); the whole histogram is 16 KiB.  After the
// block-wide inclusive prefix sum P of the merged histogram:
//   k-th smallest sample           = #{u : P[u] < k} - 128,
//   #{samples with |2x - 2x~| <= D} = P[hi(D)] - P[lo(D) - 1], a range query,
//   k-th smallest |2x - 2x~|       = #{D : count(D) < k},
// each one block-wide count, with no sort.  The threshold test
// |x - x~| > M MAD / 0.6745 is one FP64 expression per block, turned into
// the integer range [lo, hi] of values kept.  The number blanked comes from P
// too.  Eq. 4 is applied to four samples per instruction (byte-wise
// arithmetic in 32-bit words).  The blanked positions of a block are queued in
// the histogram's LDS, and all threads then compute their replacements from
// the table in FP64 and store them as single bytes.  Out of place, the block
// is copied right after it is loaded and the replacements patch the copy; in
// place, only the blanked bytes are written.
//
// Noise table: entry j of signal s is the Irwin-Hall sum of twelve 16-bit
// uniforms (U + 1/2) / 65536, minus 6.  The uniforms are the 16-bit halves
// (low, then high) of words 0..3 of Philox4x32-10 at counter (j, j >> 32, s,
// 0) and of words 0..1 at counter (j, j >> 32, s, 1), keyed by the 64-bit
// seed (Salmon, Moraes, Dror and Shaw, SC'11).  Every entry is a multiple of
// 2^-16 below 6 in magnitude, so it is exact in float.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "corr_internal.h"

namespace {

constexpr int kBlankThreads = 256;
constexpr int kBlankWaves = kBlankThreads / 64;
constexpr int kHistCopies = 16;                     // thread t adds to copy t mod 16
constexpr int kQueueCap = 256 * kHistCopies * 2;    // 16-bit positions in the histogram's memory
constexpr int kBlankMaxSignals = 65535;           // grid y
constexpr int kBlankMaxBlock = 65536;             // 16 chunks of 16 B per thread
constexpr int64_t kBlankMaxTable = 1ll << 31;

// ---------------------------------------------------------------- Philox
// One Philox4x32-10 block: ten rounds of two 32x32->64 products whose halves
// are mixed with the other two words and the round key; the key advances by
// the Weyl constants between rounds.
__device__ inline uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ inline uint32_t halves(uint32_t w) { return (w & 0xFFFFu) + (w >> 16); }

__global__ __launch_bounds__(256) void noise_table_kernel(uint32_t k0, uint32_t k1, int64_t total, int lg_L,
                                                          float *table) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const uint64_t j = (uint64_t)e & ((1ull << lg_L) - 1);
        const uint32_t s = (uint32_t)((uint64_t)e >> lg_L);
        const uint4 a = philox4x32_10(make_uint4((uint32_t)j, (uint32_t)(j >> 32), s, 0u), k0, k1);
        const uint4 b = philox4x32_10(make_uint4((uint32_t)j, (uint32_t)(j >> 32), s, 1u), k0, k1);
        const int32_t sum = (int32_t)(halves(a.x) + halves(a.y) + halves(a.z) + halves(a.w) + halves(b.x) +
                                      halves(b.y));
        // sum of (U + 1/2) / 65536 over 12, minus 6; |numerator| < 2^19: exact
        table[e] = (float)(sum + 6 - 6 * 65536) * (1.0f / 65536.0f);
    }
}

// ---------------------------------------------------------------- blanker
// Sum of v over the workgroup (every thread gets it).
__device__ inline uint32_t block_sum(uint32_t v, uint32_t *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();  // red may still be read from a previous use
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < kBlankWaves; ++w) t += red[w];
    return t;
}

// Number of samples with |2x - med2| <= D, from the inclusive prefix sums
// cum[u] over biased values u = x + 128.
__device__ inline int dev_count(const uint32_t *cum, int med2, int D) {
    const int hi = min(((med2 + D) >> 1) + 128, 255);     // floor((med2 + D) / 2)
    const int lo = max(-((D - med2) >> 1) + 128, 0);      // ceil((med2 - D) / 2)
    if (hi < lo) return 0;
    return (int)cum[hi] - (lo ? (int)cum[lo - 1] : 0);
}

// Replacement value of a blanked sample: rint(x~ + sigma z), clamped, all in
// FP64 with every product and sum rounded on its own.
__device__ inline uint32_t replacement(double half_med2, double sigma, float z) {
#pragma clang fp contract(off)
    double r = rint(half_med2 + sigma * (double)z);
    r = fmin(fmax(r, -128.0), 127.0);
    return (uint32_t)(int32_t)r & 0xFFu;
}

// Eq. 4 for four samples at once: bit 7 of byte i of the result is set when
// byte i of w (a signed sample) lies outside [lo, hi].  d = (x - lo) mod 256
// per byte, without borrows between bytes (lo_lo7 = low seven bits of lo in
// every byte, lo_hi = bit 7 of ~lo in every byte); the sample is outside when
// d > span = hi - lo.  WIDE (span >= 128): d > span <=> d >= 128 and its low
// seven bits exceed span - 128; otherwise d >= 128 or its low seven bits
// exceed span.
template <bool WIDE>
__device__ inline uint32_t outside4(uint32_t w, uint32_t lo_lo7, uint32_t lo_hi, uint32_t c7) {
    const uint32_t d = ((w | 0x80808080u) - lo_lo7) ^ (w & 0x80808080u) ^ lo_hi;
    const uint32_t gt = (d & 0x7F7F7F7Fu) + c7;  // bit 7 set <=> low seven bits > (span mod 128)
    return (WIDE ? (d & gt) : (d | gt)) & 0x80808080u;
}

// Replace the flagged bytes of one chunk (f[d]: bit 7 of byte k set = byte
// 4 d + k flagged), one at a time.
__device__ inline void replace_chunk(uint32_t w4[4], const uint32_t f[4], const float *trow, int64_t p0,
                                     int64_t Lmask, double half_med2, double sigma) {
#pragma unroll
    for (int d = 0; d < 4; ++d) {
        uint32_t m = f[d];
        while (m) {
            const int k = __builtin_ctz(m) >> 3;
            m &= m - 1;
            const uint32_t r = replacement(half_med2, sigma, trow[(p0 + 4 * d + k) & Lmask]);
            w4[d] = (w4[d] & ~(0xFFu << (8 * k))) | (r << (8 * k));
        }
    }
}

struct BlankShared {
    // 256 raw byte values x 16 copies of a 32-bit counter: bin r of copy c at
    // word 16 r + c.  After the merge the same memory holds the queue of
    // blanked positions.
    uint32_t hist[256 * kHistCopies];
    uint32_t cum[256];
    uint32_t red[kBlankWaves];
};

// One block of `len` samples (len < B only for a row's last block: TAIL).
template <int J, bool TAIL>
__device__ inline void blank_block(BlankShared &sh, const uint4 (&v)[J], int len, int8_t *orow, double M,
                                   const float *trow, int64_t Lmask, int64_t p_blk, int32_t *count_out,
                                   int32_t *stat_out, bool in_place) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    // histogram (the counters were zeroed before the first barrier): raw byte
    // r of the sample, copy tid mod 16
    uint32_t *hl = sh.hist + (tid & (kHistCopies - 1));
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int c = tid + kBlankThreads * j;
        const int nv = len - c * 16;
        if (nv <= 0) continue;
        const uint32_t w4[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (TAIL && k >= nv) break;
            __hip_atomic_fetch_add(hl + ((w4[k >> 2] >> (8 * (k & 3))) & 0xFFu) * kHistCopies, 1u,
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
    }
    __syncthreads();

    // merge: thread t owns bin u = t (raw byte u ^ 0x80) and sums its copies
    // (the start is rotated so that a wave's lanes spread over the banks),
    // then the block-wide inclusive prefix sum over bins
    const int u = tid;
    uint32_t h = 0;
    {
        const uint4 *row = reinterpret_cast<const uint4 *>(sh.hist) + (u ^ 0x80) * (kHistCopies / 4);
#pragma unroll
        for (int q = 0; q < kHistCopies / 4; ++q) {
            const uint4 r = row[(q + u) & (kHistCopies / 4 - 1)];
            h += r.x + r.y + r.z + r.w;
        }
    }
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(h, off, 64);
        if (lane >= off) h += t;
    }
    if (lane == 63) sh.red[wave] = h;
    __syncthreads();
    for (int w = 0; w < wave; ++w) h += sh.red[w];
    sh.cum[u] = h;  // cum[u] = #{samples with x + 128 <= u}

    // median (Eq. 3): the k1-th and k2-th smallest samples (equal for odd
    // len) are #{u : cum[u] < k} - 128; med2 = their sum = 2 x~
    const uint32_t k1 = (uint32_t)(len + 1) >> 1, k2 = (uint32_t)(len >> 1) + 1;
    const uint32_t cm = block_sum((h < k1 ? 1u : 0u) | (h < k2 ? 0x10000u : 0u), sh.red);
    const int med2 = (int)(cm & 0xFFFFu) + (int)(cm >> 16) - 256;

    // MAD (Eq. 3): the k1-th and k2-th smallest of d = |2x - med2| in
    // [0, 510] are #{D : count(d <= D) < k}; thread t tests D = t and t + 256
    const int cA = dev_count(sh.cum, med2, tid), cB = dev_count(sh.cum, med2, tid + 256);
    const uint32_t pd = ((uint32_t)(cA < (int)k1) + (uint32_t)(cB < (int)k1)) |
                        (((uint32_t)(cA < (int)k2) + (uint32_t)(cB < (int)k2)) << 16);
    const uint32_t cd = block_sum(pd, sh.red);
    const int mad4 = (int)(cd & 0xFFFFu) + (int)(cd >> 16);

    // Eq. 4 as an integer range: keep lo <= x <= hi; the number blanked
    // comes from the prefix sums
    int lo = -128, hi = 127;
    if (mad4 > 0) {
        const double mad = (double)mad4 * 0.25;
        const double thr2 = 2.0 * ((M * mad) / 0.6745);  // |2x - med2| > thr2 blanks
        const int dmax = thr2 >= 511.0 ? 511 : (int)floor(thr2);
        hi = min((med2 + dmax) >> 1, 127);
        lo = max(-((dmax - med2) >> 1), -128);
    }
    const int below = lo > -128 ? (int)sh.cum[lo + 127] : 0;
    const int above = hi < 127 ? len - (int)sh.cum[hi + 128] : 0;
    const int n_out = below + above;
    if (tid == 0) {
        if (count_out) *count_out = n_out;
        if (stat_out) {
            stat_out[0] = med2;
            stat_out[1] = mad4;
        }
    }
    if (n_out == 0) return;  // nothing to blank (uniform)

    // flag four samples per instruction
    const uint32_t span = (uint32_t)(hi - lo);
    const uint32_t lo_rep = (uint32_t)(lo & 0xFF) * 0x01010101u;
    const uint32_t lo_lo7 = lo_rep & 0x7F7F7F7Fu, lo_hi = ~lo_rep & 0x80808080u;
    const uint32_t c7 = (127u - (span & 127u)) * 0x01010101u;
    const bool wide = span >= 128;
    // flags of chunk j, word d (bit 7 of each outlier byte); kept in
    // registers for up to four chunks per thread, recomputed beyond
    auto flags = [&](int j, int d) -> uint32_t {
        const int nv = len - (tid + kBlankThreads * j) * 16;
        const uint32_t w = d == 0 ? v[j].x : d == 1 ? v[j].y : d == 2 ? v[j].z : v[j].w;
        uint32_t fd = wide ? outside4<true>(w, lo_lo7, lo_hi, c7) : outside4<false>(w, lo_lo7, lo_hi, c7);
        if (TAIL) {  // bytes past the row's end are never flagged
            const int keep = min(max(nv - 4 * d, 0), 4);
            fd &= keep >= 4 ? 0xFFFFFFFFu : ((1u << (8 * keep)) - 1u);
        } else if (nv <= 0) {
            fd = 0u;
        }
        return fd;
    };
    constexpr bool kKeep = J <= 4;
    uint32_t f[kKeep ? J : 1][4];
    uint32_t mine = 0;
#pragma unroll
    for (int j = 0; j < J; ++j) {
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            const uint32_t fd = flags(j, d);
            if (kKeep) f[kKeep ? j : 0][d] = fd;
            mine += (uint32_t)__builtin_popcount(fd);
        }
    }

    // block-wide exclusive scan of the per-thread counts
    uint32_t pre = mine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(pre, off, 64);
        if (lane >= off) pre += t;
    }
    __syncthreads();  // red is reused; the histogram words are free after the merge
    if (lane == 63) sh.red[wave] = pre;
    __syncthreads();
    uint32_t base = pre - mine;
    for (int w = 0; w < wave; ++w) base += sh.red[w];
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < kBlankWaves; ++w) total += sh.red[w];  // equals n_out

    const double half_med2 = 0.5 * (double)med2;
    const double sigma = ((double)mad4 * 0.25) / 0.6745;
    if (total > (uint32_t)kQueueCap) {
        // more outliers than the queue holds (possible only for blocks longer
        // than 2 kQueueCap samples, since fewer than half the samples of a
        // block lie beyond M MAD / 0.6745 >= MAD for the usual M): each thread
        // patches its own chunks
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int c = tid + kBlankThreads * j;
            const int nv = len - c * 16;
            uint32_t fj[4];
#pragma unroll
            for (int d = 0; d < 4; ++d) fj[d] = kKeep ? f[kKeep ? j : 0][d] : flags(j, d);
            if ((fj[0] | fj[1] | fj[2] | fj[3]) == 0u) continue;
            uint32_t w4[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
            replace_chunk(w4, fj, trow, p_blk + (int64_t)c * 16, Lmask, half_med2, sigma);
            if (!TAIL || nv >= 16) {
                *reinterpret_cast<uint4 *>(orow + c * 16) = make_uint4(w4[0], w4[1], w4[2], w4[3]);
            } else {
                for (int k = 0; k < nv; ++k) orow[c * 16 + k] = (int8_t)(w4[k >> 2] >> (8 * (k & 3)));
            }
        }
        return;
    }

    // queue the blanked positions, then replace them with all threads busy
    uint16_t *queue = reinterpret_cast<uint16_t *>(sh.hist);
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int c = tid + kBlankThreads * j;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t m = kKeep ? f[kKeep ? j : 0][d] : flags(j, d);
            while (m) {
                const int bit = __builtin_ctz(m);
                m &= m - 1;
                queue[base++] = (uint16_t)(c * 16 + 4 * d + (bit >> 3));
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < (int)total; e += kBlankThreads) {
        const int pos = queue[e];
        orow[pos] = (int8_t)replacement(half_med2, sigma, trow[(p_blk + pos) & Lmask]);
    }
}

template <int J>
__global__ __launch_bounds__(kBlankThreads) void blank_kernel(const int8_t *__restrict__ x, int8_t *out,
                                                              int64_t row_stride, int64_t n, int B, double M,
                                                              const float *__restrict__ table, int64_t L,
                                                              int64_t sample0, int32_t *counts, int32_t *stats,
                                                              int in_place) {
    __shared__ __attribute__((aligned(16))) BlankShared sh;
    const int tid = threadIdx.x;
    const int s = blockIdx.y;
    const int64_t i0 = (int64_t)blockIdx.x * B;
    const int len = (int)min((int64_t)B, n - i0);
    const int8_t *xr = x + (int64_t)s * row_stride + i0;
    int8_t *orow = out + (int64_t)s * row_stride + i0;

    // the block's samples, once, into registers; out of place the copy goes
    // out at once (blanked samples are patched at the end)
    uint4 v[J];
#pragma unroll
    for (int j = 0; j < J; ++j) {
        const int c = tid + kBlankThreads * j;
        v[j] = (c * 16 < len) ? *reinterpret_cast<const uint4 *>(xr + c * 16) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 256 * kHistCopies / 4 / kBlankThreads; ++q)
        reinterpret_cast<uint4 *>(sh.hist)[tid + kBlankThreads * q] = make_uint4(0, 0, 0, 0);
    if (!in_place) {
#pragma unroll
        for (int j = 0; j < J; ++j) {
            const int c = tid + kBlankThreads * j;
            const int nv = len - c * 16;
            if (nv >= 16) {
                *reinterpret_cast<uint4 *>(orow + c * 16) = v[j];
            } else if (nv > 0) {
                const uint32_t w4[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
                for (int k = 0; k < nv; ++k) orow[c * 16 + k] = (int8_t)(w4[k >> 2] >> (8 * (k & 3)));
            }
        }
    }
    __syncthreads();

    const int64_t b = (int64_t)s * gridDim.x + blockIdx.x;
    int32_t *cnt = counts ? counts + b : nullptr;
    int32_t *st = stats ? stats + 2 * b : nullptr;
    const float *trow = table + (int64_t)s * L;
    if (len == B)
        blank_block<J, false>(sh, v, len, orow, M, trow, L - 1, sample0 + i0, cnt, st, in_place != 0);
    else
        blank_block<J, true>(sh, v, len, orow, M, trow, L - 1, sample0 + i0, cnt, st, in_place != 0);
}

template <int J>
hipError_t launch_blank_j(const int8_t *x, int8_t *out, int64_t row_stride, int S, int64_t n, int B, double M,
                          const float *table, int64_t L, int64_t sample0, int32_t *counts, int32_t *stats,
                          hipStream_t st) {
    const dim3 grid((unsigned)((n + B - 1) / B), (unsigned)S);
    hipLaunchKernelGGL(blank_kernel<J>, grid, dim3(kBlankThreads), 0, st, x, out, row_stride, n, B, M, table, L,
                       sample0, counts, stats, (int)(out == x));
    return hipGetLastError();
}

thread_local char g_blank_err[512];

corr_status blank_fail(corr_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_blank_err, sizeof(g_blank_err), fmt, ap);
    va_end(ap);
    return st;
}

bool is_aligned(const void *p, size_t a) { return ((uintptr_t)p & (a - 1)) == 0; }

}  // namespace

extern "C" {

corr_status corr_blank_noise_table(uint64_t seed, int32_t S, int64_t L, float *d_table, void *stream) {
    g_blank_err[0] = 0;
    if (!d_table) return blank_fail(CORR_ERR_NULL, "d_table is required");
    if (!is_aligned(d_table, 4)) return blank_fail(CORR_ERR_ALIGN, "d_table must be 4-byte aligned");
    if (S < 1 || S > kBlankMaxSignals) return blank_fail(CORR_ERR_INVALID, "S=%d outside [1, %d]", S, kBlankMaxSignals);
    if (L < 1 || L > kBlankMaxTable || (L & (L - 1)))
        return blank_fail(CORR_ERR_INVALID, "L=%lld must be a power of two in [1, 2^31]", (long long)L);
    int lg = 0;
    while ((1ll << lg) < L) ++lg;
    const int64_t total = (int64_t)S * L;
    const int64_t want = (total + 255) / 256;
    const unsigned grid = (unsigned)(want < 65536 ? want : 65536);
    hipLaunchKernelGGL(noise_table_kernel, dim3(grid), dim3(256), 0, (hipStream_t)stream, (uint32_t)seed,
                       (uint32_t)(seed >> 32), total, lg, d_table);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? CORR_OK
                           : blank_fail(CORR_ERR_DEVICE, "noise table launch: %s", hipGetErrorString(e));
}

corr_status corr_blank_voltages(const int8_t *d_x, int64_t row_stride, int32_t S, int64_t n, int32_t block, float M,
                                const float *d_table, int64_t table_len, int64_t sample0, int8_t *d_out,
                                int32_t *d_counts, int32_t *d_stats, void *stream) {
    g_blank_err[0] = 0;
    if (!d_x || !d_table || !d_out) return blank_fail(CORR_ERR_NULL, "d_x, d_table and d_out are required");
    if (!is_aligned(d_x, 16) || !is_aligned(d_out, 16) || !is_aligned(d_table, 4) ||
        (d_counts && !is_aligned(d_counts, 4)) || (d_stats && !is_aligned(d_stats, 4)))
        return blank_fail(CORR_ERR_ALIGN, "d_x and d_out need 16-byte, d_table, d_counts and d_stats 4-byte alignment");
    if (S < 1 || S > kBlankMaxSignals) return blank_fail(CORR_ERR_INVALID, "S=%d outside [1, %d]", S, kBlankMaxSignals);
    if (n < 0) return blank_fail(CORR_ERR_INVALID, "n=%lld is negative", (long long)n);
    if (row_stride % 16 || row_stride < n)
        return blank_fail(CORR_ERR_INVALID, "row_stride=%lld must be a multiple of 16 and >= n", (long long)row_stride);
    if (block < 16 || block > kBlankMaxBlock || block % 16)
        return blank_fail(CORR_ERR_INVALID, "block=%d must be a multiple of 16 in [16, %d]", block, kBlankMaxBlock);
    if (!(M > 0.f) || !std::isfinite(M)) return blank_fail(CORR_ERR_INVALID, "threshold M must be finite and > 0");
    if (table_len < 1 || table_len > kBlankMaxTable || (table_len & (table_len - 1)))
        return blank_fail(CORR_ERR_INVALID, "table_len=%lld must be a power of two in [1, 2^31]", (long long)table_len);
    if (sample0 < 0 || sample0 > INT64_MAX - n)
        return blank_fail(CORR_ERR_INVALID, "sample0 must be >= 0 with sample0 + n <= 2^63 - 1");
    const int64_t nblk = (n + block - 1) / block;
    if (nblk > 0x7FFFFFFF) return blank_fail(CORR_ERR_INVALID, "more than 2^31 - 1 blocks per row");
    if (n == 0) return CORR_OK;
    const int J = (block + 16 * kBlankThreads - 1) / (16 * kBlankThreads);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if (J <= 1)
        e = launch_blank_j<1>(d_x, d_out, row_stride, S, n, block, (double)M, d_table, table_len, sample0, d_counts,
                              d_stats, st);
    else if (J <= 2)
        e = launch_blank_j<2>(d_x, d_out, row_stride, S, n, block, (double)M, d_table, table_len, sample0, d_counts,
                              d_stats, st);
    else if (J <= 4)
        e = launch_blank_j<4>(d_x, d_out, row_stride, S, n, block, (double)M, d_table, table_len, sample0, d_counts,
                              d_stats, st);
    else if (J <= 8)
        e = launch_blank_j<8>(d_x, d_out, row_stride, S, n, block, (double)M, d_table, table_len, sample0, d_counts,
                              d_stats, st);
    else
        e = launch_blank_j<16>(d_x, d_out, row_stride, S, n, block, (double)M, d_table, table_len, sample0, d_counts,
                               d_stats, st);
    return e == hipSuccess ? CORR_OK : blank_fail(CORR_ERR_DEVICE, "blanker launch: %s", hipGetErrorString(e));
}

const char *corr_blank_last_error(void) { return g_blank_err; }

}  // extern "C"
