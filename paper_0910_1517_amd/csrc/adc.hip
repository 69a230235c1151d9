// ADC input formats (sections 2.3.2 and 3.3): the acquisition cards digitise
// four inputs each, 8-bit (16 MHz mode) or 4-bit (33 MHz mode), and the
// compute side demultiplexes the four streams and unpacks 4-bit samples to 8
// bits before the FFT.
//
// Raw stream of a card: time-major, the four inputs of a time sample
// together.  8-bit: byte 4t + i is input i.  4-bit: byte 2t + i/2, nibble
// i mod 2 (low nibble first).  Samples are two's complement; 4-bit ones are
// sign-extended, value kept.  Output: int8 rows, row 4c + i = input i of
// card c, the layout corr_fengine reads.
//
// One thread per card and 16 consecutive time samples.  It loads the 64 (8-bit)
// or 32 (4-bit) raw bytes as 16-byte vectors, transposes them in registers,
// and stores one 16-byte vector to each of the card's four rows, so each
// wave writes whole lines.  HBM-bound: (bits/2 + 4) bytes per time sample of
// a card.

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>

#include "corr_internal.h"

namespace {

constexpr int kAdcThreads = 256;
constexpr int kAdcMaxCards = 16383;  // 4 rows per card, rows counted in int32

// byte k of w, as the low byte of a word
__device__ inline uint32_t byte_of(uint32_t w, int k) { return (w >> (8 * k)) & 0xFFu; }

// 4-bit code at nibble position p of w, sign-extended, as a byte
__device__ inline uint32_t nib_of(uint32_t w, int p) {
    return (uint32_t)__builtin_amdgcn_sbfe((int)w, 4 * p, 4) & 0xFFu;
}

template <int BITS>
__global__ __launch_bounds__(kAdcThreads) void adc_unpack_kernel(const uint8_t *__restrict__ raw, int64_t raw_stride,
                                                                 int64_t n, int8_t *__restrict__ x,
                                                                 int64_t row_stride) {
    const int card = blockIdx.y;
    const int64_t t0 = ((int64_t)blockIdx.x * kAdcThreads + threadIdx.x) * 16;
    if (t0 >= n) return;
    const uint8_t *r = raw + (int64_t)card * raw_stride;
    int8_t *row0 = x + (int64_t)(4 * card) * row_stride;
    if (t0 + 16 <= n) {
        uint32_t o[4][4];  // [input][output word]
        if (BITS == 8) {
            uint32_t d[16];  // d[q] = the four inputs of time t0 + q
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const uint4 u = *reinterpret_cast<const uint4 *>(r + 4 * t0 + 16 * v);
                d[4 * v] = u.x;
                d[4 * v + 1] = u.y;
                d[4 * v + 2] = u.z;
                d[4 * v + 3] = u.w;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    o[i][w] = byte_of(d[4 * w], i) | (byte_of(d[4 * w + 1], i) << 8) |
                              (byte_of(d[4 * w + 2], i) << 16) | (byte_of(d[4 * w + 3], i) << 24);
        } else {
            uint32_t d[8];  // d[q] = times t0 + 2q and t0 + 2q + 1, two bytes each
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const uint4 u = *reinterpret_cast<const uint4 *>(r + 2 * t0 + 16 * v);
                d[4 * v] = u.x;
                d[4 * v + 1] = u.y;
                d[4 * v + 2] = u.z;
                d[4 * v + 3] = u.w;
            }
            // input i of time 2q + h is nibble 4h + i of d[q]
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int w = 0; w < 4; ++w)
                    o[i][w] = nib_of(d[2 * w], i) | (nib_of(d[2 * w], 4 + i) << 8) |
                              (nib_of(d[2 * w + 1], i) << 16) | (nib_of(d[2 * w + 1], 4 + i) << 24);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            *reinterpret_cast<uint4 *>(row0 + (int64_t)i * row_stride + t0) = make_uint4(o[i][0], o[i][1], o[i][2], o[i][3]);
    } else {
        // the row's last, partial group: byte by byte
        for (int64_t t = t0; t < n; ++t)
            for (int i = 0; i < 4; ++i) {
                int v;
                if (BITS == 8) {
                    v = (int8_t)r[4 * t + i];
                } else {
                    const int c = (r[2 * t + i / 2] >> (4 * (i % 2))) & 0xF;
                    v = c >= 8 ? c - 16 : c;
                }
                row0[(int64_t)i * row_stride + t] = (int8_t)v;
            }
    }
}

thread_local char g_adc_err[512];

corr_status adc_fail(corr_status st, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_adc_err, sizeof(g_adc_err), fmt, ap);
    va_end(ap);
    return st;
}

}  // namespace

extern "C" {

corr_status corr_adc_unpack(const uint8_t *d_raw, int64_t raw_stride, int32_t n_cards, int64_t n, int32_t bits,
                            int8_t *d_x, int64_t row_stride, void *stream) {
    g_adc_err[0] = 0;
    if (!d_raw || !d_x) return adc_fail(CORR_ERR_NULL, "d_raw and d_x are required");
    if (((uintptr_t)d_raw & 15) || ((uintptr_t)d_x & 15))
        return adc_fail(CORR_ERR_ALIGN, "d_raw and d_x must be 16-byte aligned");
    if (bits != 4 && bits != 8) return adc_fail(CORR_ERR_INVALID, "bits=%d must be 4 or 8", bits);
    if (n_cards < 1 || n_cards > kAdcMaxCards)
        return adc_fail(CORR_ERR_INVALID, "n_cards=%d outside [1, %d]", n_cards, kAdcMaxCards);
    if (n < 0) return adc_fail(CORR_ERR_INVALID, "n=%lld is negative", (long long)n);
    if (n > ((int64_t)1 << 40)) return adc_fail(CORR_ERR_INVALID, "n=%lld above 2^40", (long long)n);
    if (raw_stride % 16 || raw_stride < n * bits / 2)
        return adc_fail(CORR_ERR_INVALID, "raw_stride=%lld must be a multiple of 16 and >= n*bits/2",
                        (long long)raw_stride);
    if (row_stride % 16 || row_stride < n)
        return adc_fail(CORR_ERR_INVALID, "row_stride=%lld must be a multiple of 16 and >= n", (long long)row_stride);
    if (n == 0) return CORR_OK;
    const dim3 grid((unsigned)((n + 16 * kAdcThreads - 1) / (16 * kAdcThreads)), (unsigned)n_cards);
    if (bits == 8)
        hipLaunchKernelGGL(adc_unpack_kernel<8>, grid, dim3(kAdcThreads), 0, (hipStream_t)stream, d_raw, raw_stride, n,
                           d_x, row_stride);
    else
        hipLaunchKernelGGL(adc_unpack_kernel<4>, grid, dim3(kAdcThreads), 0, (hipStream_t)stream, d_raw, raw_stride, n,
                           d_x, row_stride);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? CORR_OK : adc_fail(CORR_ERR_DEVICE, "unpack launch: %s", hipGetErrorString(e));
}

const char *corr_adc_last_error(void) { return g_adc_err; }

}  // extern "C"
