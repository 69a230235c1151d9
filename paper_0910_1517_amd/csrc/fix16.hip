// fix16.hip -- the 16-bit fixed-point numerics of the paper's real-time
// pipeline, for comparison with the FP32, int8 and e4m3 paths (section 3.1:
// the 16-bit fixed-point FFT output; section 4.1: the integer fringe table
// scaled so that the rotated spectra keep 16 bits, 32-bit correlation
// products, accumulation in floating point).
//
//   fix16_kernel: from unrotated FP32 spectra in the X layout (the FFT output,
//     as the FP32 F-engine writes it for a geometry without fractional delay
//     or fringe terms),
//       q = sat16(rne(X / scale[s][k]))                      per component
//       j = nearest of the 1440 table steps to the Eq. 2 phase (FP64, the
//           operations of the table-mode F-engine)
//       y = sat16((q w_j + 2^13) >> 14)                      per component,
//     w_j the Q14 integer table (rint(2^14 cos, sin)); the product of two
//     int16 values and its rounding shift are exact in int32.  One thread per
//     channel and spectrum pair of a signal (one 16-byte chunk).
//   xengine16_kernel: A[k][p] = sum_m y_i conj(y_j), each product exact in
//     int32 (2 x 32767^2 < 2^31), sums in int64; optionally V = A scale_i
//     scale_j in FP64.  One thread per channel and pair.
#include <cmath>

#include "corr_internal.h"

namespace corr {
namespace {

__device__ __forceinline__ int sat16(int v) { return v > 32767 ? 32767 : (v < -32767 ? -32767 : v); }

__global__ void fix16_kernel(const float4 *spec, const corr_geom_t *geom, int64_t spectrum0, const float *scale,
                             const int2 *wtab, int S, int T, int C, double fs, double nu_bb, int sideband,
                             short2 *q16, short2 *y16) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over [T/2][C/8][S][8]
    const int64_t nchunk = (int64_t)(T / 2) * C * S;
    if (idx >= nchunk) return;
    const int kk = (int)(idx & 7);
    const int s = (int)((idx >> 3) % S);
    const int64_t rest = (idx >> 3) / S;
    const int kb = (int)(rest % (C / 8));
    const int g = (int)(rest / (C / 8));
    const int k = kb * 8 + kk;
    const float4 v = spec[idx];  // spectra 2g and 2g + 1 of channel k, signal s
    const corr_geom_t gm = geom[s];
    const float sc = scale[(int64_t)s * C + k];
    const int N = 2 * C;
    const double t_spec = (double)N / fs;
    const double fn = (double)gm.frac / (double)N;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int m = 2 * g + h;
        const float xr = h ? v.z : v.x, xi = h ? v.w : v.y;
        // the quotient correctly rounded (IEEE), then to the nearest integer, ties to even
        const int qr = sat16((int)fminf(fmaxf(rintf(__fdiv_rn(xr, sc)), -40000.f), 40000.f));
        const int qi = sat16((int)fminf(fmaxf(rintf(__fdiv_rn(xi, sc)), -40000.f), 40000.f));
        int j;
        {
#pragma clang fp contract(off)
            const double tm = ((double)(spectrum0 + m) + 0.5) * t_spec;
            double c = nu_bb * (double)gm.frac / fs + (double)sideband * (gm.psi0 + gm.rate * tm);
            c -= floor(c);
            const double r = rint((c + (double)k * fn) * 1440.0);
            j = (int)(r - 1440.0 * floor(r / 1440.0));  // r mod 1440, exact for integral r
            if (!(j >= 0 && j < kLutSteps)) j = 0;     // a non-finite phase reads entry 0, never out of the table
        }
        const int2 w = wtab[j];
        const int yr = sat16((qr * w.x - qi * w.y + 8192) >> 14);
        const int yi = sat16((qr * w.y + qi * w.x + 8192) >> 14);
        const int64_t o = ((int64_t)s * T + m) * C + k;
        if (q16) q16[o] = make_short2((short)qr, (short)qi);
        y16[o] = make_short2((short)yr, (short)yi);
    }
}

__global__ void xengine16_kernel(const short2 *y, int S, int T, int C, const float *scale, int64_t *acc,
                                 double *vis) {
    const int P = S * (S + 1) / 2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // over [P][C], channel fastest
    if (idx >= (int64_t)P * C) return;
    const int k = (int)(idx % C);
    const int p = (int)(idx / C);
    int j = 0;
    while ((j + 1) * (j + 2) / 2 <= p) ++j;
    const int i = p - j * (j + 1) / 2;
    const short2 *a = y + (int64_t)i * T * C + k;
    const short2 *b = y + (int64_t)j * T * C + k;
    int64_t re = 0, im = 0;
    for (int m = 0; m < T; ++m) {
        const short2 u = a[(int64_t)m * C], w = b[(int64_t)m * C];
        // (ur + i ui)(wr - i wi): each sum of two products is below 2^31
        re += (int64_t)((int)u.x * w.x + (int)u.y * w.y);
        im += (int64_t)((int)u.y * w.x - (int)u.x * w.y);
    }
    const int64_t o = ((int64_t)k * P + p) * 2;
    acc[o] = re;
    acc[o + 1] = im;
    if (vis) {
        const double f = (double)scale[(int64_t)i * C + k] * (double)scale[(int64_t)j * C + k];
        vis[o] = (double)re * f;
        vis[o + 1] = (double)im * f;
    }
}

}  // namespace

void fix16_table(int2 *w) {
    for (int j = 0; j < kLutSteps; ++j) {
        const double th = 2.0 * M_PI * (double)j / (double)kLutSteps;
        w[j] = make_int2((int)std::rint(16384.0 * std::cos(th)), (int)std::rint(16384.0 * std::sin(th)));
    }
}

hipError_t launch_fix16(const void *spec, const corr_geom_t *geom, int64_t spectrum0, const float *scale,
                        const int2 *wtab, int S, int T, int C, double fs, double nu_bb, int sideband, int16_t *q16,
                        int16_t *y16, hipStream_t st) {
    const int64_t n = (int64_t)(T / 2) * C * S;
    hipLaunchKernelGGL(fix16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<const float4 *>(spec), geom, spectrum0, scale, wtab, S, T, C, fs, nu_bb,
                       sideband, reinterpret_cast<short2 *>(q16), reinterpret_cast<short2 *>(y16));
    return hipGetLastError();
}

hipError_t launch_xengine16(const int16_t *y16, int S, int64_t T, int C, const float *scale, int64_t *acc,
                            double *vis, hipStream_t st) {
    const int64_t n = (int64_t)S * (S + 1) / 2 * C;
    hipLaunchKernelGGL(xengine16_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       reinterpret_cast<const short2 *>(y16), S, (int)T, C, scale, acc, vis);
    return hipGetLastError();
}

}  // namespace corr
