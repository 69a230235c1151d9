// integrate.hip -- long-term accumulation of the X-engine output.
//
// Section 4.1: the products up to the MAC are fixed point, the long-term sum
// is floating point.  Here the int32 (INT8) or FP32 (FP32 / FP8) accumulator
// splits of one integration are summed (int64 exact, or FP64), scaled by the
// recorded requantisation scales of the two signals (scale_i * scale_j, in
// FP64) and added to an FP64 state; the accumulator is zeroed for the next
// round.  A dump converts the state to complex64 visibilities (section 2.3.2:
// visibilities leave the correlator after each integration).
#include <type_traits>

#include "corr_internal.h"

namespace corr {
namespace {

template <typename A>
__global__ void integrate_kernel(A *acc, const float *scale, double *state, float *vis,
                                 const uint16_t *pairs, int C, int64_t P, int splits, int use_scale,
                                 uint32_t flags) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)C * P) return;
    const int k = (int)(idx / P);
    const int64_t p = idx % P;
    double re, im;
    if constexpr (std::is_integral<A>::value) {  // integer accumulator: exact int64 sum
        int64_t sr = 0, si = 0;
        for (int s = 0; s < splits; ++s) {
            A *a = acc + ((int64_t)s * C * P + idx) * 2;
            sr += a[0];
            si += a[1];
            a[0] = 0;
            a[1] = 0;
        }
        re = (double)sr;
        im = (double)si;
    } else {
        re = 0.0;
        im = 0.0;
        for (int s = 0; s < splits; ++s) {
            A *a = acc + ((int64_t)s * C * P + idx) * 2;
            re += (double)a[0];
            im += (double)a[1];
            a[0] = 0;
            a[1] = 0;
        }
    }
    if (use_scale) {
        const int i = pairs[2 * p], j = pairs[2 * p + 1];
        const double g = (double)scale[(int64_t)i * C + k] * (double)scale[(int64_t)j * C + k];
        re *= g;
        im *= g;
    }
    double2 v = reinterpret_cast<double2 *>(state)[idx];
    v.x += re;
    v.y += im;
    if (flags & CORR_DUMP) reinterpret_cast<float2 *>(vis)[idx] = make_float2((float)v.x, (float)v.y);
    if (flags & CORR_RESET) v = make_double2(0.0, 0.0);
    reinterpret_cast<double2 *>(state)[idx] = v;
}

}  // namespace

hipError_t launch_integrate(int precision, void *acc, const float *scale, double *state, float *vis,
                            const uint16_t *pairs, int S, int C, int splits, uint32_t flags,
                            hipStream_t st) {
    const int64_t P = (int64_t)S * (S + 1) / 2;
    const int64_t n = (int64_t)C * P;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    if (precision == CORR_INT8)
        hipLaunchKernelGGL(integrate_kernel<int32_t>, grid, block, 0, st, (int32_t *)acc, scale, state, vis,
                           pairs, C, P, splits, 1, flags);
    else
        hipLaunchKernelGGL(integrate_kernel<float>, grid, block, 0, st, (float *)acc, scale, state, vis,
                           pairs, C, P, splits, precision == CORR_FP8_E4M3 ? 1 : 0, flags);
    return hipGetLastError();
}

}  // namespace corr
