// corr_api.hip -- host side of libcorr: plan validation, tables, workspace
// layout, argument checks and kernel launches behind the C ABI of corr.h.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "corr_internal.h"

using namespace corr;

struct corr_plan {
    corr_desc_t d;
    int log2m = 0;
    int M = 0;  // complex points of the half-length transform = channels C
    int64_t P = 0;
    int splits = 1;
    WsLayout ws{};
    char *d_ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    int64_t acc_spectra = 0;  // spectra accumulated in acc since the last integrate
    int x_calls = 0;
    char err[512] = {0};
};

namespace {

thread_local char g_create_err[512];

corr_status fail(corr_plan *p, corr_status st, const char *fmt, ...) {
    char *buf = p ? p->err : g_create_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
    return st;
}

corr_status hip_fail(corr_plan *p, hipError_t e, const char *what) {
    return fail(p, CORR_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void *ptr, size_t a) { return (reinterpret_cast<uintptr_t>(ptr) % a) == 0; }

int chunk_of(int precision) { return precision == CORR_FP32 ? kChunk32 : kChunk8; }

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Default K-split of the X-engine: enough waves to fill the GPU (>= 4096
// (split, channel) waves), FP32 also keeps every wave's running FP32 sum at
// <= 1024 spectra; each split must be a whole number of 32-spectrum steps.
int choose_splits(const corr_desc_t &d, int C) {
    const int64_t steps = d.n_spectra / 32;
    int64_t target = (4096 + C - 1) / C;
    if (d.precision == CORR_FP32) target = std::max<int64_t>(target, (d.n_spectra + 1023) / 1024);
    if (d.x_split > 0) target = d.x_split;
    int best = 1;
    for (int64_t s = 1; s <= std::min<int64_t>(target, steps); ++s)
        if (steps % s == 0) best = (int)s;
    return best;
}

}  // namespace

extern "C" {

const char *corr_status_string(corr_status st) {
    switch (st) {
    case CORR_OK: return "ok";
    case CORR_ERR_INVALID: return "invalid argument";
    case CORR_ERR_NULL: return "null pointer";
    case CORR_ERR_ALIGN: return "misaligned pointer or stride";
    case CORR_ERR_UNSUPPORTED: return "unsupported on this device";
    case CORR_ERR_WORKSPACE: return "workspace missing or too small";
    case CORR_ERR_OVERFLOW: return "int32 accumulator bound exceeded";
    case CORR_ERR_DEVICE: return "HIP runtime error";
    case CORR_ERR_NOMEM: return "out of host memory";
    case CORR_ERR_STATE: return "call not allowed in this state";
    case CORR_ERR_DEVICE_ARG: return "invalid device-resident argument";
    case CORR_ERR_IO: return "file I/O error";
    default: return "unknown status";
    }
}

const char *corr_last_error(const corr_plan_t *plan) { return plan ? plan->err : g_create_err; }

corr_status corr_plan_create(const corr_desc_t *desc, corr_plan_t **out) {
    if (!desc || !out) return fail(nullptr, CORR_ERR_NULL, "desc and out must be non-null");
    *out = nullptr;
    const corr_desc_t &d = *desc;
    if (d.n_signals < 1 || d.n_signals > kMaxSignals)
        return fail(nullptr, CORR_ERR_INVALID, "n_signals %d outside 1..%d", d.n_signals, kMaxSignals);
    if (d.fft_len < 512 || d.fft_len > 16384 || (d.fft_len & (d.fft_len - 1)))
        return fail(nullptr, CORR_ERR_INVALID, "fft_len %d is not a power of two in 512..16384", d.fft_len);
    if (d.n_spectra < 32 || d.n_spectra % 32 || d.n_spectra > (int64_t)1 << 30)
        return fail(nullptr, CORR_ERR_INVALID, "n_spectra %lld must be a multiple of 32 in 32..2^30",
                    (long long)d.n_spectra);
    if ((int64_t)d.fft_len * d.n_spectra > ((int64_t)1 << 40))
        return fail(nullptr, CORR_ERR_INVALID, "fft_len * n_spectra too large");
    if (d.max_delay < 0 || d.max_delay > (1 << 26))
        return fail(nullptr, CORR_ERR_INVALID, "max_delay %d outside 0..2^26", d.max_delay);
    if (d.precision != CORR_FP32 && d.precision != CORR_INT8 && d.precision != CORR_FP8_E4M3)
        return fail(nullptr, CORR_ERR_INVALID, "unknown precision %d", d.precision);
    if (d.sideband != 1 && d.sideband != -1)
        return fail(nullptr, CORR_ERR_INVALID, "sideband must be +1 or -1 (got %d)", d.sideband);
    if (d.scale_mode != CORR_SCALE_HOLD && d.scale_mode != CORR_SCALE_COMPUTE)
        return fail(nullptr, CORR_ERR_INVALID, "unknown scale_mode %d", d.scale_mode);
    if (!(d.sample_rate > 0) || !std::isfinite(d.sample_rate) || !std::isfinite(d.nu_bb))
        return fail(nullptr, CORR_ERR_INVALID, "sample_rate must be finite and > 0, nu_bb finite");
    if (d.x_split < 0 || d.x_split > 4096)
        return fail(nullptr, CORR_ERR_INVALID, "x_split %d outside 0..4096", d.x_split);
    if (d.phase_lut != 0 && d.phase_lut != 1)
        return fail(nullptr, CORR_ERR_INVALID, "phase_lut must be 0 or 1 (got %d)", d.phase_lut);
    if (d.power_fp16 != 0 && d.power_fp16 != 1)
        return fail(nullptr, CORR_ERR_INVALID, "power_fp16 must be 0 or 1 (got %d)", d.power_fp16);
    for (int i = 0; i < 5; ++i)
        if (d.reserved[i]) return fail(nullptr, CORR_ERR_INVALID, "reserved[%d] must be zero", i);

    corr_plan *p = new (std::nothrow) corr_plan;
    if (!p) return fail(nullptr, CORR_ERR_NOMEM, "plan allocation failed");
    p->d = d;
    p->M = d.fft_len / 2;
    p->log2m = 0;
    while ((1 << p->log2m) < p->M) ++p->log2m;
    p->P = (int64_t)d.n_signals * (d.n_signals + 1) / 2;
    p->splits = choose_splits(d, p->M);

    WsLayout &w = p->ws;
    size_t o = 0;
    size_t ntw = 0;
    fengine_twiddle_table(p->log2m, nullptr, &ntw);
    w.twp = o; o = round_up(o + sizeof(float2) * std::max<size_t>(ntw, 1), 256);
    w.wn = o; o = round_up(o + sizeof(float2) * p->M, 256);
    w.pairs = o; o = round_up(o + sizeof(uint16_t) * 2 * p->P, 256);
    w.err = o; o = round_up(o + 16, 256);
    w.lut = o; o = round_up(o + sizeof(float2) * kLutSteps, 256);
    {
        const int n1 = d.fft_len / 64;
        size_t ntwb = 0;
        fengine4_tables(p->log2m, nullptr, nullptr, nullptr, &ntwb, nullptr);
        w.afrag = o; o = round_up(o + sizeof(uint16_t) * 2 * 64 * 64, 256);
        w.tw4 = o; o = round_up(o + sizeof(float2) * n1 * 32, 256);
        w.twb = o; o = round_up(o + sizeof(float2) * std::max<size_t>(ntwb, 1), 256);
        w.wsp = o; o = round_up(o + sizeof(float2) * n1, 256);
    }
    w.w16 = o; o = round_up(o + sizeof(int2) * kLutSteps, 256);
    w.part = o;
    if (d.precision != CORR_FP32 && d.scale_mode == CORR_SCALE_COMPUTE)
        o = round_up(o + sizeof(float) * d.n_signals * (d.n_spectra / 16) * p->M, 256);
    w.total = o;
    *out = p;
    return CORR_OK;
}

void corr_plan_destroy(corr_plan_t *plan) { delete plan; }

size_t corr_plan_workspace_bytes(const corr_plan_t *p) { return p ? p->ws.total : 0; }
size_t corr_plan_spectra_bytes(const corr_plan_t *p) {
    if (!p) return 0;
    const size_t per = p->d.precision == CORR_FP32 ? 8 : 2;
    return per * (size_t)p->M * p->d.n_spectra * p->d.n_signals;
}
size_t corr_plan_acc_bytes(const corr_plan_t *p) {
    return p ? (size_t)p->splits * p->M * p->P * 2 * 4 : 0;
}
size_t corr_plan_state_bytes(const corr_plan_t *p) { return p ? (size_t)p->M * p->P * 2 * 8 : 0; }
size_t corr_plan_vis_bytes(const corr_plan_t *p) { return p ? (size_t)p->M * p->P * 2 * 4 : 0; }
int32_t corr_plan_x_splits(const corr_plan_t *p) { return p ? p->splits : 0; }

const char *corr_plan_fengine_kernel(const corr_plan_t *p) {
    if (!p) return "";
    int mode = p->d.precision == CORR_FP32 ? 0 : p->d.precision == CORR_INT8 ? 1 : 2;
    if (p->d.phase_lut) mode += 4;
    static thread_local char name[64];
    snprintf(name, sizeof name, "%s<%d, %d>", use_fengine4(p->log2m, mode) ? "fengine4_kernel" : "fengine_kernel",
             p->log2m, mode);
    return name;
}

corr_status corr_plan_bind_workspace(corr_plan_t *p, void *d_ws, size_t bytes, void *stream) {
    if (!p || !d_ws) return fail(p, CORR_ERR_NULL, "plan and workspace must be non-null");
    if (!aligned(d_ws, 256)) return fail(p, CORR_ERR_ALIGN, "workspace must be 256-byte aligned");
    if (bytes < p->ws.total)
        return fail(p, CORR_ERR_WORKSPACE, "workspace of %zu bytes < %zu needed", bytes, p->ws.total);
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(p, e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return hip_fail(p, e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(p, CORR_ERR_UNSUPPORTED, "device %s is not gfx950", prop.gcnArchName);

    // Twiddle tables in FP64, rounded once to FP32.
    const int M = p->M, N = p->d.fft_len;
    size_t ntw = 0;
    fengine_twiddle_table(p->log2m, nullptr, &ntw);
    std::vector<float2> tw(std::max<size_t>(ntw, 1)), wn(M);
    fengine_twiddle_table(p->log2m, tw.data(), &ntw);
    for (int n = 0; n < M; ++n) {
        const double b = -2.0 * M_PI * (double)n / (double)N;
        wn[n] = make_float2((float)std::cos(b), (float)std::sin(b));
    }
    // phase table: cos and sin of 2 pi j / 1440 in FP64, rounded once to FP32
    std::vector<float2> lut(kLutSteps);
    for (int j = 0; j < kLutSteps; ++j) {
        const double b = 2.0 * M_PI * (double)j / (double)kLutSteps;
        lut[j] = make_float2((float)std::cos(b), (float)std::sin(b));
    }
    std::vector<uint16_t> pairs(2 * p->P);
    for (int j = 0; j < p->d.n_signals; ++j)
        for (int i = 0; i <= j; ++i) {
            const int64_t q = (int64_t)j * (j + 1) / 2 + i;
            pairs[2 * q] = (uint16_t)i;
            pairs[2 * q + 1] = (uint16_t)j;
        }
    // four-step F-engine tables
    const int n1 = N / 64;
    size_t ntwb = 0;
    fengine4_tables(p->log2m, nullptr, nullptr, nullptr, &ntwb, nullptr);
    std::vector<uint16_t> afrag(2 * 64 * 64);
    std::vector<float2> tw4((size_t)n1 * 32), twb(std::max<size_t>(ntwb, 1)), wsp(n1);
    fengine4_tables(p->log2m, afrag.data(), tw4.data(), twb.data(), &ntwb, wsp.data());
    std::vector<int2> w16(kLutSteps);
    fix16_table(w16.data());
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)d_ws;
    if ((e = hipMemcpyAsync(ws + p->ws.w16, w16.data(), sizeof(int2) * w16.size(), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(ws + p->ws.afrag, afrag.data(), sizeof(uint16_t) * afrag.size(), hipMemcpyHostToDevice,
                            st)) ||
        (e = hipMemcpyAsync(ws + p->ws.tw4, tw4.data(), sizeof(float2) * tw4.size(), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(ws + p->ws.twb, twb.data(), sizeof(float2) * twb.size(), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(ws + p->ws.wsp, wsp.data(), sizeof(float2) * wsp.size(), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(ws + p->ws.twp, tw.data(), sizeof(float2) * tw.size(), hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(ws + p->ws.wn, wn.data(), sizeof(float2) * M, hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(ws + p->ws.pairs, pairs.data(), sizeof(uint16_t) * pairs.size(),
                            hipMemcpyHostToDevice, st)) ||
        (e = hipMemcpyAsync(ws + p->ws.lut, lut.data(), sizeof(float2) * kLutSteps, hipMemcpyHostToDevice, st)) ||
        (e = hipMemsetAsync(ws + p->ws.err, 0, 16, st)) || (e = hipStreamSynchronize(st)))
        return hip_fail(p, e, "uploading plan tables");
    p->d_ws = ws;
    p->ws_bytes = bytes;
    p->bound = true;
    return CORR_OK;
}

corr_status corr_fengine(corr_plan_t *p, const int8_t *d_x, int64_t row_stride, const corr_geom_t *d_geom,
                         int64_t spectrum0, void *d_spec, float *d_scale, void *d_power, void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (!d_x || !d_geom || !d_spec) return fail(p, CORR_ERR_NULL, "d_x, d_geom and d_spec are required");
    const bool q8 = p->d.precision != CORR_FP32;
    if (q8 && !d_scale) return fail(p, CORR_ERR_NULL, "d_scale is required for INT8/FP8");
    if (!p->bound) return fail(p, CORR_ERR_WORKSPACE, "no workspace bound");
    if (!aligned(d_x, 16) || row_stride % 16) return fail(p, CORR_ERR_ALIGN, "d_x and row_stride must be 16-byte aligned");
    if (!aligned(d_geom, 8)) return fail(p, CORR_ERR_ALIGN, "d_geom must be 8-byte aligned");
    if (!aligned(d_spec, 256)) return fail(p, CORR_ERR_ALIGN, "d_spec must be 256-byte aligned");
    if (d_scale && !aligned(d_scale, 4)) return fail(p, CORR_ERR_ALIGN, "d_scale must be 4-byte aligned");
    if (d_power && !aligned(d_power, p->d.power_fp16 ? 2 : 4))
        return fail(p, CORR_ERR_ALIGN, "d_power must be %d-byte aligned", p->d.power_fp16 ? 2 : 4);
    const int64_t need = (int64_t)p->d.fft_len * p->d.n_spectra + p->d.max_delay;
    if (row_stride < need)
        return fail(p, CORR_ERR_INVALID, "row_stride %lld < T*N + max_delay = %lld", (long long)row_stride,
                    (long long)need);
    if (spectrum0 < 0) return fail(p, CORR_ERR_INVALID, "spectrum0 must be >= 0");

    FLaunch a{};
    a.x = d_x;
    a.row_stride = row_stride;
    a.geom = d_geom;
    a.spectrum0 = spectrum0;
    a.spec = d_spec;
    a.scale = d_scale;
    a.part = reinterpret_cast<float *>(p->d_ws + p->ws.part);
    a.power = d_power;
    a.power_f16 = p->d.power_fp16;
    a.power_scale = std::ldexp(1.0f, -2 * (p->log2m + 1));  // 1 / N^2
    a.twp = reinterpret_cast<const float2 *>(p->d_ws + p->ws.twp);
    a.wn = reinterpret_cast<const float2 *>(p->d_ws + p->ws.wn);
    a.err = reinterpret_cast<uint32_t *>(p->d_ws + p->ws.err);
    a.S = p->d.n_signals;
    a.T = (int)p->d.n_spectra;
    a.max_delay = p->d.max_delay;
    a.sideband = p->d.sideband;
    a.fs = p->d.sample_rate;
    a.nu_bb = p->d.nu_bb;
    a.lut = reinterpret_cast<const float2 *>(p->d_ws + p->ws.lut);
    a.afrag = reinterpret_cast<const uint16_t *>(p->d_ws + p->ws.afrag);
    a.tw4 = reinterpret_cast<const float2 *>(p->d_ws + p->ws.tw4);
    a.twb = reinterpret_cast<const float2 *>(p->d_ws + p->ws.twb);
    a.wsp = reinterpret_cast<const float2 *>(p->d_ws + p->ws.wsp);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    auto launch = [&](int mode) {
        return use_fengine4(p->log2m, mode) ? launch_fengine4(p->log2m, mode, a, st)
                                             : launch_fengine(p->log2m, mode, a, st);
    };
    if (q8 && p->d.scale_mode == CORR_SCALE_COMPUTE) {
        a.power = nullptr;
        if ((e = launch(3)) != hipSuccess) return hip_fail(p, e, "calibration pass");
        if ((e = launch_calib_reduce(a.part, a.S, p->M, a.T / 16, a.T, p->d.precision, d_scale, st)) != hipSuccess)
            return hip_fail(p, e, "calibration reduce");
    }
    a.power = d_power;
    const int mode = (p->d.precision == CORR_FP32 ? 0 : (p->d.precision == CORR_INT8 ? 1 : 2)) + (p->d.phase_lut ? 4 : 0);
    if ((e = launch(mode)) != hipSuccess) return hip_fail(p, e, "F-engine launch");
    return CORR_OK;
}

corr_status corr_xpack(corr_plan_t *p, const void *d_in, void *d_spec, void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (!d_in || !d_spec) return fail(p, CORR_ERR_NULL, "d_in and d_spec are required");
    if (!aligned(d_in, 16) || !aligned(d_spec, 256)) return fail(p, CORR_ERR_ALIGN, "d_in 16 B / d_spec 256 B alignment");
    hipError_t e = launch_xpack(p->d.precision, d_in, d_spec, p->d.n_signals, p->M, (int)p->d.n_spectra,
                                (hipStream_t)stream);
    return e == hipSuccess ? CORR_OK : hip_fail(p, e, "xpack launch");
}

corr_status corr_requantize(corr_plan_t *p, const float *d_in, const float *d_scale, void *d_out, void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (!d_in || !d_scale || !d_out) return fail(p, CORR_ERR_NULL, "d_in, d_scale and d_out are required");
    if (p->d.precision == CORR_FP32) return fail(p, CORR_ERR_UNSUPPORTED, "an FP32 plan has no codes");
    if (!aligned(d_in, 8) || !aligned(d_scale, 4) || !aligned(d_out, 2))
        return fail(p, CORR_ERR_ALIGN, "d_in 8 B, d_scale 4 B, d_out 2 B alignment");
    hipError_t e = launch_requantize(p->d.precision, d_in, d_scale, p->d.n_signals, p->d.n_spectra, p->M,
                                     static_cast<uint8_t *>(d_out), (hipStream_t)stream);
    return e == hipSuccess ? CORR_OK : hip_fail(p, e, "requantize launch");
}

corr_status corr_beamform(corr_plan_t *p, const void *d_spec, const float *d_scale, const float *d_w, float *d_inc,
                          const float *d_c, int32_t n_beams, int32_t mode, float *d_coh, int32_t tint,
                          void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (n_beams < 0 || n_beams > CORR_MAX_BEAMS)
        return fail(p, CORR_ERR_INVALID, "n_beams %d outside 0..%d", n_beams, CORR_MAX_BEAMS);
    if (mode != CORR_BEAM_INTENSITY && mode != CORR_BEAM_FULLPOL && mode != CORR_BEAM_VOLTAGE)
        return fail(p, CORR_ERR_INVALID, "unknown coherent beam mode %d", mode);
    if (tint != 1 && tint != 2 && tint != 4 && tint != 8)
        return fail(p, CORR_ERR_INVALID, "tint %d is not 1, 2, 4 or 8", tint);
    if (mode == CORR_BEAM_VOLTAGE && n_beams > 0 && tint != 1)
        return fail(p, CORR_ERR_INVALID, "voltage beams are not summed over time (tint must be 1)");
    if (!d_inc && n_beams == 0) return fail(p, CORR_ERR_INVALID, "no beam requested");
    if (!d_spec) return fail(p, CORR_ERR_NULL, "d_spec is required");
    if (d_inc && !d_w) return fail(p, CORR_ERR_NULL, "the incoherent beam needs d_w");
    if (n_beams > 0 && (!d_c || !d_coh)) return fail(p, CORR_ERR_NULL, "coherent beams need d_c and d_coh");
    if (p->d.precision != CORR_FP32 && !d_scale) return fail(p, CORR_ERR_NULL, "INT8 / FP8 spectra need d_scale");
    if (!aligned(d_spec, 256)) return fail(p, CORR_ERR_ALIGN, "d_spec must be 256-byte aligned");
    if (!aligned(d_scale, 4) || !aligned(d_w, 4) || !aligned(d_inc, 4) || !aligned(d_c, 4) ||
        !aligned(d_coh, mode == CORR_BEAM_VOLTAGE ? 8 : 4))
        return fail(p, CORR_ERR_ALIGN, "beam weights and outputs must be 4-byte aligned (8 for voltage beams)");
    hipError_t e = launch_beamform(p->d.precision, d_spec, d_scale, d_w, d_c, n_beams, p->d.n_signals, p->M,
                                   p->d.n_spectra, tint, mode, d_inc, n_beams > 0 ? d_coh : nullptr,
                                   (hipStream_t)stream);
    return e == hipSuccess ? CORR_OK : hip_fail(p, e, "beamformer launch");
}

corr_status corr_xengine(corr_plan_t *p, const void *d_spec, const uint32_t *d_keep, void *d_acc, int32_t *d_counts,
                         void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (!d_spec || !d_acc) return fail(p, CORR_ERR_NULL, "d_spec and d_acc are required");
    if (d_counts && !d_keep) return fail(p, CORR_ERR_NULL, "d_counts needs d_keep");
    if (!aligned(d_spec, 256) || !aligned(d_acc, 256)) return fail(p, CORR_ERR_ALIGN, "d_spec/d_acc must be 256-byte aligned");
    if (!aligned(d_keep, 4) || !aligned(d_counts, 4)) return fail(p, CORR_ERR_ALIGN, "d_keep/d_counts must be 4-byte aligned");
    if (d_counts && !p->bound) return fail(p, CORR_ERR_WORKSPACE, "pair counts need the bound workspace");
    if (p->d.precision == CORR_INT8 && p->acc_spectra + p->d.n_spectra > kMaxInt8Spectra)
        return fail(p, CORR_ERR_OVERFLOW, "%lld spectra since the last integrate would exceed the int32 bound (%lld)",
                    (long long)(p->acc_spectra + p->d.n_spectra), (long long)kMaxInt8Spectra);
    if (p->d.precision != CORR_FP32 && p->d.scale_mode == CORR_SCALE_COMPUTE && p->x_calls > 0)
        return fail(p, CORR_ERR_STATE, "COMPUTE scales change per call: integrate before the next X-engine call");
    hipError_t e = launch_xengine(p->d.precision, d_spec, d_keep, d_acc, p->d.n_signals, p->M, (int)p->d.n_spectra,
                                  p->splits, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(p, e, "X-engine launch");
    if (d_counts) {
        e = launch_pair_counts(d_keep, p->d.n_signals, (int)p->d.n_spectra, p->M, d_counts, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(p, e, "pair-count launch");
    }
    p->acc_spectra += p->d.n_spectra;
    p->x_calls += 1;
    return CORR_OK;
}

corr_status corr_xengine_gated(corr_plan_t *p, const void *d_spec, const uint8_t *d_gate, int32_t n_bins, void *d_acc,
                               void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (!d_spec || !d_gate || !d_acc) return fail(p, CORR_ERR_NULL, "d_spec, d_gate and d_acc are required");
    if (!aligned(d_spec, 256) || !aligned(d_acc, 256) || !aligned(d_gate, 16))
        return fail(p, CORR_ERR_ALIGN, "d_spec/d_acc 256-byte, d_gate 16-byte alignment");
    if (n_bins < 1 || n_bins > CORR_MAX_GATE_BINS)
        return fail(p, CORR_ERR_INVALID, "n_bins=%d outside [1, %d]", n_bins, CORR_MAX_GATE_BINS);
    if (p->d.precision == CORR_INT8 && p->acc_spectra + p->d.n_spectra > kMaxInt8Spectra)
        return fail(p, CORR_ERR_OVERFLOW, "%lld spectra since the last integrate would exceed the int32 bound (%lld)",
                    (long long)(p->acc_spectra + p->d.n_spectra), (long long)kMaxInt8Spectra);
    if (p->d.precision != CORR_FP32 && p->d.scale_mode == CORR_SCALE_COMPUTE && p->x_calls > 0)
        return fail(p, CORR_ERR_STATE, "COMPUTE scales change per call: integrate before the next X-engine call");
    const int64_t acc_elems = (int64_t)p->splits * p->M * ((int64_t)p->d.n_signals * (p->d.n_signals + 1) / 2) * 2;
    hipError_t e = launch_xengine_gated(p->d.precision, d_spec, d_gate, n_bins, d_acc, acc_elems, p->d.n_signals,
                                        p->M, (int)p->d.n_spectra, p->splits, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(p, e, "gated X-engine launch");
    p->acc_spectra += p->d.n_spectra;
    p->x_calls += 1;
    return CORR_OK;
}

corr_status corr_pulsar_gates(int64_t spectrum0, int64_t n_spectra, int32_t fft_len, double sample_rate, double t0,
                              double period, int32_t n_bins, uint8_t *h_gate, int64_t *h_counts) {
    if (!h_gate) return fail(nullptr, CORR_ERR_NULL, "h_gate is required");
    if (n_spectra < 0 || spectrum0 < 0 || fft_len < 1 || !(sample_rate > 0) || !std::isfinite(sample_rate) ||
        !(period > 0) || !std::isfinite(period) || !std::isfinite(t0))
        return fail(nullptr, CORR_ERR_INVALID, "n_spectra, spectrum0 >= 0, fft_len >= 1, finite sample_rate, "
                                               "period > 0 and t0 required");
    if (n_bins < 1 || n_bins > CORR_MAX_GATE_BINS)
        return fail(nullptr, CORR_ERR_INVALID, "n_bins=%d outside [1, %d]", n_bins, CORR_MAX_GATE_BINS);
    const double t_spec = (double)fft_len / sample_rate;
    for (int64_t m = 0; m < n_spectra; ++m) {
        // window centre of spectrum spectrum0 + m, then its pulse phase in [0, 1)
        const double t = ((double)(spectrum0 + m) + 0.5) * t_spec;
        const double x = (t - t0) / period;
        const double phase = x - std::floor(x);
        int b = (int)std::floor(phase * (double)n_bins);
        if (b >= n_bins) b = n_bins - 1;  // phase * n_bins rounded up to n_bins
        if (b < 0) b = 0;
        h_gate[m] = (uint8_t)b;
        if (h_counts) h_counts[b] += 1;
    }
    return CORR_OK;
}

corr_status corr_geom_from_model(int32_t n, const double *tau0, const double *taudot, double t0, double t_delay,
                                 double fs, double nu_lo, int32_t max_delay, corr_geom_t *out) {
    if (!tau0 || !taudot || !out) return fail(nullptr, CORR_ERR_NULL, "h_tau0, h_taudot and h_geom are required");
    if (n < 1) return fail(nullptr, CORR_ERR_INVALID, "n_signals %d < 1", n);
    if (!std::isfinite(t0) || !std::isfinite(t_delay) || !std::isfinite(fs) || !(fs > 0) ||
        !std::isfinite(nu_lo) || nu_lo < 0 || max_delay < 0)
        return fail(nullptr, CORR_ERR_INVALID, "t0, t_delay finite, sample_rate > 0, nu_lo >= 0 and "
                                               "max_delay >= 0 required");
    std::vector<corr_geom_t> g(n);
    for (int s = 0; s < n; ++s) {
        if (!std::isfinite(tau0[s]) || !std::isfinite(taudot[s]))
            return fail(nullptr, CORR_ERR_INVALID, "signal %d: non-finite delay model", s);
        // integer + fractional delay at t_delay, in samples
        const double x = (tau0[s] + taudot[s] * (t_delay - t0)) * fs;
        double D = std::floor(x);
        float f = (float)(x - D);  // x - D is exact in FP64 (|x| < 2^52); one rounding to float
        if (f >= 1.0f) {           // rounded up to a whole sample: carry
            D += 1.0;
            f = 0.0f;
        }
        if (!(D >= 0.0) || D > (double)max_delay)
            return fail(nullptr, CORR_ERR_INVALID, "signal %d: delay of %.6f samples outside [0, max_delay = %d]",
                        s, x, max_delay);
        // fringe phase at t = 0, nu_lo * (tau0 - taudot t0) mod 1, with error-free transforms:
        // taudot t0 = q + eq and tau0 - q = z + ez exactly, nu_lo z = p + ep exactly; the
        // fraction of p is exact and the small terms are added after it
        const double q = taudot[s] * t0;
        const double eq = std::fma(taudot[s], t0, -q);
        const double z = tau0[s] - q;
        const double bz = z - tau0[s];
        const double ez = (tau0[s] - (z - bz)) + (-q - bz);
        const double p = nu_lo * z;
        const double ep = std::fma(nu_lo, z, -p);
        // the F-engine time-stamps spectrum m at the aligned window centre t_m, while its samples
        // arrived tau later (read-pointer advance), when the fringe phase was rate * tau further on
        const double arrive = (nu_lo * taudot[s]) * (x / fs);
        double c = (p - std::floor(p)) + (ep + nu_lo * (ez - eq) + arrive);
        c -= std::floor(c);
        if (c >= 1.0) c = 0.0;  // a tiny negative c rounds to 1 above
        g[s].D = (int32_t)D;
        g[s].frac = f;
        g[s].psi0 = c;
        g[s].rate = nu_lo * taudot[s];
    }
    std::memcpy(out, g.data(), sizeof(corr_geom_t) * n);
    return CORR_OK;
}

corr_status corr_fix16_spectra(corr_plan_t *p, const void *d_spec, const corr_geom_t *d_geom, int64_t spectrum0,
                               const float *d_scale, int16_t *d_q16, int16_t *d_y16, void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (!d_spec || !d_geom || !d_scale || !d_y16) return fail(p, CORR_ERR_NULL, "d_spec, d_geom, d_scale and d_y16 are required");
    if (p->d.precision != CORR_FP32)
        return fail(p, CORR_ERR_INVALID, "the 16-bit path reads the spectra of an FP32 plan");
    if (!p->bound) return fail(p, CORR_ERR_WORKSPACE, "no workspace bound");
    if (!aligned(d_spec, 256) || !aligned(d_geom, 8) || !aligned(d_scale, 4) || !aligned(d_y16, 4) ||
        (d_q16 && !aligned(d_q16, 4)))
        return fail(p, CORR_ERR_ALIGN, "d_spec 256 B, d_geom 8 B, d_scale, d_q16 and d_y16 4 B alignment");
    if (spectrum0 < 0) return fail(p, CORR_ERR_INVALID, "spectrum0 must be >= 0");
    hipError_t e = launch_fix16(d_spec, d_geom, spectrum0, d_scale, reinterpret_cast<const int2 *>(p->d_ws + p->ws.w16),
                                p->d.n_signals, (int)p->d.n_spectra, p->M, p->d.sample_rate, p->d.nu_bb, p->d.sideband,
                                d_q16, d_y16, (hipStream_t)stream);
    return e == hipSuccess ? CORR_OK : hip_fail(p, e, "16-bit spectra launch");
}

corr_status corr_fix16_xengine(corr_plan_t *p, const int16_t *d_y16, const float *d_scale, int64_t *d_acc,
                               double *d_vis, void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (!d_y16 || !d_acc) return fail(p, CORR_ERR_NULL, "d_y16 and d_acc are required");
    if (d_vis && !d_scale) return fail(p, CORR_ERR_NULL, "d_vis needs d_scale");
    if (!aligned(d_y16, 4) || !aligned(d_acc, 8) || (d_vis && !aligned(d_vis, 8)) || (d_scale && !aligned(d_scale, 4)))
        return fail(p, CORR_ERR_ALIGN, "d_y16 4 B, d_acc and d_vis 8 B, d_scale 4 B alignment");
    hipError_t e = launch_xengine16(d_y16, p->d.n_signals, p->d.n_spectra, p->M, d_scale, d_acc, d_vis,
                                    (hipStream_t)stream);
    return e == hipSuccess ? CORR_OK : hip_fail(p, e, "16-bit X-engine launch");
}

corr_status corr_integrate(corr_plan_t *p, void *d_acc, const float *d_scale, double *d_state, float *d_vis_out,
                           uint32_t flags, void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (!d_acc || !d_state) return fail(p, CORR_ERR_NULL, "d_acc and d_state are required");
    if (p->d.precision != CORR_FP32 && !d_scale) return fail(p, CORR_ERR_NULL, "d_scale is required for INT8/FP8");
    if ((flags & CORR_DUMP) && !d_vis_out) return fail(p, CORR_ERR_NULL, "CORR_DUMP needs d_vis_out");
    if (flags & ~(CORR_DUMP | CORR_RESET)) return fail(p, CORR_ERR_INVALID, "unknown flags 0x%x", flags);
    if (!p->bound) return fail(p, CORR_ERR_WORKSPACE, "no workspace bound");
    if (!aligned(d_acc, 256) || !aligned(d_state, 16) || (d_vis_out && !aligned(d_vis_out, 8)))
        return fail(p, CORR_ERR_ALIGN, "d_acc 256 B, d_state 16 B, d_vis_out 8 B alignment");
    hipError_t e = launch_integrate(p->d.precision, d_acc, d_scale, d_state, d_vis_out,
                                    reinterpret_cast<const uint16_t *>(p->d_ws + p->ws.pairs), p->d.n_signals, p->M,
                                    p->splits, flags, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(p, e, "integrate launch");
    p->acc_spectra = 0;
    p->x_calls = 0;
    return CORR_OK;
}

corr_status corr_mad_flag(corr_plan_t *p, const void *d_power, float M, uint8_t *d_flags, void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (!d_power || !d_flags) return fail(p, CORR_ERR_NULL, "d_power and d_flags are required");
    if (!aligned(d_power, 16) || !aligned(d_flags, 16))
        return fail(p, CORR_ERR_ALIGN, "d_power and d_flags must be 16-byte aligned");
    if (p->d.n_spectra % kFlagTileSpectra || p->M % kFlagTileChannels)
        return fail(p, CORR_ERR_INVALID, "flagging needs T %% %d == 0 and C %% %d == 0", kFlagTileSpectra,
                    kFlagTileChannels);
    if (!(M > 0) || !std::isfinite(M)) return fail(p, CORR_ERR_INVALID, "threshold M must be finite and > 0");
    hipError_t e = launch_mad_flag(d_power, p->d.power_fp16 != 0, p->d.n_signals, (int)p->d.n_spectra, p->M, M,
                                   d_flags, (hipStream_t)stream);
    return e == hipSuccess ? CORR_OK : hip_fail(p, e, "MAD flag launch");
}

corr_status corr_apply_flags(corr_plan_t *p, const uint8_t *d_flags, void *d_spec, uint32_t *d_keep, void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (!d_flags || (!d_spec && !d_keep)) return fail(p, CORR_ERR_NULL, "d_flags and one of d_spec, d_keep are required");
    if (!aligned(d_spec, 256) || (d_keep && !aligned(d_keep, 4)))
        return fail(p, CORR_ERR_ALIGN, "d_spec 256 B / d_keep 4 B alignment");
    hipError_t e = launch_apply_flags(p->d.precision, d_flags, d_spec, d_keep, p->d.n_signals,
                                      (int)p->d.n_spectra, p->M, (hipStream_t)stream);
    return e == hipSuccess ? CORR_OK : hip_fail(p, e, "apply-flags launch");
}

corr_status corr_pair_counts(corr_plan_t *p, const uint32_t *d_keep, int32_t *d_counts, void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (!d_keep || !d_counts) return fail(p, CORR_ERR_NULL, "d_keep and d_counts are required");
    if (!p->bound) return fail(p, CORR_ERR_WORKSPACE, "no workspace bound");
    if (!aligned(d_keep, 4) || !aligned(d_counts, 4)) return fail(p, CORR_ERR_ALIGN, "4-byte alignment");
    hipError_t e = launch_pair_counts(d_keep, p->d.n_signals, (int)p->d.n_spectra, p->M, d_counts,
                                      (hipStream_t)stream);
    return e == hipSuccess ? CORR_OK : hip_fail(p, e, "pair-count launch");
}

size_t corr_plan_flags_bytes(const corr_plan_t *p) {
    return p ? (size_t)p->d.n_signals * p->d.n_spectra * p->M : 0;
}
size_t corr_plan_keep_bytes(const corr_plan_t *p) {
    return p ? (size_t)p->M * p->d.n_signals * (p->d.n_spectra / 32) * 4 : 0;
}
size_t corr_plan_power_bytes(const corr_plan_t *p) {
    return p ? (size_t)p->d.n_signals * p->d.n_spectra * p->M * (p->d.power_fp16 ? 2 : 4) : 0;
}

/* ------------------------------------------------------------------ batch */

struct corr_batch {
    int n = 0;
    corr_plan *plans[kMaxBatch] = {};
    corr_batch_io_t io[kMaxBatch] = {};
    bool io_set[kMaxBatch] = {};
    hipStream_t side[kMaxBatch] = {};
    hipEvent_t fork = nullptr, done[kMaxBatch] = {};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    char err[512] = {0};
};

namespace {
corr_status bfail(corr_batch *b, corr_status st, const char *msg) {
    std::snprintf(b ? b->err : g_create_err, 512, "%s", msg);
    return st;
}
}  // namespace

corr_status corr_batch_create(const corr_desc_t *descs, int n, corr_batch_t **out) {
    if (!descs || !out) return fail(nullptr, CORR_ERR_NULL, "descs and out must be non-null");
    *out = nullptr;
    if (n < 1 || n > kMaxBatch) return fail(nullptr, CORR_ERR_INVALID, "batch size %d outside 1..%d", n, kMaxBatch);
    for (int i = 0; i < n; ++i) {
        if (descs[i].precision != CORR_INT8)
            return fail(nullptr, CORR_ERR_UNSUPPORTED, "batched correlation is INT8 only (entry %d)", i);
        if (descs[i].scale_mode != CORR_SCALE_HOLD)
            return fail(nullptr, CORR_ERR_INVALID, "batched correlation needs held scales (entry %d)", i);
        // one run accumulates a whole call into the int32 accumulator before integrating it
        if (descs[i].n_spectra > kMaxInt8Spectra)
            return fail(nullptr, CORR_ERR_OVERFLOW, "entry %d: %lld spectra per run exceed the int32 bound (%lld)", i,
                        (long long)descs[i].n_spectra, (long long)kMaxInt8Spectra);
    }
    corr_batch *b = new (std::nothrow) corr_batch;
    if (!b) return fail(nullptr, CORR_ERR_NOMEM, "batch allocation failed");
    b->n = n;
    for (int i = 0; i < n; ++i) {
        corr_status st = corr_plan_create(&descs[i], &b->plans[i]);
        if (st != CORR_OK) {
            corr_batch_destroy(b);
            return st;
        }
    }
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int i = 0; i < n && e == hipSuccess; ++i) {
        e = hipStreamCreateWithFlags(&b->side[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        corr_batch_destroy(b);
        return fail(nullptr, CORR_ERR_DEVICE, "batch streams/events: %s", hipGetErrorString(e));
    }
    *out = b;
    return CORR_OK;
}

void corr_batch_destroy(corr_batch_t *b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (int i = 0; i < kMaxBatch; ++i) {
        if (b->side[i]) (void)hipStreamDestroy(b->side[i]);
        if (b->done[i]) (void)hipEventDestroy(b->done[i]);
        corr_plan_destroy(b->plans[i]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    delete b;
}

corr_plan_t *corr_batch_plan(corr_batch_t *b, int i) { return (b && i >= 0 && i < b->n) ? b->plans[i] : nullptr; }

const char *corr_batch_last_error(const corr_batch_t *b) { return b ? b->err : g_create_err; }

corr_status corr_batch_set_io(corr_batch_t *b, int i, const corr_batch_io_t *io) {
    if (!b || !io) return bfail(b, CORR_ERR_NULL, "batch and io must be non-null");
    if (i < 0 || i >= b->n) return bfail(b, CORR_ERR_INVALID, "sub-array index out of range");
    corr_plan *p = b->plans[i];
    if (!io->x || !io->geom || !io->spec || !io->scale || !io->acc || !io->state)
        return bfail(b, CORR_ERR_NULL, "x, geom, spec, scale, acc and state are required");
    if ((io->flags & CORR_DUMP) && !io->vis) return bfail(b, CORR_ERR_NULL, "CORR_DUMP needs vis");
    if (!p->bound) return bfail(b, CORR_ERR_WORKSPACE, "bind the sub-plan's workspace first");
    if (!aligned(io->x, 16) || io->row_stride % 16 || !aligned(io->spec, 256) || !aligned(io->acc, 256) ||
        !aligned(io->state, 16) || !aligned(io->geom, 8) || !aligned(io->scale, 4))
        return bfail(b, CORR_ERR_ALIGN, "misaligned batch buffer");
    if (io->row_stride < (int64_t)p->d.fft_len * p->d.n_spectra + p->d.max_delay)
        return bfail(b, CORR_ERR_INVALID, "row_stride < T*N + max_delay");
    b->io[i] = *io;
    b->io_set[i] = true;
    return CORR_OK;
}

corr_status corr_batch_run(corr_batch_t *b, void *stream) {
    if (!b) return fail(nullptr, CORR_ERR_NULL, "batch is null");
    for (int i = 0; i < b->n; ++i)
        if (!b->io_set[i]) return bfail(b, CORR_ERR_STATE, "every sub-array needs corr_batch_set_io");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    // fork: the F-engines of the sub-arrays run concurrently on side streams
    if ((e = hipEventRecord(b->fork, st)) != hipSuccess) return bfail(b, CORR_ERR_DEVICE, "fork record");
    XBatchArgs xa{};
    xa.n = b->n;
    xa.first[0] = 0;
    for (int i = 0; i < b->n; ++i) {
        corr_plan *p = b->plans[i];
        const corr_batch_io_t &io = b->io[i];
        if ((e = hipStreamWaitEvent(b->side[i], b->fork, 0)) != hipSuccess)
            return bfail(b, CORR_ERR_DEVICE, "fork wait");
        corr_status cs = corr_fengine(p, io.x, io.row_stride, io.geom, io.spectrum0, io.spec, io.scale, nullptr,
                                      b->side[i]);
        if (cs != CORR_OK) return bfail(b, cs, p->err);
        if ((e = hipEventRecord(b->done[i], b->side[i])) != hipSuccess) return bfail(b, CORR_ERR_DEVICE, "join record");
        if ((e = hipStreamWaitEvent(st, b->done[i], 0)) != hipSuccess) return bfail(b, CORR_ERR_DEVICE, "join wait");
        xa.cor[i] = XBatchEntry{io.spec, io.acc, p->d.n_signals, p->M, (int)p->d.n_spectra, p->splits};
        xa.first[i + 1] = xa.first[i] + (p->M / 8) * p->splits;
    }
    // one X-engine launch over the tasks of every sub-array
    if ((e = launch_xengine_batch(xa, st)) != hipSuccess) return bfail(b, CORR_ERR_DEVICE, hipGetErrorString(e));
    for (int i = 0; i < b->n; ++i) {
        corr_plan *p = b->plans[i];
        const corr_batch_io_t &io = b->io[i];
        if ((e = launch_integrate(CORR_INT8, io.acc, io.scale, io.state, io.vis,
                                  reinterpret_cast<const uint16_t *>(p->d_ws + p->ws.pairs), p->d.n_signals, p->M,
                                  p->splits, io.flags, st)) != hipSuccess)
            return bfail(b, CORR_ERR_DEVICE, hipGetErrorString(e));
    }
    return CORR_OK;
}

corr_status corr_batch_capture(corr_batch_t *b, void *stream) {
    if (!b) return fail(nullptr, CORR_ERR_NULL, "batch is null");
    if (!stream) return bfail(b, CORR_ERR_INVALID, "graph capture needs a non-null stream");
    hipStream_t st = (hipStream_t)stream;
    if (b->exec) { (void)hipGraphExecDestroy(b->exec); b->exec = nullptr; }
    if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(b, CORR_ERR_DEVICE, hipGetErrorString(e));
    corr_status cs = corr_batch_run(b, stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (cs != CORR_OK) { if (g) (void)hipGraphDestroy(g); return cs; }
    if (e != hipSuccess) return bfail(b, CORR_ERR_DEVICE, hipGetErrorString(e));
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) return bfail(b, CORR_ERR_DEVICE, hipGetErrorString(e));
    return CORR_OK;
}

corr_status corr_batch_launch(corr_batch_t *b, void *stream) {
    if (!b) return fail(nullptr, CORR_ERR_NULL, "batch is null");
    if (!b->exec) return bfail(b, CORR_ERR_STATE, "capture the batch first");
    hipError_t e = hipGraphLaunch(b->exec, (hipStream_t)stream);
    return e == hipSuccess ? CORR_OK : bfail(b, CORR_ERR_DEVICE, hipGetErrorString(e));
}

/* -------------------------------------------------------------- autotune */

size_t corr_autotune_scratch_bytes(const corr_desc_t *desc) {
    corr_plan_t *p = nullptr;
    if (!desc) return 0;
    corr_desc_t d = *desc;
    d.x_split = 64;  // the largest candidate sizes the accumulator
    if (corr_plan_create(&d, &p) != CORR_OK) return 0;
    const size_t n = round_up(corr_plan_spectra_bytes(p), 256) + (size_t)64 * p->M * p->P * 8;
    corr_plan_destroy(p);
    return n;
}

corr_status corr_autotune_x_split(const corr_desc_t *desc, void *d_scratch, size_t bytes, void *stream,
                                  int32_t *best_split, float *best_ms) {
    if (!desc || !d_scratch || !best_split) return fail(nullptr, CORR_ERR_NULL, "desc, scratch and best_split");
    if (!aligned(d_scratch, 256)) return fail(nullptr, CORR_ERR_ALIGN, "scratch must be 256-byte aligned");
    if (bytes < corr_autotune_scratch_bytes(desc)) return fail(nullptr, CORR_ERR_WORKSPACE, "scratch too small");
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(nullptr, CORR_ERR_DEVICE, "autotune events");
    const int64_t steps = desc->n_spectra / 32;
    float best = 1e30f;
    int bsplit = 1;
    corr_status result = CORR_OK;
    for (int cand = 1; cand <= 64 && cand <= steps; ++cand) {
        if (steps % cand) continue;
        corr_desc_t d = *desc;
        d.x_split = cand;
        corr_plan_t *p = nullptr;
        if ((result = corr_plan_create(&d, &p)) != CORR_OK) break;
        char *spec = (char *)d_scratch;
        char *acc = spec + round_up(corr_plan_spectra_bytes(p), 256);
        float ts[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        hipError_t e = hipSuccess;
        for (int rep = 0; rep < 6 && e == hipSuccess; ++rep) {  // the first launch warms up
            e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = launch_xengine(d.precision, spec, nullptr, acc, d.n_signals, p->M, (int)d.n_spectra, p->splits, st);
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ts[rep], e0, e1);
        }
        std::sort(ts + 1, ts + 6);
        const float ms = ts[3];  // median of the 5 timed launches
        corr_plan_destroy(p);
        if (e != hipSuccess) { result = fail(nullptr, CORR_ERR_DEVICE, "autotune run: %s", hipGetErrorString(e)); break; }
        if (ms < best) { best = ms; bsplit = cand; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (result != CORR_OK) return result;
    *best_split = bsplit;
    if (best_ms) *best_ms = best;
    return CORR_OK;
}

corr_status corr_check_device_errors(corr_plan_t *p, void *stream) {
    if (!p) return fail(nullptr, CORR_ERR_NULL, "plan is null");
    if (!p->bound) return fail(p, CORR_ERR_WORKSPACE, "no workspace bound");
    uint32_t w[4] = {0, 0, 0, 0};
    hipStream_t st = (hipStream_t)stream;
    hipError_t e;
    if ((e = hipMemcpyAsync(w, p->d_ws + p->ws.err, sizeof(w), hipMemcpyDeviceToHost, st)) ||
        (e = hipStreamSynchronize(st)) || (e = hipMemsetAsync(p->d_ws + p->ws.err, 0, sizeof(w), st)) ||
        (e = hipStreamSynchronize(st)))
        return hip_fail(p, e, "reading device error words");
    if (w[0] & 1u) return fail(p, CORR_ERR_DEVICE_ARG, "a signal delay was outside [0, max_delay] (clamped)");
    return CORR_OK;
}

}  // extern "C"
