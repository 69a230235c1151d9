// cnn_api.hip -- host side of the learned flagger: argument checks, workspace
// layout and launches behind the corr_cnn_* entry points of corr.h.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "corr_internal.h"

using namespace corr;

struct corr_cnn {
    corr_cnn_desc_t d;
    char *d_ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    // byte offsets of the training buffers in the workspace
    size_t o_x, o_y, o_z1, o_z2, o_z3, o_d3, o_d2, o_d1, o_part, o_lpart, o_grad, o_loss, o_err, total;
    char err[512] = {0};
};

namespace {

thread_local char g_cnn_err[512];

corr_status fail(corr_cnn *c, corr_status st, const char *fmt, ...) {
    char *buf = c ? c->err : g_cnn_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
    return st;
}

corr_status hip_fail(corr_cnn *c, hipError_t e, const char *what) {
    return fail(c, CORR_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

void layout(corr_cnn &c) {
    const size_t n = (size_t)c.d.max_tiles, plane = (size_t)kCnnPixels * sizeof(float);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = round_up(o + bytes, 256);
        return at;
    };
    c.o_x = take(n * plane);
    c.o_y = take(n * plane);
    c.o_z1 = take(n * 16 * plane);
    c.o_z2 = take(n * 16 * plane);
    c.o_z3 = take(n * plane);
    c.o_d3 = take(n * plane);
    c.o_d2 = take(n * 16 * plane);
    c.o_d1 = take(n * 16 * plane);
    c.o_part = take(n * kCnnBlocksPerTile * kCnnGradEntries * sizeof(float));
    c.o_lpart = take(kCnnLossBlocks * sizeof(double));
    c.o_grad = take(kCnnParams * sizeof(float));
    c.o_loss = take(sizeof(float));
    c.o_err = take(4 * sizeof(uint32_t));
    c.total = o;
}

CnnTrainBufs bufs(corr_cnn *c) {
    char *b = c->d_ws;
    CnnTrainBufs r;
    r.x = (float *)(b + c->o_x);
    r.y = (float *)(b + c->o_y);
    r.z1 = (float *)(b + c->o_z1);
    r.z2 = (float *)(b + c->o_z2);
    r.z3 = (float *)(b + c->o_z3);
    r.d3 = (float *)(b + c->o_d3);
    r.d2 = (float *)(b + c->o_d2);
    r.d1 = (float *)(b + c->o_d1);
    r.part = (float *)(b + c->o_part);
    r.lpart = (double *)(b + c->o_lpart);
    r.grad = (float *)(b + c->o_grad);
    r.loss = (float *)(b + c->o_loss);
    r.err = (uint32_t *)(b + c->o_err);
    return r;
}

corr_status check_shape(corr_cnn *c, int32_t S, int64_t T, int32_t C) {
    if (S < 1 || T < kFlagTileSpectra || C < kFlagTileChannels || T % kFlagTileSpectra || C % kFlagTileChannels)
        return fail(c, CORR_ERR_INVALID, "power shape S=%d T=%lld C=%d: need S >= 1, T a multiple of %d, C of %d", S,
                    (long long)T, C, kFlagTileSpectra, kFlagTileChannels);
    if ((int64_t)S * (T / kFlagTileSpectra) * (C / kFlagTileChannels) > INT32_MAX)
        return fail(c, CORR_ERR_INVALID, "more than 2^31 - 1 tiles");
    return CORR_OK;
}

corr_status check_train(corr_cnn *c, const float *d_params, const float *d_power, int32_t S, int64_t T, int32_t C,
                        const int32_t *d_tiles, int32_t n_tiles) {
    if (!c) return fail(nullptr, CORR_ERR_NULL, "cnn is null");
    if (!d_params || !d_power || !d_tiles) return fail(c, CORR_ERR_NULL, "d_params, d_power and d_tiles are required");
    if (!c->bound) return fail(c, CORR_ERR_WORKSPACE, "no workspace bound");
    if (!aligned(d_params, 4) || !aligned(d_power, 4) || !aligned(d_tiles, 4))
        return fail(c, CORR_ERR_ALIGN, "d_params, d_power and d_tiles must be 4-byte aligned");
    if (n_tiles < 1 || n_tiles > c->d.max_tiles)
        return fail(c, CORR_ERR_INVALID, "n_tiles %d outside 1..%d", n_tiles, c->d.max_tiles);
    return check_shape(c, S, T, C);
}

// FP32 forward of the listed tiles into the workspace activations.
corr_status forward(corr_cnn *c, const float *d_params, const float *d_power, const uint8_t *d_labels, int32_t S,
                    int64_t T, int32_t C, const int32_t *d_tiles, int32_t n, hipStream_t st) {
    const CnnTrainBufs b = bufs(c);
    hipError_t e = launch_cnn_gather(d_power, d_labels, S, T, C, d_tiles, n, b, st);
    if (e == hipSuccess) e = launch_cnn_forward(d_params, n, b, st);
    return e == hipSuccess ? CORR_OK : hip_fail(c, e, "CNN forward launch");
}

}  // namespace

extern "C" {

corr_status corr_cnn_create(const corr_cnn_desc_t *desc, corr_cnn_t **out) {
    if (!desc || !out) return fail(nullptr, CORR_ERR_NULL, "desc and out must be non-null");
    const corr_cnn_desc_t &d = *desc;
    if (d.max_tiles < 1 || d.max_tiles > 4096) return fail(nullptr, CORR_ERR_INVALID, "max_tiles %d outside 1..4096", d.max_tiles);
    if (!(d.lr > 0) || !std::isfinite(d.lr)) return fail(nullptr, CORR_ERR_INVALID, "lr must be finite and > 0");
    if (!(d.beta1 >= 0 && d.beta1 < 1) || !(d.beta2 >= 0 && d.beta2 < 1))
        return fail(nullptr, CORR_ERR_INVALID, "beta1 and beta2 must lie in [0, 1)");
    if (!(d.eps > 0) || !std::isfinite(d.eps)) return fail(nullptr, CORR_ERR_INVALID, "eps must be finite and > 0");
    for (int i = 0; i < 7; ++i)
        if (d.reserved[i]) return fail(nullptr, CORR_ERR_INVALID, "reserved[%d] must be zero", i);
    corr_cnn *c = new (std::nothrow) corr_cnn;
    if (!c) return fail(nullptr, CORR_ERR_NOMEM, "allocation failed");
    c->d = d;
    layout(*c);
    *out = c;
    return CORR_OK;
}

void corr_cnn_destroy(corr_cnn_t *c) { delete c; }

size_t corr_cnn_workspace_bytes(const corr_cnn_t *c) { return c ? c->total : 0; }

corr_status corr_cnn_bind_workspace(corr_cnn_t *c, void *d_ws, size_t bytes) {
    if (!c || !d_ws) return fail(c, CORR_ERR_NULL, "cnn and workspace must be non-null");
    if (!aligned(d_ws, 256)) return fail(c, CORR_ERR_ALIGN, "workspace must be 256-byte aligned");
    if (bytes < c->total) return fail(c, CORR_ERR_WORKSPACE, "workspace of %zu bytes < %zu needed", bytes, c->total);
    c->d_ws = (char *)d_ws;
    c->ws_bytes = bytes;
    hipError_t e = hipMemset(c->d_ws + c->o_err, 0, 4 * sizeof(uint32_t));
    if (e != hipSuccess) return hip_fail(c, e, "clearing the error words");
    c->bound = true;
    return CORR_OK;
}

corr_status corr_cnn_forward(corr_cnn_t *c, const float *d_params, const float *d_power, int32_t S, int64_t T,
                             int32_t C, const int32_t *d_tiles, int32_t n_tiles, float *d_logits, void *stream) {
    corr_status r = check_train(c, d_params, d_power, S, T, C, d_tiles, n_tiles);
    if (r != CORR_OK) return r;
    if (!d_logits) return fail(c, CORR_ERR_NULL, "d_logits is required");
    hipStream_t st = (hipStream_t)stream;
    if ((r = forward(c, d_params, d_power, nullptr, S, T, C, d_tiles, n_tiles, st)) != CORR_OK) return r;
    hipError_t e = hipMemcpyAsync(d_logits, bufs(c).z3, (size_t)n_tiles * kCnnPixels * sizeof(float),
                                  hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? CORR_OK : hip_fail(c, e, "copying the logits");
}

corr_status corr_cnn_loss_grad(corr_cnn_t *c, const float *d_params, const float *d_power, const uint8_t *d_labels,
                               int32_t S, int64_t T, int32_t C, const int32_t *d_tiles, int32_t n_tiles,
                               float *d_loss, float *d_grad, void *stream) {
    corr_status r = check_train(c, d_params, d_power, S, T, C, d_tiles, n_tiles);
    if (r != CORR_OK) return r;
    if (!d_labels || !d_loss) return fail(c, CORR_ERR_NULL, "d_labels and d_loss are required");
    if (!aligned(d_loss, 4) || (d_grad && !aligned(d_grad, 4))) return fail(c, CORR_ERR_ALIGN, "d_loss / d_grad alignment");
    hipStream_t st = (hipStream_t)stream;
    if ((r = forward(c, d_params, d_power, d_labels, S, T, C, d_tiles, n_tiles, st)) != CORR_OK) return r;
    const CnnTrainBufs b = bufs(c);
    hipError_t e = launch_cnn_backward(d_params, n_tiles, b, b.grad, d_loss, st);
    if (e == hipSuccess && d_grad)
        e = hipMemcpyAsync(d_grad, b.grad, kCnnParams * sizeof(float), hipMemcpyDeviceToDevice, st);
    return e == hipSuccess ? CORR_OK : hip_fail(c, e, "CNN backward launch");
}

corr_status corr_cnn_adam(corr_cnn_t *c, float *d_params, float *d_m, float *d_v, const float *d_grad, int64_t step,
                          void *stream) {
    if (!c) return fail(nullptr, CORR_ERR_NULL, "cnn is null");
    if (!d_params || !d_m || !d_v) return fail(c, CORR_ERR_NULL, "d_params, d_m and d_v are required");
    if (!d_grad && !c->bound) return fail(c, CORR_ERR_WORKSPACE, "no workspace bound (and no d_grad)");
    if (step < 1) return fail(c, CORR_ERR_INVALID, "step must be >= 1");
    if (!aligned(d_params, 4) || !aligned(d_m, 4) || !aligned(d_v, 4) || (d_grad && !aligned(d_grad, 4)))
        return fail(c, CORR_ERR_ALIGN, "parameter arrays must be 4-byte aligned");
    const corr_cnn_desc_t &d = c->d;
    // bias corrections of Adam in FP64 (beta^t underflows to 0 for large t)
    const double c1 = 1.0 / (1.0 - std::pow((double)d.beta1, (double)step));
    const double c2 = 1.0 / (1.0 - std::pow((double)d.beta2, (double)step));
    hipError_t e = launch_cnn_adam(d_params, d_m, d_v, d_grad ? d_grad : bufs(c).grad, d.lr, d.beta1, d.beta2, d.eps,
                                   (float)c1, (float)c2, (hipStream_t)stream);
    return e == hipSuccess ? CORR_OK : hip_fail(c, e, "Adam launch");
}

corr_status corr_cnn_train_step(corr_cnn_t *c, float *d_params, float *d_m, float *d_v, int64_t step,
                                const float *d_power, const uint8_t *d_labels, int32_t S, int64_t T, int32_t C,
                                const int32_t *d_tiles, int32_t n_tiles, float *d_loss, void *stream) {
    if (c && step < 1) return fail(c, CORR_ERR_INVALID, "step must be >= 1");
    if (c && (!d_m || !d_v)) return fail(c, CORR_ERR_NULL, "d_m and d_v are required");
    corr_status r = corr_cnn_loss_grad(c, d_params, d_power, d_labels, S, T, C, d_tiles, n_tiles, d_loss, nullptr,
                                       stream);
    if (r != CORR_OK) return r;
    return corr_cnn_adam(c, d_params, d_m, d_v, nullptr, step, stream);
}

corr_status corr_cnn_check_device_errors(corr_cnn_t *c, void *stream) {
    if (!c) return fail(nullptr, CORR_ERR_NULL, "cnn is null");
    if (!c->bound) return fail(c, CORR_ERR_WORKSPACE, "no workspace bound");
    hipStream_t st = (hipStream_t)stream;
    uint32_t words[4] = {0, 0, 0, 0};
    hipError_t e = hipMemcpyAsync(words, c->d_ws + c->o_err, sizeof(words), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(c, e, "reading the error words");
    if (words[0]) {
        e = hipMemsetAsync(c->d_ws + c->o_err, 0, sizeof(words), st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(c, e, "clearing the error words");
        return fail(c, CORR_ERR_DEVICE_ARG, "a tile number was outside the data (that tile read as zeros)");
    }
    return CORR_OK;
}

static corr_status cnn_infer_any(const float *d_params, const void *d_power, bool f16, int32_t S, int64_t T,
                                 int32_t C, float threshold, float guard_m, uint8_t *d_flags, float *d_logits,
                                 void *stream) {
    if (!d_params || !d_power || !d_flags) return fail(nullptr, CORR_ERR_NULL, "d_params, d_power and d_flags are required");
    if (!aligned(d_params, 4) || !aligned(d_power, f16 ? 2 : 4) || (d_logits && !aligned(d_logits, 4)))
        return fail(nullptr, CORR_ERR_ALIGN, "d_params and d_logits must be 4-byte aligned, d_power %d-byte",
                    f16 ? 2 : 4);
    if (!(threshold > 0.f && threshold < 1.f)) return fail(nullptr, CORR_ERR_INVALID, "threshold must lie in (0, 1)");
    if (!(guard_m >= 0.f) || !std::isfinite(guard_m))
        return fail(nullptr, CORR_ERR_INVALID, "guard_m must be finite and >= 0");
    corr_status r = check_shape(nullptr, S, T, C);
    if (r != CORR_OK) return r;
    if (C > kCnnMaxInferChannels)
        return fail(nullptr, CORR_ERR_INVALID, "C=%d above the inference limit %d", C, kCnnMaxInferChannels);
    // sigmoid(z) > thr  <=>  z > log(thr / (1 - thr))
    const float thr_logit = (float)std::log((double)threshold / (1.0 - (double)threshold));
    hipError_t e =
        launch_cnn_infer(d_params, d_power, f16, S, T, C, thr_logit, guard_m, d_flags, d_logits, (hipStream_t)stream);
    return e == hipSuccess ? CORR_OK : hip_fail(nullptr, e, "CNN inference launch");
}

corr_status corr_cnn_infer(const float *d_params, const float *d_power, int32_t S, int64_t T, int32_t C,
                           float threshold, uint8_t *d_flags, float *d_logits, void *stream) {
    return cnn_infer_any(d_params, d_power, false, S, T, C, threshold, 0.f, d_flags, d_logits, stream);
}

corr_status corr_cnn_infer_f16(const float *d_params, const void *d_power16, int32_t S, int64_t T, int32_t C,
                               float threshold, uint8_t *d_flags, float *d_logits, void *stream) {
    return cnn_infer_any(d_params, d_power16, true, S, T, C, threshold, 0.f, d_flags, d_logits, stream);
}

corr_status corr_cnn_infer_guarded(const float *d_params, const void *d_power, int32_t power_fp16, int32_t S,
                                   int64_t T, int32_t C, float threshold, float guard_m, uint8_t *d_flags,
                                   float *d_logits, void *stream) {
    if (power_fp16 != 0 && power_fp16 != 1) return fail(nullptr, CORR_ERR_INVALID, "power_fp16 must be 0 or 1");
    return cnn_infer_any(d_params, d_power, power_fp16 != 0, S, T, C, threshold, guard_m, d_flags, d_logits,
                         stream);
}

corr_status corr_cnn_save(const char *path, const float *d_params, const float *d_m, const float *d_v, int64_t step) {
    if (!path || !d_params) return fail(nullptr, CORR_ERR_NULL, "path and d_params are required");
    std::vector<float> h(3 * (size_t)kCnnParams, 0.f);
    const float *src[3] = {d_params, d_m, d_v};
    for (int k = 0; k < 3; ++k) {
        if (!src[k]) continue;
        hipError_t e = hipMemcpy(h.data() + k * kCnnParams, src[k], kCnnParams * sizeof(float), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(nullptr, e, "copying parameters to the host");
    }
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(nullptr, CORR_ERR_IO, "cannot open %s for writing", path);
    const int32_t count = kCnnParams;
    bool ok = std::fwrite("CORRCNN1", 1, 8, f) == 8 && std::fwrite(&step, sizeof(step), 1, f) == 1 &&
              std::fwrite(&count, sizeof(count), 1, f) == 1 && std::fwrite(h.data(), sizeof(float), h.size(), f) == h.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? CORR_OK : fail(nullptr, CORR_ERR_IO, "writing %s failed", path);
}

corr_status corr_cnn_load(const char *path, float *d_params, float *d_m, float *d_v, int64_t *step) {
    if (!path || !d_params) return fail(nullptr, CORR_ERR_NULL, "path and d_params are required");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(nullptr, CORR_ERR_IO, "cannot open %s", path);
    char magic[8];
    int64_t st = 0;
    int32_t count = 0;
    std::vector<float> h(3 * (size_t)kCnnParams);
    const bool head = std::fread(magic, 1, 8, f) == 8 && std::fread(&st, sizeof(st), 1, f) == 1 &&
                      std::fread(&count, sizeof(count), 1, f) == 1;
    if (!head || std::memcmp(magic, "CORRCNN1", 8) != 0 || count != kCnnParams) {
        std::fclose(f);
        return fail(nullptr, CORR_ERR_INVALID, "%s is not a flagger parameter file of %d parameters", path, kCnnParams);
    }
    const bool body = std::fread(h.data(), sizeof(float), h.size(), f) == h.size();
    std::fclose(f);
    if (!body) return fail(nullptr, CORR_ERR_IO, "%s is truncated", path);
    float *dst[3] = {d_params, d_m, d_v};
    for (int k = 0; k < 3; ++k) {
        if (!dst[k]) continue;
        hipError_t e = hipMemcpy(dst[k], h.data() + k * kCnnParams, kCnnParams * sizeof(float), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(nullptr, e, "copying parameters to the device");
    }
    if (step) *step = st;
    return CORR_OK;
}

const char *corr_cnn_last_error(const corr_cnn_t *c) { return c ? c->err : g_cnn_err; }

}  // extern "C"
