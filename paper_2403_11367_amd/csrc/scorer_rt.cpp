// Host side of the learned candidate scorer (declared in include/gsr_scorer.h):
// argument checks, buffer ownership and the launch sequence of each call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "gsr_scorer.h"
#include "internal.h"

using gsr::kScorerChannels;
using gsr::kScorerHidden;
using gsr::kScorerLayers;

namespace {

// Flat parameter layout: per convolution W[co][3][3][ci], b[co]; W1, b1, w2, b2.
struct Layout {
    int64_t w_off[kScorerLayers], b_off[kScorerLayers], fc_off[4], total;
    Layout() {
        int64_t o = 0;
        for (int l = 0; l < kScorerLayers; ++l) {
            w_off[l] = o;
            o += (int64_t)kScorerChannels[l + 1] * 9 * kScorerChannels[l];
            b_off[l] = o;
            o += kScorerChannels[l + 1];
        }
        const int feat = kScorerChannels[kScorerLayers];
        fc_off[0] = o;
        o += (int64_t)kScorerHidden * feat;
        fc_off[1] = o;
        o += kScorerHidden;
        fc_off[2] = o;
        o += kScorerHidden;
        fc_off[3] = o;
        o += 1;
        total = o;
    }
};
const Layout kLayout;

// float32 partial sums of the weight gradient (bounds the split of its reduction)
constexpr int64_t kPartCap = 9 << 20;

}  // namespace

struct gsr_scorer {
    gsr_ctx *ctx = nullptr;
    int device = 0;
    int H = 0, W = 0, max_batch = 0;
    int64_t step = 0;
    float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    uint8_t *decay = nullptr;
    uint16_t *wt = nullptr, *wd = nullptr;
    uint16_t *act[kScorerLayers + 1] = {};
    uint16_t *dbuf[2] = {};
    float *g = nullptr, *h = nullptr, *ds = nullptr, *dh = nullptr, *score = nullptr, *qstats = nullptr;
    float *part = nullptr;
    std::vector<void *> owned;
};

namespace gsr {
void scorer_info(const gsr_scorer *s, gsr_ctx **ctx, int *height, int *width, int *max_batch) {
    *ctx = s->ctx;
    *height = s->H;
    *width = s->W;
    *max_batch = s->max_batch;
}
}  // namespace gsr

namespace {

int fail(gsr_scorer *s, int code, const std::string &msg) { return gsr::ctx_fail(s->ctx, code, msg.c_str()); }

int alloc(gsr_scorer *s, void **p, size_t bytes, const char *what) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 256);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(s, GSR_ENOMEM, std::string("scorer: allocation of ") + what + " failed (" +
                                       std::to_string(bytes) + " bytes)");
    }
    s->owned.push_back(*p);
    return GSR_OK;
}

void free_all(gsr_scorer *s) {
    for (void *p : s->owned) (void)hipFree(p);
    s->owned.clear();
}

int check(gsr_scorer *s, const char *what) {
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? GSR_OK : gsr::ctx_hip_fail(s->ctx, e, what);
}

gsr::ScorerBufs bufs(gsr_scorer *s, const uint16_t *x) {
    gsr::ScorerBufs b;
    b.H = s->H;
    b.W = s->W;
    b.x = x;
    for (int l = 0; l <= kScorerLayers; ++l) b.act[l] = s->act[l];
    b.params = s->params;
    b.wt = s->wt;
    b.wd = s->wd;
    for (int l = 0; l < kScorerLayers; ++l) {
        b.w_off[l] = kLayout.w_off[l];
        b.b_off[l] = kLayout.b_off[l];
    }
    for (int i = 0; i < 4; ++i) b.fc_off[i] = kLayout.fc_off[i];
    b.g = s->g;
    b.h = s->h;
    b.ds = s->ds;
    b.dh = s->dh;
    b.dbuf[0] = s->dbuf[0];
    b.dbuf[1] = s->dbuf[1];
    b.part = s->part;
    b.part_cap = kPartCap;
    return b;
}

int check_batch(gsr_scorer *s, const uint16_t *x, int32_t n) {
    if (!x) return fail(s, GSR_EINVAL, "scorer: null input");
    if ((uintptr_t)x % 4) return fail(s, GSR_EINVAL, "scorer: input must be 4-byte aligned");
    if (n < 1 || n > s->max_batch)
        return fail(s, GSR_EINVAL, "scorer: batch " + std::to_string(n) + " outside [1, " +
                                       std::to_string(s->max_batch) + "]");
    return GSR_OK;
}

int set_device(gsr_scorer *s) {
    hipError_t e = hipSetDevice(s->device);
    return e == hipSuccess ? GSR_OK : gsr::ctx_hip_fail(s->ctx, e, "hipSetDevice");
}

int backward(gsr_scorer *s, const uint16_t *x, const float *labels, int32_t n, float *loss, float *grads) {
    int rc;
    if ((rc = check_batch(s, x, n))) return rc;
    if (!labels || !grads) return fail(s, GSR_EINVAL, "scorer: null labels or gradient");
    if ((rc = set_device(s))) return rc;
    hipStream_t st = gsr::ctx_stream(s->ctx);
    const gsr::ScorerBufs b = bufs(s, x);
    gsr::launch_scorer_forward(st, b, n, s->score);
    gsr::launch_scorer_backward(st, b, n, s->score, labels, grads, loss);
    return check(s, "scorer backward launch");
}

int adamw(gsr_scorer *s, const float *grads, const gsr_adamw *opt) {
    if (!grads || !opt) return fail(s, GSR_EINVAL, "scorer: null gradient or optimiser settings");
    if (!(opt->lr >= 0.f) || !(opt->beta1 >= 0.f && opt->beta1 < 1.f) || !(opt->beta2 >= 0.f && opt->beta2 < 1.f) ||
        !(opt->eps > 0.f) || !(opt->weight_decay >= 0.f))
        return fail(s, GSR_EINVAL, "scorer: AdamW settings out of range");
    int rc;
    if ((rc = set_device(s))) return rc;
    hipStream_t st = gsr::ctx_stream(s->ctx);
    const int64_t t = ++s->step;
    const float bc1 = (float)(1.0 - std::pow((double)opt->beta1, (double)t));
    const float bc2 = (float)(1.0 - std::pow((double)opt->beta2, (double)t));
    gsr::launch_adamw(st, s->params, grads, s->m, s->v, s->decay, kLayout.total, opt->lr, opt->beta1, opt->beta2,
                      opt->eps, opt->weight_decay, bc1, bc2);
    gsr::launch_scorer_weights(st, bufs(s, nullptr));
    return check(s, "scorer AdamW launch");
}

}  // namespace

extern "C" {

int64_t gsr_scorer_param_count(void) { return kLayout.total; }

int gsr_scorer_create(gsr_ctx *ctx, int32_t height, int32_t width, int32_t max_batch, gsr_scorer **out) {
    if (!out) return GSR_EINVAL;
    *out = nullptr;
    if (!ctx) return GSR_EINVAL;
    if (height < 1 || height > 4096 || width < 1 || width > 4096 || max_batch < 1 || max_batch > 65535)
        return gsr::ctx_fail(ctx, GSR_EINVAL, "scorer: size or batch out of range");
    gsr_scorer *s = new (std::nothrow) gsr_scorer;
    if (!s) return GSR_ENOMEM;
    s->ctx = ctx;
    s->device = gsr::ctx_device(ctx);
    s->H = height;
    s->W = width;
    s->max_batch = max_batch;
    int rc = set_device(s);
    int dm[kScorerLayers + 1][2];
    gsr::scorer_dims(height, width, dm);
    const int64_t np = kLayout.total, B = max_batch;
    size_t dmax = 0;
    for (int l = 1; l <= kScorerLayers && !rc; ++l) {
        const size_t e = (size_t)B * dm[l][0] * dm[l][1] * kScorerChannels[l];
        dmax = std::max(dmax, e);
        rc = alloc(s, (void **)&s->act[l], e * 2, "activations");
    }
    if (!rc) rc = alloc(s, (void **)&s->dbuf[0], dmax * 2, "gradient buffer");
    if (!rc) rc = alloc(s, (void **)&s->dbuf[1], dmax * 2, "gradient buffer");
    if (!rc) rc = alloc(s, (void **)&s->params, np * 4, "parameters");
    if (!rc) rc = alloc(s, (void **)&s->m, np * 4, "AdamW moments");
    if (!rc) rc = alloc(s, (void **)&s->v, np * 4, "AdamW moments");
    if (!rc) rc = alloc(s, (void **)&s->grad, np * 4, "gradient");
    if (!rc) rc = alloc(s, (void **)&s->decay, np, "decay mask");
    if (!rc) rc = alloc(s, (void **)&s->wt, np * 2, "bf16 weights");
    if (!rc) rc = alloc(s, (void **)&s->wd, np * 2, "bf16 weights");
    if (!rc) rc = alloc(s, (void **)&s->g, B * 128 * 4, "head buffers");
    if (!rc) rc = alloc(s, (void **)&s->h, B * kScorerHidden * 4, "head buffers");
    if (!rc) rc = alloc(s, (void **)&s->dh, B * kScorerHidden * 4, "head buffers");
    if (!rc) rc = alloc(s, (void **)&s->ds, B * 4, "head buffers");
    if (!rc) rc = alloc(s, (void **)&s->score, B * 4, "head buffers");
    if (!rc) rc = alloc(s, (void **)&s->qstats, 256, "query statistics");
    if (!rc) rc = alloc(s, (void **)&s->part, kPartCap * 4, "weight-gradient partials");
    if (!rc) {
        std::vector<uint8_t> decay(np, 0);
        for (int l = 0; l < kScorerLayers; ++l)
            for (int64_t i = kLayout.w_off[l]; i < kLayout.b_off[l]; ++i) decay[i] = 1;
        for (int64_t i = kLayout.fc_off[0]; i < kLayout.fc_off[1]; ++i) decay[i] = 1;
        for (int64_t i = kLayout.fc_off[2]; i < kLayout.fc_off[3]; ++i) decay[i] = 1;
        hipError_t e = hipMemcpy(s->decay, decay.data(), np, hipMemcpyHostToDevice);
        for (void *p : {(void *)s->params, (void *)s->m, (void *)s->v, (void *)s->grad})
            if (e == hipSuccess) e = hipMemset(p, 0, np * 4);
        if (e == hipSuccess) e = hipMemset(s->wt, 0, np * 2);
        if (e == hipSuccess) e = hipMemset(s->wd, 0, np * 2);
        if (e != hipSuccess) rc = gsr::ctx_hip_fail(ctx, e, "scorer initialisation");
    }
    if (rc) {
        free_all(s);
        delete s;
        return rc;
    }
    *out = s;
    return GSR_OK;
}

int gsr_scorer_destroy(gsr_scorer *s) {
    if (!s) return GSR_EINVAL;
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(gsr::ctx_stream(s->ctx));
    free_all(s);
    delete s;
    return GSR_OK;
}

int gsr_scorer_set_params(gsr_scorer *s, const float *params_dev) {
    if (!s) return GSR_EINVAL;
    if (!params_dev) return fail(s, GSR_EINVAL, "scorer: null parameters");
    int rc;
    if ((rc = set_device(s))) return rc;
    hipStream_t st = gsr::ctx_stream(s->ctx);
    const size_t bytes = kLayout.total * 4;
    hipError_t e = hipMemcpyAsync(s->params, params_dev, bytes, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess) e = hipMemsetAsync(s->m, 0, bytes, st);
    if (e == hipSuccess) e = hipMemsetAsync(s->v, 0, bytes, st);
    if (e != hipSuccess) return gsr::ctx_hip_fail(s->ctx, e, "scorer set params");
    s->step = 0;
    gsr::launch_scorer_weights(st, bufs(s, nullptr));
    return check(s, "scorer weight conversion");
}

int gsr_scorer_get_params(gsr_scorer *s, float *params_dev) {
    if (!s) return GSR_EINVAL;
    if (!params_dev) return fail(s, GSR_EINVAL, "scorer: null parameters");
    int rc;
    if ((rc = set_device(s))) return rc;
    hipError_t e = hipMemcpyAsync(params_dev, s->params, kLayout.total * 4, hipMemcpyDeviceToDevice,
                                  gsr::ctx_stream(s->ctx));
    return e == hipSuccess ? GSR_OK : gsr::ctx_hip_fail(s->ctx, e, "scorer get params");
}

int gsr_pool_grey(gsr_ctx *ctx, const float *rgb, int32_t n, int32_t height, int32_t width, int32_t factor,
                  float *grey) {
    if (!ctx) return GSR_EINVAL;
    if (!rgb || !grey || n < 1 || height < 1 || width < 1 || factor < 1 || height % factor || width % factor)
        return gsr::ctx_fail(ctx, GSR_EINVAL, "pool_grey: null pointer, or sizes not positive multiples of factor");
    hipError_t e = hipSetDevice(gsr::ctx_device(ctx));
    if (e != hipSuccess) return gsr::ctx_hip_fail(ctx, e, "hipSetDevice");
    gsr::launch_pool_grey(gsr::ctx_stream(ctx), rgb, n, height, width, factor, grey);
    e = hipGetLastError();
    return e == hipSuccess ? GSR_OK : gsr::ctx_hip_fail(ctx, e, "pool_grey launch");
}

int gsr_scorer_inputs(gsr_scorer *s, const float *renders, int32_t n, const float *query_grey, uint16_t *x) {
    if (!s) return GSR_EINVAL;
    int rc;
    if ((rc = check_batch(s, x, n))) return rc;
    if (!renders || !query_grey) return fail(s, GSR_EINVAL, "scorer: null render or query");
    if ((rc = set_device(s))) return rc;
    gsr::launch_scorer_input(gsr::ctx_stream(s->ctx), renders, n, s->H, s->W, query_grey, s->qstats, x);
    return check(s, "scorer input launch");
}

int gsr_scorer_forward(gsr_scorer *s, const uint16_t *x, int32_t n, float *scores) {
    if (!s) return GSR_EINVAL;
    int rc;
    if ((rc = check_batch(s, x, n))) return rc;
    if (!scores) return fail(s, GSR_EINVAL, "scorer: null scores");
    if ((rc = set_device(s))) return rc;
    gsr::launch_scorer_forward(gsr::ctx_stream(s->ctx), bufs(s, x), n, scores);
    return check(s, "scorer forward launch");
}

int gsr_scorer_backward(gsr_scorer *s, const uint16_t *x, const float *labels, int32_t n, float *loss,
                        float *grads) {
    if (!s) return GSR_EINVAL;
    return backward(s, x, labels, n, loss, grads);
}

int gsr_scorer_adamw(gsr_scorer *s, const float *grads, const gsr_adamw *opt) {
    if (!s) return GSR_EINVAL;
    return adamw(s, grads, opt);
}

int gsr_scorer_train_step(gsr_scorer *s, const uint16_t *x, const float *labels, int32_t n, const gsr_adamw *opt,
                          float *loss) {
    if (!s) return GSR_EINVAL;
    if (!opt) return fail(s, GSR_EINVAL, "scorer: null optimiser settings");
    int rc;
    if ((rc = backward(s, x, labels, n, loss, s->grad))) return rc;
    return adamw(s, s->grad, opt);
}

}  // extern "C"
