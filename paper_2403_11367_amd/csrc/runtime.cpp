// Host runtime and C ABI of libgsr (declared in include/gsr.h).
//
// The context owns a stream binding, device flags and counters, a grow-only
// workspace, internal streams, and (when profiling) HIP events around the
// stages. gsr_render enqueues the preprocess of all poses on the caller's
// stream, then splits the poses into groups (one unless asked otherwise). Each
// group runs its ordering stage (per-pose depth sort, emission sums, pair
// emission, stable bucketing by tile) and its compositing on a stream of its
// own: the caller's stream for group 0, internal streams for the others, all
// forked after the preprocess and joined back into the caller's stream. The pair count of a group is
// known only on the device; with pair_capacity == 0 the host waits once per
// render for all groups' counts and sizes the pair buffers exactly, otherwise
// each group uses the fixed capacity with no host wait and an overflow is
// flagged on the device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gsr.h"
#include "gsr_scorer.h"
#include "internal.h"

// Pose groups of a render.
constexpr int kMaxGroups = 8;

struct gsr_ctx {
    int device = 0;
    int n_cu = 0;                  // compute units of the device
    hipStream_t stream = nullptr;
    bool profile = false;
    bool capturing = false;        // between gsr_capture_begin and gsr_capture_end
    hipStream_t capture_stream = nullptr;
    unsigned int *d_queue = nullptr;  // work-queue counters of persistent blends, one per pose group
    std::string err;
    // device flags (int32) and counters (uint64)
    int *d_flags = nullptr;
    unsigned long long *d_counters = nullptr;
    // pinned host staging for small readbacks (kMaxGroups uint64) and a search batch's scores
    uint64_t *h_pin = nullptr;
    float *h_scores = nullptr;
    size_t h_scores_n = 0;
    // internal streams (default priority) for pose groups 1.., and the events
    // that chain and join them (timing disabled)
    hipStream_t aux[kMaxGroups - 1] = {};
    hipEvent_t chain[kMaxGroups] = {}, join[kMaxGroups] = {};
    // workspace
    struct Buf {
        void *p = nullptr;
        size_t bytes = 0;
    } records, rect, vmask, sort_ka, sort_va, sort_kb, sort_vb, rcnt, roff, nv, vbase, esum, pseg, ptile, pk,
        sk, ccnt, cstart, ctile, cval, block_base, bseg, offsets, keep_off, keep_state, keep_items, grey_q, partials, s_order, s_poses, s_rgb, s_depth,
        s_scores, pr_grey, pr_q3, pr_x, pr_rgb, pr_depth, bw_screen, bw_pose, h2d;
    size_t ws_limit = 0;  // bytes the workspace may hold in all (0 = no limit)
    size_t ws_bytes = 0;  // bytes it holds
    int32_t overflow_retried = 0;  // the last render overflowed its fixed capacity and was rendered again
    // layout of the last render's pose groups
    struct Group {
        int64_t p0 = 0, np = 0;        // poses [p0, p0 + np)
        uint64_t vb = 0;               // vbase / pseg: np + 1 entries from here
        uint64_t es = 0, n_eb = 0;     // emission sums from es (pair total at es + n_eb)
        uint64_t off = 0;              // list offsets: np * T + 1 entries from here
        uint64_t cst = 0;              // coarse bucket starts and bucketing block bases: np * coarse + 1
                                       // entries each from here
        uint64_t pairs = 0, cap = 0;   // pair buffers: cap entries from pairs
        uint64_t cnt = 0;              // bucketing counts
        uint64_t bsg = 0;              // bucketing block -> segment map
        uint64_t kst = 0, kit = 0;     // kept compositing states (floats) and backward items
    };
    Group groups[kMaxGroups];
    int n_groups = 0;
    int64_t last_n = 0, last_poses = 0, last_tiles = 0;
    // what the backward needs of the last render
    int64_t render_serial = 0;
    bool last_keep = false;        // the last render kept its long lists' compositing states
    const gsr_submap *last_sm = nullptr;  // single-submap render, else null
    uint64_t last_sm_version = 0;
    gsr::Camera last_cam{};
    gsr::Consts last_consts{};
    gsr::TileGrid last_tg{};
    uint64_t last_capacity = 0;  // per group
    // profiling: event sets of the renders / NCC calls profiled since the last gsr_get_stats
    struct RenderEv {
        // start, after preprocess, end (caller's stream); per group: ordering start,
        // ordering end (= compositing start), compositing end (group's stream)
        hipEvent_t e[3 + 3 * kMaxGroups] = {};
        int n_groups = 0;
    };
    struct NccEv {
        hipEvent_t e[2] = {};
    };
    std::vector<RenderEv> ev_render;
    std::vector<NccEv> ev_ncc;
    size_t n_ev_render = 0, n_ev_ncc = 0;
};

struct gsr_graph {
    gsr_ctx *ctx = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct gsr_submap {
    gsr_ctx *ctx = nullptr;
    int device = 0;
    bool identity = false;  // loaded without an index: entry g is input Gaussian g
    uint64_t version = 0;   // counts loads (a refill in place changes it)
    int64_t n = 0, cap = 0;
    float4 *packed = nullptr;  // [cap * kPackedQuads]
    unsigned long long *nonfinite = nullptr;  // Gaussians of the last load culled as non-finite
};

namespace {

int fail(gsr_ctx *ctx, int code, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return code;
}

int hip_fail(gsr_ctx *ctx, hipError_t e, const char *what) {
    return fail(ctx, e == hipErrorOutOfMemory ? GSR_ENOMEM : GSR_EHIP,
                std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPC(ctx, call)                                       \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

// Grow-only device buffer. Growing waits for the whole device: the internal
// streams of an earlier render may still read the old buffer.
int ensure(gsr_ctx *ctx, gsr_ctx::Buf &b, size_t bytes, const char *name) {
    if (bytes <= b.bytes) return GSR_OK;
    if (ctx->capturing)
        return fail(ctx, GSR_EINVAL, std::string("workspace ") + name +
                                         " would grow under graph capture; run the same call once before capturing");
    if (ctx->ws_limit && ctx->ws_bytes - b.bytes + bytes > ctx->ws_limit)
        return fail(ctx, GSR_ENOMEM, std::string("workspace ") + name + " of " + std::to_string(bytes) +
                                         " bytes would pass the workspace limit of " + std::to_string(ctx->ws_limit) +
                                         " bytes (" + std::to_string(ctx->ws_bytes - b.bytes) + " held elsewhere)");
    if (b.p) {
        HIPC(ctx, hipDeviceSynchronize());
        HIPC(ctx, hipFree(b.p));
        ctx->ws_bytes -= b.bytes;
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes + bytes / 4 + 256;
    if (ctx->ws_limit && ctx->ws_bytes + want > ctx->ws_limit) want = bytes;  // no headroom past the limit
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        want = bytes;
        e = hipMalloc(&b.p, want);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return fail(ctx, GSR_ENOMEM, std::string("device allocation of ") + name + " failed (" +
                                         std::to_string(bytes) + " bytes)");
    }
    b.bytes = want;
    ctx->ws_bytes += want;
    return GSR_OK;
}

int check_launch(gsr_ctx *ctx, const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, what);
    return GSR_OK;
}

// Next unused event set (created on first use).
template <class Set>
int next_events(gsr_ctx *ctx, std::vector<Set> &pool, size_t &used, Set **out) {
    if (used == pool.size()) {
        Set set;
        for (auto &e : set.e) HIPC(ctx, hipEventCreate(&e));
        pool.push_back(set);
    }
    *out = &pool[used++];
    return GSR_OK;
}

bool pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }
int ilog2(int x) {
    int r = 0;
    while ((1 << r) < x) ++r;
    return r;
}

}  // namespace

namespace gsr {
hipStream_t ctx_stream(gsr_ctx *ctx) { return ctx->stream; }
int ctx_device(gsr_ctx *ctx) { return ctx->device; }
int ctx_fail(gsr_ctx *ctx, int code, const char *msg) { return fail(ctx, code, msg); }
int ctx_hip_fail(gsr_ctx *ctx, hipError_t e, const char *what) { return hip_fail(ctx, e, what); }
}  // namespace gsr

extern "C" {

const char *gsr_status_string(int status) {
    switch (status) {
        case GSR_OK: return "ok";
        case GSR_EINVAL: return "invalid argument";
        case GSR_ENOMEM: return "out of memory";
        case GSR_EHIP: return "HIP runtime error";
        case GSR_ENODEV: return "no such device";
        case GSR_EOVERFLOW: return "pair buffer overflow";
        case GSR_EUNSUPPORTED: return "unsupported by this library";
        case GSR_EDEVICE: return "device-side check failed";
        default: return "unknown status";
    }
}

const char *gsr_last_error(gsr_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

int gsr_default_cfg(gsr_render_cfg *out) {
    if (!out) return GSR_EINVAL;
    std::memset(out, 0, sizeof(*out));
    out->tile_w = 16;
    out->tile_h = 16;
    out->eps_dilate = 0.3f;
    out->z_near = 0.2f;
    out->jac_clamp = 1.3f;
    out->cutoff_d2 = 9.0f;
    out->alpha_min = 1.0f / 255.0f;
    out->alpha_max = 0.99f;
    out->t_min = 1e-4f;
    out->flags = 0;
    out->pair_capacity = 0;
    out->pose_groups = 0;
    out->blend_blocks_per_cu = 0;
    out->blend_chunk = 0;
    return GSR_OK;
}

// Scratch of gsr_ncc_noalloc: a static device array (one copy per device, held
// until the process ends) in place of the context workspace. Host code uses the
// device address taken once per device at gsr_create, never the array's name.
namespace {
constexpr size_t kNccScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) unsigned char scratch[kNccScratchBytes];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch[kMaxScratchDevices] = {};

// With `device` current: record the device address of its copy of `scratch`.
int scratch_setup(gsr_ctx *ctx, int device) {
    if (device >= kMaxScratchDevices) return GSR_OK;  // gsr_ncc_noalloc then reports GSR_EUNSUPPORTED
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return GSR_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(ctx, GSR_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch[device] = static_cast<unsigned char *>(p);
    return GSR_OK;
}

unsigned char *scratch_of(int device) {
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch[device];
}
}  // namespace

int gsr_create(gsr_ctx **out, int device, void *hip_stream) {
    if (!out) return GSR_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0) {
        (void)hipGetLastError();
        return GSR_ENODEV;
    }
    if (device < 0 || device >= count) return GSR_ENODEV;
    gsr_ctx *ctx = new (std::nothrow) gsr_ctx();
    if (!ctx) return GSR_ENOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    int rc = GSR_OK;
    do {
        if (hipSetDevice(device) != hipSuccess) { rc = GSR_ENODEV; break; }
        if (hipMalloc(&ctx->d_flags, gsr::FLAG_COUNT * sizeof(int)) != hipSuccess) { rc = GSR_ENOMEM; break; }
        if (hipMalloc(&ctx->d_counters, gsr::CNT_COUNT * sizeof(unsigned long long)) != hipSuccess) { rc = GSR_ENOMEM; break; }
        if (hipHostMalloc(&ctx->h_pin, kMaxGroups * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess) { rc = GSR_ENOMEM; break; }
        for (auto &st : ctx->aux)
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) { rc = GSR_EHIP; break; }
        if (rc != GSR_OK) break;
        for (int g = 0; g < kMaxGroups && rc == GSR_OK; ++g)
            if (hipEventCreateWithFlags(&ctx->chain[g], hipEventDisableTiming) != hipSuccess ||
                hipEventCreateWithFlags(&ctx->join[g], hipEventDisableTiming) != hipSuccess)
                rc = GSR_EHIP;
        if (rc != GSR_OK) break;
        if (hipMemset(ctx->d_flags, 0, gsr::FLAG_COUNT * sizeof(int)) != hipSuccess) { rc = GSR_EHIP; break; }
        if (hipMemset(ctx->d_counters, 0, gsr::CNT_COUNT * sizeof(unsigned long long)) != hipSuccess) { rc = GSR_EHIP; break; }
        if (hipMalloc(&ctx->d_queue, kMaxGroups * sizeof(unsigned int)) != hipSuccess) { rc = GSR_ENOMEM; break; }
        if (hipDeviceGetAttribute(&ctx->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
            ctx->n_cu < 1) { rc = GSR_EHIP; break; }
        if ((rc = scratch_setup(ctx, device)) != GSR_OK) break;
    } while (0);
    if (rc != GSR_OK) {
        (void)hipGetLastError();
        gsr_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return GSR_OK;
}

int gsr_destroy(gsr_ctx *ctx) {
    if (!ctx) return GSR_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto st : ctx->aux)
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    for (int g = 0; g < kMaxGroups; ++g) {
        if (ctx->chain[g]) (void)hipEventDestroy(ctx->chain[g]);
        if (ctx->join[g]) (void)hipEventDestroy(ctx->join[g]);
    }
    gsr_ctx::Buf *bufs[] = {&ctx->records,   &ctx->rect,      &ctx->vmask,    &ctx->sort_ka,
                            &ctx->sort_va,   &ctx->sort_kb, &ctx->sort_vb,   &ctx->rcnt,      &ctx->roff,
                            &ctx->nv,        &ctx->vbase,   &ctx->esum,      &ctx->pseg,      &ctx->ptile,
                            &ctx->pk,        &ctx->sk,      &ctx->ccnt,      &ctx->cstart,    &ctx->ctile,
                            &ctx->cval,      &ctx->block_base, &ctx->bseg, &ctx->offsets, &ctx->grey_q, &ctx->partials,
                            &ctx->s_order,   &ctx->s_poses, &ctx->s_rgb,     &ctx->s_depth,   &ctx->s_scores,
                            &ctx->pr_grey,   &ctx->pr_q3,   &ctx->pr_x,      &ctx->pr_rgb,    &ctx->pr_depth,
                            &ctx->bw_screen, &ctx->bw_pose, &ctx->keep_off, &ctx->keep_state,
                            &ctx->keep_items};
    for (auto *b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (ctx->d_flags) (void)hipFree(ctx->d_flags);
    if (ctx->d_counters) (void)hipFree(ctx->d_counters);
    if (ctx->d_queue) (void)hipFree(ctx->d_queue);
    if (ctx->h_pin) (void)hipHostFree(ctx->h_pin);
    if (ctx->h_scores) (void)hipHostFree(ctx->h_scores);
    for (auto &r : ctx->ev_render)
        for (auto &e : r.e)
            if (e) (void)hipEventDestroy(e);
    for (auto &r : ctx->ev_ncc)
        for (auto &e : r.e)
            if (e) (void)hipEventDestroy(e);
    delete ctx;
    return GSR_OK;
}

int gsr_set_stream(gsr_ctx *ctx, void *hip_stream) {
    if (!ctx) return GSR_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return GSR_OK;
}

int gsr_set_profiling(gsr_ctx *ctx, int on) {
    if (!ctx) return GSR_EINVAL;
    ctx->profile = on != 0;
    return GSR_OK;
}

int gsr_submap_load(gsr_ctx *ctx, int64_t n_map, const float *means, const float *scales, const float *quats,
                    const float *opacity, const float *rgb, const int64_t *index, int64_t n_sel,
                    gsr_submap **out) {
    if (!ctx || !out) return GSR_EINVAL;
    if (n_map < 0 || n_sel < 0) return fail(ctx, GSR_EINVAL, "negative size");
    if (n_sel >= ((int64_t)1 << 32)) return fail(ctx, GSR_EINVAL, "submap larger than 2^32 - 1 Gaussians");
    if (!index && n_sel != n_map) return fail(ctx, GSR_EINVAL, "without an index, n_sel must equal n_map");
    if (n_sel > 0 && (!means || !scales || !quats || !opacity || !rgb))
        return fail(ctx, GSR_EINVAL, "null input array");
    HIPC(ctx, hipSetDevice(ctx->device));
    gsr_submap *sm = *out;
    if (sm && sm->ctx != ctx) return fail(ctx, GSR_EINVAL, "submap belongs to another context");
    if (!sm || sm->cap < n_sel) {
        gsr_submap *nsm = new (std::nothrow) gsr_submap();
        if (!nsm) return GSR_ENOMEM;
        nsm->ctx = ctx;
        nsm->device = ctx->device;
        nsm->cap = n_sel > 0 ? n_sel : 1;
        hipError_t e = hipMalloc(&nsm->packed, (size_t)nsm->cap * gsr::kPackedQuads * sizeof(float4));
        if (e == hipSuccess) e = hipMalloc(&nsm->nonfinite, sizeof(unsigned long long));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            if (nsm->packed) (void)hipFree(nsm->packed);
            delete nsm;
            return fail(ctx, GSR_ENOMEM, "submap allocation failed");
        }
        if (sm) gsr_submap_free(sm);
        sm = nsm;
        *out = sm;
    }
    sm->n = n_sel;
    sm->identity = index == nullptr;
    sm->version++;
    gsr::launch_pack(ctx->stream, n_map, means, scales, quats, opacity, rgb, index, n_sel, sm->packed, ctx->d_flags,
                     sm->nonfinite);
    return check_launch(ctx, "pack");
}

int gsr_submap_load_host(gsr_ctx *ctx, int64_t n_map, const float *means, const float *scales, const float *quats,
                         const float *opacity, const float *rgb, const int64_t *index, int64_t n_sel,
                         gsr_submap **out) {
    if (!ctx || !out) return GSR_EINVAL;
    if (n_map < 0 || n_sel < 0) return fail(ctx, GSR_EINVAL, "negative size");
    if (n_map > 0 && (!means || !scales || !quats || !opacity || !rgb)) return fail(ctx, GSR_EINVAL, "null input array");
    if (ctx->capturing) return fail(ctx, GSR_EUNSUPPORTED, "host-input load copies and waits: not under graph capture");
    HIPC(ctx, hipSetDevice(ctx->device));
    // staging: means, scales, quats, opacity, colours, then the index
    const size_t nf = (size_t)n_map * 14, bytes = nf * sizeof(float) + (index ? (size_t)n_sel * sizeof(int64_t) : 0);
    int rc;
    if ((rc = ensure(ctx, ctx->h2d, bytes + 64, "host-input staging"))) return rc;
    float *d = (float *)ctx->h2d.p;
    float *dm = d, *ds = dm + 3 * n_map, *dq = ds + 3 * n_map, *dopa = dq + 4 * n_map, *dc = dopa + n_map;
    int64_t *di = index ? reinterpret_cast<int64_t *>(d + nf + (nf & 1)) : nullptr;  // 8-byte aligned
    if (index && (size_t)((char *)(di + n_sel) - (char *)d) > ctx->h2d.bytes)
        return fail(ctx, GSR_EINVAL, "staging layout");
    const hipStream_t st = ctx->stream;
    if (n_map > 0) {
        HIPC(ctx, hipMemcpyAsync(dm, means, (size_t)n_map * 3 * sizeof(float), hipMemcpyHostToDevice, st));
        HIPC(ctx, hipMemcpyAsync(ds, scales, (size_t)n_map * 3 * sizeof(float), hipMemcpyHostToDevice, st));
        HIPC(ctx, hipMemcpyAsync(dq, quats, (size_t)n_map * 4 * sizeof(float), hipMemcpyHostToDevice, st));
        HIPC(ctx, hipMemcpyAsync(dopa, opacity, (size_t)n_map * sizeof(float), hipMemcpyHostToDevice, st));
        HIPC(ctx, hipMemcpyAsync(dc, rgb, (size_t)n_map * 3 * sizeof(float), hipMemcpyHostToDevice, st));
    }
    if (index && n_sel > 0)
        HIPC(ctx, hipMemcpyAsync(di, index, (size_t)n_sel * sizeof(int64_t), hipMemcpyHostToDevice, st));
    rc = gsr_submap_load(ctx, n_map, dm, ds, dq, dopa, dc, di, index ? n_sel : n_map, out);
    if (rc != GSR_OK) return rc;
    // the staging buffer is reused by the next call: wait for the pack here
    HIPC(ctx, hipStreamSynchronize(st));
    return GSR_OK;
}

int gsr_submap_free(gsr_submap *sm) {
    if (!sm) return GSR_EINVAL;
    // hipFree waits for work on the device that may still read the submap
    (void)hipSetDevice(sm->device);
    if (sm->packed) (void)hipFree(sm->packed);
    if (sm->nonfinite) (void)hipFree(sm->nonfinite);
    delete sm;
    return GSR_OK;
}

int64_t gsr_submap_size(const gsr_submap *sm) { return sm ? sm->n : -1; }

namespace {

// The render of gsr_render and gsr_render_multi: the poses see the submaps of
// `tab`; n_slot = the largest submap (record slots pose * n_slot + index).
int render_impl(gsr_ctx *ctx, const gsr::SubmapTable &tab, int64_t n_slot, const gsr_camera *cam, const float *poses,
                int32_t n_poses, const gsr_render_cfg *cfg_in, float *rgb, float *depth, float *tfinal,
                const gsr_submap *last_sm_hint) {
    if (!cam || !poses || !rgb || !depth) return fail(ctx, GSR_EINVAL, "null argument");
    if (n_poses < 1 || n_poses > 65535) return fail(ctx, GSR_EINVAL, "pose count out of [1, 65535]");
    if (cam->width < 1 || cam->height < 1 || cam->width > 32768 || cam->height > 32768)
        return fail(ctx, GSR_EINVAL, "image size out of [1, 32768]");
    if (!(cam->fx > 0.f) || !(cam->fy > 0.f) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy))
        return fail(ctx, GSR_EINVAL, "bad intrinsics");
    gsr_render_cfg cfg;
    if (cfg_in)
        cfg = *cfg_in;
    else
        gsr_default_cfg(&cfg);
    if (!pow2(cfg.tile_w) || !pow2(cfg.tile_h) || (cfg.flags & ~(GSR_RENDER_COUNT_EVALS | GSR_RENDER_KEEP_STATE | GSR_RENDER_RETRY_OVERFLOW)) != 0 ||
        cfg.pair_capacity < 0 || cfg.pose_groups < 0 || cfg.pose_groups > kMaxGroups)
        return fail(ctx, GSR_EINVAL, "bad render configuration");
    if (!gsr::blend_tile_supported(cfg.tile_w, cfg.tile_h))
        return fail(ctx, GSR_EUNSUPPORTED, "this library renders 16x16, 32x8 or 8x32 tiles");
    if (!(cfg.alpha_min > 0.f) || !(cfg.alpha_max <= 1.f) || !(cfg.alpha_min < cfg.alpha_max) ||
        !(cfg.t_min > 0.f) || !(cfg.cutoff_d2 > 0.f) || !(cfg.eps_dilate >= 0.f) || !(cfg.z_near >= 0.f))
        return fail(ctx, GSR_EINVAL, "bad render constants");
    HIPC(ctx, hipSetDevice(ctx->device));

    gsr::Camera c{cam->width, cam->height, cam->fx, cam->fy, cam->cx, cam->cy};
    gsr::Consts k{cfg.eps_dilate, cfg.z_near, cfg.jac_clamp, cfg.cutoff_d2, cfg.alpha_min, cfg.alpha_max, cfg.t_min};
    gsr::TileGrid tg;
    tg.tile_w = cfg.tile_w;
    tg.tile_h = cfg.tile_h;
    tg.log2_w = ilog2(cfg.tile_w);
    tg.log2_h = ilog2(cfg.tile_h);
    tg.tiles_x = (cam->width + cfg.tile_w - 1) / cfg.tile_w;
    tg.tiles_y = (cam->height + cfg.tile_h - 1) / cfg.tile_h;
    tg.n_tiles = tg.tiles_x * tg.tiles_y;

    const int64_t n = n_slot;
    const int64_t P = n_poses;
    const uint64_t T = (uint64_t)tg.n_tiles;
    const uint64_t n_lists = (uint64_t)P * T;
    if (tg.n_tiles > gsr::kMaxTilesPerPose)
        return fail(ctx, GSR_EUNSUPPORTED, "more than 16384 tiles per image");
    if (n_lists >= 0xffffffffull) return fail(ctx, GSR_EINVAL, "poses x tiles must be below 2^32");
    if ((uint64_t)P * (uint64_t)n >= 0xffffffffull)
        return fail(ctx, GSR_EINVAL, "poses x submap size must be below 2^32");
    const uint64_t pn = (uint64_t)std::max<int64_t>(1, P * n);
    const uint64_t n_regions = (uint64_t)(n + 63) / 64;
    const uint64_t nvc = std::max<uint64_t>(1, (uint64_t)P * n_regions);  // visibility-mask entries
    const uint64_t n_rc = gsr::radix_count_elems(n, n_poses);
    const bool exact = cfg.pair_capacity == 0;
    if (exact && ctx->capturing)
        return fail(ctx, GSR_EINVAL, "a render under graph capture needs a fixed pair_capacity (no host wait)");
    if (cfg.blend_blocks_per_cu < 0 || cfg.blend_blocks_per_cu > 64)
        return fail(ctx, GSR_EINVAL, "blend_blocks_per_cu out of [0, 64]");
    if (!gsr::blend_chunk_supported(cfg.blend_chunk))
        return fail(ctx, GSR_EUNSUPPORTED, "blend_chunk must be 0, 252, 124 or 60");
    const bool keep = (cfg.flags & GSR_RENDER_KEEP_STATE) != 0;
    if (keep && ((cfg.flags & GSR_RENDER_COUNT_EVALS) || (cfg.blend_chunk != 0 && cfg.blend_chunk != 252)))
        return fail(ctx, GSR_EUNSUPPORTED, "GSR_RENDER_KEEP_STATE needs 252-record chunks and no evaluation counting");

    // pose groups: automatic = one. Splitting a render of 64 poses at 1408x376 into
    // 2, 4 or 8 concurrent groups measured 1-13% slower: the ordering of a group
    // costs about as much launch latency as the ordering of all poses at once.
    int G = cfg.pose_groups ? cfg.pose_groups : 1;
    G = (int)std::min<int64_t>(G, P);
    const uint64_t NC = (uint64_t)gsr::bucket_coarse(tg.n_tiles);
    uint64_t n_es = 0, n_cst = 0;
    for (int g = 0; g < G; ++g) {
        gsr_ctx::Group &gr = ctx->groups[g];
        gr.p0 = P * g / G;
        gr.np = P * (g + 1) / G - gr.p0;
        gr.vb = (uint64_t)gr.p0 + g;
        gr.n_eb = gsr::emit_blocks((uint64_t)std::max<int64_t>(1, gr.np * n));
        gr.es = n_es;
        n_es += gsr::emit_sums_size((uint64_t)std::max<int64_t>(1, gr.np * n));
        gr.off = (uint64_t)gr.p0 * T + g;
        gr.cst = n_cst;
        n_cst += (uint64_t)gr.np * NC + 1;
    }
    ctx->n_groups = G;

    int rc;
    if ((rc = ensure(ctx, ctx->records, pn * gsr::kRecordQuads * sizeof(float4), "records")) ||
        (rc = ensure(ctx, ctx->rect, pn * sizeof(uint2), "tile rectangles")) ||
        (rc = ensure(ctx, ctx->vmask, nvc * sizeof(uint64_t), "visibility masks")) ||
        (rc = ensure(ctx, ctx->sort_ka, pn * sizeof(uint32_t), "depth sort")) ||
        (rc = ensure(ctx, ctx->sort_va, pn * sizeof(uint32_t), "depth sort")) ||
        (rc = ensure(ctx, ctx->sort_kb, pn * sizeof(uint32_t), "depth sort")) ||
        (rc = ensure(ctx, ctx->sort_vb, pn * sizeof(uint32_t), "depth sort")) ||
        (rc = ensure(ctx, ctx->rcnt, n_rc * sizeof(uint32_t), "radix counts")) ||
        (rc = ensure(ctx, ctx->roff, n_rc * sizeof(uint32_t), "radix offsets")) ||
        (rc = ensure(ctx, ctx->nv, (uint64_t)P * sizeof(uint32_t), "pose visible counts")) ||
        (rc = ensure(ctx, ctx->vbase, ((uint64_t)P + G) * sizeof(uint32_t), "pose bases")) ||
        (rc = ensure(ctx, ctx->esum, n_es * sizeof(uint64_t), "emission sums")) ||
        (rc = ensure(ctx, ctx->pseg, ((uint64_t)P + G) * sizeof(uint64_t), "pair segments")) ||
        (rc = ensure(ctx, ctx->cstart, n_cst * sizeof(uint64_t), "coarse bucket starts")) ||
        (rc = ensure(ctx, ctx->offsets, (n_lists + G) * sizeof(uint64_t), "offsets")) ||
        (rc = ensure(ctx, ctx->keep_off, (n_lists + G) * sizeof(uint32_t), "kept-state offsets")) ||
        (rc = ensure(ctx, ctx->block_base, n_cst * sizeof(uint32_t), "block bases")))
        return rc;
    // with a fixed capacity every buffer is sized now, before any launch
    auto size_pairs = [&](const uint64_t *caps) -> int {
        uint64_t n_pairs = 0, n_cnt = 0, n_bsg = 0, n_kst = 0;
        for (int g = 0; g < G; ++g) {
            gsr_ctx::Group &gr = ctx->groups[g];
            gr.cap = caps[g];
            gr.pairs = n_pairs;
            n_pairs += std::max<uint64_t>(1, gr.cap);
            gr.cnt = n_cnt;
            n_cnt += gsr::bucket_count_elems(gr.cap, (int)gr.np, tg.n_tiles);
            gr.bsg = n_bsg;
            n_bsg += gsr::bucket_blocks_max(gr.cap, (int)gr.np, tg.n_tiles);
            gr.kst = n_kst;
            if (keep) n_kst += gr.cap / gsr::kKeepRecords * 5 * 256;  // at most one state per kKeepRecords pairs
        }
        int r;
        if ((r = ensure(ctx, ctx->ptile, n_pairs * sizeof(uint16_t), "pair tiles")) ||
            (r = ensure(ctx, ctx->pk, n_pairs * sizeof(uint32_t), "pair indices")) ||
            (r = ensure(ctx, ctx->sk, n_pairs * sizeof(uint32_t), "list indices")) ||
            (r = ensure(ctx, ctx->ctile, n_pairs * sizeof(uint16_t), "bucketed pair tiles")) ||
            (r = ensure(ctx, ctx->cval, n_pairs * sizeof(uint32_t), "bucketed pair indices")) ||
            (r = ensure(ctx, ctx->ccnt, n_cnt * sizeof(uint32_t), "bucket counts")) ||
            (r = ensure(ctx, ctx->bseg, n_bsg * sizeof(uint32_t), "bucket block segments")) ||
            (keep && (r = ensure(ctx, ctx->keep_state, std::max<uint64_t>(1, n_kst) * sizeof(float), "kept states"))))
            return r;
        return GSR_OK;
    };
    uint64_t caps[kMaxGroups];
    if (!exact) {
        if ((uint64_t)cfg.pair_capacity >= 0xffffffffull) return fail(ctx, GSR_EINVAL, "pair capacity must be below 2^32");
        for (int g = 0; g < G; ++g) caps[g] = (uint64_t)cfg.pair_capacity;
        if ((rc = size_pairs(caps))) return rc;
    }

    hipStream_t s = ctx->stream;
    auto stream_of = [&](int g) { return g == 0 ? s : ctx->aux[g - 1]; };
    uint32_t *sort_ka = (uint32_t *)ctx->sort_ka.p, *sort_va = (uint32_t *)ctx->sort_va.p;
    uint32_t *sort_kb = (uint32_t *)ctx->sort_kb.p, *sort_vb = (uint32_t *)ctx->sort_vb.p;
    uint32_t *vbase = (uint32_t *)ctx->vbase.p;
    uint64_t *esum = (uint64_t *)ctx->esum.p;
    const float4 *records = (const float4 *)ctx->records.p;
    const int64_t hw = (int64_t)cam->width * cam->height;

    gsr_ctx::RenderEv *ev = nullptr;
    if (ctx->profile && !ctx->capturing) {
        if ((rc = next_events(ctx, ctx->ev_render, ctx->n_ev_render, &ev))) return rc;
        ev->n_groups = G;
        HIPC(ctx, hipEventRecord(ev->e[0], s));
    }
    gsr::launch_fill_u64(s, ctx->d_counters, gsr::CNT_COUNT, 0ull);
    gsr::launch_sum_nonfinite(s, tab, ctx->d_counters + gsr::CNT_NONFINITE);
    const bool pack = gsr::pack_sort_values(n, tg.n_tiles);  // tile counts ride in the sort values
    gsr::launch_preprocess(s, tab, n, poses, n_poses, c, k, tg, (float4 *)ctx->records.p, (uint2 *)ctx->rect.p,
                           sort_kb, sort_vb, (uint64_t *)ctx->vmask.p, pack, ctx->d_counters + gsr::CNT_WIDE_DEPTH);
    if ((rc = check_launch(ctx, "preprocess"))) return rc;
    if (ev) HIPC(ctx, hipEventRecord(ev->e[1], s));

    // the depth sort's output of group g (three or four radix passes)
    const unsigned long long *wide = ctx->d_counters + gsr::CNT_WIDE_DEPTH;
    auto sorted_run = [&](int g) {
        const uint64_t so = (uint64_t)ctx->groups[g].p0 * n;
        return gsr::SortedRun{sort_kb + so, sort_vb + so, sort_ka + so, sort_va + so, wide};
    };
    // ordering, part 1 of group g: per-pose depth order of its visible Gaussians
    // and the emission sums. Group slices: poses p0.., Gaussian slots p0 * n..
    auto order_part1 = [&](int g, hipStream_t st) {
        const gsr_ctx::Group &gr = ctx->groups[g];
        const uint64_t so = (uint64_t)gr.p0 * n, ro = gsr::radix_count_elems(n, (int)gr.p0);
        const uint64_t gpn = (uint64_t)std::max<int64_t>(1, gr.np * n);
        gsr::launch_depth_sort(st, n, (int)gr.np, (const uint64_t *)ctx->vmask.p + (uint64_t)gr.p0 * n_regions,
                               (const uint2 *)ctx->rect.p, (uint32_t)so, pack, wide, sort_ka + so, sort_va + so,
                               sort_kb + so, sort_vb + so, (uint32_t *)ctx->rcnt.p + ro,
                               (uint32_t *)ctx->roff.p + ro, (uint32_t *)ctx->nv.p + gr.p0, vbase + gr.vb);
        gsr::launch_emit_sums(st, sorted_run(g), vbase + gr.vb, (int)gr.np, gpn, esum + gr.es);
    };
    // ordering, part 2 (pair emission and stable bucketing by tile), then compositing
    auto order_part2 = [&](int g, hipStream_t st) {
        const gsr_ctx::Group &gr = ctx->groups[g];
        const uint64_t gpn = (uint64_t)std::max<int64_t>(1, gr.np * n);
        uint16_t *ptile = (uint16_t *)ctx->ptile.p + gr.pairs;
        uint32_t *pk = (uint32_t *)ctx->pk.p + gr.pairs;
        gsr::launch_pair_segments(st, sorted_run(g), vbase + gr.vb, (int)gr.np, esum + gr.es, gpn, gr.cap,
                                  (uint64_t *)ctx->pseg.p + gr.vb);
        gsr::launch_emit(st, sorted_run(g), vbase + gr.vb, (int)gr.np, (const uint2 *)ctx->rect.p, n, gpn,
                         esum + gr.es, tg, ptile, pk, gr.cap, ctx->d_flags);
        gsr::launch_bucket(st, ptile, pk, (uint64_t *)ctx->pseg.p + gr.vb, (int)gr.np, gr.cap, tg.n_tiles,
                           (uint32_t *)ctx->block_base.p + gr.cst, (uint32_t *)ctx->bseg.p + gr.bsg,
                           (uint32_t *)ctx->ccnt.p + gr.cnt,
                           (uint64_t *)ctx->cstart.p + gr.cst, (uint16_t *)ctx->ctile.p + gr.pairs,
                           (uint32_t *)ctx->cval.p + gr.pairs, (uint64_t *)ctx->offsets.p + gr.off,
                           (uint32_t *)ctx->sk.p + gr.pairs);
        if (keep)
            gsr::launch_keep_offsets(st, (const uint64_t *)ctx->offsets.p + gr.off, gr.cap, (uint32_t)(gr.np * T),
                                     (uint32_t *)ctx->keep_off.p + gr.off);
    };
    auto composite = [&](int g, hipStream_t st) {
        const gsr_ctx::Group &gr = ctx->groups[g];
        gsr::launch_blend(st, records + (uint64_t)gr.p0 * n * gsr::kRecordQuads, n, (int)gr.np,
                          (const uint32_t *)ctx->sk.p + gr.pairs, (const uint64_t *)ctx->offsets.p + gr.off, gr.cap, c,
                          k, tg, rgb + gr.p0 * 3 * hw, depth + gr.p0 * hw, tfinal ? tfinal + gr.p0 * hw : nullptr,
                          (cfg.flags & GSR_RENDER_COUNT_EVALS) != 0, ctx->d_counters,
                          cfg.blend_blocks_per_cu * ctx->n_cu, ctx->d_queue + g, cfg.blend_chunk,
                          keep ? (const uint32_t *)ctx->keep_off.p + gr.off : nullptr,
                          keep ? (float *)ctx->keep_state.p + gr.kst : nullptr);
    };

    if (exact) {
        // all groups' part 1 on the caller's stream, one host wait for every group's pair count
        for (int g = 0; g < G; ++g) {
            order_part1(g, s);
            HIPC(ctx, hipMemcpyAsync(ctx->h_pin + g, esum + ctx->groups[g].es + ctx->groups[g].n_eb, sizeof(uint64_t),
                                     hipMemcpyDeviceToHost, s));
        }
        if ((rc = check_launch(ctx, "depth sort"))) return rc;
        HIPC(ctx, hipStreamSynchronize(s));
        for (int g = 0; g < G; ++g) {
            caps[g] = ctx->h_pin[g];
            if (caps[g] >= 0xffffffffull) return fail(ctx, GSR_EINVAL, "pair count must be below 2^32");
        }
        if ((rc = size_pairs(caps))) return rc;
    }
    // every group starts once the preprocess (and in exact mode part 1 of all
    // groups) is done; the groups' ordering kernels, which are bound by latency,
    // then run side by side, and a group's compositing overlaps what is left of
    // the others' ordering
    if (G > 1) HIPC(ctx, hipEventRecord(ctx->chain[0], s));
    for (int g = 0; g < G; ++g) {
        hipStream_t st = stream_of(g);
        if (g > 0) HIPC(ctx, hipStreamWaitEvent(st, ctx->chain[0], 0));
        if (ev) HIPC(ctx, hipEventRecord(ev->e[3 + 3 * g], st));
        if (!exact) order_part1(g, st);
        order_part2(g, st);
        if ((rc = check_launch(ctx, "pair ordering"))) return rc;
        if (ev) HIPC(ctx, hipEventRecord(ev->e[4 + 3 * g], st));
        composite(g, st);
        if ((rc = check_launch(ctx, "blend"))) return rc;
        if (ev) HIPC(ctx, hipEventRecord(ev->e[5 + 3 * g], st));
    }
    for (int g = 1; g < G; ++g) {
        HIPC(ctx, hipEventRecord(ctx->join[g], stream_of(g)));
        HIPC(ctx, hipStreamWaitEvent(s, ctx->join[g], 0));
    }
    if (ev) HIPC(ctx, hipEventRecord(ev->e[2], s));

    ctx->last_n = n;
    ctx->last_poses = P;
    ctx->last_tiles = tg.n_tiles;
    ctx->last_capacity = exact ? 0 : (uint64_t)cfg.pair_capacity;
    ctx->render_serial++;
    ctx->last_sm = tab.count == 1 ? last_sm_hint : nullptr;
    ctx->last_sm_version = last_sm_hint ? last_sm_hint->version : 0;
    ctx->last_cam = c;
    ctx->last_keep = keep;
    ctx->last_consts = k;
    ctx->last_tg = tg;
    return GSR_OK;
}

}  // namespace

namespace {

// render_impl, and with GSR_RENDER_RETRY_OVERFLOW and a fixed pair capacity: wait
// for the device's overflow flag and, if the capacity was exceeded, render again
// with the pair buffers sized exactly.
int render_retry(gsr_ctx *ctx, const gsr::SubmapTable &tab, int64_t n_slot, const gsr_camera *cam, const float *poses,
                 int32_t n_poses, const gsr_render_cfg *cfg_in, float *rgb, float *depth, float *tfinal,
                 const gsr_submap *hint) {
    ctx->overflow_retried = 0;
    if (!cfg_in || !(cfg_in->flags & GSR_RENDER_RETRY_OVERFLOW))
        return render_impl(ctx, tab, n_slot, cam, poses, n_poses, cfg_in, rgb, depth, tfinal, hint);
    if (ctx->capturing)
        return fail(ctx, GSR_EUNSUPPORTED, "GSR_RENDER_RETRY_OVERFLOW waits on the host: not under graph capture");
    gsr_render_cfg cfg = *cfg_in;
    cfg.flags &= ~GSR_RENDER_RETRY_OVERFLOW;
    HIPC(ctx, hipSetDevice(ctx->device));
    int flags[gsr::FLAG_COUNT];
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    HIPC(ctx, hipMemcpy(flags, ctx->d_flags, sizeof(flags), hipMemcpyDeviceToHost));
    if (flags[gsr::FLAG_OVERFLOW]) return fail(ctx, GSR_EOVERFLOW, "an earlier render overflowed (not yet reported)");
    int rc = render_impl(ctx, tab, n_slot, cam, poses, n_poses, &cfg, rgb, depth, tfinal, hint);
    if (rc != GSR_OK || cfg.pair_capacity == 0) return rc;
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    HIPC(ctx, hipMemcpy(flags, ctx->d_flags, sizeof(flags), hipMemcpyDeviceToHost));
    if (!flags[gsr::FLAG_OVERFLOW]) return GSR_OK;
    flags[gsr::FLAG_OVERFLOW] = 0;
    HIPC(ctx, hipMemcpy(ctx->d_flags, flags, sizeof(flags), hipMemcpyHostToDevice));
    cfg.pair_capacity = 0;
    rc = render_impl(ctx, tab, n_slot, cam, poses, n_poses, &cfg, rgb, depth, tfinal, hint);
    ctx->overflow_retried = 1;
    return rc;
}

}  // namespace

int gsr_set_workspace_limit(gsr_ctx *ctx, int64_t bytes) {
    if (!ctx || bytes < 0) return GSR_EINVAL;
    ctx->ws_limit = (size_t)bytes;
    return GSR_OK;
}

int gsr_render(gsr_ctx *ctx, const gsr_submap *sm, const gsr_camera *cam, const float *poses, int32_t n_poses,
               const gsr_render_cfg *cfg, float *rgb, float *depth, float *tfinal) {
    if (!ctx) return GSR_EINVAL;
    if (!sm) return fail(ctx, GSR_EINVAL, "null argument");
    if (sm->ctx != ctx) return fail(ctx, GSR_EINVAL, "submap belongs to another context");
    gsr::SubmapTable tab{};
    tab.count = 1;
    tab.pose_end[0] = n_poses;
    tab.n[0] = sm->n;
    tab.packed[0] = sm->packed;
    tab.nonfinite[0] = sm->nonfinite;
    return render_retry(ctx, tab, sm->n, cam, poses, n_poses, cfg, rgb, depth, tfinal, sm);
}

int gsr_render_backward(gsr_ctx *ctx, const gsr_submap *sm, const float *scales, const float *quats,
                        const float *poses, int32_t n_poses, const float *rgb, const float *depth,
                        const float *grad_rgb, const float *grad_depth, float *g_means, float *g_scales,
                        float *g_quats, float *g_opacity, float *g_rgb) {
    if (!ctx) return GSR_EINVAL;
    if (!sm || !scales || !quats || !poses || !rgb || !depth || !grad_rgb || !grad_depth || !g_means || !g_scales ||
        !g_quats || !g_opacity || !g_rgb)
        return fail(ctx, GSR_EINVAL, "null argument");
    if (ctx->capturing) return fail(ctx, GSR_EINVAL, "the backward is not captured");
    if (!sm->identity) return fail(ctx, GSR_EINVAL, "the submap must be loaded without an index");
    if (ctx->last_sm != sm || ctx->last_sm_version != sm->version || ctx->last_poses != n_poses ||
        ctx->last_n != sm->n)
        return fail(ctx, GSR_EINVAL, "the last render of this context is not a render of this submap at these poses");
    HIPC(ctx, hipSetDevice(ctx->device));
    const int64_t n = sm->n, P = n_poses;
    const uint64_t pn = (uint64_t)std::max<int64_t>(1, P * n);
    const int ns = gsr::kScreenGrads, np = gsr::pose_grads_per_gaussian();
    int rc;
    if ((rc = ensure(ctx, ctx->bw_screen, pn * ns * sizeof(float), "screen-space gradients")) ||
        (rc = ensure(ctx, ctx->bw_pose, pn * np * sizeof(float), "per-pose gradients")))
        return rc;
    hipStream_t s = ctx->stream;
    const gsr::TileGrid &tg = ctx->last_tg;
    const int64_t hw = (int64_t)ctx->last_cam.width * ctx->last_cam.height;
    float *gscreen = (float *)ctx->bw_screen.p;
    gsr::launch_fill_u32(s, (uint32_t *)gscreen, (uint64_t)P * n * ns, 0u);
    const float4 *records = (const float4 *)ctx->records.p;
    // one backward block per (list, kept-state segment); without kept states one per list
    const uint64_t T = (uint64_t)tg.n_tiles;
    uint64_t blocks[kMaxGroups] = {}, n_items = 0;
    for (int g = 0; g < ctx->n_groups; ++g) {
        const gsr_ctx::Group &gr = ctx->groups[g];
        blocks[g] = (uint64_t)gr.np * T + (ctx->last_keep ? gr.cap / gsr::kKeepRecords : 0);
        n_items += blocks[g];
    }
    if ((rc = ensure(ctx, ctx->keep_items, std::max<uint64_t>(1, n_items) * sizeof(uint32_t), "backward blocks")))
        return rc;
    uint64_t item0 = 0;
    for (int g = 0; g < ctx->n_groups; ++g) {
        const gsr_ctx::Group &gr = ctx->groups[g];
        if (gr.np <= 0) continue;
        const uint32_t n_lists = (uint32_t)(gr.np * T);
        uint32_t *keep_off = (uint32_t *)ctx->keep_off.p + gr.off;
        if (!ctx->last_keep) gsr::launch_fill_u32(s, keep_off, (uint64_t)n_lists + 1, 0u);
        uint32_t *items = (uint32_t *)ctx->keep_items.p + item0;
        gsr::launch_keep_items(s, keep_off, n_lists, items);
        gsr::launch_blend_backward(s, records + (uint64_t)gr.p0 * n * gsr::kRecordQuads, n, (int)gr.np,
                                   (const uint32_t *)ctx->sk.p + gr.pairs, (const uint64_t *)ctx->offsets.p + gr.off,
                                   gr.cap, ctx->last_cam, ctx->last_consts, tg, rgb + gr.p0 * 3 * hw,
                                   depth + gr.p0 * hw, grad_rgb + gr.p0 * 3 * hw, grad_depth + gr.p0 * hw,
                                   gscreen + (uint64_t)gr.p0 * n * ns, keep_off,
                                   ctx->last_keep ? (const float *)ctx->keep_state.p + gr.kst : nullptr, items,
                                   blocks[g]);
        item0 += blocks[g];
    }
    gsr::launch_project_backward(s, sm->packed, n, poses, n_poses, ctx->last_cam, ctx->last_consts,
                                 (const uint64_t *)ctx->vmask.p, gscreen, (float *)ctx->bw_pose.p);
    gsr::launch_param_grads(s, (const float *)ctx->bw_pose.p, n, n_poses, scales, quats, g_means, g_scales, g_quats,
                            g_opacity, g_rgb);
    return check_launch(ctx, "render backward");
}

int gsr_render_multi(gsr_ctx *ctx, const gsr_submap *const *submaps, const int32_t *poses_per_submap,
                     int32_t n_submaps, const gsr_camera *cam, const float *poses, const gsr_render_cfg *cfg, float *rgb,
                     float *depth, float *tfinal) {
    if (!ctx) return GSR_EINVAL;
    if (!submaps || !poses_per_submap) return fail(ctx, GSR_EINVAL, "null argument");
    if (n_submaps < 1 || n_submaps > gsr::kMaxBatchSubmaps)
        return fail(ctx, GSR_EINVAL, "submap count out of [1, 16]");
    gsr::SubmapTable tab{};
    tab.count = n_submaps;
    int64_t P = 0, n_slot = 0;
    for (int q = 0; q < n_submaps; ++q) {
        const gsr_submap *sm = submaps[q];
        if (!sm) return fail(ctx, GSR_EINVAL, "null submap");
        if (sm->ctx != ctx) return fail(ctx, GSR_EINVAL, "submap belongs to another context");
        if (poses_per_submap[q] < 1) return fail(ctx, GSR_EINVAL, "every submap needs at least one pose");
        P += poses_per_submap[q];
        if (P > 65535) return fail(ctx, GSR_EINVAL, "pose count out of [1, 65535]");
        tab.pose_end[q] = (int)P;
        tab.n[q] = sm->n;
        tab.packed[q] = sm->packed;
        tab.nonfinite[q] = sm->nonfinite;
        n_slot = std::max<int64_t>(n_slot, sm->n);
    }
    return render_retry(ctx, tab, n_slot, cam, poses, (int32_t)P, cfg, rgb, depth, tfinal, nullptr);
}

int gsr_ncc(gsr_ctx *ctx, const float *query, const float *renders, int32_t n_poses, int32_t height, int32_t width,
            float *scores) {
    if (!ctx) return GSR_EINVAL;
    if (!query || !renders || !scores) return fail(ctx, GSR_EINVAL, "null argument");
    if (n_poses < 1 || n_poses > 65535 || height < 1 || width < 1 || (int64_t)height * width > ((int64_t)1 << 31))
        return fail(ctx, GSR_EINVAL, "size out of range");
    HIPC(ctx, hipSetDevice(ctx->device));
    const int64_t hw = (int64_t)height * width;
    const int64_t nb = (hw + gsr::ncc_pixels_per_block() - 1) / gsr::ncc_pixels_per_block();
    int rc;
    if ((rc = ensure(ctx, ctx->grey_q, (size_t)hw * sizeof(float), "grey query")) ||
        (rc = ensure(ctx, ctx->partials, (size_t)n_poses * nb * 6 * sizeof(double), "ncc partials")))
        return rc;
    gsr_ctx::NccEv *ev = nullptr;
    if (ctx->profile) {
        if ((rc = next_events(ctx, ctx->ev_ncc, ctx->n_ev_ncc, &ev))) return rc;
        HIPC(ctx, hipEventRecord(ev->e[0], ctx->stream));
    }
    gsr::launch_ncc(ctx->stream, query, renders, n_poses, height, width, (float *)ctx->grey_q.p,
                    (double *)ctx->partials.p, scores);
    if ((rc = check_launch(ctx, "ncc"))) return rc;
    if (ev) HIPC(ctx, hipEventRecord(ev->e[1], ctx->stream));
    return GSR_OK;
}

int gsr_ncc_noalloc(gsr_ctx *ctx, const float *query, const float *renders, int32_t n_poses, int32_t height,
                    int32_t width, float *scores) {
    if (!ctx) return GSR_EINVAL;
    if (!query || !renders || !scores) return fail(ctx, GSR_EINVAL, "null argument");
    if (n_poses < 1 || n_poses > 65535 || height < 1 || width < 1 || (int64_t)height * width > ((int64_t)1 << 31))
        return fail(ctx, GSR_EINVAL, "size out of range");
    const int64_t hw = (int64_t)height * width;
    const int64_t nb = (hw + gsr::ncc_pixels_per_block() - 1) / gsr::ncc_pixels_per_block();
    // grey query, then the per-block partial moments (6 doubles each); both are
    // written in full before they are read, so nothing is cleared
    const size_t grey_bytes = ((size_t)hw * sizeof(float) + 255) & ~(size_t)255;
    const size_t need = grey_bytes + (size_t)n_poses * (size_t)nb * 6 * sizeof(double);
    if (need > kNccScratchBytes)
        return fail(ctx, GSR_EINVAL, "gsr_ncc_noalloc: " + std::to_string(need) + " bytes of scratch needed, more than the " +
                                         std::to_string(kNccScratchBytes) + " of the static scratch (use gsr_ncc)");
    unsigned char *base = scratch_of(ctx->device);
    if (!base) return fail(ctx, GSR_EUNSUPPORTED, "gsr_ncc_noalloc: no static scratch on this device");
    HIPC(ctx, hipSetDevice(ctx->device));
    gsr::launch_ncc(ctx->stream, query, renders, n_poses, height, width, reinterpret_cast<float *>(base),
                    reinterpret_cast<double *>(base + grey_bytes), scores);
    return check_launch(ctx, "ncc_noalloc");
}

int gsr_topk(gsr_ctx *ctx, const float *scores, int32_t n_poses, int32_t k, int32_t *idx) {
    if (!ctx) return GSR_EINVAL;
    if (!scores || !idx) return fail(ctx, GSR_EINVAL, "null argument");
    if (n_poses < 1 || n_poses > 8192 || k < 1 || k > n_poses) return fail(ctx, GSR_EINVAL, "need 1 <= k <= P <= 8192");
    HIPC(ctx, hipSetDevice(ctx->device));
    gsr::launch_topk(ctx->stream, scores, n_poses, k, idx);
    return check_launch(ctx, "topk");
}

int gsr_search(gsr_ctx *ctx, const gsr_submap *sm, const gsr_camera *cam, const float *poses, int32_t n_poses,
               const int32_t *order, int32_t batch, int32_t max_eval, float threshold, const float *query,
               const gsr_render_cfg *cfg, float *scores, int32_t *best, float *best_score, int32_t *n_scored) {
    if (!ctx) return GSR_EINVAL;
    if (!sm || !cam || !poses || !order || !query || !scores || !best || !best_score || !n_scored)
        return fail(ctx, GSR_EINVAL, "null argument");
    if (n_poses < 1 || n_poses > 65535 || batch < 1 || max_eval < 1 || max_eval > n_poses)
        return fail(ctx, GSR_EINVAL, "need 1 <= max_eval <= P <= 65535 and batch >= 1");
    if (std::isnan(threshold)) return fail(ctx, GSR_EINVAL, "threshold is NaN");
    // order must be a permutation of the candidates
    std::vector<char> seen((size_t)n_poses, 0);
    for (int32_t i = 0; i < n_poses; ++i) {
        if (order[i] < 0 || order[i] >= n_poses || seen[(size_t)order[i]])
            return fail(ctx, GSR_EINVAL, "order is not a permutation of [0, P)");
        seen[(size_t)order[i]] = 1;
    }
    HIPC(ctx, hipSetDevice(ctx->device));
    const int32_t B = std::min(batch, max_eval);
    const int64_t hw = (int64_t)cam->width * cam->height;
    int rc;
    if ((rc = ensure(ctx, ctx->s_order, (size_t)n_poses * sizeof(int32_t), "search order")) ||
        (rc = ensure(ctx, ctx->s_poses, (size_t)B * 12 * sizeof(float), "search poses")) ||
        (rc = ensure(ctx, ctx->s_rgb, (size_t)B * 3 * hw * sizeof(float), "search renders")) ||
        (rc = ensure(ctx, ctx->s_depth, (size_t)B * hw * sizeof(float), "search depths")) ||
        (rc = ensure(ctx, ctx->s_scores, (size_t)B * sizeof(float), "search scores")))
        return rc;
    // pinned staging for a batch's scores (grown as needed)
    if ((size_t)B > ctx->h_scores_n) {
        if (ctx->h_scores) HIPC(ctx, hipHostFree(ctx->h_scores));
        ctx->h_scores = nullptr;
        ctx->h_scores_n = 0;
        HIPC(ctx, hipHostMalloc(&ctx->h_scores, (size_t)B * sizeof(float), hipHostMallocDefault));
        ctx->h_scores_n = (size_t)B;
    }
    hipStream_t s = ctx->stream;
    int32_t *order_d = (int32_t *)ctx->s_order.p;
    HIPC(ctx, hipMemcpyAsync(order_d, order, (size_t)n_poses * sizeof(int32_t), hipMemcpyHostToDevice, s));
    int32_t b_best = -1;
    float b_score = -INFINITY;
    int32_t n = 0;
    while (n < max_eval) {
        const int32_t nb = std::min(B, max_eval - n);
        gsr::launch_gather_poses(s, poses, order_d + n, nb, (float *)ctx->s_poses.p);
        if ((rc = check_launch(ctx, "search poses"))) return rc;
        if ((rc = gsr_render(ctx, sm, cam, (const float *)ctx->s_poses.p, nb, cfg, (float *)ctx->s_rgb.p,
                             (float *)ctx->s_depth.p, nullptr)))
            return rc;
        if ((rc = gsr_ncc(ctx, query, (const float *)ctx->s_rgb.p, nb, cam->height, cam->width,
                          (float *)ctx->s_scores.p)))
            return rc;
        gsr::launch_scatter_scores(s, (const float *)ctx->s_scores.p, order_d + n, nb, scores);
        if ((rc = check_launch(ctx, "search scores"))) return rc;
        HIPC(ctx, hipMemcpyAsync(ctx->h_scores, ctx->s_scores.p, (size_t)nb * sizeof(float), hipMemcpyDeviceToHost,
                                 s));
        HIPC(ctx, hipStreamSynchronize(s));
        for (int32_t i = 0; i < nb; ++i) {
            const float v = ctx->h_scores[i];
            const int32_t c = order[n + i];
            if (v > b_score || (v == b_score && c < b_best)) {
                b_score = v;
                b_best = c;
            }
        }
        n += nb;
        if (b_score >= threshold) break;
    }
    *best = b_best;
    *best_score = b_score;
    *n_scored = n;
    return GSR_OK;
}

int gsr_search_pruned(gsr_ctx *ctx, gsr_scorer *scorer, const gsr_submap *sm, const gsr_camera *cam,
                      const gsr_camera *cam_low, const float *poses, int32_t n_poses, int32_t batch,
                      const float *query, int32_t k, const gsr_render_cfg *cfg, float *pred, int32_t *top,
                      float *ncc, int32_t *best, float *best_score) {
    if (!ctx) return GSR_EINVAL;
    if (!sm || !cam || !cam_low || !poses || !query || !pred || !top || !ncc || !best || !best_score)
        return fail(ctx, GSR_EINVAL, "null argument");
    if (n_poses < 1 || n_poses > 8192 || k < 1 || k > n_poses || batch < 0)
        return fail(ctx, GSR_EINVAL, "need 1 <= k <= P <= 8192 and batch >= 0");
    const int h = cam_low->height, w = cam_low->width;
    if (h < 1 || w < 1 || cam->height % h || cam->width % w || cam->height / h != cam->width / w)
        return fail(ctx, GSR_EINVAL, "the full-resolution image must be an integer multiple of the low-resolution one");
    const int f = cam->height / h;
    int32_t B = batch ? batch : std::min<int32_t>(n_poses, 256);
    if (scorer) {
        int sh = 0, sw = 0, smax = 0;
        gsr_ctx *sctx = nullptr;
        gsr::scorer_info(scorer, &sctx, &sh, &sw, &smax);
        if (sctx != ctx) return fail(ctx, GSR_EINVAL, "the scorer belongs to another context");
        if (sh != h || sw != w) return fail(ctx, GSR_EINVAL, "scorer input size differs from the low-resolution camera");
        B = std::min<int32_t>(B, smax);
    }
    B = std::min<int32_t>(B, n_poses);
    HIPC(ctx, hipSetDevice(ctx->device));
    const int64_t hw = (int64_t)h * w, HW = (int64_t)cam->height * cam->width;
    int rc;
    if ((rc = ensure(ctx, ctx->pr_grey, hw * sizeof(float), "pooled query")) ||
        (rc = ensure(ctx, ctx->pr_q3, 3 * hw * sizeof(float), "pooled query")) ||
        (rc = ensure(ctx, ctx->pr_x, (size_t)B * hw * 2 * sizeof(uint16_t), "scorer inputs")) ||
        (rc = ensure(ctx, ctx->s_rgb, (size_t)B * 3 * hw * sizeof(float), "low-resolution renders")) ||
        (rc = ensure(ctx, ctx->s_depth, (size_t)B * hw * sizeof(float), "low-resolution depths")) ||
        (rc = ensure(ctx, ctx->s_poses, (size_t)k * 12 * sizeof(float), "kept poses")) ||
        (rc = ensure(ctx, ctx->pr_rgb, (size_t)k * 3 * HW * sizeof(float), "full-resolution renders")) ||
        (rc = ensure(ctx, ctx->pr_depth, (size_t)k * HW * sizeof(float), "full-resolution depths")))
        return rc;
    hipStream_t s = ctx->stream;
    float *grey = (float *)ctx->pr_grey.p, *q3 = (float *)ctx->pr_q3.p;
    if ((rc = gsr_pool_grey(ctx, query, 1, cam->height, cam->width, f, grey))) return rc;
    if (!scorer)  // the low-resolution query for NCC: its grey in all three planes
        for (int c = 0; c < 3; ++c)
            HIPC(ctx, hipMemcpyAsync(q3 + c * hw, grey, hw * sizeof(float), hipMemcpyDeviceToDevice, s));
    float *lrgb = (float *)ctx->s_rgb.p, *ldep = (float *)ctx->s_depth.p;
    for (int32_t b0 = 0; b0 < n_poses; b0 += B) {
        const int32_t nb = std::min(B, n_poses - b0);
        if ((rc = gsr_render(ctx, sm, cam_low, poses + (int64_t)b0 * 12, nb, cfg, lrgb, ldep, nullptr))) return rc;
        if (scorer) {
            uint16_t *x = (uint16_t *)ctx->pr_x.p;
            if ((rc = gsr_scorer_inputs(scorer, lrgb, nb, grey, x))) return rc;
            if ((rc = gsr_scorer_forward(scorer, x, nb, pred + b0))) return rc;
        } else if ((rc = gsr_ncc(ctx, q3, lrgb, nb, h, w, pred + b0))) {
            return rc;
        }
    }
    if ((rc = gsr_topk(ctx, pred, n_poses, k, top))) return rc;
    gsr::launch_gather_poses(s, poses, top, k, (float *)ctx->s_poses.p);
    if ((rc = check_launch(ctx, "kept poses"))) return rc;
    if ((rc = gsr_render(ctx, sm, cam, (const float *)ctx->s_poses.p, k, cfg, (float *)ctx->pr_rgb.p,
                         (float *)ctx->pr_depth.p, nullptr)))
        return rc;
    if ((rc = gsr_ncc(ctx, query, (const float *)ctx->pr_rgb.p, k, cam->height, cam->width, ncc))) return rc;
    std::vector<int32_t> ht((size_t)k);
    std::vector<float> hs((size_t)k);
    HIPC(ctx, hipMemcpyAsync(ht.data(), top, (size_t)k * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPC(ctx, hipMemcpyAsync(hs.data(), ncc, (size_t)k * sizeof(float), hipMemcpyDeviceToHost, s));
    HIPC(ctx, hipStreamSynchronize(s));
    int32_t b_best = -1;
    float b_score = -INFINITY;
    for (int32_t i = 0; i < k; ++i)
        if (hs[i] > b_score || (hs[i] == b_score && ht[i] < b_best)) {
            b_score = hs[i];
            b_best = ht[i];
        }
    *best = b_best;
    *best_score = b_score;
    return GSR_OK;
}

int gsr_capture_begin(gsr_ctx *ctx) {
    if (!ctx) return GSR_EINVAL;
    if (ctx->capturing) return fail(ctx, GSR_EINVAL, "already capturing");
    if (!ctx->stream) return fail(ctx, GSR_EINVAL, "graph capture needs a stream other than the null stream");
    HIPC(ctx, hipSetDevice(ctx->device));
    HIPC(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    ctx->capturing = true;
    ctx->capture_stream = ctx->stream;
    return GSR_OK;
}

int gsr_capture_end(gsr_ctx *ctx, gsr_graph **out) {
    if (!ctx || !out) return GSR_EINVAL;
    *out = nullptr;
    if (!ctx->capturing) return fail(ctx, GSR_EINVAL, "not capturing");
    ctx->capturing = false;
    HIPC(ctx, hipSetDevice(ctx->device));
    hipGraph_t graph = nullptr;
    HIPC(ctx, hipStreamEndCapture(ctx->capture_stream, &graph));
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(ctx, e, "hipGraphInstantiate");
    }
    gsr_graph *g = new (std::nothrow) gsr_graph;
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return GSR_ENOMEM;
    }
    g->ctx = ctx;
    g->graph = graph;
    g->exec = exec;
    *out = g;
    return GSR_OK;
}

int gsr_graph_launch(gsr_graph *g) {
    if (!g) return GSR_EINVAL;
    gsr_ctx *ctx = g->ctx;
    if (ctx->capturing) return fail(ctx, GSR_EINVAL, "cannot launch a graph while capturing");
    HIPC(ctx, hipSetDevice(ctx->device));
    HIPC(ctx, hipGraphLaunch(g->exec, ctx->stream));
    return GSR_OK;
}

int gsr_graph_destroy(gsr_graph *g) {
    if (!g) return GSR_EINVAL;
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
    return GSR_OK;
}

int gsr_sync(gsr_ctx *ctx) {
    if (!ctx) return GSR_EINVAL;
    HIPC(ctx, hipSetDevice(ctx->device));
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    int flags[gsr::FLAG_COUNT];
    HIPC(ctx, hipMemcpy(flags, ctx->d_flags, sizeof(flags), hipMemcpyDeviceToHost));
    if (flags[gsr::FLAG_OVERFLOW] || flags[gsr::FLAG_BAD_INDEX]) {
        HIPC(ctx, hipMemset(ctx->d_flags, 0, sizeof(flags)));
        if (flags[gsr::FLAG_OVERFLOW]) return fail(ctx, GSR_EOVERFLOW, "pair buffer overflow in a render");
        return fail(ctx, GSR_EDEVICE, "submap index out of range");
    }
    return GSR_OK;
}

int gsr_get_stats(gsr_ctx *ctx, gsr_stats *out) {
    if (!ctx || !out) return GSR_EINVAL;
    HIPC(ctx, hipSetDevice(ctx->device));
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    std::memset(out, 0, sizeof(*out));
    unsigned long long cnt[gsr::CNT_COUNT];
    int flags[gsr::FLAG_COUNT];
    HIPC(ctx, hipMemcpy(cnt, ctx->d_counters, sizeof(cnt), hipMemcpyDeviceToHost));
    HIPC(ctx, hipMemcpy(flags, ctx->d_flags, sizeof(flags), hipMemcpyDeviceToHost));
    out->n_submap = ctx->last_n;
    out->n_poses = ctx->last_poses;
    out->pair_capacity = (int64_t)ctx->last_capacity;
    out->n_groups = ctx->n_groups;
    out->render_serial = ctx->render_serial;
    if (ctx->last_poses > 0) {
        for (int g = 0; g < ctx->n_groups; ++g) {
            const gsr_ctx::Group &gr = ctx->groups[g];
            uint32_t nv = 0;
            uint64_t np = 0;
            HIPC(ctx, hipMemcpy(&nv, (uint32_t *)ctx->vbase.p + gr.vb + gr.np, sizeof(nv), hipMemcpyDeviceToHost));
            HIPC(ctx, hipMemcpy(&np, (uint64_t *)ctx->esum.p + gr.es + gr.n_eb, sizeof(np), hipMemcpyDeviceToHost));
            out->n_visible += (int64_t)nv;
            out->n_pairs += (int64_t)np;
        }
    }
    out->overflow = flags[gsr::FLAG_OVERFLOW];
    out->bad_index = flags[gsr::FLAG_BAD_INDEX];
    out->evals_contrib = (int64_t)cnt[gsr::CNT_EVALS_CONTRIB];
    out->evals_lanes = (int64_t)cnt[gsr::CNT_EVALS_LANES];
    out->n_culled_nonfinite = (int64_t)cnt[gsr::CNT_NONFINITE];
    out->workspace_bytes = (int64_t)ctx->ws_bytes;
    out->overflow_retried = ctx->overflow_retried;
    double pre = 0, sort = 0, blend = 0, whole = 0;
    size_t n_group_runs = 0;
    for (size_t i = 0; i < ctx->n_ev_render; ++i) {
        const auto &r = ctx->ev_render[i];
        float ms = 0.f;
        HIPC(ctx, hipEventElapsedTime(&ms, r.e[0], r.e[1]));
        pre += ms;
        HIPC(ctx, hipEventElapsedTime(&ms, r.e[0], r.e[2]));
        whole += ms;
        for (int g = 0; g < r.n_groups; ++g) {
            HIPC(ctx, hipEventElapsedTime(&ms, r.e[3 + 3 * g], r.e[4 + 3 * g]));
            sort += ms;
            HIPC(ctx, hipEventElapsedTime(&ms, r.e[4 + 3 * g], r.e[5 + 3 * g]));
            blend += ms;
            ++n_group_runs;
        }
    }
    double ncc = 0;
    for (size_t i = 0; i < ctx->n_ev_ncc; ++i) {
        float ms = 0.f;
        HIPC(ctx, hipEventElapsedTime(&ms, ctx->ev_ncc[i].e[0], ctx->ev_ncc[i].e[1]));
        ncc += ms;
    }
    out->n_profiled_renders = (int32_t)ctx->n_ev_render;
    out->n_profiled_ncc = (int32_t)ctx->n_ev_ncc;
    if (ctx->n_ev_render) {
        out->ms_preprocess = (float)(pre / ctx->n_ev_render);
        out->ms_render = (float)(whole / ctx->n_ev_render);
    }
    if (n_group_runs) {
        out->ms_sort = (float)(sort / n_group_runs);
        out->ms_blend = (float)(blend / n_group_runs);
    }
    if (ctx->n_ev_ncc) out->ms_ncc = (float)(ncc / ctx->n_ev_ncc);
    ctx->n_ev_render = 0;
    ctx->n_ev_ncc = 0;
    return GSR_OK;
}

namespace {

// Pairs of every group of the last render that fit its buffer (host wait).
int group_pairs(gsr_ctx *ctx, uint64_t *pairs) {
    for (int g = 0; g < ctx->n_groups; ++g) {
        const gsr_ctx::Group &gr = ctx->groups[g];
        uint64_t np = 0;
        HIPC(ctx, hipMemcpy(&np, (uint64_t *)ctx->esum.p + gr.es + gr.n_eb, sizeof(np), hipMemcpyDeviceToHost));
        pairs[g] = std::min(np, gr.cap);
    }
    return GSR_OK;
}

}  // namespace

int gsr_debug_size(gsr_ctx *ctx, int which, int64_t *bytes) {
    if (!ctx || !bytes) return GSR_EINVAL;
    const int64_t pn = ctx->last_poses * ctx->last_n;
    const int64_t lists = ctx->last_poses * ctx->last_tiles;
    switch (which) {
        case GSR_BUF_RECORDS: *bytes = pn * gsr::kRecordQuads * (int64_t)sizeof(float4); break;
        case GSR_BUF_NTILES: *bytes = pn * (int64_t)sizeof(uint32_t); break;
        case GSR_BUF_OFFSETS: *bytes = (ctx->last_poses ? lists + 1 : 0) * (int64_t)sizeof(uint64_t); break;
        case GSR_BUF_PAIRS: {
            HIPC(ctx, hipDeviceSynchronize());
            uint64_t pairs[kMaxGroups] = {};
            int rc = group_pairs(ctx, pairs);
            if (rc) return rc;
            int64_t total = 0;
            for (int g = 0; g < ctx->n_groups; ++g) total += (int64_t)pairs[g];
            *bytes = total * (int64_t)sizeof(uint32_t);
            break;
        }
        default: return fail(ctx, GSR_EINVAL, "unknown buffer");
    }
    return GSR_OK;
}

int gsr_debug_copy(gsr_ctx *ctx, int which, void *dst, int64_t bytes) {
    if (!ctx || !dst) return GSR_EINVAL;
    int64_t want = 0;
    int rc = gsr_debug_size(ctx, which, &want);
    if (rc) return rc;
    if (bytes != want) return fail(ctx, GSR_EINVAL, "byte count differs from gsr_debug_size");
    if (bytes == 0) return GSR_OK;
    HIPC(ctx, hipDeviceSynchronize());
    if (which == GSR_BUF_RECORDS) {
        HIPC(ctx, hipMemcpy(dst, ctx->records.p, (size_t)bytes, hipMemcpyDeviceToHost));
        return GSR_OK;
    }
    if (which == GSR_BUF_NTILES) {
        // from the visibility masks and the tile rectangles of the visible entries
        const int64_t n = ctx->last_n, P = ctx->last_poses, nr = (n + 63) / 64;
        std::vector<uint64_t> mask((size_t)(P * nr));
        std::vector<uint2> rect((size_t)(P * n));
        HIPC(ctx, hipMemcpy(mask.data(), ctx->vmask.p, mask.size() * sizeof(uint64_t), hipMemcpyDeviceToHost));
        HIPC(ctx, hipMemcpy(rect.data(), ctx->rect.p, rect.size() * sizeof(uint2), hipMemcpyDeviceToHost));
        uint32_t *out = (uint32_t *)dst;
        for (int64_t p = 0; p < P; ++p)
            for (int64_t g = 0; g < n; ++g) {
                const uint2 r = rect[(size_t)(p * n + g)];
                const bool vis = (mask[(size_t)(p * nr + g / 64)] >> (g % 64)) & 1ull;
                out[p * n + g] = vis ? ((r.x >> 16) - (r.x & 0xffffu) + 1u) * ((r.y >> 16) - (r.y & 0xffffu) + 1u) : 0u;
            }
        return GSR_OK;
    }
    // the groups' pair lists laid end to end, and their list offsets shifted to match
    uint64_t pairs[kMaxGroups] = {};
    if ((rc = group_pairs(ctx, pairs))) return rc;
    const uint64_t T = (uint64_t)ctx->last_tiles;
    uint64_t base = 0;
    for (int g = 0; g < ctx->n_groups; ++g) {
        const gsr_ctx::Group &gr = ctx->groups[g];
        if (which == GSR_BUF_PAIRS) {
            HIPC(ctx, hipMemcpy((uint32_t *)dst + base, (const uint32_t *)ctx->sk.p + gr.pairs,
                                pairs[g] * sizeof(uint32_t), hipMemcpyDeviceToHost));
        } else {
            uint64_t *o = (uint64_t *)dst + (uint64_t)gr.p0 * T;
            const uint64_t n_off = (uint64_t)gr.np * T + (g == ctx->n_groups - 1 ? 1 : 0);
            HIPC(ctx, hipMemcpy(o, (const uint64_t *)ctx->offsets.p + gr.off, n_off * sizeof(uint64_t),
                                hipMemcpyDeviceToHost));
            for (uint64_t i = 0; i < n_off; ++i) o[i] += base;
        }
        base += pairs[g];
    }
    return GSR_OK;
}

}  // extern "C"
