// Host runtime and C ABI of libgsr (declared in include/gsr.h).
//
// The context owns a stream binding, device flags and counters, a grow-only
// workspace, and (when profiling) HIP events around the stages. gsr_render
// enqueues: preprocess (screen records, tile counts, per-wave packing of the
// visible Gaussians) -> per-pose depth sort -> scan of the tile counts in depth
// order -> pair emission -> stable bucketing by tile -> blend.
// The pair count is known only on the device after the scan; with
// pair_capacity == 0 the host waits for that one number and sizes the pair
// buffer exactly, otherwise the fixed capacity is used with no host wait and
// an overflow is flagged on the device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gsr.h"
#include "internal.h"

struct gsr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool profile = false;
    std::string err;
    // device flags (int32) and counters (uint64)
    int *d_flags = nullptr;
    unsigned long long *d_counters = nullptr;
    // pinned host staging for small readbacks
    uint64_t *h_pin = nullptr;
    // workspace
    struct Buf {
        void *p = nullptr;
        size_t bytes = 0;
    } records, ntiles, rect, vcount, sort_ka, sort_va, sort_kb, sort_vb, rcnt, roff, nv, vbase, esum, pseg, scan_tmp,
        ptile, pk, sk, cnt, total, block_base, offsets, grey_q, partials;
    // last render
    int64_t last_n = 0, last_poses = 0, last_tiles = 0;
    uint64_t last_capacity = 0;
    int64_t last_pairs = -1;  // known on host in exact mode
    // profiling: event sets of the calls profiled since the last gsr_get_stats
    struct RenderEv {
        hipEvent_t e[4] = {};
    };
    struct NccEv {
        hipEvent_t e[2] = {};
    };
    std::vector<RenderEv> ev_render;
    std::vector<NccEv> ev_ncc;
    size_t n_ev_render = 0, n_ev_ncc = 0;
};

struct gsr_submap {
    gsr_ctx *ctx = nullptr;
    int device = 0;
    int64_t n = 0, cap = 0;
    float4 *packed = nullptr;  // [cap * kPackedQuads]
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

// Grow-only device buffer.
int ensure(gsr_ctx *ctx, gsr_ctx::Buf &b, size_t bytes, const char *name) {
    if (bytes <= b.bytes) return GSR_OK;
    if (b.p) {
        HIPC(ctx, hipStreamSynchronize(ctx->stream));
        HIPC(ctx, hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes + bytes / 4 + 256;
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

extern "C" {

const char *gsr_status_string(int status) {
    switch (status) {
        case GSR_OK: return "ok";
        case GSR_EINVAL: return "invalid argument";
        case GSR_ENOMEM: return "out of memory";
        case GSR_EHIP: return "HIP runtime error";
        case GSR_ENODEV: return "no such device";
        case GSR_EOVERFLOW: return "pair buffer overflow";
        case GSR_EUNSUPPORTED: return "unsupported by this build";
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
    return GSR_OK;
}

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
        if (hipHostMalloc(&ctx->h_pin, 64, hipHostMallocDefault) != hipSuccess) { rc = GSR_ENOMEM; break; }
        if (hipMemset(ctx->d_flags, 0, gsr::FLAG_COUNT * sizeof(int)) != hipSuccess) { rc = GSR_EHIP; break; }
        if (hipMemset(ctx->d_counters, 0, gsr::CNT_COUNT * sizeof(unsigned long long)) != hipSuccess) { rc = GSR_EHIP; break; }
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
    gsr_ctx::Buf *bufs[] = {&ctx->records, &ctx->ntiles,  &ctx->rect,     &ctx->vcount,  &ctx->sort_ka,
                            &ctx->sort_va, &ctx->sort_kb, &ctx->sort_vb,  &ctx->rcnt,    &ctx->roff,    &ctx->nv,
                            &ctx->vbase,   &ctx->esum,    &ctx->pseg,     &ctx->scan_tmp, &ctx->ptile,
                            &ctx->pk,      &ctx->sk,      &ctx->cnt,      &ctx->total,   &ctx->block_base,
                            &ctx->offsets, &ctx->grey_q,  &ctx->partials};
    for (auto *b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (ctx->d_flags) (void)hipFree(ctx->d_flags);
    if (ctx->d_counters) (void)hipFree(ctx->d_counters);
    if (ctx->h_pin) (void)hipHostFree(ctx->h_pin);
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
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete nsm;
            return fail(ctx, GSR_ENOMEM, "submap allocation failed");
        }
        if (sm) gsr_submap_free(sm);
        sm = nsm;
        *out = sm;
    }
    sm->n = n_sel;
    gsr::launch_pack(ctx->stream, n_map, means, scales, quats, opacity, rgb, index, n_sel, sm->packed, ctx->d_flags);
    return check_launch(ctx, "pack");
}

int gsr_submap_free(gsr_submap *sm) {
    if (!sm) return GSR_EINVAL;
    // hipFree waits for work on the device that may still read the submap
    (void)hipSetDevice(sm->device);
    if (sm->packed) (void)hipFree(sm->packed);
    delete sm;
    return GSR_OK;
}

int64_t gsr_submap_size(const gsr_submap *sm) { return sm ? sm->n : -1; }

int gsr_render(gsr_ctx *ctx, const gsr_submap *sm, const gsr_camera *cam, const float *poses, int32_t n_poses,
               const gsr_render_cfg *cfg_in, float *rgb, float *depth, float *tfinal) {
    if (!ctx) return GSR_EINVAL;
    if (!sm || !cam || !poses || !rgb || !depth) return fail(ctx, GSR_EINVAL, "null argument");
    if (sm->ctx != ctx) return fail(ctx, GSR_EINVAL, "submap belongs to another context");
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
    if (!pow2(cfg.tile_w) || !pow2(cfg.tile_h) || (cfg.flags & ~GSR_RENDER_COUNT_EVALS) != 0 ||
        cfg.pair_capacity < 0)
        return fail(ctx, GSR_EINVAL, "bad render configuration");
    if (cfg.tile_w != 16 || cfg.tile_h != 16) return fail(ctx, GSR_EUNSUPPORTED, "this build renders 16x16 tiles");
    if (!(cfg.alpha_min > 0.f) || !(cfg.alpha_max <= 1.f) || !(cfg.alpha_min < cfg.alpha_max) ||
        !(cfg.t_min > 0.f) || !(cfg.cutoff_d2 > 0.f) || !(cfg.eps_dilate >= 0.f))
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

    const int64_t n = sm->n;
    const int64_t P = n_poses;
    const uint64_t n_lists = (uint64_t)P * tg.n_tiles;
    if (tg.n_tiles > gsr::kMaxTilesPerPose)
        return fail(ctx, GSR_EUNSUPPORTED, "more than 16384 tiles per image");
    if (n_lists >= 0xffffffffull) return fail(ctx, GSR_EINVAL, "poses x tiles must be below 2^32");
    if ((uint64_t)P * (uint64_t)n >= 0xffffffffull)
        return fail(ctx, GSR_EINVAL, "poses x submap size must be below 2^32");
    const uint64_t pn = (uint64_t)std::max<int64_t>(1, P * n);
    const uint64_t n_regions = (uint64_t)(n + 63) / 64;
    const uint64_t nvc = std::max<uint64_t>(1, (uint64_t)P * n_regions);  // visible-count entries
    const uint64_t n_rc = gsr::radix_count_elems(n, n_poses);
    int rc;
    if ((rc = ensure(ctx, ctx->records, pn * gsr::kRecordQuads * sizeof(float4), "records")) ||
        (rc = ensure(ctx, ctx->ntiles, pn * sizeof(uint32_t), "ntiles")) ||
        (rc = ensure(ctx, ctx->rect, pn * sizeof(uint2), "tile rectangles")) ||
        (rc = ensure(ctx, ctx->vcount, nvc * sizeof(uint32_t), "visible counts")) ||
        (rc = ensure(ctx, ctx->sort_ka, pn * sizeof(uint32_t), "depth sort")) ||
        (rc = ensure(ctx, ctx->sort_va, pn * sizeof(uint32_t), "depth sort")) ||
        (rc = ensure(ctx, ctx->sort_kb, pn * sizeof(uint32_t), "depth sort")) ||
        (rc = ensure(ctx, ctx->sort_vb, pn * sizeof(uint32_t), "depth sort")) ||
        (rc = ensure(ctx, ctx->rcnt, n_rc * sizeof(uint32_t), "radix counts")) ||
        (rc = ensure(ctx, ctx->roff, n_rc * sizeof(uint32_t), "radix offsets")) ||
        (rc = ensure(ctx, ctx->nv, (uint64_t)P * sizeof(uint32_t), "pose visible counts")) ||
        (rc = ensure(ctx, ctx->vbase, ((uint64_t)P + 1) * sizeof(uint32_t), "pose bases")) ||
        (rc = ensure(ctx, ctx->esum, (gsr::emit_blocks(pn) + 1) * sizeof(uint64_t), "emission sums")) ||
        (rc = ensure(ctx, ctx->pseg, ((uint64_t)P + 1) * sizeof(uint64_t), "pair segments")) ||
        (rc = ensure(ctx, ctx->scan_tmp, gsr::scan_tmp_elems(std::max(pn, n_lists)) * sizeof(uint64_t),
                     "scan")) ||
        (rc = ensure(ctx, ctx->offsets, (n_lists + 1) * sizeof(uint64_t), "offsets")) ||
        (rc = ensure(ctx, ctx->total, n_lists * sizeof(uint32_t), "list totals")) ||
        (rc = ensure(ctx, ctx->block_base, ((uint64_t)P + 1) * sizeof(uint32_t), "block bases")))
        return rc;
    hipStream_t s = ctx->stream;
    uint32_t *ntiles = (uint32_t *)ctx->ntiles.p;
    uint32_t *sort_kb = (uint32_t *)ctx->sort_kb.p, *sort_vb = (uint32_t *)ctx->sort_vb.p;
    uint32_t *vbase = (uint32_t *)ctx->vbase.p;
    uint32_t *roff = (uint32_t *)ctx->roff.p;
    uint64_t *esum = (uint64_t *)ctx->esum.p;  // scanned block sums; the pair total at [emit_blocks]
    const uint64_t n_eb = gsr::emit_blocks(pn);
    uint64_t *pseg = (uint64_t *)ctx->pseg.p;
    uint64_t *scan_tmp = (uint64_t *)ctx->scan_tmp.p;
    const float4 *records = (const float4 *)ctx->records.p;
    uint64_t *offsets = (uint64_t *)ctx->offsets.p;
    int tile_bits = 1;
    while ((1 << tile_bits) < tg.n_tiles) ++tile_bits;

    gsr_ctx::RenderEv *ev = nullptr;
    if (ctx->profile) {
        if ((rc = next_events(ctx, ctx->ev_render, ctx->n_ev_render, &ev))) return rc;
        HIPC(ctx, hipEventRecord(ev->e[0], s));
    }
    gsr::launch_fill_u64(s, ctx->d_counters, gsr::CNT_COUNT, 0ull);
    gsr::launch_preprocess(s, sm->packed, n, poses, n_poses, c, k, tg, (float4 *)ctx->records.p, ntiles,
                           (uint2 *)ctx->rect.p, sort_kb, sort_vb, (uint32_t *)ctx->vcount.p);
    if ((rc = check_launch(ctx, "preprocess"))) return rc;
    if (ev) HIPC(ctx, hipEventRecord(ev->e[1], s));
    // S2-S3: per-pose depth order of the visible Gaussians, then pair offsets in that order
    gsr::launch_depth_sort(s, n, n_poses, (const uint32_t *)ctx->vcount.p, ntiles, (uint32_t *)ctx->sort_ka.p,
                           (uint32_t *)ctx->sort_va.p, sort_kb, sort_vb, (uint32_t *)ctx->rcnt.p, roff,
                           (uint32_t *)ctx->nv.p, vbase);
    gsr::launch_emit_sums(s, sort_kb, vbase, n_poses, pn, esum);
    gsr::launch_block_scan(s, esum, n_eb, nullptr, esum + n_eb);
    if ((rc = check_launch(ctx, "depth sort"))) return rc;

    uint64_t capacity;
    if (cfg.pair_capacity == 0) {
        HIPC(ctx, hipMemcpyAsync(ctx->h_pin, esum + n_eb, sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        HIPC(ctx, hipStreamSynchronize(s));
        capacity = ctx->h_pin[0];
        ctx->last_pairs = (int64_t)capacity;
    } else {
        capacity = (uint64_t)cfg.pair_capacity;
        ctx->last_pairs = -1;
    }
    if (capacity >= 0xffffffffull) return fail(ctx, GSR_EINVAL, "pair count must be below 2^32");
    const uint64_t cap1 = std::max<uint64_t>(1, capacity);
    const uint64_t nbm = gsr::bucket_blocks_max(capacity, n_poses);
    if ((rc = ensure(ctx, ctx->ptile, cap1 * sizeof(uint16_t), "pair tiles")) ||
        (rc = ensure(ctx, ctx->pk, cap1 * sizeof(uint32_t), "pair indices")) ||
        (rc = ensure(ctx, ctx->sk, cap1 * sizeof(uint32_t), "list indices")) ||
        (rc = ensure(ctx, ctx->cnt, nbm * tg.n_tiles * sizeof(uint32_t), "bucket counts")))
        return rc;
    uint16_t *ptile = (uint16_t *)ctx->ptile.p;
    uint32_t *pk = (uint32_t *)ctx->pk.p, *sk = (uint32_t *)ctx->sk.p;
    gsr::launch_pair_segments(s, sort_kb, vbase, n_poses, esum, pn, capacity, pseg);
    gsr::launch_emit(s, sort_kb, sort_vb, vbase, n_poses, (const uint2 *)ctx->rect.p, n, pn, esum, tg, ptile, pk,
                     capacity, ctx->d_flags);
    // S3-S4: stable bucketing by tile keeps the depth order inside every list
    gsr::launch_bucket(s, ptile, pk, pseg, n_poses, capacity, tg.n_tiles, tile_bits, (uint32_t *)ctx->block_base.p,
                       (uint32_t *)ctx->cnt.p, (uint32_t *)ctx->total.p, offsets, scan_tmp, sk);
    if ((rc = check_launch(ctx, "pair sort"))) return rc;
    if (ev) HIPC(ctx, hipEventRecord(ev->e[2], s));
    gsr::launch_blend(s, records, n, n_poses, sk, offsets, capacity, c, k, tg, rgb, depth, tfinal,
                      (cfg.flags & GSR_RENDER_COUNT_EVALS) != 0, ctx->d_counters);
    if ((rc = check_launch(ctx, "blend"))) return rc;
    if (ev) HIPC(ctx, hipEventRecord(ev->e[3], s));

    ctx->last_n = n;
    ctx->last_poses = P;
    ctx->last_tiles = tg.n_tiles;
    ctx->last_capacity = capacity;
    return GSR_OK;
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

int gsr_topk(gsr_ctx *ctx, const float *scores, int32_t n_poses, int32_t k, int32_t *idx) {
    if (!ctx) return GSR_EINVAL;
    if (!scores || !idx) return fail(ctx, GSR_EINVAL, "null argument");
    if (n_poses < 1 || n_poses > 8192 || k < 1 || k > n_poses) return fail(ctx, GSR_EINVAL, "need 1 <= k <= P <= 8192");
    HIPC(ctx, hipSetDevice(ctx->device));
    gsr::launch_topk(ctx->stream, scores, n_poses, k, idx);
    return check_launch(ctx, "topk");
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
    if (ctx->last_poses > 0) {
        uint32_t nv = 0;
        HIPC(ctx, hipMemcpy(&nv, (uint32_t *)ctx->vbase.p + ctx->last_poses, sizeof(nv), hipMemcpyDeviceToHost));
        out->n_visible = (int64_t)nv;
        uint64_t v = 0;
        const uint64_t pn = (uint64_t)std::max<int64_t>(1, ctx->last_poses * ctx->last_n);
        HIPC(ctx, hipMemcpy(&v, (uint64_t *)ctx->esum.p + gsr::emit_blocks(pn), sizeof(v), hipMemcpyDeviceToHost));
        out->n_pairs = (int64_t)v;
    }
    out->overflow = flags[gsr::FLAG_OVERFLOW];
    out->bad_index = flags[gsr::FLAG_BAD_INDEX];
    out->evals_contrib = (int64_t)cnt[gsr::CNT_EVALS_CONTRIB];
    out->evals_lanes = (int64_t)cnt[gsr::CNT_EVALS_LANES];
    double sum[4] = {0, 0, 0, 0};
    for (size_t i = 0; i < ctx->n_ev_render; ++i) {
        const auto &r = ctx->ev_render[i];
        for (int st = 0; st < 3; ++st) {
            float ms = 0.f;
            HIPC(ctx, hipEventElapsedTime(&ms, r.e[st], r.e[st + 1]));
            sum[st] += ms;
        }
    }
    for (size_t i = 0; i < ctx->n_ev_ncc; ++i) {
        float ms = 0.f;
        HIPC(ctx, hipEventElapsedTime(&ms, ctx->ev_ncc[i].e[0], ctx->ev_ncc[i].e[1]));
        sum[3] += ms;
    }
    out->n_profiled_renders = (int32_t)ctx->n_ev_render;
    out->n_profiled_ncc = (int32_t)ctx->n_ev_ncc;
    if (ctx->n_ev_render) {
        out->ms_preprocess = (float)(sum[0] / ctx->n_ev_render);
        out->ms_sort = (float)(sum[1] / ctx->n_ev_render);
        out->ms_blend = (float)(sum[2] / ctx->n_ev_render);
    }
    if (ctx->n_ev_ncc) out->ms_ncc = (float)(sum[3] / ctx->n_ev_ncc);
    ctx->n_ev_render = 0;
    ctx->n_ev_ncc = 0;
    return GSR_OK;
}

int gsr_debug_size(gsr_ctx *ctx, int which, int64_t *bytes) {
    if (!ctx || !bytes) return GSR_EINVAL;
    const int64_t pn = ctx->last_poses * ctx->last_n;
    const int64_t lists = ctx->last_poses * ctx->last_tiles;
    switch (which) {
        case GSR_BUF_RECORDS: *bytes = pn * gsr::kRecordQuads * (int64_t)sizeof(float4); break;
        case GSR_BUF_NTILES: *bytes = pn * (int64_t)sizeof(uint32_t); break;
        case GSR_BUF_OFFSETS: *bytes = (ctx->last_poses ? lists + 1 : 0) * (int64_t)sizeof(uint64_t); break;
        case GSR_BUF_PAIRS: {
            gsr_stats st;
            int rc = gsr_get_stats(ctx, &st);
            if (rc) return rc;
            *bytes = std::min<int64_t>(st.n_pairs, (int64_t)ctx->last_capacity) * (int64_t)sizeof(uint32_t);
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
    HIPC(ctx, hipStreamSynchronize(ctx->stream));
    const void *src = which == GSR_BUF_RECORDS   ? ctx->records.p
                      : which == GSR_BUF_NTILES  ? ctx->ntiles.p
                      : which == GSR_BUF_OFFSETS ? ctx->offsets.p
                                                 : ctx->sk.p;
    HIPC(ctx, hipMemcpy(dst, src, (size_t)bytes, hipMemcpyDeviceToHost));
    return GSR_OK;
}

}  // extern "C"
