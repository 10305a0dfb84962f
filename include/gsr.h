/*
 * gsr.h - C ABI of the MI355X (gfx950) render + NCC hot path of 3DGS-ReLoc
 * (arXiv 2403.11367): render RGB and depth of a cropped 3D Gaussian submap for
 * many candidate camera poses, then score every render against the query image
 * by normalised cross-correlation, on one GPU.
 *
 * Paper passages each call follows:
 *   gsr_submap_load  Sec. III-A (Gaussian parameters mu, S, R = q2R(q), colour,
 *                    opacity; Sigma = R S S^T R^T) and Sec. III-B2 (RGB colour,
 *                    no spherical harmonics; submaps cut from a voxel map).
 *   gsr_render       Sec. III-A, Eq. 1-5: transform by the world-to-camera pose
 *                    W_t, EWA screen covariance (Eq. 3) with the Jacobian of the
 *                    projection (Eq. 4), depth sort, front-to-back compositing of
 *                    colour (Eq. 1) with footprint (Eq. 2) and of depth (Eq. 5).
 *   gsr_ncc          Sec. III-C1, Eq. 10: zero-mean normalised cross-correlation
 *                    between the query and each render.
 *   gsr_topk         Sec. III-C1: the brute-force search keeps the most similar
 *                    render(s).
 *   gsr_crop         Sec. III-B2 / III-C1: 2D voxel grid with a hash per cell and
 *                    a KD-tree over cell centres answering a radius query around
 *                    the prior pose (host code; not on the timed path).
 *
 * Conventions (readings of points the paper leaves open):
 *   - pose = world-to-camera [R | t], 3x4 row-major float32; OpenCV camera axes
 *     (x right, y down, z forward); pixel (i, j) is sampled at (i+0.5, j+0.5).
 *   - Eq. 2 footprint q = o * exp(-d^2/2) (normalisation factor read as 1);
 *     screen covariance dilated by eps on the diagonal; a pair contributes only
 *     where d^2 <= cutoff_d2, alpha = min(alpha_max, q) >= alpha_min; a pixel
 *     stops after the layer that takes its transmittance below t_min (that layer
 *     counts). Background 0. Depth is camera-space z of the mean, not divided
 *     by coverage. Near plane: cull unless t_z > z_near.
 *   - Grey for NCC = 0.299 R + 0.587 G + 0.114 B; NCC = 0 if either image has
 *     zero variance.
 *
 * Memory and ownership: every pointer argument named *_dev is device memory
 * owned by the caller (e.g. a torch tensor's data_ptr()); *_host is host
 * memory owned by the caller. The library owns the context, the submap copy
 * and its workspace. All calls enqueue on the context's stream and return
 * without waiting for the device, except where noted. Argument errors are
 * returned at once; device-side conditions (pair-buffer overflow, bad submap
 * index) are raised as flags and reported by gsr_sync / gsr_get_stats.
 *
 * Threading: a context belongs to one host thread at a time. Calls on two
 * contexts may run concurrently.
 */
#ifndef GSR_H
#define GSR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes: 0 = success, negative = error. */
#define GSR_OK 0
#define GSR_EINVAL (-1)       /* bad argument (null pointer, size, layout) */
#define GSR_ENOMEM (-2)       /* device or host allocation failed */
#define GSR_EHIP (-3)         /* a HIP runtime call failed; see gsr_last_error */
#define GSR_ENODEV (-4)       /* no usable GPU / bad device ordinal */
#define GSR_EOVERFLOW (-5)    /* fixed pair capacity exceeded in a render */
#define GSR_EUNSUPPORTED (-6) /* valid request this library does not implement */
#define GSR_EDEVICE (-7)      /* device-side check failed (e.g. index out of range) */

typedef struct gsr_ctx gsr_ctx;
typedef struct gsr_submap gsr_submap;
typedef struct gsr_graph gsr_graph;

/* Pinhole intrinsics K (Sec. III-A): image width x height in pixels, focal
 * lengths and principal point in pixels. 1 <= width, height <= 32768. */
typedef struct {
    int32_t width, height;
    float fx, fy, cx, cy;
} gsr_camera;

/* Render constants. gsr_default_cfg fills the defaults given in brackets. */
typedef struct {
    int32_t tile_w, tile_h;  /* screen tile in pixels [16, 16]: 16 x 16, 32 x 8 or 8 x 32 (else
                              * GSR_EUNSUPPORTED); the tile lists and so the images depend on it
                              * within float32 rounding of the compositing */
    float eps_dilate;        /* screen-covariance dilation, px^2 [0.3] */
    float z_near;            /* near plane, metres, >= 0; cull unless t_z > z_near [0.2] */
    float jac_clamp;         /* Jacobian point clamp, x of half field of view [1.3] */
    float cutoff_d2;         /* footprint support d^2 <= cutoff_d2 [9] */
    float alpha_min;         /* skip layers with alpha < alpha_min [float32(1/255)] */
    float alpha_max;         /* alpha = min(alpha_max, q) [0.99] */
    float t_min;             /* stop after transmittance drops below t_min [1e-4] */
    int32_t flags;           /* GSR_RENDER_* bits [0] */
    int64_t pair_capacity;   /* (Gaussian, tile) pair buffer of each pose group: 0 = size
                              * exactly, with one host wait per gsr_render for the pair
                              * counts; > 0 = fixed capacity per group, no host wait; an
                              * overflow leaves the images undefined and is reported by
                              * gsr_sync as GSR_EOVERFLOW */
    int32_t pose_groups;     /* the poses are rendered in this many groups, in [1, 8]; 0 =
                              * automatic (one group) [0]. Each group orders its pairs and
                              * then composites on a stream of its own (the context's
                              * stream for the first), concurrently with the other groups;
                              * the images do not depend on the grouping */
    int32_t blend_blocks_per_cu; /* compositing launch: 0 = one block per (pose, tile) [0];
                              * 1..64 = persistent: this many blocks per compute unit take
                              * (pose, tile) items from a work queue until it is empty.
                              * The images do not depend on it */
    int32_t blend_chunk;     /* records staged in LDS per compositing step: 0 = 252 [0];
                              * 252, 124 or 60 (shorter steps stop sooner on short lists).
                              * The images do not depend on it */
} gsr_render_cfg;

/* gsr_render_cfg.flags: count compositing work into gsr_stats (evals_*), for
 * measurement; a slower kernel variant, same images. */
#define GSR_RENDER_COUNT_EVALS 1
/* gsr_render_cfg.flags: keep the compositing state of every tile list longer
 * than 2016 records (each pixel's transmittance, colour and depth sums before
 * list positions 2016, 4032, ...) for a following gsr_render_backward, which
 * then walks such a list as independent segments instead of one serial walk.
 * Same images. The states take 5 KB per 2016 records of pair capacity (context
 * memory, kept until the next render). Not with GSR_RENDER_COUNT_EVALS (else
 * GSR_EUNSUPPORTED); blend_chunk must be 0 or 252 (else GSR_EUNSUPPORTED);
 * blend_blocks_per_cu is not used (grid launch). */
#define GSR_RENDER_KEEP_STATE 2
/* gsr_render_cfg.flags: with a fixed pair_capacity, wait after the render for
 * the device's overflow flag and, if the capacity was exceeded, render again with
 * the pair buffers sized exactly (gsr_stats.overflow_retried = 1); the images are
 * then those of an exact render. Two host waits per render; refused under graph
 * capture (GSR_EUNSUPPORTED). An overflow of an earlier render that gsr_sync has
 * not yet reported makes the call fail with GSR_EOVERFLOW. */
#define GSR_RENDER_RETRY_OVERFLOW 4

/* Counters of the most recent gsr_render / gsr_ncc on the context. */
typedef struct {
    int64_t n_submap;        /* Gaussians in the rendered submap */
    int64_t n_poses;         /* poses of the last render */
    int64_t n_visible;       /* (pose, Gaussian) records that survived culling */
    int64_t n_pairs;         /* (pose, Gaussian, tile) pairs */
    int64_t pair_capacity;   /* pair buffer size used */
    int64_t evals_contrib;   /* with GSR_RENDER_COUNT_EVALS: (pixel, Gaussian) pairs that
                              * contributed to a pixel before it stopped */
    int64_t evals_lanes;     /* with GSR_RENDER_COUNT_EVALS: lane slots spent on evaluations */
    int32_t overflow;        /* 1 if the pair buffer overflowed */
    int32_t bad_index;       /* 1 if gsr_submap_load saw an index out of range */
    /* Stage times from HIP events recorded on the stream each stage runs on, when
     * profiling is on: means over the calls profiled since the previous
     * gsr_get_stats. Groups overlap, so ms_render is less than the sum. */
    int32_t n_profiled_renders;
    int32_t n_profiled_ncc;
    float ms_preprocess;     /* counter reset + preprocess, per render */
    float ms_sort;           /* ordering of one pose group (depth sort, emission, bucketing) */
    float ms_blend;          /* one compositing launch (one pose group) */
    float ms_ncc;            /* whole gsr_ncc */
    float ms_render;         /* whole gsr_render, first launch to the join */
    int32_t n_groups;        /* pose groups of the last render */
    int64_t render_serial;   /* renders made on this context so far (gsr_render_backward
                              * differentiates the latest) */
    int64_t n_culled_nonfinite; /* Gaussians of the rendered submap(s), as last loaded, with a
                              * non-finite mean, covariance, opacity or colour entry: culled
                              * at every pose (summed over the submaps of a batched render) */
    int64_t workspace_bytes; /* device memory the context's workspace holds */
    int32_t overflow_retried; /* 1 if the last render overflowed its fixed capacity and was
                              * rendered again (GSR_RENDER_RETRY_OVERFLOW) */
} gsr_stats;

/* Create a context on GPU `device`, enqueueing on `hip_stream` (a hipStream_t;
 * NULL = the null stream). Returns GSR_ENODEV if the device is absent. */
int gsr_create(gsr_ctx **out, int device, void *hip_stream);
/* Waits for the context's stream, then frees the context and its workspace.
 * Submaps must be freed first. */
int gsr_destroy(gsr_ctx *ctx);
/* Switch the stream later calls enqueue on. */
int gsr_set_stream(gsr_ctx *ctx, void *hip_stream);
/* Limit the device memory the context's grow-only workspace may hold, in bytes
 * (0 = no limit, the default). A call whose workspace would pass it fails with
 * GSR_ENOMEM and allocates nothing; submaps and static scratch are not counted. */
int gsr_set_workspace_limit(gsr_ctx *ctx, int64_t bytes);
/* 1 = record HIP events around the stages of gsr_render / gsr_ncc. */
int gsr_set_profiling(gsr_ctx *ctx, int on);
/* Fill `out` with the default constants (see gsr_render_cfg). */
int gsr_default_cfg(gsr_render_cfg *out);

/* Pack a submap on the device (Sec. III-A): for i in [0, n_sel), Gaussian
 * src = index_dev ? index_dev[i] : i of the caller's map is normalised
 * (quaternion), turned into Sigma = R diag(s)^2 R^T and stored with its mean,
 * opacity and colour in a library-owned record.
 *   n_map                  Gaussians in the caller's arrays
 *   means_dev   [n_map,3]  float32 world positions
 *   scales_dev  [n_map,3]  float32 linear scales (> 0)
 *   quats_dev   [n_map,4]  float32 rotation quaternions (w, x, y, z), any nonzero norm
 *   opacity_dev [n_map]    float32 opacities in (0, 1] (post-sigmoid)
 *   rgb_dev     [n_map,3]  float32 colours
 *   index_dev   [n_sel]    int64 indices into the map, or NULL (then n_sel == n_map);
 *                          the index order is the submap order (ties in depth sort by
 *                          submap position). Out-of-range entries raise bad_index.
 * If *out is a submap of this context with capacity >= n_sel it is refilled in
 * place without allocating; otherwise a new submap is allocated and *out set.
 * The inputs are only read by work enqueued here: the caller may free them
 * once the stream has passed this call. */
int gsr_submap_load(gsr_ctx *ctx, int64_t n_map, const float *means_dev, const float *scales_dev,
                    const float *quats_dev, const float *opacity_dev, const float *rgb_dev,
                    const int64_t *index_dev, int64_t n_sel, gsr_submap **out);
/* gsr_submap_load from host memory (Sec. III-B2: the submap retrieved around the
 * prior is uploaded once per query): the same arguments, with every array in host
 * memory, copied into a context staging buffer and packed. Waits until the
 * packing is done, so the caller may free or reuse the inputs on return. Refused
 * under graph capture (GSR_EUNSUPPORTED). */
int gsr_submap_load_host(gsr_ctx *ctx, int64_t n_map, const float *means_host, const float *scales_host,
                         const float *quats_host, const float *opacity_host, const float *rgb_host,
                         const int64_t *index_host, int64_t n_sel, gsr_submap **out);
int gsr_submap_free(gsr_submap *sm);
int64_t gsr_submap_size(const gsr_submap *sm);

/* Render the submap at P poses (Sec. III-A, Eq. 1-5). P x tiles < 2^32.
 *   poses_dev  [P,3,4]  float32 world-to-camera [R | t], device memory
 *   rgb_dev    [P,3,H,W] float32 output, planar colour
 *   depth_dev  [P,H,W]   float32 output, Eq. 5 depth
 *   tfinal_dev [P,H,W]   float32 output, final transmittance, or NULL
 * cfg may be NULL (defaults). 1 <= P <= 65535. */
int gsr_render(gsr_ctx *ctx, const gsr_submap *sm, const gsr_camera *cam, const float *poses_dev,
               int32_t n_poses, const gsr_render_cfg *cfg, float *rgb_dev, float *depth_dev,
               float *tfinal_dev);

/* Gradient of a loss through the most recent render of this context, given the
 * gradients of its images (Sec. III-A, Eq. 1-5, differentiated; the map-training
 * side of the paper). That render must be a gsr_render of `sm` at these poses, with
 * no render and no reload of sm since; sm must be loaded without an index, so that
 * submap entry g is input Gaussian g. The contributing set of every pixel (support
 * cutoff, alpha floor, stop after t_min) is taken as fixed; where alpha is clamped at
 * alpha_max it is constant. Per-pixel transmittance is recomputed front to back
 * with the forward's arithmetic, not stored; if the render had
 * GSR_RENDER_KEEP_STATE, each 2016-record segment of a long list starts from the
 * state the forward kept there (equal, bit for bit, to the serial walk's state).
 *   scales_dev [n,3], quats_dev [n,4]: the arrays sm was loaded from
 *   poses_dev  [P,3,4]: the render's poses
 *   rgb_dev, depth_dev: the render's images [P,3,H,W], [P,H,W]
 *   grad_rgb_dev, grad_depth_dev: dL/d images, same shapes
 *   outputs dL/d means [n,3], scales [n,3] (linear), quats [n,4] (raw, before
 *   normalisation), opacity [n] (after the sigmoid), rgb [n,3].
 * Gradients are summed with float atomics across pixels: the last bits vary from
 * run to run. */
int gsr_render_backward(gsr_ctx *ctx, const gsr_submap *sm, const float *scales_dev, const float *quats_dev,
                        const float *poses_dev, int32_t n_poses, const float *rgb_dev, const float *depth_dev,
                        const float *grad_rgb_dev, const float *grad_depth_dev, float *grad_means_dev,
                        float *grad_scales_dev, float *grad_quats_dev, float *grad_opacity_dev, float *grad_rgb_out_dev);

/* A batch of queries in one render: submap q is rendered at poses_per_submap[q]
 * consecutive poses (Sec. III-C1 for several queries at once, each with its own
 * submap), with one launch per stage for all of them. 1 <= n_submaps <= 16,
 * poses_per_submap[q] >= 1, total P <= 65535; poses_dev [P,3,4] in submap order;
 * rgb_dev / depth_dev / tfinal_dev as for gsr_render with P images. The images
 * are those of separate gsr_render calls, bit for bit. Record slots are laid out
 * per pose for the largest submap (P x max n < 2^32); gsr_debug_* then report
 * that layout. */
int gsr_render_multi(gsr_ctx *ctx, const gsr_submap *const *submaps, const int32_t *poses_per_submap,
                     int32_t n_submaps, const gsr_camera *cam, const float *poses_dev, const gsr_render_cfg *cfg,
                     float *rgb_dev, float *depth_dev, float *tfinal_dev);

/* HIP graph capture of the context's stream. Between gsr_capture_begin and
 * gsr_capture_end the calls of this context are recorded, not run; the graph
 * then replays them with one launch. Rules: the stream must not be the null
 * stream; renders need a fixed pair_capacity (no host wait); every workspace
 * must already be large enough (run the same calls once before capturing),
 * else the call fails with GSR_EINVAL; profiling is off; the library records no
 * memset into the graph. A replay reads the inputs and writes the outputs at the
 * addresses given during capture. gsr_graph_launch enqueues on the context's
 * current stream. */
int gsr_capture_begin(gsr_ctx *ctx);
int gsr_capture_end(gsr_ctx *ctx, gsr_graph **out);
int gsr_graph_launch(gsr_graph *graph);
/* Waits for the context's stream and frees the graph. */
int gsr_graph_destroy(gsr_graph *graph);

/* NCC (Eq. 10) of the query against each of P renders, on grey images.
 *   query_dev   [3,H,W]   float32 planar RGB
 *   renders_dev [P,3,H,W] float32 planar RGB
 *   scores_dev  [P]       float32 output in [-1, 1] */
int gsr_ncc(gsr_ctx *ctx, const float *query_dev, const float *renders_dev, int32_t n_poses,
            int32_t height, int32_t width, float *scores_dev);

/* gsr_ncc without any allocation, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and scores, with the grey query and the per-block partial sums in
 * a static device array of 8 MiB per device (each device holds its copy until the
 * process ends) instead of the context's workspace. It calls no hipMalloc or
 * hipFree and records no profiling events. Sizes whose scratch,
 * 4 H W (rounded up to 256 B) + 48 P ceil(H W / 4096) bytes, exceeds 8 MiB are
 * refused with GSR_EINVAL (1408 x 376 fits up to about 1000 renders per call).
 * Every call on a device shares that device's array: calls that overlap on one
 * device, from any context or stream, race. Arguments as gsr_ncc. */
int gsr_ncc_noalloc(gsr_ctx *ctx, const float *query_dev, const float *renders_dev, int32_t n_poses,
                    int32_t height, int32_t width, float *scores_dev);

/* Indices of the k best scores, best first; ties go to the lower index
 * (Sec. III-C1 keeps the most similar render). 1 <= k <= P <= 8192.
 *   scores_dev [P] float32, idx_dev [k] int32 output. */
int gsr_topk(gsr_ctx *ctx, const float *scores_dev, int32_t n_poses, int32_t k, int32_t *idx_dev);

/* Random-order candidate search with an early stop (Sec. IV, initial
 * relocalisation: a random search over the first share of the candidates that
 * stops on an NCC criterion; read here as "the best NCC so far reaches
 * `threshold`"). Candidates are rendered and scored in the order given, `batch`
 * at a time; the search stops after the first batch whose best score is >=
 * threshold, or once `max_eval` candidates are scored (e.g. 20% of P). One host
 * wait per batch.
 *   poses_dev  [P,3,4] float32, as for gsr_render
 *   order_host [P] int32, a permutation of [0, P) (the random order, drawn by the caller)
 *   query_dev  [3,H,W] float32; cfg as for gsr_render (NULL = defaults)
 *   scores_dev [P] float32: the NCC of every scored candidate is written at its
 *              index; entries of unscored candidates are left as they were
 *   best / best_score: the best scored candidate (ties: lowest index) and its NCC
 *   n_scored: candidates scored (a multiple of batch, or max_eval)
 * Renders go to library-owned buffers of `batch` images.
 * Errors: GSR_EINVAL for null pointers, 1 <= max_eval <= P <= 65535 or batch < 1
 * violated, a NaN threshold, or an order that is not a permutation. */
int gsr_search(gsr_ctx *ctx, const gsr_submap *sm, const gsr_camera *cam, const float *poses_dev,
               int32_t n_poses, const int32_t *order_host, int32_t batch, int32_t max_eval, float threshold,
               const float *query_dev, const gsr_render_cfg *cfg, float *scores_dev, int32_t *best,
               float *best_score, int32_t *n_scored);

/* Wait for the context's stream. Returns GSR_EOVERFLOW / GSR_EDEVICE if a
 * device-side flag was raised since the last gsr_sync (and clears it). */
int gsr_sync(gsr_ctx *ctx);
/* Wait for the stream and read the counters of the last render / ncc, and the
 * mean stage times of the calls profiled since the previous call. */
int gsr_get_stats(gsr_ctx *ctx, gsr_stats *out);

/* Introspection of the last gsr_render for tests (waits for the stream, then
 * copies a library buffer to host memory `dst_host` of `bytes` bytes, which
 * must equal the size reported by gsr_debug_size). Buffers:
 *   GSR_BUF_RECORDS    [P][N][12] float32 screen records: u, v, conic A, B, C,
 *                      opacity, r, g, b, z, rect_x = i0 | i1 << 16,
 *                      rect_y = j0 | j1 << 16 (the last two as uint32 bits);
 *                      valid where the tile count is nonzero
 *   GSR_BUF_NTILES     [P][N] uint32 tiles touched (0 = culled)
 *   GSR_BUF_OFFSETS    [P*T + 1] uint64 start of each (pose, tile) list in the
 *                      pair list; the last entry is the pair count
 *   GSR_BUF_PAIRS      [n_pairs] uint32 submap index of each pair; each (pose,
 *                      tile) list is in front-to-back order: ascending depth
 *                      bits, then ascending submap index
 */
#define GSR_BUF_RECORDS 0
#define GSR_BUF_NTILES 1
#define GSR_BUF_OFFSETS 2
#define GSR_BUF_PAIRS 3
int gsr_debug_size(gsr_ctx *ctx, int which, int64_t *bytes);
int gsr_debug_copy(gsr_ctx *ctx, int which, void *dst_host, int64_t bytes);

/* Submap retrieval on the host (Sec. III-B2, III-C1): Gaussians are binned in
 * a 2D grid of `cell`-metre cells keyed by (floor(x/cell), floor(y/cell)) in a
 * hash map; a KD-tree over the occupied cell centres returns the cells whose
 * centre lies within `radius` of (px, py); their Gaussians' indices are written
 * to idx_host in Morton order of their `voxel`-metre 3D voxels (v =
 * floor(coord / voxel) + 2^20 clamped to [0, 2^21 - 1]; x, y, z bit b -> code
 * bit 3b, 3b+1, 3b+2), ties by ascending index; voxel <= 0: ascending index.
 * A spatially coherent submap order keeps the per-tile pair lists local in
 * memory, which gsr_render relies on for speed (any order renders correctly).
 *   means_host [n,3] float32; idx_host [cap] int64 output; *n_out = count
 *   (GSR_EINVAL with *n_out set if cap is too small). Synchronous, no GPU. */
int gsr_crop(const float *means_host, int64_t n, double cell, double px, double py, double radius, double voxel,
             int64_t *idx_host, int64_t cap, int64_t *n_out);

const char *gsr_status_string(int status);
/* Message of the last error on this context (empty if none). */
const char *gsr_last_error(gsr_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* GSR_H */
