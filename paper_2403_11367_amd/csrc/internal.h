// Internal declarations shared by the kernel translation units and the host
// runtime of libgsr. Not part of the public ABI (see include/gsr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "gsr.h"
#include "gsr_scorer.h"

namespace gsr {

// Device flag slots (int32 each), raised by kernels, read and cleared by gsr_sync.
enum : int { FLAG_OVERFLOW = 0, FLAG_BAD_INDEX = 1, FLAG_COUNT = 4 };
// Device counter slots (uint64 each), reset at the start of a render.
// CNT_WIDE_DEPTH: nonzero when some visible depth key reaches 2^kNarrowKeyBits.
enum : int { CNT_EVALS_CONTRIB = 0, CNT_EVALS_LANES = 1, CNT_NONFINITE = 2, CNT_WIDE_DEPTH = 3, CNT_COUNT = 8 };

// Depth keys: float32 depth bits minus the near plane's (the near plane is not
// negative, so every visible depth is positive and keys order like depths).
// Keys below 2^kNarrowKeyBits (depths up to about 2^16 times a positive near
// plane) sort in three 9-bit radix passes; the preprocess flags any larger key
// in CNT_WIDE_DEPTH, and a fourth pass then runs.
constexpr int kNarrowKeyBits = 27;

// Packed submap record: 4 float4 (64 B) per Gaussian.
//   q0 = (mu_x, mu_y, mu_z, opacity)
//   q1 = (S00, S01, S02, S11)        3D covariance, unique entries
//   q2 = (S12, S22, r, g)
//   q3 = (b, 0, 0, 0)
constexpr int kPackedQuads = 4;

// Screen record: 3 float4 (48 B) per (pose, Gaussian).
//   q0 = (u, v, conic A, conic B)    d^2 = A dx^2 + 2 B dx dy + C dy^2
//   q1 = (conic C, opacity, r, g)
//   q2 = (b, z, rect_x bits, rect_y bits)   rect_x = i0 | i1 << 16
constexpr int kRecordQuads = 3;


// XCDs (accelerator complex dies) of the part; workgroups are dealt to them
// round robin by linear id, and each has its own L2.
constexpr uint32_t kXcdCount = 8;

// Tiles per pose the LDS bucketing handles (larger images are rejected).
constexpr int kMaxTilesPerPose = 16384;

struct Camera {
    int width, height;
    float fx, fy, cx, cy;
};

struct Consts {
    float eps;        // screen-covariance dilation
    float z_near;     // near plane
    float jac_clamp;  // Jacobian point clamp (x half field of view)
    float cutoff_d2;  // footprint support
    float alpha_min;
    float alpha_max;
    float t_min;
};

struct TileGrid {
    int tile_w, tile_h;    // 16 x 16, 32 x 8 or 8 x 32
    int log2_w, log2_h;
    int tiles_x, tiles_y;  // tiles per image row / column
    int n_tiles;           // tiles per pose
};

// ---- geometry.hip (strict float32, no contraction) ----
void launch_pack(hipStream_t s, int64_t n_map, const float *means, const float *scales,
                 const float *quats, const float *opacity, const float *rgb, const int64_t *index,
                 int64_t n_sel, float4 *packed, int *flags, unsigned long long *nonfinite);
// The submaps of one render: poses [pose_end[q-1], pose_end[q]) see submap q
// (n[q] Gaussians, packed records). One entry for an ordinary render; up to
// kMaxBatchSubmaps for a batch of queries. Record slots are pose * n_slot + g
// with n_slot = the largest n[q]; slots g >= n[q] of a pose are culled.
constexpr int kMaxBatchSubmaps = 16;
struct SubmapTable {
    int count;
    int pose_end[kMaxBatchSubmaps];
    int64_t n[kMaxBatchSubmaps];
    const float4 *packed[kMaxBatchSubmaps];
    const unsigned long long *nonfinite[kMaxBatchSubmaps];  // per submap: Gaussians culled as non-finite
};
// Adds the non-finite counts of the table's submaps to *total (one launch).
void launch_sum_nonfinite(hipStream_t s, const SubmapTable &tab, unsigned long long *total);
// Blocks of the preprocess grid along the Gaussians.
int64_t preprocess_blocks(int64_t n);
// Screen records and tile rectangles rect[p][g] = (tx0 | tx1 << 16, ty0 | ty1
// << 16) of the visible Gaussians (entries of culled ones are left as they
// were); per pose and 64-Gaussian region, the visibility mask (bit l: Gaussian
// 64 region + l) in vmask[p * ceil(n / 64) + region], and the (depth key, sort
// value) of the visible Gaussians packed at the front of the region's slots of
// vz / vg (P * n each); *wide (a CNT_WIDE_DEPTH counter) is raised when a depth
// key reaches 2^kNarrowKeyBits.
// Sort values: the record slot (pose * n + index) of each visible Gaussian, or,
// where pack_sort_values(n, n_tiles), (index) | (tile count << kPackIndexBits),
// which the depth sort's last pass turns back into the slot and the count.
constexpr int kPackIndexBits = 19;
inline bool pack_sort_values(int64_t n, int n_tiles) {
    return n <= (int64_t(1) << kPackIndexBits) && n_tiles < (1 << (32 - kPackIndexBits));
}
void launch_preprocess(hipStream_t s, const SubmapTable &tab, int64_t n, const float *poses, int n_poses,
                       const Camera &cam, const Consts &k, const TileGrid &tg, float4 *records,
                       uint2 *rect, uint32_t *vz, uint32_t *vg, uint64_t *vmask, bool pack,
                       unsigned long long *wide);
// The depth sort's output (tile counts and record slots, front to back): in the
// "b" buffers after three radix passes, in the "a" buffers after four (when
// *wide is raised).
struct SortedRun {
    const uint32_t *cnt_b, *slot_b, *cnt_a, *slot_a;
    const unsigned long long *wide;
};
// Pair emission in front-to-back order. The depth-sorted visible Gaussians
// (snt: tile counts, sg: record slots p * n + g; pose p owns [vbase[p],
// vbase[p+1]), at most n_max = P * n of them) are cut into nb = emit_blocks(n_max)
// blocks, grouped in spans. The emission sums es (emit_sums_size(n_max) entries):
//   es[b], b < nb:          tile counts of the blocks of b's span before b
//   es[nb]:                 the pair total
//   es[nb + 1]:             the number of spans that hold elements
//   es[nb + 2 + s]:         first pair of span s
//   launch_emit_sums:     all of es (the span sums scanned by launch_block_scan)
//   launch_pair_segments: pseg[p] = min(first pair of pose p, capacity), p in [0, P]
//   launch_emit:          ptile / pk = tile id within the pose / submap index per pair
uint64_t emit_blocks(uint64_t n_max);
uint64_t emit_sums_size(uint64_t n_max);
void launch_emit_sums(hipStream_t s, const SortedRun &run, const uint32_t *vbase, int n_poses, uint64_t n_max,
                      uint64_t *es);
void launch_pair_segments(hipStream_t s, const SortedRun &run, const uint32_t *vbase, int n_poses,
                          const uint64_t *es, uint64_t n_max, uint64_t capacity, uint64_t *pseg);
void launch_emit(hipStream_t s, const SortedRun &run, const uint32_t *vbase, int n_poses,
                 const uint2 *rect, int64_t n, uint64_t n_max, const uint64_t *es, const TileGrid &tg,
                 uint16_t *ptile, uint32_t *pk, uint64_t capacity, int *flags);

// ---- sort.hip ----
void launch_fill_u32(hipStream_t s, uint32_t *p, uint64_t n, uint32_t value);
void launch_fill_u64(hipStream_t s, unsigned long long *p, uint64_t n, unsigned long long value);
// Per-pose stable sort of the visible Gaussians by depth key. Input: the
// preprocess's regions in (kb, vb) with vmask. Output: vb[vbase[p] ..
// vbase[p+1]) = pose p's record slots front to back, kb = their tile counts, or
// the same in (va, ka) when *wide is raised (see SortedRun); vbase[P] = visible
// total; nv[p] = pose p's visible count.
// ka, va, kb, vb hold P * n entries; rcnt and roff radix_count_elems each.
uint64_t radix_blocks_per_pose(int64_t n);
uint64_t radix_count_elems(int64_t n, int n_poses);
// slot0: the first pose's first record slot (record slots are pose * n + index
// over all poses of the render); pack: the values are packed (as the preprocess
// wrote them).
void launch_depth_sort(hipStream_t s, int64_t n, int n_poses, const uint64_t *vmask, const uint2 *rect,
                       uint32_t slot0, bool pack, const unsigned long long *wide, uint32_t *ka, uint32_t *va,
                       uint32_t *kb, uint32_t *vb, uint32_t *rcnt, uint32_t *roff, uint32_t *nv, uint32_t *vbase);
// Exclusive scan of sums[0 .. nb_max) in place (only the first *d_nb with d_nb),
// total to *total. One block.
void launch_block_scan(hipStream_t s, uint64_t *sums, uint64_t nb_max, const uint64_t *d_nb, uint64_t *total);
// Stable sort of the emitted pairs by tile within each pose, in two stable
// passes (coarse buckets of 64 tiles, then tiles within a bucket). Writes the
// per-(pose, tile) list offsets [P*T + 1] and the bucketed indices sk.
// Workspace: block_base P * bucket_coarse(T) + 1 entries, bseg
// bucket_blocks_max(capacity, P, T), cnt bucket_count_elems(capacity, P, T),
// cstart P * bucket_coarse(T) + 1, ctile and cval capacity. n_poses >= 1 and
// n_tiles <= kMaxTilesPerPose.
int bucket_coarse(int n_tiles);
uint64_t bucket_blocks_max(uint64_t capacity, int n_poses, int n_tiles);
uint64_t bucket_count_elems(uint64_t capacity, int n_poses, int n_tiles);
void launch_bucket(hipStream_t s, const uint16_t *ptile, const uint32_t *pk, const uint64_t *pseg, int n_poses,
                   uint64_t capacity, int n_tiles, uint32_t *block_base, uint32_t *bseg, uint32_t *cnt,
                   uint64_t *cstart, uint16_t *ctile, uint32_t *cval, uint64_t *offsets, uint32_t *sk);

// Kept compositing states (see kKeepRecords): keep_off[l] = states of lists j < l,
// l in [0, n_lists], from the list offsets clipped to the capacity. One block.
void launch_keep_offsets(hipStream_t s, const uint64_t *offsets, uint64_t capacity, uint32_t n_lists,
                         uint32_t *keep_off);
// items[b] = list of backward block b: list l owns blocks l + keep_off[l] ..
// l + keep_off[l + 1] (one per segment).
void launch_keep_items(hipStream_t s, const uint32_t *keep_off, uint32_t n_lists, uint32_t *items);

// ---- blend.hip ----
// With keep_off (GSR_RENDER_KEEP_STATE): the 252-record grid launch that also
// writes the kept compositing states of long lists (see kKeepRecords);
// count_evals, persistent_blocks and chunk are then not used.
void launch_blend(hipStream_t s, const float4 *records, int64_t n, int n_poses, const uint32_t *pairs,
                  const uint64_t *offsets, uint64_t capacity, const Camera &cam, const Consts &k,
                  const TileGrid &tg, float *rgb, float *depth, float *tfinal, bool count_evals,
                  unsigned long long *counters, int persistent_blocks, unsigned int *queue, int chunk,
                  const uint32_t *keep_off, float *keep_state);
// Records per compositing chunk the blend is built for (0 = the default, 252).
bool blend_chunk_supported(int chunk);
// Tile shapes the compositing kernels implement: 16x16, 32x8, 8x32.
bool blend_tile_supported(int tile_w, int tile_h);
// Screen-space gradients per (pose, Gaussian): u, v, conic A, B, C, opacity, r, g, b, z.
constexpr int kScreenGrads = 10;
// Records between kept compositing states of a long tile list (8 chunks of 252):
// the forward with GSR_RENDER_KEEP_STATE stores each pixel's T, colour and depth
// sums [5][256] before list positions kKeepRecords, 2 kKeepRecords, ..., so that
// the backward can walk a long list as several independent segments.
constexpr uint64_t kKeepRecords = 2016;
// Backward of the compositing: adds the screen-space gradients of every (pose,
// Gaussian) pair into gscreen [n_poses, n, kScreenGrads] (which the caller zeroes).
// One block per (list, segment): keep_off [lists + 1] the kept states per list
// (all zero when none were kept), items [max_blocks] the list of each block
// (launch_keep_items), max_blocks at least lists + kept states.
void launch_blend_backward(hipStream_t s, const float4 *records, int64_t n, int n_poses, const uint32_t *pairs,
                           const uint64_t *offsets, uint64_t capacity, const Camera &cam, const Consts &k,
                           const TileGrid &tg, const float *img_rgb, const float *img_depth, const float *g_rgb,
                           const float *g_depth, float *gscreen, const uint32_t *keep_off, const float *keep_state,
                           const uint32_t *items, uint64_t max_blocks);

// ---- ncc.hip ----
int ncc_pixels_per_block();
void launch_ncc(hipStream_t s, const float *query, const float *renders, int n_poses, int height,
                int width, float *grey_q, double *partials, float *scores);
void launch_topk(hipStream_t s, const float *scores, int n, int k, int32_t *idx);
// out[i] = poses[order[i]] (3x4 each), i < nb; scores[order[i]] = batch_scores[i].
void launch_gather_poses(hipStream_t s, const float *poses, const int32_t *order, int nb, float *out);
void launch_scatter_scores(hipStream_t s, const float *batch_scores, const int32_t *order, int nb, float *scores);

// ---- backward.hip ----
// Gradients per (pose, Gaussian) in parameter space (mean 3, covariance entries 6,
// opacity, r, g, b).
int pose_grads_per_gaussian();
void launch_project_backward(hipStream_t s, const float4 *packed, int64_t n, const float *poses, int n_poses,
                             const Camera &cam, const Consts &k, const uint64_t *vmask, const float *gscreen,
                             float *gpose);
void launch_param_grads(hipStream_t s, const float *gpose, int64_t n, int n_poses, const float *scales,
                        const float *quats, float *g_means, float *g_scales, float *g_quats, float *g_opacity,
                        float *g_rgb);

// ---- scorer.hip ----
constexpr int kScorerLayers = 5;
constexpr int kScorerChannels[kScorerLayers + 1] = {2, 32, 64, 64, 128, 128};
constexpr int kScorerStride[kScorerLayers] = {2, 1, 2, 1, 2};
constexpr int kScorerHidden = 128;

// Device buffers of one scorer call. Convolution weights in bf16 are kept in
// two copies indexed like the flat parameters: wt in the parameter layout
// [co][tap][ci], wd in [tap][ci][co]; w_off, b_off, fc_off are offsets into
// the flat parameter vector (fc: W1, b1, w2, b2). act[l] (l = 1..5) holds
// layer l's output [B][h_l][w_l][c_l] in bf16; dbuf[2] are gradient ping-pong
// buffers of the largest activation; part holds part_cap float32 partial sums.
struct ScorerBufs {
    int H, W;
    const uint16_t *x;
    uint16_t *act[kScorerLayers + 1];
    const float *params;
    uint16_t *wt, *wd;
    int64_t w_off[kScorerLayers], b_off[kScorerLayers], fc_off[4];
    float *g, *h, *ds, *dh;  // [B][128] pooled features, hidden units, [B] dscore, [B][128] dhidden
    uint16_t *dbuf[2];
    float *part;
    int64_t part_cap;
};
// dims[l] = (height, width) of the input of layer l (dims[5] = last output).
void scorer_dims(int H, int W, int dims[kScorerLayers + 1][2]);
// out[p] = f x f mean pool of the grey of rgb[p] ([3][H][W] planar).
void launch_pool_grey(hipStream_t s, const float *rgb, int P, int H, int W, int f, float *out);
// Network input x [B][h][w][2] bf16 from renders rgb [B][3][h][w] and the
// pooled query grey q [h][w]; qstats holds 2 floats of scratch.
void launch_scorer_input(hipStream_t s, const float *rgb, int B, int h, int w, const float *q, float *qstats,
                         uint16_t *x);
void launch_scorer_forward(hipStream_t s, const ScorerBufs &b, int B, float *score);
// After launch_scorer_forward on the same buffers: gradient of the mean squared
// error against label[B] into grad (flat parameter layout), the loss into
// loss[0] (or not, if null).
void launch_scorer_backward(hipStream_t s, const ScorerBufs &b, int B, const float *score, const float *label,
                            float *grad, float *loss);
void launch_scorer_weights(hipStream_t s, const ScorerBufs &b);
void launch_adamw(hipStream_t s, float *p, const float *g, float *m, float *v, const uint8_t *decay, int64_t n,
                  float lr, float b1, float b2, float eps, float wd, float bc1, float bc2);

// ---- scorer_rt.cpp ----
// Context, input size and batch limit of a scorer.
void scorer_info(const gsr_scorer *s, gsr_ctx **ctx, int *height, int *width, int *max_batch);

// ---- runtime.cpp: context access for the other host units ----
hipStream_t ctx_stream(gsr_ctx *ctx);
int ctx_device(gsr_ctx *ctx);
int ctx_fail(gsr_ctx *ctx, int code, const char *msg);
int ctx_hip_fail(gsr_ctx *ctx, hipError_t e, const char *what);

}  // namespace gsr
