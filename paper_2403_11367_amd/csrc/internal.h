// Internal declarations shared by the kernel translation units and the host
// runtime of libgsr. Not part of the public ABI (see include/gsr.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace gsr {

// Device flag slots (int32 each), raised by kernels, read and cleared by gsr_sync.
enum : int { FLAG_OVERFLOW = 0, FLAG_BAD_INDEX = 1, FLAG_COUNT = 4 };
// Device counter slots (uint64 each), reset at the start of a render.
// CNT_QUEUE + 0..2: lists queued per size class for the list sort.
enum : int { CNT_EVALS_CONTRIB = 0, CNT_EVALS_LANES = 1, CNT_QUEUE = 2, CNT_COUNT = 8 };

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
    int tile_w, tile_h;    // 16 x 16 in this build
    int log2_w, log2_h;
    int tiles_x, tiles_y;  // tiles per image row / column
    int n_tiles;           // tiles per pose
};

// ---- geometry.hip (strict float32, no contraction) ----
void launch_pack(hipStream_t s, int64_t n_map, const float *means, const float *scales,
                 const float *quats, const float *opacity, const float *rgb, const int64_t *index,
                 int64_t n_sel, float4 *packed, int *flags);
// Blocks of the preprocess grid along the Gaussians (vcount has P * this entries).
int64_t preprocess_blocks(int64_t n);
void launch_preprocess(hipStream_t s, const float4 *packed, int64_t n, const float *poses, int n_poses,
                       const Camera &cam, const Consts &k, const TileGrid &tg, float4 *records,
                       uint32_t *ntiles, uint4 *einfo, uint32_t *vcount);
// Pairs in (pose, index) order: tile id within the pose, depth bits, submap index.
// einfo[p][g] = (depth bits, tx0 | tx1 << 16, ty0 | ty1 << 16, 0), written by the preprocess.
void launch_emit(hipStream_t s, const uint4 *einfo, const uint32_t *ntiles, int64_t n, int n_poses,
                 const uint64_t *pair_off, const TileGrid &tg, uint32_t *ptile, uint32_t *pz, uint32_t *pk,
                 uint64_t capacity, int *flags);

// ---- sort.hip ----
void launch_fill_u32(hipStream_t s, uint32_t *p, uint64_t n, uint32_t value);
void launch_fill_u64(hipStream_t s, unsigned long long *p, uint64_t n, unsigned long long value);
// Exclusive scan of count[0..n) into offsets[0..n), total into offsets[n]. With
// d_n, only the first min(*d_n, n) counts are read and offsets written.
// tmp must hold scan_tmp_elems(n) uint64.
uint64_t scan_tmp_elems(uint64_t n);
void launch_scan(hipStream_t s, const uint32_t *count, uint64_t n, uint64_t *offsets, uint64_t *tmp,
                 const uint64_t *d_n);
// Stable counting sort of the emitted pairs by tile within each pose. Writes
// the per-(pose, tile) list offsets [P*T + 1] and the bucketed (depth bits,
// index) arrays sz, sk. cnt holds bucket_blocks_max(capacity, P) * T entries,
// total P * T, block_base P + 1; n_tiles <= kMaxTilesPerPose.
uint64_t bucket_blocks_max(uint64_t capacity, int n_poses);
void launch_bucket(hipStream_t s, const uint32_t *ptile, const uint32_t *pz, const uint32_t *pk,
                   const uint64_t *pair_off, int64_t n, int n_poses, uint64_t capacity, int n_tiles, int tile_bits,
                   uint32_t *block_base, uint32_t *cnt, uint32_t *total, uint64_t *offsets, uint64_t *scan_tmp,
                   uint32_t *sz, uint32_t *sk);
// Sorts every list by depth bits (stable); sk ends in front-to-back order.
// tz, tk: scratch as large as sz, sk; queue: 3 * P * T entries.
void launch_list_sort(hipStream_t s, uint32_t *sz, uint32_t *sk, uint32_t *tz, uint32_t *tk, const uint64_t *offsets,
                      int n_tiles, int n_poses, uint32_t *queue, unsigned long long *counters);

// ---- blend.hip ----
void launch_blend(hipStream_t s, const float4 *records, int64_t n, int n_poses, const uint32_t *pairs,
                  const uint64_t *offsets, uint64_t capacity, const Camera &cam, const Consts &k,
                  const TileGrid &tg, float *rgb, float *depth, float *tfinal, bool count_evals,
                  unsigned long long *counters);

// ---- ncc.hip ----
int ncc_pixels_per_block();
void launch_ncc(hipStream_t s, const float *query, const float *renders, int n_poses, int height,
                int width, float *grey_q, double *partials, float *scores);
void launch_topk(hipStream_t s, const float *scores, int n, int k, int32_t *idx);

}  // namespace gsr
