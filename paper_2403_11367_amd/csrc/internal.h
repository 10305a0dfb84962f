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
enum : int { CNT_VISIBLE = 0, CNT_LONG_TILES = 1, CNT_EVALS_CONTRIB = 2, CNT_EVALS_LANES = 3, CNT_COUNT = 4 };

// Packed submap record: 4 float4 (64 B) per Gaussian, in spatial (internal) order.
//   q0 = (mu_x, mu_y, mu_z, opacity)
//   q1 = (S00, S01, S02, S11)        3D covariance, unique entries
//   q2 = (S12, S22, r, g)
//   q3 = (b, submap index bits, 0, 0)
constexpr int kPackedQuads = 4;

// Screen record: 3 float4 (48 B) per (pose, Gaussian).
//   q0 = (u, v, conic A, conic B)    d^2 = A dx^2 + 2 B dx dy + C dy^2
//   q1 = (conic C, opacity, r, g)
//   q2 = (b, z, rect_x bits, rect_y bits)   rect_x = i0 | i1 << 16
constexpr int kRecordQuads = 3;

// Per-tile lists of up to kSmallSortCap pairs are sorted in LDS by k_tile_sort
// (16 KB of LDS per block, high occupancy). Longer lists are queued and sorted
// by k_long_sort: in LDS (64 KB) up to kMidSortCap, else by a radix sort in
// global memory.
constexpr int kSmallSortCap = 2048;
constexpr int kMidSortCap = 8192;

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
// Scratch of the submap pack (sizes for n Gaussians).
struct PackScratch {
    float4 *packed_tmp;     // [n * kPackedQuads]
    uint32_t *code, *order, *code_tmp, *order_tmp;  // [n] each
    uint64_t *radix_tmp;    // [radix_tmp_elems(n)]
    uint32_t *bbox;         // [6]
};
// Packs the selection, then orders it spatially (Morton order of the means):
// packed[k] holds submap entry perm[k]; inv_perm is the inverse.
void launch_pack(hipStream_t s, int64_t n_map, const float *means, const float *scales,
                 const float *quats, const float *opacity, const float *rgb, const int64_t *index,
                 int64_t n_sel, PackScratch sc, float4 *packed, uint32_t *perm, uint32_t *inv_perm,
                 int *flags);
void launch_preprocess(hipStream_t s, const float4 *packed, int64_t n, const float *poses, int n_poses,
                       const Camera &cam, const Consts &k, const TileGrid &tg, float4 *records,
                       uint32_t *ntiles, uint32_t *tile_count, unsigned long long *counters);
void launch_scatter(hipStream_t s, const float4 *packed, const float4 *records, const uint32_t *ntiles,
                    int64_t n, int n_poses, const TileGrid &tg, const uint64_t *offsets, uint32_t *cursor,
                    uint64_t *pairs, uint64_t capacity, int *flags);

// ---- sort.hip ----
void launch_fill_u32(hipStream_t s, uint32_t *p, uint64_t n, uint32_t value);
void launch_fill_u64(hipStream_t s, unsigned long long *p, uint64_t n, unsigned long long value);
// exclusive scan of count[0..n) into offsets[0..n], offsets[n] = total.
// tmp must hold scan_tmp_elems(n) uint64.
uint64_t scan_tmp_elems(uint64_t n);
void launch_scan(hipStream_t s, const uint32_t *count, uint64_t n, uint64_t *offsets, uint64_t *tmp);
// Sorts the P * n_tiles lists by (depth bits, submap index), then rewrites the
// low 32 bits of each pair to the Gaussian's internal position (inv_perm);
// long_list must hold P * n_tiles entries and pairs_tmp as many pairs as pairs.
void launch_tile_sort(hipStream_t s, uint64_t *pairs, uint64_t *pairs_tmp, const uint64_t *offsets,
                      int n_tiles, int n_poses, uint64_t capacity, const uint32_t *inv_perm,
                      uint32_t *long_list, unsigned long long *counters);
// Device-wide stable LSD radix sort of n (key, value) pairs on the low `bits`
// key bits; tmp must hold radix_tmp_elems(n) uint64.
uint64_t radix_tmp_elems(uint64_t n);
void launch_radix_sort_u32(hipStream_t s, uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp,
                           uint64_t n, int bits, uint64_t *tmp);

// ---- blend.hip ----
void launch_blend(hipStream_t s, const float4 *records, int64_t n, int n_poses, const uint64_t *pairs,
                  const uint64_t *offsets, uint64_t capacity, const Camera &cam, const Consts &k,
                  const TileGrid &tg, float *rgb, float *depth, float *tfinal, bool count_evals,
                  unsigned long long *counters);

// ---- ncc.hip ----
int ncc_pixels_per_block();
void launch_ncc(hipStream_t s, const float *query, const float *renders, int n_poses, int height,
                int width, float *grey_q, double *partials, float *scores);
void launch_topk(hipStream_t s, const float *scores, int n, int k, int32_t *idx);

}  // namespace gsr
