// Submap packing, EWA preprocessing and (Gaussian, tile) pair scatter.
//
// Built with -ffp-contract=off and correctly rounded float32 division and
// square root, so that every record and depth key is a deterministic function
// of the float32 inputs with the operation order written below (each
// parenthesised sum is evaluated as written; no fused multiply-add).
//
// Paper: Sec. III-A. A Gaussian has mean mu, covariance Sigma = R S S^T R^T with
// S = diag(s) and R = q2R(q), q = (w, x, y, z), colour c and opacity o. For a
// camera with intrinsics K and world-to-camera pose W_t it is moved to camera
// space, projected by m(mu) = K (W mu / (W mu)_z) (Eq. 4) and given the screen
// covariance J W Sigma W^T J^T (Eq. 3, top-left 2x2), with J the Jacobian of m.
#include "internal.h"

namespace gsr {

namespace {

constexpr int kThreads = 256;
constexpr int kPosesPerThread = 8;

// Order-preserving map of a float to uint32 (for atomic min / max).
__device__ __forceinline__ uint32_t f2ord(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t o) {
    return __uint_as_float((o & 0x80000000u) ? (o & 0x7fffffffu) : ~o);
}

// Bounding box of the selected means (finite ones): bbox[0..2] = min, [3..5] = max.
__global__ __launch_bounds__(kThreads) void k_bbox(int64_t n_map, const float *__restrict__ means,
                                                   const int64_t *__restrict__ index, int64_t n_sel,
                                                   uint32_t *__restrict__ bbox) {
    __shared__ uint32_t s_b[6];
    if (threadIdx.x < 6) s_b[threadIdx.x] = threadIdx.x < 3 ? 0xffffffffu : 0u;
    __syncthreads();
    uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n_sel; i += (int64_t)gridDim.x * kThreads) {
        const int64_t src = index ? index[i] : i;
        if (src < 0 || src >= n_map) continue;
        const float x = means[src * 3 + 0], y = means[src * 3 + 1], z = means[src * 3 + 2];
        if (!(__builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z))) continue;
        const uint32_t o[3] = {f2ord(x), f2ord(y), f2ord(z)};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = min(lo[a], o[a]);
            hi[a] = max(hi[a], o[a]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        atomicMin(&s_b[a], lo[a]);
        atomicMax(&s_b[3 + a], hi[a]);
    }
    __syncthreads();
    if (threadIdx.x < 3) atomicMin(&bbox[threadIdx.x], s_b[threadIdx.x]);
    else if (threadIdx.x < 6) atomicMax(&bbox[threadIdx.x], s_b[threadIdx.x]);
}

__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 10 bits -> every third bit
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t quant10(float x, float lo, float inv_ext) {
    const float t = (x - lo) * inv_ext;
    return (uint32_t)fminf(fmaxf(t, 0.f), 1023.f);
}

// S0: q normalised, R = q2R(q), M = R diag(s), Sigma = M M^T (6 unique entries),
// stored in submap order, plus a 30-bit Morton code of the mean in the bounding
// box (the spatial sort key; NaN / out-of-range entries sort last).
__global__ __launch_bounds__(kThreads) void k_pack(int64_t n_map, const float *__restrict__ means,
                                                   const float *__restrict__ scales,
                                                   const float *__restrict__ quats,
                                                   const float *__restrict__ opacity,
                                                   const float *__restrict__ rgb,
                                                   const int64_t *__restrict__ index, int64_t n_sel,
                                                   const uint32_t *__restrict__ bbox, float4 *__restrict__ packed,
                                                   uint32_t *__restrict__ code, uint32_t *__restrict__ order,
                                                   int *__restrict__ flags) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n_sel) return;
    const int64_t src = index ? index[i] : i;
    float4 *out = packed + i * kPackedQuads;
    order[i] = (uint32_t)i;
    if (src < 0 || src >= n_map) {
        // an invalid entry becomes a Gaussian that every pose culls (NaN depth)
        const float nan = __builtin_nanf("");
        out[0] = make_float4(nan, nan, nan, 0.f);
        out[1] = make_float4(0.f, 0.f, 0.f, 0.f);
        out[2] = make_float4(0.f, 0.f, 0.f, 0.f);
        out[3] = make_float4(0.f, 0.f, 0.f, 0.f);
        code[i] = 0x3fffffffu;
        atomicOr(&flags[FLAG_BAD_INDEX], 1);
        return;
    }
    float w = quats[src * 4 + 0], x = quats[src * 4 + 1], y = quats[src * 4 + 2], z = quats[src * 4 + 3];
    const float n = sqrtf(((w * w + x * x) + y * y) + z * z);
    w = w / n;
    x = x / n;
    y = y / n;
    z = z / n;
    const float r00 = 1.0f - 2.0f * (y * y + z * z);
    const float r01 = 2.0f * (x * y - w * z);
    const float r02 = 2.0f * (x * z + w * y);
    const float r10 = 2.0f * (x * y + w * z);
    const float r11 = 1.0f - 2.0f * (x * x + z * z);
    const float r12 = 2.0f * (y * z - w * x);
    const float r20 = 2.0f * (x * z - w * y);
    const float r21 = 2.0f * (y * z + w * x);
    const float r22 = 1.0f - 2.0f * (x * x + y * y);
    const float sx = scales[src * 3 + 0], sy = scales[src * 3 + 1], sz = scales[src * 3 + 2];
    const float m00 = r00 * sx, m01 = r01 * sy, m02 = r02 * sz;
    const float m10 = r10 * sx, m11 = r11 * sy, m12 = r12 * sz;
    const float m20 = r20 * sx, m21 = r21 * sy, m22 = r22 * sz;
    const float s00 = (m00 * m00 + m01 * m01) + m02 * m02;
    const float s01 = (m00 * m10 + m01 * m11) + m02 * m12;
    const float s02 = (m00 * m20 + m01 * m21) + m02 * m22;
    const float s11 = (m10 * m10 + m11 * m11) + m12 * m12;
    const float s12 = (m10 * m20 + m11 * m21) + m12 * m22;
    const float s22 = (m20 * m20 + m21 * m21) + m22 * m22;
    const float px = means[src * 3 + 0], py = means[src * 3 + 1], pz = means[src * 3 + 2];
    out[0] = make_float4(px, py, pz, opacity[src]);
    out[1] = make_float4(s00, s01, s02, s11);
    out[2] = make_float4(s12, s22, rgb[src * 3 + 0], rgb[src * 3 + 1]);
    out[3] = make_float4(rgb[src * 3 + 2], __uint_as_float((uint32_t)i), 0.f, 0.f);
    if (__builtin_isfinite(px) && __builtin_isfinite(py) && __builtin_isfinite(pz)) {
        float lo[3], inv[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            lo[a] = ord2f(bbox[a]);
            const float ext = ord2f(bbox[3 + a]) - lo[a];
            inv[a] = ext > 0.f ? 1024.f / ext : 0.f;
        }
        code[i] = (spread3(quant10(px, lo[0], inv[0])) << 2) | (spread3(quant10(py, lo[1], inv[1])) << 1) |
                  spread3(quant10(pz, lo[2], inv[2]));
    } else {
        code[i] = 0x3fffffffu;
    }
}

// packed[k] = packed_tmp[order[k]] (spatial order); inv_perm[order[k]] = k.
__global__ __launch_bounds__(kThreads) void k_pack_permute(const float4 *__restrict__ tmp,
                                                           const uint32_t *__restrict__ order, int64_t n,
                                                           float4 *__restrict__ packed, uint32_t *__restrict__ perm,
                                                           uint32_t *__restrict__ inv_perm) {
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    const uint32_t i = order[k];
    const float4 *src = tmp + (int64_t)i * kPackedQuads;
    float4 *dst = packed + k * kPackedQuads;
    dst[0] = src[0];
    dst[1] = src[1];
    dst[2] = src[2];
    dst[3] = src[3];
    perm[k] = i;
    inv_perm[i] = (uint32_t)k;
}

// Wave-aggregated update of per-tile counters: every lane holds a tile
// rectangle (n_mine tiles, row-major from (tx0, ty0) with width wx) or none.
// Lanes that name the same tile in the same round share one atomic. With
// `reserve`, the leader's atomic returns the group's first slot and each lane
// gets its own consecutive slot, delivered through emit(tile, slot).
template <bool kReserve, typename Emit>
__device__ __forceinline__ void wave_tile_atomics(uint32_t *counters, int tiles_x, int tx0, int ty0, int wx,
                                                  int n_mine, Emit emit) {
    const int lane = threadIdx.x & 63;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int c = 0;; ++c) {
        const bool has = c < n_mine;
        uint64_t pending = __ballot(has);
        if (pending == 0) break;
        const int t = has ? (ty0 + c / wx) * tiles_x + tx0 + c % wx : -1;
        while (pending) {
            const int leader = (int)__builtin_ctzll(pending);
            const int tl = __builtin_amdgcn_readlane(t, leader);
            const uint64_t peers = __ballot(t == tl);
            uint32_t base = 0;
            if (lane == leader) {
                if (kReserve)
                    base = atomicAdd(&counters[tl], (uint32_t)__popcll(peers));
                else
                    atomicAdd(&counters[tl], (uint32_t)__popcll(peers));
            }
            if (kReserve) {
                base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
                if (t == tl) emit(tl, base + (uint32_t)__popcll(peers & lt_mask));
            }
            pending &= ~peers;
        }
    }
}

// S1 + tile histogram. One thread per Gaussian, looping over a chunk of poses
// (blockIdx.y), so the packed record is read once per chunk. For each pose the
// screen record is written, the number of tiles its 3-sigma rectangle touches
// is stored (0 = culled), and every touched (pose, tile) counter is incremented.
__global__ __launch_bounds__(kThreads) void k_preprocess(
    const float4 *__restrict__ packed, int64_t n, const float *__restrict__ poses, int n_poses, Camera cam,
    Consts k, TileGrid tg, float4 *__restrict__ records, uint32_t *__restrict__ ntiles,
    uint32_t *__restrict__ tile_count, unsigned long long *__restrict__ counters) {
    __shared__ unsigned s_vis;
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int p0 = blockIdx.y * kPosesPerThread;
    const int p1 = min(p0 + kPosesPerThread, n_poses);
    const bool in = g < n;
    if (threadIdx.x == 0) s_vis = 0;
    __syncthreads();
    float4 q0 = make_float4(0.f, 0.f, 0.f, 0.f), q1 = q0, q2 = q0, q3 = q0;
    if (in) {
        const float4 *src = packed + g * kPackedQuads;
        q0 = src[0];
        q1 = src[1];
        q2 = src[2];
        q3 = src[3];
    }
    const float mx = q0.x, my = q0.y, mz = q0.z;
    const float s00 = q1.x, s01 = q1.y, s02 = q1.z, s11 = q1.w, s12 = q2.x, s22 = q2.y;
    // Jacobian clamp limits: 1.3 x tan(half field of view)
    const float lim_x = k.jac_clamp * ((0.5f * (float)cam.width) / cam.fx);
    const float lim_y = k.jac_clamp * ((0.5f * (float)cam.height) / cam.fy);
    const float wmax = (float)(cam.width - 1), hmax = (float)(cam.height - 1);
    unsigned vis_count = 0;
    for (int p = p0; p < p1; ++p) {
        const float *P = poses + p * 12;  // [R | t] row-major, uniform across the block
        const float R00 = P[0], R01 = P[1], R02 = P[2], T0 = P[3];
        const float R10 = P[4], R11 = P[5], R12 = P[6], T1 = P[7];
        const float R20 = P[8], R21 = P[9], R22 = P[10], T2 = P[11];
        uint32_t nt = 0;
        int tr[3] = {0, 0, 1};  // tile rect origin and width, for the histogram
        if (in) {
            const float tx = ((R00 * mx + R01 * my) + R02 * mz) + T0;
            const float ty = ((R10 * mx + R11 * my) + R12 * mz) + T1;
            const float tz = ((R20 * mx + R21 * my) + R22 * mz) + T2;
            if (tz > k.z_near) {
                const float xt = tx / tz, yt = ty / tz;
                const float xc = fminf(fmaxf(xt, -lim_x), lim_x);
                const float yc = fminf(fmaxf(yt, -lim_y), lim_y);
                const float j00 = cam.fx / tz;
                const float j02 = -(cam.fx * xc) / tz;
                const float j11 = cam.fy / tz;
                const float j12 = -(cam.fy * yc) / tz;
                // T = J R_w (2x3)
                const float t00 = j00 * R00 + j02 * R20, t01 = j00 * R01 + j02 * R21, t02 = j00 * R02 + j02 * R22;
                const float t10 = j11 * R10 + j12 * R20, t11 = j11 * R11 + j12 * R21, t12 = j11 * R12 + j12 * R22;
                // U = T Sigma (2x3)
                const float u00 = (t00 * s00 + t01 * s01) + t02 * s02;
                const float u01 = (t00 * s01 + t01 * s11) + t02 * s12;
                const float u02 = (t00 * s02 + t01 * s12) + t02 * s22;
                const float u10 = (t10 * s00 + t11 * s01) + t12 * s02;
                const float u11 = (t10 * s01 + t11 * s11) + t12 * s12;
                const float u12 = (t10 * s02 + t11 * s12) + t12 * s22;
                const float a = ((u00 * t00 + u01 * t01) + u02 * t02) + k.eps;
                const float b = (u00 * t10 + u01 * t11) + u02 * t12;
                const float c = ((u10 * t10 + u11 * t11) + u12 * t12) + k.eps;
                const float det = a * c - b * b;
                if (det > 0.f) {
                    const float ca = c / det, cb = (-b) / det, cc = a / det;
                    const float rx = 3.0f * sqrtf(a), ry = 3.0f * sqrtf(c);
                    const float u = cam.fx * xt + cam.cx;
                    const float v = cam.fy * yt + cam.cy;
                    const bool fin = __builtin_isfinite(u) && __builtin_isfinite(v) && __builtin_isfinite(rx) &&
                                     __builtin_isfinite(ry) && __builtin_isfinite(ca) &&
                                     __builtin_isfinite(cb) && __builtin_isfinite(cc);
                    if (fin) {
                        const float i0f = fmaxf(ceilf((u - rx) - 0.5f), 0.f);
                        const float i1f = fminf(floorf((u + rx) - 0.5f), wmax);
                        const float j0f = fmaxf(ceilf((v - ry) - 0.5f), 0.f);
                        const float j1f = fminf(floorf((v + ry) - 0.5f), hmax);
                        if (i0f <= i1f && j0f <= j1f) {
                            const int i0 = (int)i0f, i1 = (int)i1f, j0 = (int)j0f, j1 = (int)j1f;
                            const int tx0 = i0 >> tg.log2_w, tx1 = i1 >> tg.log2_w;
                            const int ty0 = j0 >> tg.log2_h, ty1 = j1 >> tg.log2_h;
                            nt = (uint32_t)((tx1 - tx0 + 1) * (ty1 - ty0 + 1));
                            float4 *r = records + ((int64_t)p * n + g) * kRecordQuads;
                            r[0] = make_float4(u, v, ca, cb);
                            r[1] = make_float4(cc, q0.w, q2.z, q2.w);
                            r[2] = make_float4(q3.x, tz, __uint_as_float((uint32_t)i0 | ((uint32_t)i1 << 16)),
                                               __uint_as_float((uint32_t)j0 | ((uint32_t)j1 << 16)));
                            tr[0] = tx0;
                            tr[1] = ty0;
                            tr[2] = tx1 - tx0 + 1;
                        }
                    }
                }
            }
            ntiles[(int64_t)p * n + g] = nt;
        }
        vis_count += (nt != 0);
        wave_tile_atomics<false>(tile_count + (int64_t)p * tg.n_tiles, tg.tiles_x, tr[0], tr[1], tr[2], (int)nt,
                                 [](int, uint32_t) {});
    }
    // one counter update per block
    if (vis_count) atomicAdd(&s_vis, vis_count);
    __syncthreads();
    if (threadIdx.x == 0 && s_vis) atomicAdd(&counters[CNT_VISIBLE], (unsigned long long)s_vis);
}

// S2: every (pose, Gaussian, tile) pair takes a slot in its tile's list, with
// key (depth bits << 32 | submap index). Slots are reserved one atomic per
// (wave, tile) group, so a wave's pairs for one tile land contiguously; their
// order inside a list is otherwise arbitrary and k_tile_sort orders each list
// by the key, which is unique.
__global__ __launch_bounds__(kThreads) void k_scatter(const float4 *__restrict__ packed,
                                                      const float4 *__restrict__ records,
                                                      const uint32_t *__restrict__ ntiles, int64_t n,
                                                      int n_poses, TileGrid tg,
                                                      const uint64_t *__restrict__ offsets,
                                                      uint32_t *__restrict__ cursor, uint64_t *__restrict__ pairs,
                                                      uint64_t capacity, int *__restrict__ flags) {
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const bool in = g < n;
    const int p0 = blockIdx.y * kPosesPerThread;
    const int p1 = min(p0 + kPosesPerThread, n_poses);
    const uint32_t sub_index = in ? __float_as_uint(packed[g * kPackedQuads + 3].y) : 0u;
    bool over = false;
    for (int p = p0; p < p1; ++p) {
        const int64_t rg = (int64_t)p * n + g;
        const uint32_t nt = in ? ntiles[rg] : 0u;
        int tx0 = 0, ty0 = 0, wx = 1;
        uint64_t key = 0;
        if (nt) {
            const float4 q2 = records[rg * kRecordQuads + 2];
            const uint32_t rxb = __float_as_uint(q2.z), ryb = __float_as_uint(q2.w);
            tx0 = (int)(rxb & 0xffffu) >> tg.log2_w;
            ty0 = (int)(ryb & 0xffffu) >> tg.log2_h;
            wx = ((int)(rxb >> 16) >> tg.log2_w) - tx0 + 1;
            key = ((uint64_t)__float_as_uint(q2.y) << 32) | sub_index;
        }
        const int64_t base = (int64_t)p * tg.n_tiles;
        wave_tile_atomics<true>(cursor + base, tg.tiles_x, tx0, ty0, wx, (int)nt, [&](int t, uint32_t slot) {
            const uint64_t pos = offsets[base + t] + slot;
            if (pos < capacity)
                pairs[pos] = key;
            else
                over = true;
        });
    }
    if (over) atomicOr(&flags[FLAG_OVERFLOW], 1);
}

}  // namespace

void launch_pack(hipStream_t s, int64_t n_map, const float *means, const float *scales, const float *quats,
                 const float *opacity, const float *rgb, const int64_t *index, int64_t n_sel, PackScratch sc,
                 float4 *packed, uint32_t *perm, uint32_t *inv_perm, int *flags) {
    if (n_sel <= 0) return;
    const unsigned blocks = (unsigned)((n_sel + kThreads - 1) / kThreads);
    launch_fill_u32(s, sc.bbox, 3, 0xffffffffu);
    launch_fill_u32(s, sc.bbox + 3, 3, 0u);
    hipLaunchKernelGGL(k_bbox, dim3(std::min(blocks, 1024u)), dim3(kThreads), 0, s, n_map, means, index, n_sel,
                       sc.bbox);
    hipLaunchKernelGGL(k_pack, dim3(blocks), dim3(kThreads), 0, s, n_map, means, scales, quats, opacity, rgb, index,
                       n_sel, sc.bbox, sc.packed_tmp, sc.code, sc.order, flags);
    launch_radix_sort_u32(s, sc.code, sc.order, sc.code_tmp, sc.order_tmp, (uint64_t)n_sel, 30, sc.radix_tmp);
    hipLaunchKernelGGL(k_pack_permute, dim3(blocks), dim3(kThreads), 0, s, sc.packed_tmp, sc.order, n_sel, packed,
                       perm, inv_perm);
}

void launch_preprocess(hipStream_t s, const float4 *packed, int64_t n, const float *poses, int n_poses,
                       const Camera &cam, const Consts &k, const TileGrid &tg, float4 *records,
                       uint32_t *ntiles, uint32_t *tile_count, unsigned long long *counters) {
    if (n <= 0) return;
    const dim3 grid((unsigned)((n + kThreads - 1) / kThreads), (unsigned)((n_poses + kPosesPerThread - 1) / kPosesPerThread));
    hipLaunchKernelGGL(k_preprocess, grid, dim3(kThreads), 0, s, packed, n, poses, n_poses, cam, k, tg, records,
                       ntiles, tile_count, counters);
}

void launch_scatter(hipStream_t s, const float4 *packed, const float4 *records, const uint32_t *ntiles, int64_t n,
                    int n_poses, const TileGrid &tg, const uint64_t *offsets, uint32_t *cursor, uint64_t *pairs,
                    uint64_t capacity, int *flags) {
    if (n <= 0) return;
    const dim3 grid((unsigned)((n + kThreads - 1) / kThreads), (unsigned)((n_poses + kPosesPerThread - 1) / kPosesPerThread));
    hipLaunchKernelGGL(k_scatter, grid, dim3(kThreads), 0, s, packed, records, ntiles, n, n_poses, tg, offsets,
                       cursor, pairs, capacity, flags);
}

}  // namespace gsr
