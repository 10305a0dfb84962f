// Submap packing (S0), EWA preprocessing (S1) and the per-Gaussian steps of
// the pair ordering (S2): per-wave packing of the visible entries and pair
// emission.
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

// S0: q normalised, R = q2R(q), M = R diag(s), Sigma = M M^T (6 unique entries).
__global__ __launch_bounds__(kThreads) void k_pack(int64_t n_map, const float *__restrict__ means,
                                                   const float *__restrict__ scales,
                                                   const float *__restrict__ quats,
                                                   const float *__restrict__ opacity,
                                                   const float *__restrict__ rgb,
                                                   const int64_t *__restrict__ index, int64_t n_sel,
                                                   float4 *__restrict__ packed, int *__restrict__ flags,
                                                   unsigned long long *__restrict__ nonfinite) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n_sel) return;
    const int64_t src = index ? index[i] : i;
    float4 *out = packed + i * kPackedQuads;
    if (src < 0 || src >= n_map) {
        // an invalid entry becomes a Gaussian that every pose culls (NaN depth)
        const float nan = __builtin_nanf("");
        out[0] = make_float4(nan, nan, nan, 0.f);
        out[1] = make_float4(0.f, 0.f, 0.f, 0.f);
        out[2] = make_float4(0.f, 0.f, 0.f, 0.f);
        out[3] = make_float4(0.f, 0.f, 0.f, 0.f);
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
    float mx = means[src * 3 + 0], my = means[src * 3 + 1], mz = means[src * 3 + 2];
    const float o = opacity[src], cr = rgb[src * 3 + 0], cg = rgb[src * 3 + 1], cb = rgb[src * 3 + 2];
    // a Gaussian with any non-finite entry is counted and culled at every pose (NaN mean)
    const bool finite = __builtin_isfinite(mx) && __builtin_isfinite(my) && __builtin_isfinite(mz) &&
                        __builtin_isfinite(s00) && __builtin_isfinite(s01) && __builtin_isfinite(s02) &&
                        __builtin_isfinite(s11) && __builtin_isfinite(s12) && __builtin_isfinite(s22) &&
                        __builtin_isfinite(o) && __builtin_isfinite(cr) && __builtin_isfinite(cg) &&
                        __builtin_isfinite(cb);
    if (!finite) {
        mx = my = mz = __builtin_nanf("");
        atomicAdd(nonfinite, 1ull);
    }
    out[0] = make_float4(mx, my, mz, o);
    out[1] = make_float4(s00, s01, s02, s11);
    out[2] = make_float4(s12, s22, cr, cg);
    out[3] = make_float4(cb, 0.f, 0.f, 0.f);
}

// Adds each submap's count of non-finite Gaussians to *total.
__global__ void k_sum_nonfinite(const SubmapTable tab, unsigned long long *__restrict__ total) {
    const int q = threadIdx.x;
    if (q < tab.count) atomicAdd(total, *tab.nonfinite[q]);
}

// S1. One thread per Gaussian slot, looping over a chunk of poses (blockIdx.y),
// so the packed record is read once per chunk (again where the chunk crosses
// into the next submap of a batch; slot g of a pose whose submap has no
// Gaussian g is culled). For each pose the screen record and the tile
// rectangle of a visible Gaussian are written, and each wave packs the (depth
// key, sort value) of its visible Gaussians, in index order, at the front of
// its 64-slot region of vz / vg, with the region's visibility mask (bit l: slot
// 64 region + l is visible) in vmask[pose * n_regions + region]: the input of
// the per-pose depth sort. (The mask replaces a 4-byte tile count per pose and
// Gaussian: 8 bytes per 64 slots; the count is in the sort value and follows
// from the tile rectangle.) The depth key is the depth's float32 bits minus the
// near plane's; a key of 2^kNarrowKeyBits or more raises *wide.
__global__ __launch_bounds__(kThreads) void k_preprocess(
    const SubmapTable tab, int64_t n, const float *__restrict__ poses, int n_poses, Camera cam,
    Consts k, TileGrid tg, float4 *__restrict__ records, uint2 *__restrict__ rect, uint32_t *__restrict__ vz,
    uint32_t *__restrict__ vg, uint64_t *__restrict__ vmask, bool pack, unsigned long long *__restrict__ wide) {
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int p0 = blockIdx.y * kPosesPerThread;
    const int p1 = min(p0 + kPosesPerThread, n_poses);
    const int lane = threadIdx.x & 63;
    const int64_t region = g >> 6;  // the same for the whole wave
    const int64_t n_regions = (n + 63) >> 6;
    const bool region_in = (region << 6) < n;
    const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    // submap of the chunk's first pose (uniform across the block)
    int q = 0;
    while (q + 1 < tab.count && p0 >= tab.pose_end[q]) ++q;
    bool in = false;
    float4 q0, q1, q2, q3;
    auto load = [&](int sq) {
        in = g < tab.n[sq];
        q0 = make_float4(0.f, 0.f, 0.f, 0.f);
        q1 = q0;
        q2 = q0;
        q3 = q0;
        if (in) {
            const float4 *src = tab.packed[sq] + g * kPackedQuads;
            q0 = src[0];
            q1 = src[1];
            q2 = src[2];
            q3 = src[3];
        }
    };
    load(q);
    // Jacobian clamp limits: 1.3 x tan(half field of view)
    const float lim_x = k.jac_clamp * ((0.5f * (float)cam.width) / cam.fx);
    const float lim_y = k.jac_clamp * ((0.5f * (float)cam.height) / cam.fy);
    const float wmax = (float)(cam.width - 1), hmax = (float)(cam.height - 1);
    // visible depths exceed z_near >= 0, so their bits exceed these
    const uint32_t zoff = k.z_near > 0.f ? __float_as_uint(k.z_near) : 0u;
    for (int p = p0; p < p1; ++p) {
        if (p >= tab.pose_end[q]) {
            while (p >= tab.pose_end[q]) ++q;
            load(q);
        }
        const float mx = q0.x, my = q0.y, mz = q0.z;
        const float s00 = q1.x, s01 = q1.y, s02 = q1.z, s11 = q1.w, s12 = q2.x, s22 = q2.y;
        const float *P = poses + p * 12;  // [R | t] row-major, uniform across the block
        const float R00 = P[0], R01 = P[1], R02 = P[2], T0 = P[3];
        const float R10 = P[4], R11 = P[5], R12 = P[6], T1 = P[7];
        const float R20 = P[8], R21 = P[9], R22 = P[10], T2 = P[11];
        uint32_t nt = 0, zb = 0;
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
                            rect[(int64_t)p * n + g] = make_uint2((uint32_t)tx0 | ((uint32_t)tx1 << 16),
                                                                  (uint32_t)ty0 | ((uint32_t)ty1 << 16));
                            zb = __float_as_uint(tz) - zoff;
                        }
                    }
                }
            }
        }
        const uint64_t vis = __ballot(nt != 0);
        if (__ballot(nt != 0 && zb >= (1u << kNarrowKeyBits)) != 0ull && lane == 0) atomicOr(wide, 1ull);
        if (region_in) {
            if (lane == 0) vmask[(int64_t)p * n_regions + region] = vis;
            if (nt != 0) {
                const int64_t slot = (int64_t)p * n + (region << 6) + __popcll(vis & lt_mask);
                vz[slot] = zb;
                // the record slot of (pose, Gaussian), or its index and tile count
                vg[slot] = pack ? (uint32_t)g | (nt << kPackIndexBits) : (uint32_t)((int64_t)p * n + g);
            }
        }
    }
}

// S2, pair emission in front-to-back order. The depth-sorted visible Gaussians of
// all poses are cut into emission blocks of kEmitTile elements (pose p owns
// [vbase[p], vbase[p+1]); the sorted run holds their tile counts and record
// slots). The tile counts are summed per block, the block sums prefixed in two
// levels (within spans of kSumSpan blocks, then across spans by a scan in
// sort.hip), and each block then lays its pairs out contiguously from its
// prefix: element i writes one pair per tile of its rectangle (row-major): the
// tile id within the pose and the submap index.
constexpr int kEmitItems = 2;
constexpr int kEmitTile = kThreads * kEmitItems;
constexpr int kSumSpan = 8;

// First pair of emission block b: its span's prefix plus its prefix within the span
// (the layout of the emission sums is in internal.h).
__device__ __forceinline__ uint64_t emit_block_prefix(const uint64_t *__restrict__ es, uint64_t n_blocks,
                                                      uint64_t b) {
    return es[n_blocks + 2 + b / kSumSpan] + es[b];
}

// Exclusive scan of one uint32 per thread across a kThreads block; *total = sum.
__device__ uint32_t emit_block_scan(uint32_t x, uint32_t *s_wave /*[4]*/, uint32_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < wave; ++w) add += s_wave[w];
    *total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    __syncthreads();
    return add + inc - x;
}

// The emission sums, before the scan of the span sums: one workgroup per span of
// kSumSpan emission blocks, wave w summing blocks 2w and 2w + 1 (lane l takes
// elements k * 64 + l of a block, coalesced). Spans past the visible total
// write nothing.
static_assert(kSumSpan == 2 * (kThreads / 64), "two emission blocks per wave");
__global__ __launch_bounds__(kThreads) void k_emit_sums(const SortedRun run, const uint32_t *__restrict__ vbase,
                                                        int P, uint64_t n_blocks, uint64_t *__restrict__ es) {
    __shared__ uint32_t s_sum[kSumSpan];
    const uint32_t *__restrict__ snt = *run.wide ? run.cnt_a : run.cnt_b;
    const uint64_t nv = vbase[P];
    const uint64_t blocks_used = (nv + kEmitTile - 1) / kEmitTile;
    if (blockIdx.x == 0 && threadIdx.x == 0) es[n_blocks + 1] = (blocks_used + kSumSpan - 1) / kSumSpan;
    const uint64_t span = blockIdx.x, b0 = span * kSumSpan;
    if (b0 >= blocks_used) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // unconditional loads (an element past the end reads element 0 and adds
    // nothing), so that all of them are in flight at once
    uint32_t sum[2] = {0u, 0u};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint64_t e0 = (b0 + 2 * wave + h) * kEmitTile;
#pragma unroll
        for (int k = 0; k < kEmitTile / 64; ++k) {
            const uint64_t e = e0 + (uint64_t)k * 64 + lane;
            const uint32_t c = snt[e < nv ? e : 0];
            sum[h] += e < nv ? c : 0u;
        }
    }
    // tile counts per element are < 2^15 and a span has 4096 elements: fits 32 bits
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) sum[h] += __shfl_xor(sum[h], o, 64);
    }
    if (lane == 0) {
        s_sum[2 * wave] = sum[0];
        s_sum[2 * wave + 1] = sum[1];
    }
    __syncthreads();
    if (threadIdx.x < kSumSpan) {
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int i = 0; i < kSumSpan; ++i) {
            const uint32_t x = s_sum[i];
            if (i < (int)threadIdx.x) before += x;
            all += x;
        }
        if (b0 + threadIdx.x < n_blocks) es[b0 + threadIdx.x] = before;
        if (threadIdx.x == 0) es[n_blocks + 2 + span] = all;
    }
}

// pseg[p] = min(first pair of pose p, capacity) for p in [0, P], from the
// scanned emission sums es (es[n_blocks]: the pair total).
__global__ __launch_bounds__(kThreads) void k_pair_segments(const SortedRun run, const uint32_t *__restrict__ vbase,
                                                            int P, const uint64_t *__restrict__ es, uint64_t n_blocks,
                                                            uint64_t capacity, uint64_t *__restrict__ pseg) {
    __shared__ uint32_t s_wave[4];
    const uint32_t *__restrict__ snt = *run.wide ? run.cnt_a : run.cnt_b;
    const int p = blockIdx.x;
    const uint64_t e = vbase[p], nv = vbase[P];
    if (e >= nv) {
        if (threadIdx.x == 0) pseg[p] = min(es[n_blocks], capacity);
        return;
    }
    const uint64_t b = e / kEmitTile, e0 = b * kEmitTile;
    uint32_t part = 0;
    for (uint64_t i = e0 + threadIdx.x; i < e; i += kThreads) part += snt[i];
    uint32_t total = 0;
    (void)emit_block_scan(part, s_wave, &total);
    if (threadIdx.x == 0) pseg[p] = min(emit_block_prefix(es, n_blocks, b) + total, capacity);
}

// The submap index of record slot x = pose * n + index (n >= 1): the quotient
// x / n is the pose, below 65536, so the float product (relative error a few
// 2^-24) is within 0.02 of it and its truncation off by at most one; the
// remainder is then corrected into [0, n) exactly.
__device__ __forceinline__ uint32_t slot_index(uint32_t x, uint32_t n, float inv_n) {
    const int64_t q = (int64_t)((float)x * inv_n);
    int64_t r = (int64_t)x - q * (int64_t)n;
    if (r < 0) r += n;
    if (r >= (int64_t)n) r -= n;
    return (uint32_t)r;
}

// One block per emission block. The block scans its elements' tile counts, then
// lays the pairs out window by window in LDS: every thread expands its own
// elements' rectangles (row-major) into the window slots given by the scan, and
// the block copies the window to the output with coalesced stores.
constexpr int kEmitWin = 4096;  // pairs per LDS window

__global__ __launch_bounds__(kThreads) void k_emit(const SortedRun run, const uint32_t *__restrict__ vbase, int P,
                                                   const uint2 *__restrict__ rect, int64_t n,
                                                   const uint64_t *__restrict__ es, uint64_t n_blocks, TileGrid tg,
                                                   uint16_t *__restrict__ ptile, uint32_t *__restrict__ pk,
                                                   uint64_t capacity, int *__restrict__ flags) {
    __shared__ uint16_t s_tile[kEmitWin];
    __shared__ uint32_t s_key[kEmitWin];
    __shared__ uint32_t s_wave[4];
    const bool wide = *run.wide != 0ull;
    const uint32_t *__restrict__ snt = wide ? run.cnt_a : run.cnt_b;
    const uint32_t *__restrict__ slots = wide ? run.slot_a : run.slot_b;
    // Workgroups go to the 8 XCDs round robin by linear id; block b below takes
    // emission block (b % 8) * per + b / 8 with per = ceil(nb / 8) for the nb
    // blocks that hold elements, so each XCD walks one eighth of the elements in
    // order (about one pose at a time), and the rectangles its blocks gather come
    // through one L2 instead of eight. The grid (a multiple of 8, sized for every
    // slot visible) has at least 8 * per blocks.
    const uint64_t nv = vbase[P];
    const uint64_t nb = (nv + kEmitTile - 1) / kEmitTile;
    const uint64_t per = (nb + kXcdCount - 1) / kXcdCount;
    const uint64_t turn = blockIdx.x / kXcdCount;  // this block's place in its XCD's walk
    if (turn >= per) return;
    const uint64_t eb = (uint64_t)(blockIdx.x % kXcdCount) * per + turn;
    const uint64_t e0 = eb * kEmitTile;
    if (e0 >= nv) return;
    const float inv_n = 1.0f / (float)n;
    // this thread's elements: e0 + t * kEmitItems + k (consecutive, for the scan)
    const uint64_t et = e0 + (uint64_t)threadIdx.x * kEmitItems;
    // tile counts and record slots together, then the rectangles (one round trip
    // fewer than loading the slots after the scan). No load is conditional: an
    // element past the end reads the block's first element and counts nothing, so
    // the loads of all items are in flight at once (a load under a branch is
    // waited for where the branches join, one item at a time).
    uint32_t cnt[kEmitItems], slot[kEmitItems], sum = 0;
#pragma unroll
    for (int k = 0; k < kEmitItems; ++k) {
        const bool in = et + k < nv;
        const uint64_t e = in ? et + k : e0;
        const uint32_t c = snt[e];
        cnt[k] = in ? c : 0u;
        slot[k] = slots[e];
    }
    uint32_t key[kEmitItems];
    uint2 rc[kEmitItems];
#pragma unroll
    for (int k = 0; k < kEmitItems; ++k) {
        sum += cnt[k];
        rc[k] = rect[slot[k]];
        key[k] = slot_index(slot[k], (uint32_t)n, inv_n);  // submap index
    }
    uint32_t total = 0;
    const uint32_t first = emit_block_scan(sum, s_wave, &total);
    const uint64_t base = emit_block_prefix(es, n_blocks, eb);
    bool over = false;
    for (uint32_t w0 = 0; w0 < total; w0 += kEmitWin) {
        const uint32_t w1 = min(total, w0 + kEmitWin);
        uint32_t pos = first;
#pragma unroll
        for (int k = 0; k < kEmitItems; ++k) {
            const uint32_t c = cnt[k];
            // this element's pairs [pos, pos + c) clipped to the window
            const uint32_t j0 = pos < w0 ? w0 - pos : 0u;
            const uint32_t j1 = min(c, w1 > pos ? w1 - pos : 0u);
            if (j0 < j1) {
                const uint32_t tx0 = rc[k].x & 0xffffu, tx1 = rc[k].x >> 16, ty0 = rc[k].y & 0xffffu;
                const uint32_t w = tx1 - tx0 + 1;
                uint32_t ty = ty0 + j0 / w, tx = tx0 + j0 % w;
                for (uint32_t j = j0; j < j1; ++j) {
                    const uint32_t q = pos + j - w0;
                    s_tile[q] = (uint16_t)(ty * (uint32_t)tg.tiles_x + tx);
                    s_key[q] = key[k];
                    if (++tx > tx1) {
                        tx = tx0;
                        ++ty;
                    }
                }
            }
            pos += c;
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < w1 - w0; i += kThreads) {
            const uint64_t o = base + w0 + i;
            if (o < capacity) {
                ptile[o] = s_tile[i];
                pk[o] = s_key[i];
            } else {
                over = true;
            }
        }
        __syncthreads();
    }
    if (over) atomicOr(&flags[FLAG_OVERFLOW], 1);
}

}  // namespace

void launch_pack(hipStream_t s, int64_t n_map, const float *means, const float *scales, const float *quats,
                 const float *opacity, const float *rgb, const int64_t *index, int64_t n_sel, float4 *packed,
                 int *flags, unsigned long long *nonfinite) {
    launch_fill_u64(s, nonfinite, 1, 0ull);
    if (n_sel <= 0) return;
    const unsigned blocks = (unsigned)((n_sel + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_pack, dim3(blocks), dim3(kThreads), 0, s, n_map, means, scales, quats, opacity, rgb,
                       index, n_sel, packed, flags, nonfinite);
}

void launch_sum_nonfinite(hipStream_t s, const SubmapTable &tab, unsigned long long *total) {
    static_assert(kMaxBatchSubmaps <= 64, "one lane per submap");
    hipLaunchKernelGGL(k_sum_nonfinite, dim3(1), dim3(64), 0, s, tab, total);
}

int64_t preprocess_blocks(int64_t n) { return (n + kThreads - 1) / kThreads; }

void launch_preprocess(hipStream_t s, const SubmapTable &tab, int64_t n, const float *poses, int n_poses,
                       const Camera &cam, const Consts &k, const TileGrid &tg, float4 *records, uint2 *rect,
                       uint32_t *vz, uint32_t *vg, uint64_t *vmask, bool pack, unsigned long long *wide) {
    if (n <= 0) return;
    const dim3 grid((unsigned)preprocess_blocks(n), (unsigned)((n_poses + kPosesPerThread - 1) / kPosesPerThread));
    hipLaunchKernelGGL(k_preprocess, grid, dim3(kThreads), 0, s, tab, n, poses, n_poses, cam, k, tg, records,
                       rect, vz, vg, vmask, pack, wide);
}

uint64_t emit_blocks(uint64_t n_max) { return std::max<uint64_t>(1, (n_max + kEmitTile - 1) / kEmitTile); }

uint64_t emit_sums_size(uint64_t n_max) {
    const uint64_t nb = emit_blocks(n_max);
    return nb + 2 + (nb + kSumSpan - 1) / kSumSpan;
}

void launch_emit_sums(hipStream_t s, const SortedRun &run, const uint32_t *vbase, int n_poses, uint64_t n_max,
                      uint64_t *es) {
    const uint64_t nb = emit_blocks(n_max), spans = (nb + kSumSpan - 1) / kSumSpan;
    hipLaunchKernelGGL(k_emit_sums, dim3((unsigned)spans), dim3(kThreads), 0, s, run, vbase, n_poses, nb, es);
    // the span sums, scanned in place (only the spans in use); the pair total to es[nb]
    launch_block_scan(s, es + nb + 2, spans, es + nb + 1, es + nb);
}

void launch_pair_segments(hipStream_t s, const SortedRun &run, const uint32_t *vbase, int n_poses,
                          const uint64_t *es, uint64_t n_max, uint64_t capacity, uint64_t *pseg) {
    hipLaunchKernelGGL(k_pair_segments, dim3((unsigned)n_poses + 1), dim3(kThreads), 0, s, run, vbase, n_poses,
                       es, emit_blocks(n_max), capacity, pseg);
}

void launch_emit(hipStream_t s, const SortedRun &run, const uint32_t *vbase, int n_poses,
                 const uint2 *rect, int64_t n, uint64_t n_max, const uint64_t *es, const TileGrid &tg,
                 uint16_t *ptile, uint32_t *pk, uint64_t capacity, int *flags) {
    if (n <= 0) return;
    const uint64_t grid = (emit_blocks(n_max) + kXcdCount - 1) / kXcdCount * kXcdCount;  // see k_emit
    hipLaunchKernelGGL(k_emit, dim3((unsigned)grid), dim3(kThreads), 0, s, run, vbase, n_poses,
                       rect, n, es, emit_blocks(n_max), tg, ptile, pk, capacity, flags);
}

}  // namespace gsr
