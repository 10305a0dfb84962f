// Front-to-back compositing of colour and depth per 16x16 tile (S5).
//
// Paper: Sec. III-A, Eq. 1 and Eq. 5 with the footprint of Eq. 2:
//   C(x) = sum_i c_i a_i T_i,  D(x) = sum_i z_i a_i T_i,  T_i = prod_{j<i} (1 - a_j),
//   a_i = min(alpha_max, o_i exp(-d_i^2 / 2)) where d_i^2 <= cutoff and a_i >= alpha_min,
// over the depth-sorted list of the tile. A pixel stops after the layer that
// takes T below t_min (that layer counts).
//
// One 256-thread block per (tile, pose); wave w owns pixel rows 4w..4w+3 of the
// tile (a 16x4 band), one pixel per lane. The block walks the tile's list in
// chunks of 256 records: every thread stages one record in LDS (with the conic
// pre-scaled by -log2(e)/2 and a per-record log2 threshold that folds both the
// cutoff and the alpha floor into one compare) and marks which bands its pixel
// rectangle overlaps; a ballot per band turns the marks into one 256-bit mask
// per wave. Each wave then visits only the set bits, in list order, so a record
// costs a band nothing unless it can reach it. A wave stops when all of its
// pixels have stopped; the block stops loading when all waves have.
#include "internal.h"

namespace gsr {

namespace {

constexpr int kThreads = 256;
constexpr int kChunk = kThreads;
constexpr float kLog2e = 1.4426950408889634f;

struct BlendConsts {
    float neg_half_log2e;  // -log2(e)/2: p2 = -log2(e)/2 * d^2
    float cut_p2;          // -log2(e)/2 * cutoff_d2
    float log2_amin;       // log2(alpha_min)
    float alpha_max;
    float t_min;
};

template <bool kCount>
__global__ __launch_bounds__(kThreads) void k_blend(const float4 *__restrict__ records, int64_t n,
                                                    const uint32_t *__restrict__ pairs,
                                                    const uint64_t *__restrict__ offsets, uint64_t capacity,
                                                    int width, int height, int tiles_x, int n_tiles,
                                                    BlendConsts k, float *__restrict__ out_rgb,
                                                    float *__restrict__ out_depth, float *__restrict__ out_t,
                                                    unsigned long long *__restrict__ counters) {
    __shared__ float4 s_rec[kChunk * 3];
    __shared__ uint64_t s_mask[4][4];  // [band][wave that staged the records]

    const int tile = blockIdx.x, pose = blockIdx.y;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int pi = tx * 16 + (lane & 15);
    const int pj = ty * 16 + wave * 4 + (lane >> 4);
    const float px = (float)pi + 0.5f, py = (float)pj + 0.5f;
    const bool in_image = pi < width && pj < height;
    const int row0 = ty * 16;

    const uint64_t list = (uint64_t)pose * n_tiles + tile;
    const uint64_t beg = offsets[list];
    const uint64_t end = min(offsets[list + 1], capacity);
    const float4 *rec_pose = records + (int64_t)pose * n * 3;

    float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f, dep = 0.f;
    bool live = in_image;
    unsigned n_contrib = 0, n_visits = 0;  // only with kCount

    for (uint64_t c0 = beg; c0 < end; c0 += kChunk) {
        // stage one record per thread
        const uint64_t kk = c0 + tid;
        uint32_t bands = 0;
        if (kk < end) {
            const uint32_t g = pairs[kk];
            const float4 *r = rec_pose + (int64_t)g * 3;
            const float4 q0 = r[0], q1 = r[1], q2 = r[2];
            const float o = q1.y;
            const float thr = fmaxf(k.cut_p2, k.log2_amin - __log2f(o));
            s_rec[tid * 3 + 0] = make_float4(q0.x, q0.y, q0.z * k.neg_half_log2e, q0.w * (2.f * k.neg_half_log2e));
            s_rec[tid * 3 + 1] = make_float4(q1.x * k.neg_half_log2e, thr, o, q2.y);
            s_rec[tid * 3 + 2] = make_float4(q1.z, q1.w, q2.x, 0.f);
            const uint32_t ry = __float_as_uint(q2.w);
            const int j0 = (int)(ry & 0xffffu), j1 = (int)(ry >> 16);
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int b0 = row0 + 4 * b, b1 = b0 + 3;
                if (j0 <= b1 && j1 >= b0) bands |= 1u << b;
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint64_t m = __ballot((bands >> b) & 1u);
            if (lane == 0) s_mask[b][wave] = m;
        }
        __syncthreads();

        if (__ballot(live) != 0) {
            for (int sw = 0; sw < 4; ++sw) {
                // the mask is the same in every lane: move it to scalar registers so
                // the walk over its set bits is scalar control flow
                const uint64_t mv = s_mask[wave][sw];
                uint64_t m = ((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(mv >> 32)) << 32) |
                             (uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)mv);
                while (m) {
                    const int j = (int)__builtin_ctzll(m);
                    m &= m - 1;
                    const int idx = sw * 64 + j;
                    const float4 a = s_rec[idx * 3 + 0];
                    const float4 b = s_rec[idx * 3 + 1];
                    const float4 c = s_rec[idx * 3 + 2];
                    const float dx = px - a.x, dy = py - a.y;
                    const float p2 = (a.z * dx + a.w * dy) * dx + b.x * dy * dy;
                    float al = fminf(k.alpha_max, b.z * __builtin_amdgcn_exp2f(p2));
                    const bool ok = live && p2 >= b.y;
                    al = ok ? al : 0.f;
                    if (kCount) {
                        n_contrib += ok;
                        ++n_visits;
                    }
                    const float w = al * T;
                    cr += c.x * w;
                    cg += c.y * w;
                    cb += c.z * w;
                    dep += b.w * w;
                    T -= w;
                    live = live && !(T < k.t_min);
                }
                if (__ballot(live) == 0) goto wave_done;
            }
        }
    wave_done:
        if (__syncthreads_count(live) == 0) break;
    }

    if (kCount) {
        // contributions summed over the wave; visits are per wave (64 lane slots each)
        unsigned c = n_contrib;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        if (lane == 0) {
            atomicAdd(&counters[CNT_EVALS_CONTRIB], (unsigned long long)c);
            atomicAdd(&counters[CNT_EVALS_LANES], 64ull * n_visits);
        }
    }

    if (in_image) {
        const int64_t hw = (int64_t)width * height;
        const int64_t pix = (int64_t)pj * width + pi;
        float *rgb = out_rgb + (int64_t)pose * 3 * hw;
        rgb[pix] = cr;
        rgb[hw + pix] = cg;
        rgb[2 * hw + pix] = cb;
        out_depth[(int64_t)pose * hw + pix] = dep;
        if (out_t) out_t[(int64_t)pose * hw + pix] = T;
    }
}

}  // namespace

void launch_blend(hipStream_t s, const float4 *records, int64_t n, int n_poses, const uint32_t *pairs,
                  const uint64_t *offsets, uint64_t capacity, const Camera &cam, const Consts &k,
                  const TileGrid &tg, float *rgb, float *depth, float *tfinal, bool count_evals,
                  unsigned long long *counters) {
    BlendConsts bc;
    bc.neg_half_log2e = -0.5f * kLog2e;
    bc.cut_p2 = -0.5f * kLog2e * k.cutoff_d2;
    bc.log2_amin = log2f(k.alpha_min);
    bc.alpha_max = k.alpha_max;
    bc.t_min = k.t_min;
    const dim3 grid((unsigned)tg.n_tiles, (unsigned)n_poses);
    if (count_evals)
        hipLaunchKernelGGL(k_blend<true>, grid, dim3(kThreads), 0, s, records, n, pairs, offsets, capacity,
                           cam.width, cam.height, tg.tiles_x, tg.n_tiles, bc, rgb, depth, tfinal, counters);
    else
        hipLaunchKernelGGL(k_blend<false>, grid, dim3(kThreads), 0, s, records, n, pairs, offsets, capacity,
                           cam.width, cam.height, tg.tiles_x, tg.n_tiles, bc, rgb, depth, tfinal, counters);
}

}  // namespace gsr
