// Normalised cross-correlation of the query against every render (S6) and
// selection of the best candidates (S7).
//
// Paper: Sec. III-C1, Eq. 10: NCC = sum (q - mean_q)(g - mean_g) /
// (sqrt(sum (q - mean_q)^2) sqrt(sum (g - mean_g)^2)) over all pixels; the
// brute-force search keeps the most similar render.
//
// Grey = 0.299 R + 0.587 G + 0.114 B. Each block reads 4096 pixels of one render
// once (12 B/px, coalesced, 16 B per lane and load where the layout allows) plus the query's grey image (4 B/px, shared by all
// renders and so mostly served from cache), computes the block's counts,
// means, centred sums of squares and co-moment by a two-pass reduction about a
// shift (the block's first pixel, so a constant block gives exactly zero
// spread), and stores them in float64. One block per render then merges the
// partials in a fixed order with the pairwise (Chan et al.) update, so the
// score is deterministic. A render or query with zero spread scores 0.
#include "internal.h"

namespace gsr {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kPix = kThreads * kItems;  // pixels per partial block
constexpr int kPartial = 6;              // n, mean_q, mean_g, m2_q, m2_g, c_qg

__device__ __forceinline__ float grey(float r, float g, float b) { return 0.299f * r + 0.587f * g + 0.114f * b; }

__global__ __launch_bounds__(kThreads) void k_grey(const float *__restrict__ rgb, int64_t hw, float *__restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < hw; i += (int64_t)gridDim.x * kThreads)
        out[i] = grey(rgb[i], rgb[hw + i], rgb[2 * hw + i]);
}

// Sum of three floats across the block (fixed order: in-wave butterfly, then waves 0..3).
__device__ void block_sum3(float &a, float &b, float &c, float *s /*[3][4]*/) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o, 64);
        b += __shfl_xor(b, o, 64);
        c += __shfl_xor(c, o, 64);
    }
    if (lane == 0) {
        s[wave] = a;
        s[4 + wave] = b;
        s[8 + wave] = c;
    }
    __syncthreads();
    a = (s[0] + s[1]) + (s[2] + s[3]);
    b = (s[4] + s[5]) + (s[6] + s[7]);
    c = (s[8] + s[9]) + (s[10] + s[11]);
    __syncthreads();
}

// kVec (4 | hw and 16-byte aligned planes): each thread reads 4 consecutive
// pixels per load (float4), 16 pixels in 4 loads per plane; otherwise one pixel
// per load, 256 apart.
template <bool kVec>
__global__ __launch_bounds__(kThreads) void k_ncc_partial(const float *__restrict__ qgrey,
                                                          const float *__restrict__ renders, int64_t hw,
                                                          int n_blocks, double *__restrict__ partials) {
    __shared__ float s_red[12];
    const int blk = blockIdx.x, pose = blockIdx.y;
    const float *rgb = renders + (int64_t)pose * 3 * hw;
    const int64_t base = (int64_t)blk * kPix;
    const int64_t nvalid = min((int64_t)kPix, hw - base);
    // block-relative position of this thread's item i (kVec: 4 | nvalid, so a group
    // of 4 is valid or not as a whole)
    auto item_loc = [&](int i) -> int64_t {
        if constexpr (kVec)
            return ((int64_t)(i >> 2) * kThreads + threadIdx.x) * 4 + (i & 3);
        else
            return (int64_t)i * kThreads + threadIdx.x;
    };
    float q[kItems], g[kItems];
    const float sq = qgrey[base];
    const float sg = grey(rgb[base], rgb[hw + base], rgb[2 * hw + base]);
    float aq = 0.f, ag = 0.f, dummy = 0.f;
    if constexpr (kVec) {
#pragma unroll
        for (int i = 0; i < kItems / 4; ++i) {
            const int64_t loc = item_loc(4 * i);
            if (loc < nvalid) {
                const int64_t pix = base + loc;
                const float4 qv = *reinterpret_cast<const float4 *>(qgrey + pix);
                const float4 rv = *reinterpret_cast<const float4 *>(rgb + pix);
                const float4 gv = *reinterpret_cast<const float4 *>(rgb + hw + pix);
                const float4 bv = *reinterpret_cast<const float4 *>(rgb + 2 * hw + pix);
                q[4 * i + 0] = qv.x - sq;
                q[4 * i + 1] = qv.y - sq;
                q[4 * i + 2] = qv.z - sq;
                q[4 * i + 3] = qv.w - sq;
                g[4 * i + 0] = grey(rv.x, gv.x, bv.x) - sg;
                g[4 * i + 1] = grey(rv.y, gv.y, bv.y) - sg;
                g[4 * i + 2] = grey(rv.z, gv.z, bv.z) - sg;
                g[4 * i + 3] = grey(rv.w, gv.w, bv.w) - sg;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    aq += q[4 * i + k];
                    ag += g[4 * i + k];
                }
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    q[4 * i + k] = 0.f;
                    g[4 * i + k] = 0.f;
                }
            }
        }
    } else {
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            const int64_t loc = item_loc(i);
            const int64_t pix = base + loc;
            if (loc < nvalid) {
                q[i] = qgrey[pix] - sq;
                g[i] = grey(rgb[pix], rgb[hw + pix], rgb[2 * hw + pix]) - sg;
                aq += q[i];
                ag += g[i];
            } else {
                q[i] = 0.f;
                g[i] = 0.f;
            }
        }
    }
    block_sum3(aq, ag, dummy, s_red);
    const float inv_n = 1.f / (float)nvalid;
    const float mq = aq * inv_n, mg = ag * inv_n;  // means relative to the shifts
    float m2q = 0.f, m2g = 0.f, cqg = 0.f;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        if (item_loc(i) < nvalid) {
            const float dq = q[i] - mq, dg = g[i] - mg;
            m2q += dq * dq;
            m2g += dg * dg;
            cqg += dq * dg;
        }
    }
    block_sum3(m2q, m2g, cqg, s_red);
    if (threadIdx.x == 0) {
        double *o = partials + ((int64_t)pose * n_blocks + blk) * kPartial;
        o[0] = (double)nvalid;
        o[1] = (double)sq + (double)mq;
        o[2] = (double)sg + (double)mg;
        o[3] = (double)m2q;
        o[4] = (double)m2g;
        o[5] = (double)cqg;
    }
}

struct Moments {
    double n, mq, mg, m2q, m2g, c;
};

__device__ Moments merge(const Moments &a, const Moments &b) {
    if (a.n == 0.0) return b;
    if (b.n == 0.0) return a;
    Moments r;
    r.n = a.n + b.n;
    const double dq = b.mq - a.mq, dg = b.mg - a.mg;
    const double f = a.n * b.n / r.n;
    r.mq = a.mq + dq * (b.n / r.n);
    r.mg = a.mg + dg * (b.n / r.n);
    r.m2q = a.m2q + b.m2q + dq * dq * f;
    r.m2g = a.m2g + b.m2g + dg * dg * f;
    r.c = a.c + b.c + dq * dg * f;
    return r;
}

__global__ __launch_bounds__(kThreads) void k_ncc_final(const double *__restrict__ partials, int n_blocks,
                                                        float *__restrict__ scores) {
    __shared__ Moments s[kThreads];
    const int pose = blockIdx.x;
    Moments acc = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < n_blocks; b += kThreads) {
        const double *p = partials + ((int64_t)pose * n_blocks + b) * kPartial;
        const Moments m = {p[0], p[1], p[2], p[3], p[4], p[5]};
        acc = merge(acc, m);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) s[threadIdx.x] = merge(s[threadIdx.x], s[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const Moments &m = s[0];
        double v = 0.0;
        if (m.m2q > 0.0 && m.m2g > 0.0) v = m.c / (sqrt(m.m2q) * sqrt(m.m2g));
        scores[pose] = (float)v;
    }
}

// Ascending order of the key = descending score, then ascending index; a NaN
// score ranks after every number (-inf included).
__device__ __forceinline__ uint64_t rank_key(float score, uint32_t idx) {
    if (__builtin_isnan(score)) return (0xffffffffull << 32) | idx;
    uint32_t b = __float_as_uint(score);
    b = (b & 0x80000000u) ? ~b : (b | 0x80000000u);  // ascending in score
    return ((uint64_t)(~b) << 32) | idx;
}

constexpr int kTopkCap = 8192;

__global__ __launch_bounds__(1024) void k_topk(const float *__restrict__ scores, int n, int k,
                                               int32_t *__restrict__ out) {
    __shared__ uint64_t s[kTopkCap];
    int m = 1;
    while (m < n) m <<= 1;
    for (int i = threadIdx.x; i < m; i += blockDim.x) s[i] = i < n ? rank_key(scores[i], (uint32_t)i) : ~0ull;
    __syncthreads();
    for (int kk = 2; kk <= m; kk <<= 1) {
        for (int j = kk >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < (m >> 1); i += blockDim.x) {
                const int lo = 2 * j * (i / j) + (i % j), hi = lo + j;
                const bool up = (lo & kk) == 0;
                const uint64_t a = s[lo], b = s[hi];
                if ((a > b) == up) {
                    s[lo] = b;
                    s[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < k; i += blockDim.x) out[i] = (int32_t)(uint32_t)(s[i] & 0xffffffffu);
}

// Random-order search (S7): the poses of one batch, poses[order[i]], gathered into
// a dense [nb][3][4] array; and the batch's scores written back to their candidates.
__global__ void k_gather_poses(const float *__restrict__ poses, const int32_t *__restrict__ order, int nb,
                               float *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb * 12) return;
    out[i] = poses[(int64_t)order[i / 12] * 12 + i % 12];
}

__global__ void k_scatter_scores(const float *__restrict__ batch_scores, const int32_t *__restrict__ order, int nb,
                                 float *__restrict__ scores) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) scores[order[i]] = batch_scores[i];
}

}  // namespace

int ncc_pixels_per_block() { return kPix; }

void launch_ncc(hipStream_t s, const float *query, const float *renders, int n_poses, int height, int width,
                float *grey_q, double *partials, float *scores) {
    const int64_t hw = (int64_t)height * width;
    const int nb = (int)((hw + kPix - 1) / kPix);
    const unsigned gblocks = (unsigned)std::min<int64_t>((hw + kThreads - 1) / kThreads, 2048);
    hipLaunchKernelGGL(k_grey, dim3(gblocks), dim3(kThreads), 0, s, query, hw, grey_q);
    // whole float4 groups: 4 | hw (so every block's pixel count and every plane's
    // start are multiples of 4) and 16-byte aligned bases
    const bool vec = hw % 4 == 0 && reinterpret_cast<uintptr_t>(renders) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(grey_q) % 16 == 0;
    if (vec)
        hipLaunchKernelGGL(k_ncc_partial<true>, dim3((unsigned)nb, (unsigned)n_poses), dim3(kThreads), 0, s, grey_q,
                           renders, hw, nb, partials);
    else
        hipLaunchKernelGGL(k_ncc_partial<false>, dim3((unsigned)nb, (unsigned)n_poses), dim3(kThreads), 0, s, grey_q,
                           renders, hw, nb, partials);
    hipLaunchKernelGGL(k_ncc_final, dim3((unsigned)n_poses), dim3(kThreads), 0, s, partials, nb, scores);
}

void launch_topk(hipStream_t s, const float *scores, int n, int k, int32_t *idx) {
    hipLaunchKernelGGL(k_topk, dim3(1), dim3(1024), 0, s, scores, n, k, idx);
}

void launch_gather_poses(hipStream_t s, const float *poses, const int32_t *order, int nb, float *out) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_gather_poses, dim3((unsigned)((nb * 12 + 255) / 256)), dim3(256), 0, s, poses, order, nb, out);
}

void launch_scatter_scores(hipStream_t s, const float *batch_scores, const int32_t *order, int nb, float *scores) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_scatter_scores, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, batch_scores, order, nb,
                       scores);
}

}  // namespace gsr
