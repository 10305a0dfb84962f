// Learned candidate scorer: a small CNN that predicts the NCC of a candidate
// from its low-resolution render and the low-resolution query, used to prune
// the candidate set before the full-resolution comparison of Eq. 10.
//
// Network (NHWC activations, 3x3 convolutions with zero padding 1):
//   conv 2->32 /2, ReLU; conv 32->64, ReLU; conv 64->64 /2, ReLU;
//   conv 64->128, ReLU; conv 128->128 /2, ReLU; global average pool;
//   linear 128->128, ReLU; linear 128->1.
// Weights and activations are bfloat16 (round to nearest even), sums are
// float32 on the matrix cores (v_mfma_f32_32x32x16_bf16); the pooled features,
// the two linear layers, the loss and AdamW are float32 on the vector ALUs.
//
// The three convolution products are implicit GEMMs:
//   forward        rows = output channels, cols = output pixels, K = (tap, c_in)
//                  (so a lane's accumulators hold four consecutive channels of
//                  one pixel at a time, which leave in one 8-byte store)
//   backward data  rows = input pixels of one sub-pixel class (for stride 2 the
//                  four (y mod 2, x mod 2) classes each see a fixed set of taps,
//                  so no MFMA is spent on taps that skip the pixel),
//                  cols = input channels, K = (tap, c_out)
//   backward weight rows = output channels, cols = (tap, c_in), K = output
//                  pixels, split over row ranges into float32 partial sums that
//                  a second kernel adds in a fixed order (deterministic).
// MFMA operand layout of 32x32x16: lane l supplies row (or column) l % 32 and
// the eight K entries 8 (l / 32) .. 8 (l / 32) + 7; accumulator element i of
// lane l is row 8 (i / 4) + 4 (l / 32) + i % 4, column l % 32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace gsr {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef uint16_t u16;

__device__ inline u16 to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40u);  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}
__device__ inline float from_bf16(u16 h) { return __uint_as_float((uint32_t)h << 16); }

__device__ inline bf16x8 load8(const u16 *p) { return __builtin_bit_cast(bf16x8, *(const u32x4 *)p); }
__device__ inline bf16x8 zero8() {
    u32x4 z = {0u, 0u, 0u, 0u};
    return __builtin_bit_cast(bf16x8, z);
}
__device__ inline bf16x8 pack8(const uint32_t (&w)[4]) {
    u32x4 v = {w[0], w[1], w[2], w[3]};
    return __builtin_bit_cast(bf16x8, v);
}
__device__ inline f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// relu(acc + bias) of four consecutive output channels as bfloat16 (round to
// nearest even, as to_bf16: the hardware conversion of finite and infinite
// values), packed for one 8-byte store.
__device__ inline uint2 relu_bf16x4(float a0, float a1, float a2, float a3, float4 b) {
    const f32x2 lo = {fmaxf(a0 + b.x, 0.f), fmaxf(a1 + b.y, 0.f)};
    const f32x2 hi = {fmaxf(a2 + b.z, 0.f), fmaxf(a3 + b.w, 0.f)};
    return make_uint2(__builtin_bit_cast(uint32_t, __builtin_convertvector(lo, bf16x2)),
                      __builtin_bit_cast(uint32_t, __builtin_convertvector(hi, bf16x2)));
}

// Forward epilogue of a wave whose accumulators hold D[c_out][pixel] (the
// weights are the MFMA's A operand, the pixels its B operand): lane l holds the
// pixel in column l % 32 of each pixel block r and, for g = 0..3, the output
// channels 32 c + 8 g + 4 (l / 32) .. + 3 of each channel block c. Lanes l and
// l + 32 hold the same pixel, so one lane-half swap (v_permlane32_swap, lanes
// 32..63 of the first operand with lanes 0..31 of the second) per register of
// groups g and g + 1 gives lane l channels 16 h .. 16 h + 7 and lane l + 32
// channels 16 h + 8 .. 16 h + 15 (h = g / 2), each leaving as one 16-byte store
// (two per 32 channels instead of four 8-byte stores). dst[r]: the lane's
// pixel's first output channel of the wave's channel range (null: the pixel is
// outside the output, for both lanes of the pair).
// The biases a lane's accumulators need (its RN channel blocks from `bias`), for
// store_relu_bf16: loaded ahead of the main loop, so that their latency is not
// waited out in the epilogue.
template <int RN>
struct LaneBias {
    float4 v[RN][4];
};
template <int RN>
__device__ inline LaneBias<RN> load_lane_bias(const float *bias) {
    const int kq = (threadIdx.x & 63) >> 5;
    LaneBias<RN> b;
#pragma unroll
    for (int c = 0; c < RN; ++c)
#pragma unroll
        for (int g = 0; g < 4; ++g) b.v[c][g] = *(const float4 *)(bias + 32 * c + 8 * g + 4 * kq);
    return b;
}

template <int RM, int RN>
__device__ inline void store_relu_bf16(const f32x16 (&acc)[RM][RN], u16 *const (&dst)[RM], const LaneBias<RN> &bv) {
    const int kq = (threadIdx.x & 63) >> 5;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        if (!dst[r]) continue;
#pragma unroll
        for (int c = 0; c < RN; ++c) {
            uint2 q[4];
#pragma unroll
            for (int g = 0; g < 4; ++g)
                q[g] = relu_bf16x4(acc[r][c][4 * g], acc[r][c][4 * g + 1], acc[r][c][4 * g + 2],
                                   acc[r][c][4 * g + 3], bv.v[c][g]);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const auto sx = __builtin_amdgcn_permlane32_swap(q[2 * h].x, q[2 * h + 1].x, false, false);
                const auto sy = __builtin_amdgcn_permlane32_swap(q[2 * h].y, q[2 * h + 1].y, false, false);
                *(uint4 *)(dst[r] + 32 * c + 16 * h + 8 * kq) = make_uint4(sx[0], sy[0], sx[1], sy[1]);
            }
        }
    }
}

template <typename T>
__device__ inline T block_sum(T v, T *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    T s = 0;
    for (int w = 0; w < nw; ++w) s += red[w];
    return s;
}

// ---- input preparation ----

__device__ inline float grey_of(float r, float g, float b) { return 0.299f * r + 0.587f * g + 0.114f * b; }

// out[p][y][x] = mean over the f x f block of the grey of rgb[p][3][H][W].
__global__ void k_pool_grey(const float *__restrict__ rgb, int P, int H, int W, int f, float *__restrict__ out) {
    const int h = H / f, w = W / f;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)P * h * w) return;
    const int p = (int)(i / ((int64_t)h * w));
    const int r = (int)(i - (int64_t)p * h * w), y = r / w, x = r - y * w;
    const int64_t plane = (int64_t)H * W;
    const float *src = rgb + (int64_t)p * 3 * plane;
    float s = 0.f;
    for (int dy = 0; dy < f; ++dy)
        for (int dx = 0; dx < f; ++dx) {
            const int64_t o = (int64_t)(y * f + dy) * W + x * f + dx;
            s += grey_of(src[o], src[plane + o], src[2 * plane + o]);
        }
    out[i] = s / (float)(f * f);
}

// Mean and reciprocal standard deviation of an image, summed in float64 (the
// sum of a constant image is then exact and its variance exactly 0); rstd = 0
// for a constant image, which then standardises to zeros.
__device__ inline void image_stats(double sum, double m2, int n, float &mean, float &rstd) {
    mean = (float)(sum / n);
    rstd = m2 > 0.0 ? (float)(1.0 / sqrt(m2 / n)) : 0.f;
}

// stats[0], stats[1] = mean and rstd of the query grey image q[n].
__global__ __launch_bounds__(1024) void k_query_stats(const float *__restrict__ q, int n, float *__restrict__ stats) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += q[i];
    const double sum = block_sum(s, red), mu = sum / n;
    double m2 = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double d = q[i] - mu;
        m2 += d * d;
    }
    m2 = block_sum(m2, red);
    if (threadIdx.x == 0) {
        float mean, rstd;
        image_stats(sum, m2, n, mean, rstd);
        stats[0] = mean;
        stats[1] = rstd;
    }
}

// x[b][y][x][0] = standardised grey of render b, x[b][y][x][1] = standardised
// query; one block per render.
__global__ __launch_bounds__(1024) void k_scorer_input(const float *__restrict__ rgb, int h, int w,
                                                        const float *__restrict__ q, const float *__restrict__ qstats,
                                                        u16 *__restrict__ x) {
    __shared__ double red[16];
    const int n = h * w;
    const float *src = rgb + (int64_t)blockIdx.x * 3 * n;
    // four pixels per thread and step, their loads in flight together (clamped)
    const int stride = blockDim.x;
    auto grey4 = [&](int i0, float (&gv)[4]) {
        float r[4], g[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = min(i0 + u * stride, n - 1);
            r[u] = src[i];
            g[u] = src[n + i];
            b[u] = src[2 * n + i];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) gv[u] = grey_of(r[u], g[u], b[u]);
    };
    double s = 0.0;
    for (int i0 = threadIdx.x; i0 < n; i0 += 4 * stride) {
        float gv[4];
        grey4(i0, gv);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + u * stride < n) s += gv[u];
    }
    const double sum = block_sum(s, red), mu = sum / n;
    double m2 = 0.0;
    for (int i0 = threadIdx.x; i0 < n; i0 += 4 * stride) {
        float gv[4];
        grey4(i0, gv);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + u * stride < n) {
                const double d = gv[u] - mu;
                m2 += d * d;
            }
    }
    m2 = block_sum(m2, red);
    float mean, rstd;
    image_stats(sum, m2, n, mean, rstd);
    const float qm = qstats[0], qr = qstats[1];
    uint32_t *dst = (uint32_t *)(x + (int64_t)blockIdx.x * 2 * n);
    for (int i0 = threadIdx.x; i0 < n; i0 += 4 * stride) {
        float gv[4], qv[4];
        grey4(i0, gv);
#pragma unroll
        for (int u = 0; u < 4; ++u) qv[u] = q[min(i0 + u * stride, n - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + u * stride < n) {
                const float g = (gv[u] - mean) * rstd;
                const float v = (qv[u] - qm) * qr;
                dst[i0 + u * stride] = (uint32_t)to_bf16(g) | ((uint32_t)to_bf16(v) << 16);
            }
    }
}

// ---- convolutions ----

struct ConvDims {
    int n, H, W, Ho, Wo;  // images, input height and width, output height and width
};

// Forward: y = relu(conv(x, W) + b) in bf16. Block = 4 waves in a WGM x WGN
// grid; each wave owns RM x RN accumulator tiles of 32 x 32; block (x, n) takes
// output pixels [BM x, BM x + BM) of image n.
template <int CI, int CO, int S, int RM, int RN, int WGN>
__global__ __launch_bounds__(256) void k_conv_fwd(const u16 *__restrict__ x, ConvDims d, const u16 *__restrict__ wt,
                                                   const float *__restrict__ bias, u16 *__restrict__ y) {
    constexpr int WGM = 4 / WGN, BM = WGM * RM * 32;
    static_assert(WGN * RN * 32 == CO, "wave grid must cover the output channels");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    const int r32 = lane & 31, kq = lane >> 5;
    const int hw = d.Ho * d.Wo;
    const int n = blockIdx.y;
    const int m0 = blockIdx.x * BM + wm * RM * 32;  // within image n
    int iy0[RM], ix0[RM];
    int64_t img[RM];
    bool live[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const int m = m0 + 32 * r + r32;
        live[r] = m < hw;
        const int mm = live[r] ? m : 0;
        const int oy = mm / d.Wo, ox = mm - oy * d.Wo;
        iy0[r] = oy * S - 1;
        ix0[r] = ox * S - 1;
        img[r] = (int64_t)n * d.H * d.W;
    }
    f32x16 acc[RM][RN];
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int c = 0; c < RN; ++c)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[r][c][i] = 0.f;
    const int cob = wn * RN * 32;
    if constexpr (CI == 2) {
        // K = 18 = (tap, c_in), padded to 32: two K steps of 16.
#pragma unroll
        for (int sub = 0; sub < 2; ++sub) {
            bf16x8 a[RM], b[RN];
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                uint32_t wv[4];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    // (loaded from a clamped address, not under a branch, so that the
                    // eight loads of a lane are in flight together)
                    const int tap = 8 * sub + 4 * kq + jj;
                    const int iy = iy0[r] + tap / 3, ix = ix0[r] + tap % 3;
                    const bool ok = live[r] && tap < 9 && iy >= 0 && iy < d.H && ix >= 0 && ix < d.W;
                    const int64_t o = img[r] + (ok ? (int64_t)iy * d.W + ix : 0);
                    const uint32_t v = *(const uint32_t *)(x + o * 2);
                    wv[jj] = ok ? v : 0u;
                }
                a[r] = pack8(wv);
            }
#pragma unroll
            for (int c = 0; c < RN; ++c) {
                uint32_t wv[4];
                const int co = cob + 32 * c + r32;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    const int tap = 8 * sub + 4 * kq + jj;
                    const uint32_t v = *(const uint32_t *)(wt + co * 18 + 2 * (tap < 9 ? tap : 0));
                    wv[jj] = tap < 9 ? v : 0u;
                }
                b[c] = pack8(wv);
            }
#pragma unroll
            for (int r = 0; r < RM; ++r)
#pragma unroll
                for (int c = 0; c < RN; ++c) acc[r][c] = mfma(b[c], a[r], acc[r][c]);  // D[c_out][pixel]
        }
    } else {
        for (int tap = 0; tap < 9; ++tap) {
            const int kh = tap / 3, kw = tap - 3 * kh;
            const u16 *src[RM];
            bool ok[RM];
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                const int iy = iy0[r] + kh, ix = ix0[r] + kw;
                ok[r] = live[r] && iy >= 0 && iy < d.H && ix >= 0 && ix < d.W;
                src[r] = x + (img[r] + (int64_t)(ok[r] ? iy : 0) * d.W + (ok[r] ? ix : 0)) * CI + 8 * kq;
            }
            const u16 *wsrc = wt + ((int64_t)(cob + r32) * 9 + tap) * CI + 8 * kq;
#pragma unroll
            for (int c0 = 0; c0 < CI; c0 += 16) {
                bf16x8 a[RM], b[RN];
#pragma unroll
                for (int r = 0; r < RM; ++r) a[r] = ok[r] ? load8(src[r] + c0) : zero8();
#pragma unroll
                for (int c = 0; c < RN; ++c) b[c] = load8(wsrc + (int64_t)32 * c * 9 * CI + c0);
#pragma unroll
                for (int r = 0; r < RM; ++r)
#pragma unroll
                    for (int c = 0; c < RN; ++c) acc[r][c] = mfma(b[c], a[r], acc[r][c]);  // D[c_out][pixel]
            }
        }
    }
    if constexpr (WGN == 1) {
        // A wave's RM x 32 pixels are consecutive in the output and it holds all
        // of their channels: the results go through LDS (rows padded by 16 bytes)
        // and leave in 16-byte stores of consecutive addresses, instead of 8-byte
        // stores a pixel row (CO x 2 bytes) apart.
        constexpr int PXW = RM * 32, ROWB = CO * 2 + 16, PPP = CO * 2 / 16;  // pixels, row bytes, pieces per pixel
        __shared__ __align__(16) unsigned char s_out[4][PXW * ROWB];
        unsigned char *so = s_out[wave];
        const LaneBias<RN> bv = load_lane_bias<RN>(bias);
#pragma unroll
        for (int r = 0; r < RM; ++r)
#pragma unroll
            for (int c = 0; c < RN; ++c)
#pragma unroll
                for (int g = 0; g < 4; ++g)
                    *(uint2 *)(so + (32 * r + r32) * ROWB + (32 * c + 8 * g + 4 * kq) * 2) =
                        relu_bf16x4(acc[r][c][4 * g], acc[r][c][4 * g + 1], acc[r][c][4 * g + 2],
                                    acc[r][c][4 * g + 3], bv.v[c][g]);
        __builtin_amdgcn_wave_barrier();  // (one wave's LDS accesses complete in program order)
#pragma unroll
        for (int t = lane; t < PXW * PPP; t += 64) {
            const int px = t / PPP, part = t - px * PPP;
            if (m0 + px < hw)
                *(uint4 *)(y + ((int64_t)n * hw + m0 + px) * CO + 8 * part) =
                    *(const uint4 *)(so + px * ROWB + 16 * part);
        }
    } else {
        u16 *dst[RM];
#pragma unroll
        for (int r = 0; r < RM; ++r)
            dst[r] = live[r] ? y + ((int64_t)n * hw + m0 + 32 * r + r32) * CO + cob : nullptr;
        store_relu_bf16<RM, RN>(acc, dst, load_lane_bias<RN>(bias + cob));
    }
}

// Forward for c_in >= 32, LDS-staged: one block computes a TH x TW tile of output
// pixels of one image for all output channels. Per chunk of 32 input channels
// the block stages the tile's input halo ((TH-1) S + 3 rows x (TW-1) S + 3
// columns) in LDS once, and all nine taps read their B fragments from it; the
// taps' weights [c_out][32] go through two LDS buffers, each tap's fetched into
// registers two taps ahead, with one barrier per tap. (Staging all nine taps'
// weights at once needs up to 135 KB of LDS, one block per compute unit, and
// measured 1.5x slower.) Rows of
// 32 channels are padded to 80 bytes, so the 16-byte fragment reads of 16
// consecutive pixels (or channels) hit distinct banks; for stride 2 the halo is
// stored as even and odd column planes, so that strided pixels are consecutive
// in LDS as well. PIPE: the taps of all chunks form one pipeline (the next
// chunk's halo is loaded into registers while this chunk's taps compute);
// otherwise each chunk loads its halo and first weights before its taps.
template <int CI, int CO, int S, int TH, int TW, int WGN, bool PIPE>
__global__ __launch_bounds__(256) void k_conv_fwd_lds(const u16 *__restrict__ x, ConvDims d,
                                                       const u16 *__restrict__ wt, const float *__restrict__ bias,
                                                       u16 *__restrict__ y) {
    constexpr int WGM = 4 / WGN, BM = TH * TW;
    constexpr int RM = BM / (WGM * 32), RN = CO / (WGN * 32);
    static_assert(RM >= 1 && RN >= 1 && WGM * RM * 32 == BM && WGN * RN * 32 == CO, "tile and wave grid");
    static_assert(CI % 32 == 0, "channel chunks of 32");
    constexpr int HH = (TH - 1) * S + 3, HWD = (TW - 1) * S + 3;
    constexpr int PW = S == 1 ? HWD : (HWD + 1) / 2;  // columns per plane
    constexpr int SLOTS = S == 1 ? HH * HWD : HH * 2 * PW;
    constexpr int ROW = 40;                              // bf16 per LDS row (32 + 8 padding)
    __shared__ __align__(16) u16 s_halo[SLOTS * ROW];
    __shared__ __align__(16) u16 s_b[2][CO * ROW];  // the weights of taps t (t & 1) and t + 1

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    const int r32 = lane & 31, kq = lane >> 5;
    const int n = blockIdx.z, oy0 = blockIdx.y * TH, ox0 = blockIdx.x * TW;
    const int iy0 = oy0 * S - 1, ix0 = ox0 * S - 1;
    const u16 *ximg = x + (int64_t)n * d.H * d.W * CI;
    auto slot_of = [](int hy, int hx) { return S == 1 ? hy * HWD + hx : (hy * 2 + (hx & 1)) * PW + (hx >> 1); };

    // this lane's output pixels (tile-local) for each of its row blocks
    int ty[RM], tx[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const int m = wm * RM * 32 + 32 * r + r32;
        ty[r] = m / TW;
        tx[r] = m - ty[r] * TW;
    }
    f32x16 acc[RM][RN];
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int c = 0; c < RN; ++c)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[r][c][i] = 0.f;

    constexpr int BPIECES = CO * 4;                      // 16-byte pieces of one tap's weights
    constexpr int BPER = (BPIECES + 255) / 256;
    u32x4 bpre[BPER];
    auto fetch_b = [&](int tap, int ci0) {
#pragma unroll
        for (int j = 0; j < BPER; ++j) {
            const int p = tid + 256 * j;
            if (p < BPIECES) {
                const int co = p >> 2, q = p & 3;
                bpre[j] = *(const u32x4 *)(wt + ((int64_t)co * 9 + tap) * CI + ci0 + 8 * q);
            }
        }
    };
    auto store_b = [&](int buf) {
#pragma unroll
        for (int j = 0; j < BPER; ++j) {
            const int p = tid + 256 * j;
            if (p < BPIECES) *(u32x4 *)(s_b[buf] + (p >> 2) * ROW + 8 * (p & 3)) = bpre[j];
        }
    };

    if constexpr (PIPE) {
        // the halo's 16-byte pieces of one chunk of 32 input channels, loaded from
        // clamped addresses (none under a branch, so that a thread's loads are in
        // flight together)
        constexpr int NCH = CI / 32, HPIECES = HH * HWD * 4, HPER = (HPIECES + 255) / 256;
        static_assert(HPER <= 32, "one mask bit per piece");
        u32x4 hv[HPER];
        uint32_t hin = 0;  // bit j: piece j lies inside the image (else it goes to LDS as zeros)
        auto load_halo = [&](int ci0) {
            hin = 0;
#pragma unroll
            for (int j = 0; j < HPER; ++j) {
                const int p = min(tid + 256 * j, HPIECES - 1);
                const int pix = p >> 2, q = p & 3;
                const int hy = pix / HWD, hx = pix - hy * HWD;
                const int iy = iy0 + hy, ix = ix0 + hx;
                const bool in = iy >= 0 && iy < d.H && ix >= 0 && ix < d.W;
                // (kept as loaded: a select here would wait for the load at once)
                hv[j] = *(const u32x4 *)(ximg + ((int64_t)(in ? iy : 0) * d.W + (in ? ix : 0)) * CI + ci0 + 8 * q);
                hin |= (uint32_t)in << j;
            }
        };
        auto store_halo = [&]() {
#pragma unroll
            for (int j = 0; j < HPER; ++j) {
                const int p = tid + 256 * j;
                if (p < HPIECES) {
                    const int pix = p >> 2, q = p & 3;
                    const int hy = pix / HWD, hx = pix - hy * HWD;
                    const u32x4 z = {0u, 0u, 0u, 0u};
                    *(u32x4 *)(s_halo + slot_of(hy, hx) * ROW + 8 * q) = ((hin >> j) & 1u) ? hv[j] : z;
                }
            }
        };
        // Steps st = 9 chunk + tap over all chunks: the weights of step st + 1 (fetched
        // during step st - 1) go to the buffer that step st - 1 read, past the last
        // barrier, and those of st + 2 are fetched while st computes; the next
        // chunk's halo is loaded into registers while this chunk's taps compute.
        constexpr int STEPS = 9 * NCH;
        load_halo(0);
        store_halo();
        fetch_b(0, 0);
        store_b(0);
        fetch_b(1, 0);
        if (NCH > 1) load_halo(32);
        __syncthreads();
        for (int st = 0; st < STEPS; ++st) {
            const int ch = st / 9, tap = st - 9 * ch;
            const int kh = tap / 3, kw = tap - 3 * kh;
            if (st + 1 < STEPS) {
                store_b((st + 1) & 1);
                if (st + 2 < STEPS) fetch_b((st + 2) % 9, 32 * ((st + 2) / 9));
            }
#pragma unroll
            for (int kk = 0; kk < 2; ++kk) {
                bf16x8 a[RM], b[RN];
#pragma unroll
                for (int r = 0; r < RM; ++r)
                    a[r] = __builtin_bit_cast(
                        bf16x8, *(const u32x4 *)(s_halo + slot_of(ty[r] * S + kh, tx[r] * S + kw) * ROW + 16 * kk + 8 * kq));
#pragma unroll
                for (int c = 0; c < RN; ++c)
                    b[c] = __builtin_bit_cast(
                        bf16x8, *(const u32x4 *)(s_b[st & 1] + (wn * RN * 32 + 32 * c + r32) * ROW + 16 * kk + 8 * kq));
#pragma unroll
                for (int r = 0; r < RM; ++r)
#pragma unroll
                    for (int c = 0; c < RN; ++c) acc[r][c] = mfma(b[c], a[r], acc[r][c]);  // D[c_out][pixel]
            }
            if (st + 1 < STEPS) {
                __syncthreads();  // step st + 1's weights are in LDS, and step st's buffer is free
                if (tap == 8) {
                    // every wave is done with this chunk's halo: the next one replaces it
                    store_halo();
                    if (ch + 2 < NCH) load_halo(32 * (ch + 2));
                    __syncthreads();
                }
            }
        }
    } else {
        for (int ci0 = 0; ci0 < CI; ci0 += 32) {
            // the halo's 16-byte pieces: all of a thread's loads are issued before its
            // first LDS store (unconditional, from a clamped address, so that none waits
            // for another), and land in LDS after the barrier
            constexpr int HPIECES = HH * HWD * 4, HPER = (HPIECES + 255) / 256;
            static_assert(HPER <= 32, "one mask bit per piece");
            u32x4 hv[HPER];
            uint32_t hin = 0;  // bit j: piece j lies inside the image (else it goes to LDS as zeros)
#pragma unroll
            for (int j = 0; j < HPER; ++j) {
                const int p = min(tid + 256 * j, HPIECES - 1);
                const int pix = p >> 2, q = p & 3;
                const int hy = pix / HWD, hx = pix - hy * HWD;
                const int iy = iy0 + hy, ix = ix0 + hx;
                const bool in = iy >= 0 && iy < d.H && ix >= 0 && ix < d.W;
                // (kept as loaded: a select here would wait for the load before the barrier)
                hv[j] = *(const u32x4 *)(ximg + ((int64_t)(in ? iy : 0) * d.W + (in ? ix : 0)) * CI + ci0 + 8 * q);
                hin |= (uint32_t)in << j;
            }
            __syncthreads();  // the previous chunk is done with the LDS
#pragma unroll
            for (int j = 0; j < HPER; ++j) {
                const int p = tid + 256 * j;
                if (p < HPIECES) {
                    const int pix = p >> 2, q = p & 3;
                    const int hy = pix / HWD, hx = pix - hy * HWD;
                    const u32x4 z = {0u, 0u, 0u, 0u};
                    *(u32x4 *)(s_halo + slot_of(hy, hx) * ROW + 8 * q) = ((hin >> j) & 1u) ? hv[j] : z;
                }
            }
            fetch_b(0, ci0);
            store_b(0);
            fetch_b(1, ci0);
            __syncthreads();
            for (int tap = 0; tap < 9; ++tap) {
                const int kh = tap / 3, kw = tap - 3 * kh;
                // The weights of tap + 1 (fetched during the previous tap) go to the other
                // buffer, whose readers (tap - 1) are past the last barrier; those of
                // tap + 2 are fetched while this tap computes. One barrier per tap.
                if (tap < 8) {
                    store_b((tap + 1) & 1);
                    if (tap < 7) fetch_b(tap + 2, ci0);
                }
#pragma unroll
                for (int kk = 0; kk < 2; ++kk) {
                    bf16x8 a[RM], b[RN];
#pragma unroll
                    for (int r = 0; r < RM; ++r)
                        a[r] = __builtin_bit_cast(
                            bf16x8, *(const u32x4 *)(s_halo + slot_of(ty[r] * S + kh, tx[r] * S + kw) * ROW + 16 * kk +
                                                     8 * kq));
#pragma unroll
                    for (int c = 0; c < RN; ++c)
                        b[c] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(s_b[tap & 1] + (wn * RN * 32 + 32 * c + r32) * ROW +
                                                                            16 * kk + 8 * kq));
#pragma unroll
                    for (int r = 0; r < RM; ++r)
#pragma unroll
                        for (int c = 0; c < RN; ++c) acc[r][c] = mfma(b[c], a[r], acc[r][c]);  // D[c_out][pixel]
                }
                if (tap < 8) __syncthreads();  // tap + 1's weights are in LDS, and this tap's buffer is free
            }
        }
    }
    u16 *dst[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const int oy = oy0 + ty[r], ox = ox0 + tx[r];
        dst[r] = oy < d.Ho && ox < d.Wo ? y + (((int64_t)n * d.Ho + oy) * d.Wo + ox) * CO + wn * RN * 32 : nullptr;
    }
    store_relu_bf16<RM, RN>(acc, dst, load_lane_bias<RN>(bias + wn * RN * 32));
}

// Forward, persistent: each block stages the nine taps' weights for its COG
// output channels and all c_in in LDS once, then takes TH x TW output tiles t =
// blockIdx.x, blockIdx.x + gridDim.x, ... (channel group blockIdx.y). The next
// tile's input halo (all c_in, in chunks of 32 channels) is loaded into
// registers while the current tile computes and goes to LDS between two
// barriers; the taps run with no barrier in between. Halo layout and row
// padding as in k_conv_fwd_lds. BPC blocks share a compute unit (their LDS), so
// each wave keeps to 512 / BPC registers. (Two or three tiles' halos in flight,
// and fragment reads pipelined up to six K steps ahead of the multiplies,
// measured no faster.)
template <int CI, int CO, int S, int TH, int TW, int COG, int WGN, int BPC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(BPC))) void k_conv_fwd_pers(
    const u16 *__restrict__ x, ConvDims d, const u16 *__restrict__ wt, const float *__restrict__ bias,
    u16 *__restrict__ y, int tiles_x, int tiles_y) {
    constexpr int WGM = 4 / WGN, BM = TH * TW, NCH = CI / 32;
    constexpr int RM = BM / (WGM * 32), RN = COG / (WGN * 32);
    static_assert(RM >= 1 && RN >= 1 && WGM * RM * 32 == BM && WGN * RN * 32 == COG && CO % COG == 0,
                  "tile, channel group and wave grid");
    static_assert(CI % 32 == 0, "channel chunks of 32");
    constexpr int HH = (TH - 1) * S + 3, HWD = (TW - 1) * S + 3;
    constexpr int PW = S == 1 ? HWD : (HWD + 1) / 2;  // columns per plane
    constexpr int SLOTS = S == 1 ? HH * HWD : HH * 2 * PW;
    constexpr int ROW = 40;                              // bf16 per LDS row (32 + 8 padding)
    __shared__ __align__(16) u16 s_halo[NCH * SLOTS * ROW];  // [chunk][slot][32 + 8]
    __shared__ __align__(16) u16 s_w[9 * NCH * COG * ROW];   // [tap][chunk][c_out][32 + 8]

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    const int r32 = lane & 31, kq = lane >> 5;
    const int co0 = blockIdx.y * COG;
    const int n_tiles = d.n * tiles_y * tiles_x;
    auto slot_of = [](int hy, int hx) { return S == 1 ? hy * HWD + hx : (hy * 2 + (hx & 1)) * PW + (hx >> 1); };

    int ty[RM], tx[RM];  // this lane's output pixels (tile-local)
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const int m = wm * RM * 32 + 32 * r + r32;
        ty[r] = m / TW;
        tx[r] = m - ty[r] * TW;
    }

    // loaded once, so that no tile's epilogue waits for them
    const LaneBias<RN> lane_bias = load_lane_bias<RN>(bias + co0 + wn * RN * 32);
    // the weights, once: piece p = ((tap NCH + chunk) COG + c_out) 4 + quarter
    constexpr int WPIECES = 9 * NCH * COG * 4;
    for (int p = tid; p < WPIECES; p += 256) {
        const int row = p >> 2, co = row % COG, tc = row / COG, tap = tc / NCH, ch = tc - tap * NCH;
        *(u32x4 *)(s_w + row * ROW + 8 * (p & 3)) =
            *(const u32x4 *)(wt + ((int64_t)(co0 + co) * 9 + tap) * CI + 32 * ch + 8 * (p & 3));
    }

    // a tile's halo, piece p = (chunk HH HWD + pixel) 4 + quarter, loaded from
    // clamped addresses (none under a branch) and kept as loaded until its LDS
    // store: a select right after the load would wait for it there
    constexpr int HPIX = HH * HWD, HPIECES = NCH * HPIX * 4, HPER = (HPIECES + 255) / 256;
    static_assert(HPER <= 32, "one mask bit per piece");
    u32x4 hv[HPER];
    uint32_t hin = 0;  // bit j: piece j lies inside the image (else zeros go to LDS)
    auto load_halo = [&](int t) {
        hin = 0;
        const int txi = t % tiles_x, rest = t / tiles_x, tyi = rest % tiles_y, n = rest / tiles_y;
        const int iy0 = tyi * TH * S - 1, ix0 = txi * TW * S - 1;
        const u16 *ximg = x + (int64_t)n * d.H * d.W * CI;
#pragma unroll
        for (int j = 0; j < HPER; ++j) {
            const int p = min(tid + 256 * j, HPIECES - 1);
            const int ch = (p >> 2) / HPIX, pix = (p >> 2) - ch * HPIX, q = p & 3;
            const int hy = pix / HWD, hx = pix - hy * HWD;
            const int iy = iy0 + hy, ix = ix0 + hx;
            const bool in = iy >= 0 && iy < d.H && ix >= 0 && ix < d.W;
            hv[j] = *(const u32x4 *)(ximg + ((int64_t)(in ? iy : 0) * d.W + (in ? ix : 0)) * CI + 32 * ch + 8 * q);
            hin |= (uint32_t)in << j;
        }
    };
    int t = blockIdx.x;
    if (t < n_tiles) load_halo(t);
    for (; t < n_tiles; t += gridDim.x) {
        __syncthreads();  // the previous tile is done with the halo (and the weights are stored)
#pragma unroll
        for (int j = 0; j < HPER; ++j) {
            const int p = tid + 256 * j;
            if (p < HPIECES) {
                const int ch = (p >> 2) / HPIX, pix = (p >> 2) - ch * HPIX, q = p & 3;
                const int hy = pix / HWD, hx = pix - hy * HWD;
                const u32x4 z = {0u, 0u, 0u, 0u};
                *(u32x4 *)(s_halo + (ch * SLOTS + slot_of(hy, hx)) * ROW + 8 * q) = ((hin >> j) & 1u) ? hv[j] : z;
            }
        }
        __syncthreads();
        if (t + (int)gridDim.x < n_tiles) load_halo(t + gridDim.x);  // in flight during this tile
        f32x16 acc[RM][RN];
#pragma unroll
        for (int r = 0; r < RM; ++r)
#pragma unroll
            for (int c = 0; c < RN; ++c)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[r][c][i] = 0.f;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int kh = tap / 3, kw = tap - 3 * kh;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                for (int kk = 0; kk < 2; ++kk) {
                    bf16x8 a[RN], b[RM];
#pragma unroll
                    for (int c = 0; c < RN; ++c)
                        a[c] = __builtin_bit_cast(bf16x8, *(const u32x4 *)(s_w +
                                                                          ((tap * NCH + ch) * COG + wn * RN * 32 +
                                                                           32 * c + r32) * ROW +
                                                                          16 * kk + 8 * kq));
#pragma unroll
                    for (int r = 0; r < RM; ++r)
                        b[r] = __builtin_bit_cast(
                            bf16x8, *(const u32x4 *)(s_halo + (ch * SLOTS + slot_of(ty[r] * S + kh, tx[r] * S + kw)) *
                                                                  ROW +
                                                     16 * kk + 8 * kq));
#pragma unroll
                    for (int r = 0; r < RM; ++r)
#pragma unroll
                        for (int c = 0; c < RN; ++c) acc[r][c] = mfma(a[c], b[r], acc[r][c]);  // D[c_out][pixel]
                }
        }
        const int txi = t % tiles_x, rest = t / tiles_x, tyi = rest % tiles_y, n = rest / tiles_y;
        u16 *dst[RM];
#pragma unroll
        for (int r = 0; r < RM; ++r) {
            const int oy = tyi * TH + ty[r], ox = txi * TW + tx[r];
            dst[r] = oy < d.Ho && ox < d.Wo ? y + (((int64_t)n * d.Ho + oy) * d.Wo + ox) * CO + co0 + wn * RN * 32
                                           : nullptr;
        }
        store_relu_bf16<RM, RN>(acc, dst, lane_bias);
    }
}

// Backward data: dx = (conv^T(dy, W)) * (a_in > 0) in bf16, for the input
// pixels of sub-pixel class blockIdx.y (stride 2: (y mod 2, x mod 2)).
// wd is the weight in [tap][c_in][c_out] layout.
template <int CI, int CO, int S, int RM, int RN, int WGN>
__global__ __launch_bounds__(256) void k_conv_bwd_data(const u16 *__restrict__ dy, ConvDims d,
                                                        const u16 *__restrict__ wd, const u16 *__restrict__ a_in,
                                                        u16 *__restrict__ dx) {
    constexpr int WGM = 4 / WGN, BM = WGM * RM * 32;
    static_assert(WGN * RN * 32 == CI, "wave grid must cover the input channels");
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave % WGM, wn = wave / WGM;
    const int r32 = lane & 31, kq = lane >> 5;
    const int py = S == 2 ? (int)(blockIdx.y >> 1) : 0, px = S == 2 ? (int)(blockIdx.y & 1) : 0;
    const int Hc = (d.H - py + S - 1) / S, Wc = (d.W - px + S - 1) / S;
    const int64_t Mc = (int64_t)d.n * Hc * Wc;
    if ((int64_t)blockIdx.x * BM >= Mc) return;
    const int64_t m0 = (int64_t)blockIdx.x * BM + wm * RM * 32;
    const int hwc = Hc * Wc;
    int iy[RM], ix[RM], nn[RM];
    bool live[RM];
#pragma unroll
    for (int r = 0; r < RM; ++r) {
        const int64_t m = m0 + 32 * r + r32;
        live[r] = m < Mc;
        const int64_t mm = live[r] ? m : 0;
        nn[r] = (int)(mm / hwc);
        const int rem = (int)(mm - (int64_t)nn[r] * hwc);
        const int a = rem / Wc, b = rem - a * Wc;
        iy[r] = S * a + py;
        ix[r] = S * b + px;
    }
    f32x16 acc[RM][RN];
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int c = 0; c < RN; ++c)
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[r][c][i] = 0.f;
    const int cib = wn * RN * 32;
    for (int kh = 0; kh < 3; ++kh) {
        if (S == 2 && ((py + 1 - kh) & 1)) continue;
        for (int kw = 0; kw < 3; ++kw) {
            if (S == 2 && ((px + 1 - kw) & 1)) continue;
            const int tap = kh * 3 + kw;
            const u16 *src[RM];
            bool ok[RM];
#pragma unroll
            for (int r = 0; r < RM; ++r) {
                const int ty = iy[r] + 1 - kh, tx = ix[r] + 1 - kw;
                const int oy = ty / S, ox = tx / S;  // exact: ty, tx are multiples of S here
                ok[r] = live[r] && ty >= 0 && tx >= 0 && oy < d.Ho && ox < d.Wo;
                src[r] = dy + (((int64_t)nn[r] * d.Ho + (ok[r] ? oy : 0)) * d.Wo + (ok[r] ? ox : 0)) * CO + 8 * kq;
            }
            const u16 *wsrc = wd + ((int64_t)tap * CI + cib + r32) * CO + 8 * kq;
#pragma unroll
            for (int c0 = 0; c0 < CO; c0 += 16) {
                bf16x8 a[RM], b[RN];
#pragma unroll
                for (int r = 0; r < RM; ++r) a[r] = ok[r] ? load8(src[r] + c0) : zero8();
#pragma unroll
                for (int c = 0; c < RN; ++c) b[c] = load8(wsrc + (int64_t)32 * c * CO + c0);
#pragma unroll
                for (int r = 0; r < RM; ++r)
#pragma unroll
                    for (int c = 0; c < RN; ++c) acc[r][c] = mfma(a[r], b[c], acc[r][c]);
            }
        }
    }
#pragma unroll
    for (int r = 0; r < RM; ++r)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int64_t m = m0 + 32 * r + 8 * (i / 4) + 4 * kq + (i % 4);
            if (m >= Mc) continue;
            const int n = (int)(m / hwc), rem = (int)(m - (int64_t)n * hwc);
            const int a = rem / Wc, b = rem - a * Wc;
            const int64_t pix = ((int64_t)n * d.H + S * a + py) * d.W + S * b + px;
#pragma unroll
            for (int c = 0; c < RN; ++c) {
                const int ci = cib + 32 * c + r32;
                const bool on = from_bf16(a_in[pix * CI + ci]) > 0.f;
                dx[pix * CI + ci] = to_bf16(on ? acc[r][c][i] : 0.f);
            }
        }
}

// Backward weight, partial sums: part_w[split][co][tap][ci] = sum over the
// output pixels of rows [split * rows, (split + 1) * rows) (a row is one
// (image, output y)) of dy[pixel][co] * x[input pixel of tap][ci];
// part_b[split][co] = sum of dy[pixel][co] over the same pixels.
// Block: 4 waves, one 32 x 32 tile each: co block = blockIdx.y, column block
// (tap, ci) = 4 blockIdx.x + wave. K runs over 16 consecutive output x at a time.
template <int CI, int CO, int S>
__global__ __launch_bounds__(256) void k_conv_wgrad(const u16 *__restrict__ x, const u16 *__restrict__ dy, ConvDims d,
                                                     int rows_per_split, float *__restrict__ part_w,
                                                     float *__restrict__ part_b) {
    constexpr int NCOL = 9 * CI;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r32 = lane & 31, kq = lane >> 5;
    const int colblk = blockIdx.x * 4 + wave;
    if (colblk * 32 >= NCOL) return;
    const int col = colblk * 32 + r32;
    const bool col_ok = col < NCOL;
    const int tap = col_ok ? col / CI : 0, ci = col_ok ? col - tap * CI : 0;
    const int kh = tap / 3, kw = tap - 3 * kh;
    const int co = blockIdx.y * 32 + r32;
    const int split = blockIdx.z;
    const int R = d.n * d.Ho;
    const int rb = split * rows_per_split, re = min(R, rb + rows_per_split);
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
    float bsum = 0.f;
    for (int row = rb; row < re; ++row) {
        const int n = row / d.Ho, oy = row - n * d.Ho;
        const int iy = oy * S - 1 + kh;
        const bool row_ok = col_ok && iy >= 0 && iy < d.H;
        const u16 *dyrow = dy + (int64_t)row * d.Wo * CO + co;
        const u16 *xrow = x + ((int64_t)n * d.H + (row_ok ? iy : 0)) * d.W * CI + ci;
        for (int ox0 = 0; ox0 < d.Wo; ox0 += 16) {
            uint32_t aw[4], bw[4];
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
                uint32_t av2 = 0, bv2 = 0;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int ox = ox0 + 8 * kq + 2 * jj + h;
                    const bool okp = ox < d.Wo;
                    const uint32_t av = okp ? dyrow[(int64_t)(okp ? ox : 0) * CO] : 0u;
                    const int ix = ox * S - 1 + kw;
                    const bool okx = okp && row_ok && ix >= 0 && ix < d.W;
                    const uint32_t bv = okx ? xrow[(int64_t)(okx ? ix : 0) * CI] : 0u;
                    av2 |= av << (16 * h);
                    bv2 |= bv << (16 * h);
                    if (colblk == 0) bsum += from_bf16((u16)av);
                }
                aw[jj] = av2;
                bw[jj] = bv2;
            }
            acc = mfma(pack8(aw), pack8(bw), acc);
        }
    }
    if (col_ok) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int rco = blockIdx.y * 32 + 8 * (i / 4) + 4 * kq + (i % 4);
            part_w[((int64_t)split * CO + rco) * NCOL + col] = acc[i];
        }
    }
    if (colblk == 0) {
        bsum += __shfl_xor(bsum, 32, 64);
        if (kq == 0) part_b[(int64_t)split * CO + co] = bsum;
    }
}

// Backward weight for c_in a multiple of 32, the same partial sums as
// k_conv_wgrad, with the operands staged through LDS. A wave owns one 32 x 32
// tile (32 output channels x 32 input channels of one tap) and walks the output
// pixels of its rows 16 at a time. Per step it loads, for 16 consecutive output
// pixels, the 32 channels of dy and the 32 channels of x at its tap (8-byte
// loads of 4 channels of 2 neighbouring pixels per lane; steps go in pairs,
// the next pair's loads in flight during this pair), writes both transposed
// into its own LDS rows ([channel][pixel], 48-byte rows) as 32-bit words of two
// pixels, and reads the MFMA fragments (8 consecutive pixels of one channel)
// back as 16-byte reads: in place of 16 scalar 2-byte global loads per lane and
// MFMA. One wave's LDS accesses complete in program order, so no barrier is
// needed.
template <int CI, int CO, int S, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_conv_wgrad_lds(const u16 *__restrict__ x, const u16 *__restrict__ dy,
                                                         ConvDims d, int rows_per_split, float *__restrict__ part_w,
                                                         float *__restrict__ part_b) {
    static_assert(CI % 32 == 0 && CO % 32 == 0, "32-channel tiles");
    constexpr int NCOL = 9 * CI, PITCH = 24;  // halves per LDS row: 16 pixels + 8 padding
    __shared__ __align__(16) u16 s_t[WPB][2][32 * PITCH];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r32 = lane & 31, kq = lane >> 5;
    const int colblk = blockIdx.x * WPB + wave;
    if (colblk * 32 >= NCOL) return;  // (a whole wave; there is no block barrier)
    const int tap = colblk * 32 / CI, ci0 = colblk * 32 - tap * CI;
    const int kh = tap / 3, kw = tap - 3 * kh;
    const int co0 = blockIdx.y * 32;
    const int split = blockIdx.z;
    const int R = d.n * d.Ho;
    const int rb = split * rows_per_split, re = min(R, rb + rows_per_split);
    u16 *sd = s_t[wave][0], *sx = s_t[wave][1];
    const int pp = lane >> 3, cq = lane & 7;  // staging: pixels 2 pp and 2 pp + 1, channels 4 cq .. 4 cq + 3
    const int nch = (d.Wo + 15) / 16;
    const int64_t K = (int64_t)max(0, re - rb) * nch;
    // step k's loads: v[0], v[1] = dy of the two pixels, v[2], v[3] = x; ok bit j: v[j] holds data
    auto load = [&](int64_t k, uint2 (&v)[4], uint32_t &ok) {
        const int row = rb + (int)(k / nch), ox0 = (int)(k % nch) * 16;
        const int n = row / d.Ho, oy = row - n * d.Ho;
        const int iy = oy * S - 1 + kh;
        const bool row_ok = iy >= 0 && iy < d.H;
        ok = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int ox = ox0 + 2 * pp + h;
            const bool okp = ox < d.Wo;
            const int ix = ox * S - 1 + kw;
            const bool okx = okp && row_ok && ix >= 0 && ix < d.W;
            // (clamped addresses, no load under a branch)
            v[h] = *(const uint2 *)(dy + ((int64_t)row * d.Wo + (okp ? ox : 0)) * CO + co0 + 4 * cq);
            v[2 + h] = *(const uint2 *)(x + (((int64_t)n * d.H + (row_ok ? iy : 0)) * d.W + (okx ? ix : 0)) * CI +
                                       ci0 + 4 * cq);
            ok |= ((uint32_t)okp << h) | ((uint32_t)okx << (2 + h));
        }
    };
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
    float bsum = 0.f;
    // one step: the loaded values to LDS, transposed (row = channel, two pixels
    // per 32-bit word), then the fragments back and one MFMA
    auto step = [&](uint2 (&v)[4], uint32_t ok) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (!((ok >> j) & 1u)) v[j] = make_uint2(0u, 0u);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            u16 *dst = t == 0 ? sd : sx;
            const uint2 a = v[2 * t], b = v[2 * t + 1];
            uint32_t *w = reinterpret_cast<uint32_t *>(dst + 4 * cq * PITCH + 2 * pp);
            w[0] = (a.x & 0xffffu) | (b.x << 16);
            w[PITCH / 2] = (a.x >> 16) | (b.x & 0xffff0000u);
            w[PITCH] = (a.y & 0xffffu) | (b.y << 16);
            w[3 * PITCH / 2] = (a.y >> 16) | (b.y & 0xffff0000u);
        }
        const u32x4 fa = *(const u32x4 *)(sd + r32 * PITCH + 8 * kq);  // dy[8 pixels][c_out r32]
        const u32x4 fb = *(const u32x4 *)(sx + r32 * PITCH + 8 * kq);  // x[8 pixels][c_in r32]
        acc = mfma(__builtin_bit_cast(bf16x8, fa), __builtin_bit_cast(bf16x8, fb), acc);
        if (colblk == 0) {
#pragma unroll
            for (int e = 0; e < 4; ++e) bsum += __uint_as_float(fa[e] << 16) + __uint_as_float(fa[e] & 0xffff0000u);
        }
    };
    // steps in pairs, the next pair's loads in flight during this pair
    uint2 c0[4], c1[4], n0[4], n1[4];
    uint32_t ok0 = 0, ok1 = 0, okn0 = 0, okn1 = 0;
    if (K > 0) load(0, c0, ok0);
    if (K > 1) load(1, c1, ok1);
    for (int64_t k = 0; k < K; k += 2) {
        if (k + 2 < K) load(k + 2, n0, okn0);
        if (k + 3 < K) load(k + 3, n1, okn1);
        step(c0, ok0);
        if (k + 1 < K) step(c1, ok1);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            c0[j] = n0[j];
            c1[j] = n1[j];
        }
        ok0 = okn0;
        ok1 = okn1;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int rco = co0 + 8 * (i / 4) + 4 * kq + (i % 4);
        part_w[((int64_t)split * CO + rco) * NCOL + colblk * 32 + r32] = acc[i];
    }
    if (colblk == 0) {
        bsum += __shfl_xor(bsum, 32, 64);
        if (kq == 0) part_b[(int64_t)split * CO + co0 + r32] = bsum;
    }
}

// grad_w[e] = sum over splits of part_w, grad_b likewise, in a fixed order: a
// block takes 32 elements, and its 8 groups of 32 threads sum the splits g, g +
// 8, g + 16, ... of them (4 loads in flight per thread), then the 8 group sums
// are added in group order. (One thread per element walking all splits in turn
// left most of the machine idle behind a chain of a few hundred loads.)
constexpr int kRedElems = 32, kRedGroups = 8;
__global__ __launch_bounds__(kRedElems * kRedGroups) void k_wgrad_reduce(const float *__restrict__ part_w,
                                                                         const float *__restrict__ part_b, int nsplit,
                                                                         int nw, int nb, float *__restrict__ grad_w,
                                                                         float *__restrict__ grad_b) {
    __shared__ float s_sum[kRedGroups][kRedElems];
    const int el = threadIdx.x % kRedElems, g = threadIdx.x / kRedElems;
    const int e = blockIdx.x * kRedElems + el;
    const bool is_w = e < nw;
    const float *src = is_w ? part_w + e : part_b + (e - nw);
    const int64_t stride = is_w ? nw : nb;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    if (e < nw + nb) {
        int k = g;
        for (; k + 3 * kRedGroups < nsplit; k += 4 * kRedGroups) {
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] += src[(int64_t)(k + u * kRedGroups) * stride];
        }
        for (; k < nsplit; k += kRedGroups) acc[0] += src[(int64_t)k * stride];
    }
    s_sum[g][el] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (g == 0 && e < nw + nb) {
        float t = 0.f;
#pragma unroll
        for (int h = 0; h < kRedGroups; ++h) t += s_sum[h][el];
        if (is_w)
            grad_w[e] = t;
        else
            grad_b[e - nw] = t;
    }
}

// ---- head: global average pool and the two linear layers ----

constexpr int kFeat = 128, kHidden = 128;

// One block of 256 threads per candidate: g = mean over pixels of a5,
// h = relu(W1 g + b1), score = w2 . h + b2.
__global__ __launch_bounds__(256) void k_head_fwd(const u16 *__restrict__ a5, int npix, const float *__restrict__ w1,
                                                   const float *__restrict__ b1, const float *__restrict__ w2,
                                                   const float *__restrict__ b2, float *__restrict__ g_out,
                                                   float *__restrict__ h_out, float *__restrict__ score) {
    static_assert(kFeat == 128, "16 groups of 8 channels");
    __shared__ float s_part[16][kFeat], s_g[kFeat], s_h[kHidden], red[4];
    const int t = threadIdx.x;
    // global average pool: thread t sums channels 8 (t % 16) .. + 7 (one 16-byte
    // load per pixel) over pixels t / 16, t / 16 + 16, ..., four pixels per step
    // with their loads in flight together
    {
        const int cg = t & 15, pg = t >> 4;
        const u16 *src = a5 + (int64_t)blockIdx.x * npix * kFeat + 8 * cg;
        float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int p0 = pg; p0 < npix; p0 += 64) {
            u32x4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = *(const u32x4 *)(src + (int64_t)min(p0 + 16 * u, npix - 1) * kFeat);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (p0 + 16 * u < npix) {
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        acc[2 * k] += __uint_as_float(v[u][k] << 16);
                        acc[2 * k + 1] += __uint_as_float(v[u][k] & 0xffff0000u);
                    }
                }
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) s_part[pg][8 * cg + k] = acc[k];
    }
    __syncthreads();
    if (t < kFeat) {
        float sum = 0.f;
#pragma unroll
        for (int pg = 0; pg < 16; ++pg) sum += s_part[pg][t];
        const float g = sum / (float)npix;
        s_g[t] = g;
        g_out[(int64_t)blockIdx.x * kFeat + t] = g;
    }
    __syncthreads();
    if (t < kHidden) {
        float v = b1[t];
        const float *row = w1 + t * kFeat;
#pragma unroll 8
        for (int i = 0; i < kFeat; i += 4) {
            const float4 w = *(const float4 *)(row + i);
            v += w.x * s_g[i] + w.y * s_g[i + 1] + w.z * s_g[i + 2] + w.w * s_g[i + 3];
        }
        v = v > 0.f ? v : 0.f;
        s_h[t] = v;
        h_out[(int64_t)blockIdx.x * kHidden + t] = v;
    }
    __syncthreads();
    float v = t < kHidden ? w2[t] * s_h[t] : 0.f;
    v = block_sum(v, red);
    if (t == 0) score[blockIdx.x] = v + b2[0];
}

// Per candidate: ds = 2 (score - label) / B, dh = ds w2 (h > 0),
// dg = W1^T dh, dy5 = dg / npix where a5 > 0 (bf16).
__global__ __launch_bounds__(256) void k_head_bwd(const float *__restrict__ score, const float *__restrict__ label,
                                                   int B, const float *__restrict__ h, const float *__restrict__ w1,
                                                   const float *__restrict__ w2, const u16 *__restrict__ a5, int npix,
                                                   float *__restrict__ ds_out, float *__restrict__ dh_out,
                                                   u16 *__restrict__ dy5) {
    __shared__ float s_dh[kHidden], s_dg[kFeat];
    const int t = threadIdx.x, b = blockIdx.x;
    const float ds = 2.f * (score[b] - label[b]) / (float)B;
    if (t == 0) ds_out[b] = ds;
    if (t < kHidden) {
        const float v = h[(int64_t)b * kHidden + t] > 0.f ? ds * w2[t] : 0.f;
        s_dh[t] = v;
        dh_out[(int64_t)b * kHidden + t] = v;
    }
    __syncthreads();
    if (t < kFeat) {
        float v = 0.f;
        for (int o = 0; o < kHidden; ++o) v += s_dh[o] * w1[o * kFeat + t];
        s_dg[t] = v / (float)npix;
    }
    __syncthreads();
    const int64_t base = (int64_t)b * npix * kFeat;
    for (int e = t; e < npix * kFeat; e += blockDim.x) {
        const bool on = from_bf16(a5[base + e]) > 0.f;
        dy5[base + e] = to_bf16(on ? s_dg[e & (kFeat - 1)] : 0.f);
    }
}

// Gradients of the linear layers and the loss, summed over the batch in order:
//   dW1[o][i] = sum_b dh[b][o] g[b][i], db1[o] = sum_b dh[b][o],
//   dw2[i] = sum_b ds[b] h[b][i], db2 = sum_b ds[b], loss = mean (score - label)^2.
__global__ void k_head_grads(const float *__restrict__ ds, const float *__restrict__ dh, const float *__restrict__ g,
                             const float *__restrict__ h, const float *__restrict__ score,
                             const float *__restrict__ label, int B, float *__restrict__ gw1,
                             float *__restrict__ gb1, float *__restrict__ gw2, float *__restrict__ gb2,
                             float *__restrict__ loss) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    float s = 0.f;
    if (e < kHidden * kFeat) {
        const int o = e / kFeat, i = e - o * kFeat;
        for (int b = 0; b < B; ++b) s += dh[(int64_t)b * kHidden + o] * g[(int64_t)b * kFeat + i];
        gw1[e] = s;
    } else if (e < kHidden * kFeat + kHidden) {
        const int o = e - kHidden * kFeat;
        for (int b = 0; b < B; ++b) s += dh[(int64_t)b * kHidden + o];
        gb1[o] = s;
    } else if (e < kHidden * kFeat + 2 * kHidden) {
        const int i = e - kHidden * kFeat - kHidden;
        for (int b = 0; b < B; ++b) s += ds[b] * h[(int64_t)b * kHidden + i];
        gw2[i] = s;
    } else if (e == kHidden * kFeat + 2 * kHidden) {
        for (int b = 0; b < B; ++b) s += ds[b];
        gb2[0] = s;
    } else if (e == kHidden * kFeat + 2 * kHidden + 1 && loss) {
        for (int b = 0; b < B; ++b) {
            const float r = score[b] - label[b];
            s += r * r;
        }
        loss[0] = s / (float)B;
    }
}

// ---- parameters ----

// AdamW on the flat float32 parameters: m, v moments; bc1 = 1 - beta1^t,
// bc2 = 1 - beta2^t; decoupled weight decay on entries with decay[i] != 0.
__global__ void k_adamw(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                        float *__restrict__ v, const uint8_t *__restrict__ decay, int64_t n, float lr, float b1,
                        float b2, float eps, float wd, float bc1, float bc2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / bc1, vh = vi / bc2;
    float pi = p[i];
    if (decay[i]) pi -= lr * wd * pi;
    p[i] = pi - lr * mh / (sqrtf(vh) + eps);
}

// bf16 copies of the convolution weights: wt in the parameter layout
// [co][tap][ci] and wd in [tap][ci][co], for layer l's slice.
__global__ void k_conv_weights(const float *__restrict__ p, int64_t off, int CI, int CO, u16 *__restrict__ wt,
                               u16 *__restrict__ wd) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= CO * 9 * CI) return;
    const int co = e / (9 * CI), r = e - co * 9 * CI, tap = r / CI, ci = r - tap * CI;
    const u16 h = to_bf16(p[off + e]);
    wt[e] = h;
    wd[((int64_t)tap * CI + ci) * CO + co] = h;
}

template <int CI, int CO, int S, int RM, int RN, int WGN>
void fwd_layer(hipStream_t s, const u16 *x, ConvDims d, const u16 *wt, const float *bias, u16 *y) {
    constexpr int BM = (4 / WGN) * RM * 32;
    const int hw = d.Ho * d.Wo;
    hipLaunchKernelGGL((k_conv_fwd<CI, CO, S, RM, RN, WGN>), dim3((unsigned)((hw + BM - 1) / BM), (unsigned)d.n),
                       dim3(256), 0, s, x, d, wt, bias, y);
}

template <int CI, int CO, int S, int TH, int TW, int WGN, bool PIPE>
void fwd_layer_lds(hipStream_t s, const u16 *x, ConvDims d, const u16 *wt, const float *bias, u16 *y) {
    const dim3 grid((unsigned)((d.Wo + TW - 1) / TW), (unsigned)((d.Ho + TH - 1) / TH), (unsigned)d.n);
    hipLaunchKernelGGL((k_conv_fwd_lds<CI, CO, S, TH, TW, WGN, PIPE>), grid, dim3(256), 0, s, x, d, wt, bias, y);
}

template <int CI, int CO, int S, int TH, int TW, int COG, int WGN, int BPC>
void fwd_layer_pers(hipStream_t s, const u16 *x, ConvDims d, const u16 *wt, const float *bias, u16 *y) {
    const int tiles_x = (d.Wo + TW - 1) / TW, tiles_y = (d.Ho + TH - 1) / TH;
    const int n_tiles = d.n * tiles_x * tiles_y;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // as many blocks as fit on the device at once (their LDS), each taking tiles in turn
    const int blocks = std::max(1, std::min(n_tiles, BPC * cus));
    hipLaunchKernelGGL((k_conv_fwd_pers<CI, CO, S, TH, TW, COG, WGN, BPC>), dim3((unsigned)blocks, CO / COG), dim3(256), 0,
                       s, x, d, wt, bias, y, tiles_x, tiles_y);
}

template <int CI, int CO, int S, int RM, int RN, int WGN>
void bwd_data_layer(hipStream_t s, const u16 *dy, ConvDims d, const u16 *wd, const u16 *a_in, u16 *dx) {
    constexpr int BM = (4 / WGN) * RM * 32;
    const int64_t Hc = (d.H + S - 1) / S, Wc = (d.W + S - 1) / S;  // largest class
    const int64_t M = (int64_t)d.n * Hc * Wc;
    hipLaunchKernelGGL((k_conv_bwd_data<CI, CO, S, RM, RN, WGN>), dim3((unsigned)((M + BM - 1) / BM), S * S),
                       dim3(256), 0, s, dy, d, wd, a_in, dx);
}

template <int CI, int CO, int S>
void wgrad_layer(hipStream_t s, const u16 *x, const u16 *dy, ConvDims d, float *part_w, int64_t part_cap,
                 float *grad_w, float *grad_b) {
    constexpr int NCOL = 9 * CI, NCB = (NCOL + 31) / 32;  // 32-column blocks
    // column blocks (waves) per block: 3 for c_in 32 (9 blocks, none idle; 716
    // against 738 us), else 4 (c_in 64 with 3 per block measured slower: layer 4
    // 800 against 704 us, layer 3 494 against 395)
    constexpr int WPB = CI == 32 ? 3 : 4;
    const int colgroups = (NCB + WPB - 1) / WPB;
    const int coblocks = CO / 32;
    const int R = d.n * d.Ho;
    // about 2048 blocks, and no more splits than the partial buffer holds
    int nsplit = std::max(1, 2048 / (colgroups * coblocks));
    nsplit = (int)std::min<int64_t>(nsplit, std::min<int64_t>(R, part_cap / ((int64_t)CO * NCOL + CO)));
    nsplit = std::max(1, nsplit);
    const int rows = (R + nsplit - 1) / nsplit;
    nsplit = (R + rows - 1) / rows;
    if constexpr (CI % 32 == 0)
        hipLaunchKernelGGL((k_conv_wgrad_lds<CI, CO, S, WPB>), dim3(colgroups, coblocks, nsplit), dim3(64 * WPB), 0, s,
                           x, dy, d, rows, part_w, part_w + (int64_t)nsplit * CO * NCOL);
    else
        hipLaunchKernelGGL((k_conv_wgrad<CI, CO, S>), dim3(colgroups, coblocks, nsplit), dim3(256), 0, s, x, dy, d,
                           rows, part_w, part_w + (int64_t)nsplit * CO * NCOL);
    const int nw = CO * NCOL;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((nw + CO + kRedElems - 1) / kRedElems), dim3(kRedElems * kRedGroups), 0, s,
                       part_w, part_w + (int64_t)nsplit * CO * NCOL, nsplit, nw, CO, grad_w, grad_b);
}

}  // namespace

// ---- launchers (declared in internal.h) ----

void launch_pool_grey(hipStream_t s, const float *rgb, int P, int H, int W, int f, float *out) {
    const int64_t n = (int64_t)P * (H / f) * (W / f);
    hipLaunchKernelGGL(k_pool_grey, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rgb, P, H, W, f, out);
}

void launch_scorer_input(hipStream_t s, const float *rgb, int B, int h, int w, const float *q, float *qstats,
                         uint16_t *x) {
    hipLaunchKernelGGL(k_query_stats, dim3(1), dim3(1024), 0, s, q, h * w, qstats);
    hipLaunchKernelGGL(k_scorer_input, dim3(B), dim3(1024), 0, s, rgb, h, w, q, qstats, x);
}

void scorer_dims(int H, int W, int dims[kScorerLayers + 1][2]) {
    dims[0][0] = H;
    dims[0][1] = W;
    for (int l = 0; l < kScorerLayers; ++l) {
        const int st = kScorerStride[l];
        dims[l + 1][0] = (dims[l][0] - 1) / st + 1;
        dims[l + 1][1] = (dims[l][1] - 1) / st + 1;
    }
}

void launch_scorer_forward(hipStream_t s, const ScorerBufs &b, int B, float *score) {
    int dm[kScorerLayers + 1][2];
    scorer_dims(b.H, b.W, dm);
    auto D = [&](int l) { return ConvDims{B, dm[l][0], dm[l][1], dm[l + 1][0], dm[l + 1][1]}; };
    const float *p = b.params;
    fwd_layer<2, 32, 2, 2, 1, 1>(s, b.x, D(0), b.wt + b.w_off[0], p + b.b_off[0], b.act[1]);
    fwd_layer_pers<32, 64, 1, 16, 16, 64, 1, 2>(s, b.act[1], D(1), b.wt + b.w_off[1], p + b.b_off[1], b.act[2]);
    fwd_layer_pers<64, 64, 2, 8, 8, 64, 2, 1>(s, b.act[2], D(2), b.wt + b.w_off[2], p + b.b_off[2], b.act[3]);
    // (the continuous tap pipeline measured 11% faster on the 64->128 layer and 5%
    // slower on the 128->128 one; 12 x 8 tiles fit that layer's 12-row output,
    // where 8 x 16 tiles computed 45% padding)
    fwd_layer_lds<64, 128, 1, 8, 16, 2, true>(s, b.act[3], D(3), b.wt + b.w_off[3], p + b.b_off[3], b.act[4]);
    fwd_layer_lds<128, 128, 2, 12, 8, 4, false>(s, b.act[4], D(4), b.wt + b.w_off[4], p + b.b_off[4], b.act[5]);
    const int npix = dm[5][0] * dm[5][1];
    hipLaunchKernelGGL(k_head_fwd, dim3(B), dim3(256), 0, s, b.act[5], npix, p + b.fc_off[0], p + b.fc_off[1],
                       p + b.fc_off[2], p + b.fc_off[3], b.g, b.h, score);
}

void launch_scorer_backward(hipStream_t s, const ScorerBufs &b, int B, const float *score, const float *label,
                            float *grad, float *loss) {
    int dm[kScorerLayers + 1][2];
    scorer_dims(b.H, b.W, dm);
    auto D = [&](int l) { return ConvDims{B, dm[l][0], dm[l][1], dm[l + 1][0], dm[l + 1][1]}; };
    const float *p = b.params;
    const int npix = dm[5][0] * dm[5][1];
    u16 *dA = b.dbuf[0], *dB = b.dbuf[1];
    hipLaunchKernelGGL(k_head_bwd, dim3(B), dim3(256), 0, s, score, label, B, b.h, p + b.fc_off[0],
                       p + b.fc_off[2], b.act[5], npix, b.ds, b.dh, dA);
    const int nhead = kHidden * kFeat + 2 * kHidden + 2;
    hipLaunchKernelGGL(k_head_grads, dim3((nhead + 255) / 256), dim3(256), 0, s, b.ds, b.dh, b.g, b.h, score, label,
                       B, grad + b.fc_off[0], grad + b.fc_off[1], grad + b.fc_off[2], grad + b.fc_off[3], loss);
    // layer 5: dy in dA
    wgrad_layer<128, 128, 2>(s, b.act[4], dA, D(4), b.part, b.part_cap, grad + b.w_off[4], grad + b.b_off[4]);
    bwd_data_layer<128, 128, 2, 2, 2, 2>(s, dA, D(4), b.wd + b.w_off[4], b.act[4], dB);
    // layer 4: dy in dB
    wgrad_layer<64, 128, 1>(s, b.act[3], dB, D(3), b.part, b.part_cap, grad + b.w_off[3], grad + b.b_off[3]);
    bwd_data_layer<64, 128, 1, 2, 2, 1>(s, dB, D(3), b.wd + b.w_off[3], b.act[3], dA);
    // layer 3: dy in dA
    wgrad_layer<64, 64, 2>(s, b.act[2], dA, D(2), b.part, b.part_cap, grad + b.w_off[2], grad + b.b_off[2]);
    bwd_data_layer<64, 64, 2, 2, 2, 1>(s, dA, D(2), b.wd + b.w_off[2], b.act[2], dB);
    // layer 2: dy in dB
    wgrad_layer<32, 64, 1>(s, b.act[1], dB, D(1), b.part, b.part_cap, grad + b.w_off[1], grad + b.b_off[1]);
    bwd_data_layer<32, 64, 1, 2, 1, 1>(s, dB, D(1), b.wd + b.w_off[1], b.act[1], dA);
    // layer 1: dy in dA
    wgrad_layer<2, 32, 2>(s, b.x, dA, D(0), b.part, b.part_cap, grad + b.w_off[0], grad + b.b_off[0]);
}

void launch_scorer_weights(hipStream_t s, const ScorerBufs &b) {
    for (int l = 0; l < kScorerLayers; ++l) {
        const int ci = kScorerChannels[l], co = kScorerChannels[l + 1];
        const int n = co * 9 * ci;
        hipLaunchKernelGGL(k_conv_weights, dim3((n + 255) / 256), dim3(256), 0, s, b.params, b.w_off[l], ci, co,
                           b.wt + b.w_off[l], b.wd + b.w_off[l]);
    }
}

void launch_adamw(hipStream_t s, float *p, const float *g, float *m, float *v, const uint8_t *decay, int64_t n,
                  float lr, float b1, float b2, float eps, float wd, float bc1, float bc2) {
    hipLaunchKernelGGL(k_adamw, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, decay, n, lr, b1, b2,
                       eps, wd, bc1, bc2);
}

}  // namespace gsr
