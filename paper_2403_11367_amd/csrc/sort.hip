// Ordering of the (Gaussian, tile) pairs of every pose (S2-S4).
//
// Paper: Sec. III-A - the Gaussians are sorted by depth and composited front to
// back. Per (pose, tile) the blend needs its Gaussians in ascending depth, with
// equal depths in ascending submap index (a total order).
//
// Depth does not depend on the tile, so the order is built in two stable sorts:
//   1. per pose, the visible Gaussians are sorted by their float32 depth bits
//      with a stable LSD radix sort (four 8-bit digits). Its input is in index
//      order, so equal depths stay in index order;
//   2. the pairs are emitted in that order (geometry.hip) and a stable counting
//      sort by tile buckets them into per-(pose, tile) lists, which keeps the
//      depth order inside every list.
// Every rank is computed from counts and prefix sums (no ordering by atomics),
// so the result does not depend on scheduling.
#include "internal.h"

namespace gsr {

namespace {

constexpr int kThreads = 256;
constexpr int kScanItems = 8;  // per thread
constexpr int kScanTile = kThreads * kScanItems;

__global__ void k_fill_u32(uint32_t *__restrict__ p, uint64_t n, uint32_t v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *__restrict__ p, uint64_t n, unsigned long long v) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Inclusive scan of one uint64 per thread across a 256-thread block.
__device__ uint64_t block_inclusive_scan(uint64_t x, uint64_t *s_wave /*[4]*/) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) s_wave[wave] = x;
    __syncthreads();
    uint64_t add = 0;
    for (int w = 0; w < wave; ++w) add += s_wave[w];
    __syncthreads();
    return x + add;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t *__restrict__ count, uint64_t n_max,
                                                          const uint32_t *__restrict__ d_n,
                                                          uint64_t *__restrict__ block_sums) {
    __shared__ uint64_t s_wave[4];
    const uint64_t n = d_n ? min((uint64_t)*d_n, n_max) : n_max;
    if ((uint64_t)blockIdx.x * kScanTile >= n) {  // whole block past the end
        if (threadIdx.x == 0) block_sums[blockIdx.x] = 0;
        return;
    }
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) sum += count[base + i];
    const uint64_t inc = block_inclusive_scan(sum, s_wave);
    if (threadIdx.x == kThreads - 1) block_sums[blockIdx.x] = inc;
}

// Single block of kBigThreads: exclusive scan of the block sums in place (4 per
// thread per round); total to out_total. With d_nb only the first *d_nb sums are
// scanned (the rest are zero and left alone).
constexpr int kBigThreads = 1024;
constexpr int kBigItems = 4;

__global__ __launch_bounds__(kBigThreads) void k_scan_blocks(uint64_t *__restrict__ block_sums, uint64_t nb_max,
                                                             const uint64_t *__restrict__ d_nb,
                                                             uint64_t *__restrict__ out_total) {
    __shared__ uint64_t s_wave[kBigThreads / 64];
    __shared__ uint64_t s_carry;
    const uint64_t nb = d_nb ? min(*d_nb, nb_max) : nb_max;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint64_t c0 = 0; c0 < nb; c0 += (uint64_t)kBigThreads * kBigItems) {
        const uint64_t i0 = c0 + (uint64_t)threadIdx.x * kBigItems;
        uint64_t v[kBigItems], sum = 0;
#pragma unroll
        for (int k = 0; k < kBigItems; ++k) {
            v[k] = i0 + k < nb ? block_sums[i0 + k] : 0;
            sum += v[k];
        }
        uint64_t inc = sum;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t y = __shfl_up(inc, o, 64);
            if (lane >= o) inc += y;
        }
        if (lane == 63) s_wave[wave] = inc;
        __syncthreads();
        uint64_t run = s_carry + inc - sum;
        for (int w = 0; w < wave; ++w) run += s_wave[w];
#pragma unroll
        for (int k = 0; k < kBigItems; ++k) {
            if (i0 + k < nb) block_sums[i0 + k] = run;
            run += v[k];
        }
        __syncthreads();
        if (threadIdx.x == kBigThreads - 1) s_carry = run;
        __syncthreads();
    }
    if (threadIdx.x == 0) *out_total = s_carry;
}

__global__ __launch_bounds__(kThreads) void k_scan_apply(const uint32_t *__restrict__ count, uint64_t n_max,
                                                         const uint32_t *__restrict__ d_n,
                                                         const uint64_t *__restrict__ block_prefix,
                                                         uint64_t *__restrict__ offsets) {
    __shared__ uint64_t s_wave[4];
    const uint64_t n = d_n ? min((uint64_t)*d_n, n_max) : n_max;
    if ((uint64_t)blockIdx.x * kScanTile >= n) return;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < n ? count[base + i] : 0u;
        sum += v[i];
    }
    uint64_t run = block_inclusive_scan(sum, s_wave) - sum + block_prefix[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) offsets[base + i] = run;
        run += v[i];
    }
}

// ---- per-pose depth sort: stable LSD radix sort of the visible Gaussians ----
// Keys are float32 depth bits (depths are above the near plane, so positive,
// and order like their bits); values are record slots (pose * n + submap
// index), which within a pose order like the indices. A pose's elements are
// cut into radix blocks of kRB; per pass every block counts its digits, one
// block per pose scans the counts in (digit, block) order into each block's
// output position for its first element of every digit, and the block writes
// its elements there in order. The first pass reads the preprocess's 64-slot regions (visible
// entries packed at the front of each), later passes the dense per-pose
// segments [vbase[p], vbase[p+1]).
constexpr int kRBWaves = 8;                // waves per radix block
constexpr int kRBThreads = 64 * kRBWaves;
constexpr int kRBWave = 1024;              // elements per wave, contiguous
constexpr int kRB = kRBWaves * kRBWave;    // elements per radix block
constexpr int kRBChunks = kRBWave / 64;    // 64-element chunks per wave
constexpr int kRegionsPerBlock = kRB / 64;
constexpr int kDigits = 256;

struct RadixSrc {
    const uint32_t *keys, *vals;
    const uint32_t *vcount;  // non-null: region layout (first pass)
    int64_t n;               // Gaussians per pose (region layout)
    const uint32_t *vbase;   // dense layout: segment starts, P + 1 entries
};

// Element `c * 64 + lane` of wave `wave`'s share of radix block (p, j): returns
// whether it exists and sets its position in keys / vals.
__device__ __forceinline__ bool radix_elem(const RadixSrc &src, int p, uint32_t j, int wave, int c, int lane,
                                           uint64_t &idx) {
    if (src.vcount) {
        const int64_t n_regions = (src.n + 63) >> 6;
        const int64_t reg = (int64_t)j * kRegionsPerBlock + wave * kRBChunks + c;
        if (reg >= n_regions) return false;
        const uint32_t cnt = src.vcount[(int64_t)p * n_regions + reg];
        idx = (uint64_t)p * (uint64_t)src.n + ((uint64_t)reg << 6) + (uint64_t)lane;
        return (uint32_t)lane < cnt;
    }
    const uint64_t i = (uint64_t)src.vbase[p] + (uint64_t)j * kRB + (uint64_t)wave * kRBWave + (uint64_t)c * 64 + lane;
    idx = i;
    return i < (uint64_t)src.vbase[p + 1];
}

// cnt[(p * nbp + j) * 256 + digit] = elements of radix block (p, j) with that digit.
__global__ __launch_bounds__(kRBThreads) void k_radix_count(RadixSrc src, int shift, uint32_t nbp,
                                                          uint32_t *__restrict__ cnt) {
    __shared__ uint32_t s_h[kDigits];
    const int p = blockIdx.y;
    const uint32_t j = blockIdx.x;
    if (!src.vcount && (uint64_t)src.vbase[p] + (uint64_t)j * kRB >= src.vbase[p + 1]) return;  // empty block
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (threadIdx.x < kDigits) s_h[threadIdx.x] = 0;
    __syncthreads();
    for (int c = 0; c < kRBChunks; ++c) {
        uint64_t idx = 0;
        if (radix_elem(src, p, j, wave, c, lane, idx)) atomicAdd(&s_h[(src.keys[idx] >> shift) & 0xffu], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kDigits) cnt[((uint64_t)p * nbp + j) * kDigits + threadIdx.x] = s_h[threadIdx.x];
}

// Exclusive scan of one uint32 per thread across a 256-thread block; *total gets the sum.
__device__ uint32_t block_exclusive_scan_u32(uint32_t x, uint32_t *s_wave /*[4]*/, uint32_t *total) {
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

// Per pose (one block, thread = digit): off[(p * nbp + j) * 256 + d] = position,
// relative to the pose's first element, of radix block j's first element with
// digit d (digits in order, blocks in order within a digit). With nv non-null
// (first pass) the pose's element count is stored there.
__global__ __launch_bounds__(kThreads) void k_radix_offsets(const uint32_t *__restrict__ cnt, uint32_t nbp,
                                                            const uint32_t *__restrict__ vbase,
                                                            uint32_t *__restrict__ off, uint32_t *__restrict__ nv) {
    __shared__ uint32_t s_wave[4];
    const int p = blockIdx.x;
    const int d = threadIdx.x;
    const uint32_t nb = nv ? nbp : (uint32_t)(((uint64_t)vbase[p + 1] - vbase[p] + kRB - 1) / kRB);
    const uint32_t *c = cnt + (uint64_t)p * nbp * kDigits + d;
    uint32_t tot = 0;
    for (uint32_t j = 0; j < nb; ++j) tot += c[(uint64_t)j * kDigits];
    uint32_t all = 0;
    uint32_t run = block_exclusive_scan_u32(tot, s_wave, &all);
    uint32_t *o = off + (uint64_t)p * nbp * kDigits + d;
    for (uint32_t j = 0; j < nb; ++j) {
        const uint32_t x = c[(uint64_t)j * kDigits];
        o[(uint64_t)j * kDigits] = run;
        run += x;
    }
    if (nv && d == 0) nv[p] = all;
}

// vbase[p] = sum of nv[q] over q < p, for p in [0, P]. One block.
__global__ __launch_bounds__(kThreads) void k_pose_bases(const uint32_t *__restrict__ nv, int P,
                                                         uint32_t *__restrict__ vbase) {
    __shared__ uint32_t s_wave[4];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 <= P; c0 += kThreads) {
        const int p = c0 + threadIdx.x;
        const uint32_t x = p < P ? nv[p] : 0u;
        uint32_t all = 0;
        const uint32_t ex = block_exclusive_scan_u32(x, s_wave, &all);
        const uint32_t carry = s_carry;
        if (p <= P) vbase[p] = carry + ex;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + all;
        __syncthreads();
    }
}

// Stable scatter of radix block (p, j). Each wave walks its share 64 elements at
// a time: lanes with equal digits are matched with ballots and ranked in lane
// order; the group's leader adds the group size to a per-wave, per-digit LDS
// counter and the value it returns (the wave's earlier elements with that
// digit) is broadcast to the group. One wave's LDS operations complete in
// program order, so the counters carry the order across chunks without a
// barrier, and the chunks' atomics need not wait for each other. The block then
// turns the per-wave counts into output positions from off[]. With kLast the
// keys are not written: vout gets the sorted record slots and kout their tile
// counts, the input of the pair emission.
template <bool kLast>
__global__ __launch_bounds__(kRBThreads) void k_radix_scatter(RadixSrc src, int shift, uint32_t nbp,
                                                            const uint32_t *__restrict__ off,
                                                            uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                            const uint32_t *__restrict__ ntiles, int64_t n) {
    __shared__ uint32_t s_cnt[kRBWaves][kDigits];
    const int p = blockIdx.y;
    const uint32_t j = blockIdx.x;
    const uint32_t pose_base = src.vbase[p];
    if (!src.vcount && (uint64_t)pose_base + (uint64_t)j * kRB >= src.vbase[p + 1]) return;  // empty block
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kRBWaves * kDigits; i += kRBThreads) (&s_cnt[0][0])[i] = 0;
    __syncthreads();
    const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint32_t key[kRBChunks], val[kRBChunks], rnk[kRBChunks];
    uint32_t vmask = 0;  // bit c: this lane's element of chunk c exists
#pragma unroll
    for (int c = 0; c < kRBChunks; ++c) {
        uint64_t idx = 0;
        const bool valid = radix_elem(src, p, j, wave, c, lane, idx);
        key[c] = valid ? src.keys[idx] : 0u;
        val[c] = valid ? src.vals[idx] : 0u;
        vmask |= (uint32_t)valid << c;
    }
#pragma unroll
    for (int c = 0; c < kRBChunks; ++c) {
        const bool valid = (vmask >> c) & 1u;
        const uint32_t d = (key[c] >> shift) & 0xffu;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t r = (uint32_t)__popcll(peers & lt_mask);
        uint32_t old = 0;
        if (valid && r == 0) old = atomicAdd(&s_cnt[wave][d], (uint32_t)__popcll(peers));
        const int leader = (int)__builtin_ctzll(peers | (1ull << 63));
        const uint32_t base = (uint32_t)__shfl((int)old, leader, 64);
        rnk[c] = valid ? base + r : 0xffffffffu;
    }
    __syncthreads();
    if (threadIdx.x < kDigits) {
        // s_cnt[w][d] <- output position of wave w's first element with digit d
        const int d = threadIdx.x;
        uint32_t run = pose_base + off[((uint64_t)p * nbp + j) * kDigits + d];
#pragma unroll
        for (int w = 0; w < kRBWaves; ++w) {
            const uint32_t c = s_cnt[w][d];
            s_cnt[w][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kRBChunks; ++c) {
        if (rnk[c] == 0xffffffffu) continue;
        const uint32_t pos = s_cnt[wave][(key[c] >> shift) & 0xffu] + rnk[c];
        if (kLast) {
            vout[pos] = val[c];
            kout[pos] = ntiles[val[c]];  // values are record slots (pose * n + index)
        } else {
            kout[pos] = key[c];
            vout[pos] = val[c];
        }
    }
}

// ---- tile bucketing: a stable counting sort of the pairs by tile, per pose ----
// The pairs of pose p occupy [pseg[p], pseg[p+1]) of the emission arrays, in
// front-to-back order. They are cut into blocks of kBP pairs; each block
// counts its pairs per tile, the counts are summed per (pose, tile) and
// scanned into list offsets, and each block then writes its pairs to
// offset(list) + (pairs of the list in earlier blocks) + (rank within the
// block), which keeps the emission order inside every list.
constexpr int kBP = 4096;

// block_base[p] = sum over q < p of ceil(len(q) / kBP), for p in [0, P]. One block.
__global__ __launch_bounds__(kThreads) void k_seg_blocks(const uint64_t *__restrict__ pseg, int P,
                                                         uint32_t *__restrict__ block_base) {
    __shared__ uint64_t s_wave[4];
    __shared__ uint64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 <= P; c0 += kThreads) {
        const int p = c0 + threadIdx.x;
        uint64_t nb = 0;
        if (p < P) nb = (pseg[p + 1] - pseg[p] + kBP - 1) / kBP;
        const uint64_t inc = block_inclusive_scan(nb, s_wave);
        const uint64_t carry = s_carry;
        if (p <= P) block_base[p] = (uint32_t)(carry + inc - nb);
        __syncthreads();
        if (threadIdx.x == kThreads - 1) s_carry = carry + inc;
        __syncthreads();
    }
}

// Pose of bucketing block gb (block_base is non-decreasing); -1 past the last block.
__device__ __forceinline__ int block_pose(const uint32_t *block_base, int P, uint32_t gb) {
    if (gb >= block_base[P]) return -1;
    int lo = 0, hi = P - 1;  // largest p with block_base[p] <= gb
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (block_base[mid] <= gb)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(kThreads) void k_tile_count(const uint16_t *__restrict__ ptile,
                                                         const uint64_t *__restrict__ pseg, int P,
                                                         const uint32_t *__restrict__ block_base, int n_tiles,
                                                         uint32_t *__restrict__ cnt) {
    extern __shared__ uint32_t s_hist[];
    const uint32_t gb = blockIdx.x;
    const int p = block_pose(block_base, P, gb);
    if (p < 0) return;
    for (int t = threadIdx.x; t < n_tiles; t += kThreads) s_hist[t] = 0;
    __syncthreads();
    const uint64_t beg = pseg[p] + (uint64_t)(gb - block_base[p]) * kBP;
    const uint64_t end = min(beg + kBP, pseg[p + 1]);
    for (uint64_t i = beg + threadIdx.x; i < end; i += kThreads) atomicAdd(&s_hist[ptile[i]], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < n_tiles; t += kThreads) cnt[(uint64_t)gb * n_tiles + t] = s_hist[t];
}

// total[p * T + t] = pairs of list (p, t), summed over the pose's blocks
// (8 rows per step, so several loads are in flight per thread).
__global__ void k_col_sum(const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ block_base, int P,
                          int n_tiles, uint32_t *__restrict__ total) {
    const uint64_t l = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= (uint64_t)P * n_tiles) return;
    const int p = (int)(l / n_tiles), t = (int)(l % n_tiles);
    const uint32_t gb1 = block_base[p + 1];
    uint32_t gb = block_base[p], sum = 0;
    for (; gb + 8 <= gb1; gb += 8) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = cnt[(uint64_t)(gb + u) * n_tiles + t];
#pragma unroll
        for (int u = 0; u < 8; ++u) sum += v[u];
    }
    for (; gb < gb1; ++gb) sum += cnt[(uint64_t)gb * n_tiles + t];
    total[l] = sum;
}

// cnt[gb][t] <- first output position of block gb's pairs of list (p, t). The
// lists of a pose hold exactly the pose's pairs [pseg[p], pseg[p+1]), so the
// exclusive scan of the totals over all P * T lists is the list start.
__global__ void k_col_prefix(uint32_t *__restrict__ cnt, const uint32_t *__restrict__ block_base, int P, int n_tiles,
                             const uint64_t *__restrict__ offsets) {
    const uint64_t l = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= (uint64_t)P * n_tiles) return;
    const int p = (int)(l / n_tiles), t = (int)(l % n_tiles);
    const uint32_t gb1 = block_base[p + 1];
    uint32_t gb = block_base[p];
    uint32_t run = (uint32_t)offsets[l];
    for (; gb + 8 <= gb1; gb += 8) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = cnt[(uint64_t)(gb + u) * n_tiles + t];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            cnt[(uint64_t)(gb + u) * n_tiles + t] = run;
            run += v[u];
        }
    }
    for (; gb < gb1; ++gb) {
        const uint64_t i = (uint64_t)gb * n_tiles + t;
        const uint32_t c = cnt[i];
        cnt[i] = run;
        run += c;
    }
}

// One wave per block walks its pairs in order, 64 at a time (loads issued
// kAhead chunks ahead): lanes that name the same tile are matched with
// tile_bits ballots, take consecutive slots in lane order, and the group's
// leader advances that tile's cursor in LDS with an atomic whose return value
// (the group's first slot) is broadcast to the group.
constexpr int kAhead = 4;

template <int kTileBits>
__global__ __launch_bounds__(64) void k_tile_scatter(const uint16_t *__restrict__ ptile,
                                                     const uint32_t *__restrict__ pk,
                                                     const uint64_t *__restrict__ pseg, int P,
                                                     const uint32_t *__restrict__ block_base,
                                                     const uint32_t *__restrict__ cnt, int n_tiles,
                                                     uint32_t *__restrict__ sk) {
    extern __shared__ uint32_t s_run[];
    const uint32_t gb = blockIdx.x;
    const int p = block_pose(block_base, P, gb);
    if (p < 0) return;
    const int lane = threadIdx.x;
    for (int t = lane; t < n_tiles; t += 64) s_run[t] = cnt[(uint64_t)gb * n_tiles + t];
    __syncthreads();
    const uint64_t beg = pseg[p] + (uint64_t)(gb - block_base[p]) * kBP;
    const uint64_t end = min(beg + kBP, pseg[p + 1]);
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (uint64_t c0 = beg; c0 < end; c0 += 64 * kAhead) {
        uint32_t tt[kAhead], kk[kAhead];
#pragma unroll
        for (int a = 0; a < kAhead; ++a) {
            const uint64_t i = c0 + a * 64 + lane;
            const bool valid = i < end;
            tt[a] = valid ? (uint32_t)ptile[i] : 0xffffffffu;
            kk[a] = valid ? pk[i] : 0u;
        }
#pragma unroll
        for (int a = 0; a < kAhead; ++a) {
            const uint32_t t = tt[a];
            const bool valid = t != 0xffffffffu;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < kTileBits; ++b) {
                const bool bit = (t >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            if (!valid) peers = 0;
            const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
            // one wave: its LDS operations complete in program order, so no barrier
            // (which would also wait for the scattered global stores)
            uint32_t old = 0;
            if (valid && rank == 0) old = atomicAdd(&s_run[t], (uint32_t)__popcll(peers));
            const int leader = (int)__builtin_ctzll(peers | (1ull << 63));
            const uint32_t base = (uint32_t)__shfl((int)old, leader, 64);
            if (valid) sk[base + rank] = kk[a];
        }
    }
}

}  // namespace

void launch_fill_u32(hipStream_t s, uint32_t *p, uint64_t n, uint32_t value) {
    if (n == 0) return;
    const uint64_t blocks = std::min<uint64_t>((n + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(kThreads), 0, s, p, n, value);
}

void launch_fill_u64(hipStream_t s, unsigned long long *p, uint64_t n, unsigned long long value) {
    if (n == 0) return;
    const uint64_t blocks = std::min<uint64_t>((n + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)blocks), dim3(kThreads), 0, s, p, n, value);
}

uint64_t scan_tmp_elems(uint64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

void launch_scan(hipStream_t s, const uint32_t *count, uint64_t n, uint64_t *offsets, uint64_t *tmp,
                 const uint32_t *d_n) {
    const uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        launch_fill_u64(s, reinterpret_cast<unsigned long long *>(offsets), 1, 0ull);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kThreads), 0, s, count, n, d_n, tmp);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kBigThreads), 0, s, tmp, nb, nullptr, offsets + n);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, count, n, d_n, tmp, offsets);
}

void launch_block_scan(hipStream_t s, uint64_t *sums, uint64_t nb_max, const uint64_t *d_nb, uint64_t *total) {
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kBigThreads), 0, s, sums, nb_max, d_nb, total);
}

uint64_t radix_blocks_per_pose(int64_t n) { return std::max<uint64_t>(1, ((uint64_t)n + kRB - 1) / kRB); }

uint64_t radix_count_elems(int64_t n, int n_poses) {
    return (uint64_t)n_poses * kDigits * radix_blocks_per_pose(n);
}

void launch_depth_sort(hipStream_t s, int64_t n, int n_poses, const uint32_t *vcount, const uint32_t *ntiles,
                       uint32_t *ka, uint32_t *va, uint32_t *kb, uint32_t *vb, uint32_t *rcnt, uint32_t *roff,
                       uint32_t *nv, uint32_t *vbase) {
    const uint32_t nbp = (uint32_t)radix_blocks_per_pose(n);
    const dim3 grid(nbp, (unsigned)n_poses);
    // pass 0: regions in (kb, vb) -> dense (ka, va); passes 1, 2 ping-pong; pass 3 -> (kb = tile counts, vb = index)
    const uint32_t *kin = kb, *vin = vb;
    for (int pass = 0; pass < 4; ++pass) {
        RadixSrc src{kin, vin, pass == 0 ? vcount : nullptr, n, vbase};
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_radix_count, grid, dim3(kRBThreads), 0, s, src, shift, nbp, rcnt);
        hipLaunchKernelGGL(k_radix_offsets, dim3((unsigned)n_poses), dim3(kThreads), 0, s, rcnt, nbp, vbase, roff,
                           pass == 0 ? nv : nullptr);
        if (pass == 0) hipLaunchKernelGGL(k_pose_bases, dim3(1), dim3(kThreads), 0, s, nv, n_poses, vbase);
        uint32_t *ko = (pass & 1) ? kb : ka, *vo = (pass & 1) ? vb : va;
        if (pass == 3)
            hipLaunchKernelGGL(k_radix_scatter<true>, grid, dim3(kRBThreads), 0, s, src, shift, nbp, roff, ko, vo, ntiles,
                               n);
        else
            hipLaunchKernelGGL(k_radix_scatter<false>, grid, dim3(kRBThreads), 0, s, src, shift, nbp, roff, ko, vo,
                               ntiles, n);
        kin = ko;
        vin = vo;
    }
}

uint64_t bucket_blocks_max(uint64_t capacity, int n_poses) { return (capacity + kBP - 1) / kBP + (uint64_t)n_poses; }

void launch_bucket(hipStream_t s, const uint16_t *ptile, const uint32_t *pk, const uint64_t *pseg, int n_poses,
                   uint64_t capacity, int n_tiles, int tile_bits, uint32_t *block_base, uint32_t *cnt,
                   uint32_t *total, uint64_t *offsets, uint64_t *scan_tmp, uint32_t *sk) {
    const uint64_t nbm = bucket_blocks_max(capacity, n_poses);
    const size_t lds = (size_t)n_tiles * sizeof(uint32_t);
    hipLaunchKernelGGL(k_seg_blocks, dim3(1), dim3(kThreads), 0, s, pseg, n_poses, block_base);
    hipLaunchKernelGGL(k_tile_count, dim3((unsigned)nbm), dim3(kThreads), lds, s, ptile, pseg, n_poses, block_base,
                       n_tiles, cnt);
    const uint64_t n_lists = (uint64_t)n_poses * n_tiles;
    const unsigned lblocks = (unsigned)((n_lists + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_col_sum, dim3(lblocks), dim3(kThreads), 0, s, cnt, block_base, n_poses, n_tiles, total);
    launch_scan(s, total, n_lists, offsets, scan_tmp, nullptr);
    hipLaunchKernelGGL(k_col_prefix, dim3(lblocks), dim3(kThreads), 0, s, cnt, block_base, n_poses, n_tiles, offsets);
    const dim3 grid((unsigned)nbm), block(64);
    switch (tile_bits) {
#define GSR_SCATTER(B)                                                                                          \
    case B:                                                                                                     \
        hipLaunchKernelGGL(k_tile_scatter<B>, grid, block, lds, s, ptile, pk, pseg, n_poses, block_base, cnt,   \
                           n_tiles, sk);                                                                        \
        break;
        GSR_SCATTER(1) GSR_SCATTER(2) GSR_SCATTER(3) GSR_SCATTER(4) GSR_SCATTER(5) GSR_SCATTER(6) GSR_SCATTER(7)
        GSR_SCATTER(8) GSR_SCATTER(9) GSR_SCATTER(10) GSR_SCATTER(11) GSR_SCATTER(12) GSR_SCATTER(13)
        GSR_SCATTER(14)
#undef GSR_SCATTER
        default: break;  // n_tiles <= kMaxTilesPerPose = 2^14 is checked by the caller
    }
}

}  // namespace gsr
