// Ordering of the (Gaussian, tile) pairs of every pose (S2-S4).
//
// Paper: Sec. III-A - the Gaussians are sorted by depth and composited front to
// back. Per (pose, tile) the blend needs its Gaussians in ascending depth, with
// equal depths in ascending submap index (a total order).
//
// The pairs are emitted in (pose, submap index) order (geometry.hip). Then:
//   1. a stable counting sort by tile, per pose, buckets them into per-(pose,
//      tile) lists that keep index order (one pass over the pairs, no atomics
//      outside LDS);
//   2. every list is sorted by the depth bits with a stable LSD radix sort
//      (8-bit digits, only the digits that vary in the list): in LDS for short
//      and medium lists, in global memory by one block for very long ones.
// Stability carries the index order through, so each list ends in (depth bits,
// index) order. The result does not depend on scheduling.
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
                                                          const uint64_t *__restrict__ d_n,
                                                          uint64_t *__restrict__ block_sums) {
    __shared__ uint64_t s_wave[4];
    const uint64_t n = d_n ? min(*d_n, n_max) : n_max;
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanItems;
    uint64_t sum = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) sum += count[base + i];
    const uint64_t inc = block_inclusive_scan(sum, s_wave);
    if (threadIdx.x == kThreads - 1) block_sums[blockIdx.x] = inc;
}

// Single block: exclusive scan of the block sums in place; total to out_total.
__global__ __launch_bounds__(kThreads) void k_scan_blocks(uint64_t *__restrict__ block_sums, uint64_t nb,
                                                          uint64_t *__restrict__ out_total) {
    __shared__ uint64_t s_wave[4];
    __shared__ uint64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint64_t c0 = 0; c0 < nb; c0 += kThreads) {
        const uint64_t i = c0 + threadIdx.x;
        const uint64_t x = i < nb ? block_sums[i] : 0;
        const uint64_t inc = block_inclusive_scan(x, s_wave);
        const uint64_t carry = s_carry;
        if (i < nb) block_sums[i] = carry + inc - x;
        __syncthreads();
        if (threadIdx.x == kThreads - 1) s_carry = carry + inc;
        __syncthreads();
    }
    if (threadIdx.x == 0) *out_total = s_carry;
}

__global__ __launch_bounds__(kThreads) void k_scan_apply(const uint32_t *__restrict__ count, uint64_t n_max,
                                                         const uint64_t *__restrict__ d_n,
                                                         const uint64_t *__restrict__ block_prefix,
                                                         uint64_t *__restrict__ offsets) {
    __shared__ uint64_t s_wave[4];
    const uint64_t n = d_n ? min(*d_n, n_max) : n_max;
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

// ---- tile bucketing: a stable counting sort of the pairs by tile, per pose ----
// The pairs of pose p occupy [seg(p), seg(p+1)) of the emission arrays, in
// (submap index, tile) order. They are cut into blocks of kBP pairs; each block
// counts its pairs per tile, the counts are summed per (pose, tile) and
// scanned into list offsets, and each block then writes its pairs to
// offset(list) + (pairs of the list in earlier blocks) + (rank within the
// block), which keeps the emission order inside every list.
constexpr int kBP = 4096;

__device__ __forceinline__ uint64_t seg_start(const uint64_t *pair_off, int64_t n, int p, uint64_t capacity) {
    return min(pair_off[(int64_t)p * n], capacity);
}

// block_base[p] = sum over q < p of ceil(len(q) / kBP), for p in [0, P]. One block.
__global__ __launch_bounds__(kThreads) void k_seg_blocks(const uint64_t *__restrict__ pair_off, int64_t n, int P,
                                                         uint64_t capacity, uint32_t *__restrict__ block_base) {
    __shared__ uint64_t s_wave[4];
    __shared__ uint64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 <= P; c0 += kThreads) {
        const int p = c0 + threadIdx.x;
        uint64_t nb = 0;
        if (p < P) {
            const uint64_t len = seg_start(pair_off, n, p + 1, capacity) - seg_start(pair_off, n, p, capacity);
            nb = (len + kBP - 1) / kBP;
        }
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

__global__ __launch_bounds__(kThreads) void k_tile_count(const uint32_t *__restrict__ ptile,
                                                         const uint64_t *__restrict__ pair_off, int64_t n, int P,
                                                         uint64_t capacity, const uint32_t *__restrict__ block_base,
                                                         int n_tiles, uint32_t *__restrict__ cnt) {
    extern __shared__ uint32_t s_hist[];
    const uint32_t gb = blockIdx.x;
    const int p = block_pose(block_base, P, gb);
    if (p < 0) return;
    for (int t = threadIdx.x; t < n_tiles; t += kThreads) s_hist[t] = 0;
    __syncthreads();
    const uint64_t beg = seg_start(pair_off, n, p, capacity) + (uint64_t)(gb - block_base[p]) * kBP;
    const uint64_t end = min(beg + kBP, seg_start(pair_off, n, p + 1, capacity));
    for (uint64_t i = beg + threadIdx.x; i < end; i += kThreads) atomicAdd(&s_hist[ptile[i]], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < n_tiles; t += kThreads) cnt[(uint64_t)gb * n_tiles + t] = s_hist[t];
}

// total[p * T + t] = pairs of list (p, t), summed over the pose's blocks.
__global__ void k_col_sum(const uint32_t *__restrict__ cnt, const uint32_t *__restrict__ block_base, int P,
                          int n_tiles, uint32_t *__restrict__ total) {
    const uint64_t l = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= (uint64_t)P * n_tiles) return;
    const int p = (int)(l / n_tiles), t = (int)(l % n_tiles);
    uint32_t sum = 0;
    for (uint32_t gb = block_base[p]; gb < block_base[p + 1]; ++gb) sum += cnt[(uint64_t)gb * n_tiles + t];
    total[l] = sum;
}

// cnt[gb][t] <- first output position of block gb's pairs of list (p, t).
__global__ void k_col_prefix(uint32_t *__restrict__ cnt, const uint32_t *__restrict__ block_base, int P, int n_tiles,
                             const uint64_t *__restrict__ offsets) {
    const uint64_t l = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= (uint64_t)P * n_tiles) return;
    const int p = (int)(l / n_tiles), t = (int)(l % n_tiles);
    uint32_t run = (uint32_t)offsets[l];
    for (uint32_t gb = block_base[p]; gb < block_base[p + 1]; ++gb) {
        const uint64_t i = (uint64_t)gb * n_tiles + t;
        const uint32_t c = cnt[i];
        cnt[i] = run;
        run += c;
    }
}

// One wave per block walks its pairs in order, 64 at a time (loads issued
// kAhead chunks ahead): lanes that name the same tile are matched with
// tile_bits ballots, take consecutive slots in lane order, and the group's
// leader advances that tile's cursor in LDS.
constexpr int kAhead = 4;

__global__ __launch_bounds__(64) void k_tile_scatter(const uint32_t *__restrict__ ptile, const uint32_t *__restrict__ pz,
                                                     const uint32_t *__restrict__ pk,
                                                     const uint64_t *__restrict__ pair_off, int64_t n, int P,
                                                     uint64_t capacity, const uint32_t *__restrict__ block_base,
                                                     const uint32_t *__restrict__ cnt, int n_tiles, int tile_bits,
                                                     uint32_t *__restrict__ sz, uint32_t *__restrict__ sk) {
    extern __shared__ uint32_t s_run[];
    const uint32_t gb = blockIdx.x;
    const int p = block_pose(block_base, P, gb);
    if (p < 0) return;
    const int lane = threadIdx.x;
    for (int t = lane; t < n_tiles; t += 64) s_run[t] = cnt[(uint64_t)gb * n_tiles + t];
    __syncthreads();
    const uint64_t beg = seg_start(pair_off, n, p, capacity) + (uint64_t)(gb - block_base[p]) * kBP;
    const uint64_t end = min(beg + kBP, seg_start(pair_off, n, p + 1, capacity));
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (uint64_t c0 = beg; c0 < end; c0 += 64 * kAhead) {
        uint32_t tt[kAhead], zz[kAhead], kk[kAhead];
#pragma unroll
        for (int a = 0; a < kAhead; ++a) {
            const uint64_t i = c0 + a * 64 + lane;
            const bool valid = i < end;
            tt[a] = valid ? ptile[i] : 0xffffffffu;
            zz[a] = valid ? pz[i] : 0u;
            kk[a] = valid ? pk[i] : 0u;
        }
#pragma unroll
        for (int a = 0; a < kAhead; ++a) {
            const uint32_t t = tt[a];
            const bool valid = t != 0xffffffffu;
            uint64_t peers = __ballot(valid);
            for (int b = 0; b < tile_bits; ++b) {
                const bool bit = (t >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            if (!valid) peers = 0;
            const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
            // one wave: its LDS reads and writes take effect in program order, so no
            // barrier (which would also wait for the scattered global stores)
            const uint32_t base = valid ? s_run[t] : 0u;
            if (valid && rank == 0) s_run[t] = base + (uint32_t)__popcll(peers);
            if (valid) {
                sz[base + rank] = zz[a];
                sk[base + rank] = kk[a];
            }
        }
    }
}

// ---- per-list depth sort: stable LSD radix sort on the depth bits ----
// Keys are the float32 depth bits (positive, so they order like the depths);
// values are submap indices. The bucketing left each list in index order, so
// the stable sort yields (depth bits, index) order. Only digits that differ
// within the list are sorted.
constexpr int kWaveList = 256;    // sorted in registers, one wave per list (k_list_sort)
constexpr int kLdsList1 = 1024;   // sorted in LDS by one wave (k_wave_radix, 16 KB)
constexpr int kLdsList2 = 3840;   // sorted in LDS by one wave (k_wave_radix, 61 KB); longer: k_long_sort

struct SortScratch {
    uint32_t off[256];
    uint32_t wcnt[4 * 256];
    uint32_t red[2];
    uint32_t wtmp[4];
};

// Exclusive scan of a 256-entry LDS array in place (256 threads).
__device__ __forceinline__ void scan256(uint32_t *a, uint32_t *s_tmp) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t h = a[tid];
    uint32_t x = h;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_tmp[wave] = x;
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < wave; ++w) add += s_tmp[w];
    __syncthreads();
    a[tid] = x - h + add;
    __syncthreads();
}

// Sort (k0, v0)[0, len) by key; (k1, v1) is the ping-pong buffer. Returns true
// if the result ends in (k0, v0). 256 threads; pointers may be LDS or global.
__device__ __forceinline__ bool block_sort_zk(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1, uint32_t len,
                                              SortScratch &sc) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (tid == 0) {
        sc.red[0] = 0u;
        sc.red[1] = 0xffffffffu;
    }
    for (int i = tid; i < 4 * 256; i += kThreads) sc.wcnt[i] = 0;
    __syncthreads();
    uint32_t o = 0u, a = 0xffffffffu;
    for (uint32_t i = tid; i < len; i += kThreads) {
        o |= k0[i];
        a &= k0[i];
    }
    atomicOr(&sc.red[0], o);
    atomicAnd(&sc.red[1], a);
    __syncthreads();
    const uint32_t vary = sc.red[0] ^ sc.red[1];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    uint32_t *sk = k0, *sv = v0, *dk = k1, *dv = v1;
    bool first = true;
    for (int shift = 0; shift < 32; shift += 8) {
        if (((vary >> shift) & 0xffu) == 0) continue;
        sc.off[tid] = 0;
        __syncthreads();
        for (uint32_t i = tid; i < len; i += kThreads) atomicAdd(&sc.off[(sk[i] >> shift) & 0xffu], 1u);
        __syncthreads();
        scan256(sc.off, sc.wtmp);
        for (uint32_t c0 = 0; c0 < len; c0 += kThreads) {
            const uint32_t i = c0 + tid;
            const bool valid = i < len;
            const uint32_t key = valid ? sk[i] : 0u;
            const uint32_t val = valid ? sv[i] : 0u;
            const uint32_t d = (key >> shift) & 0xffu;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t m = __ballot(bit);
                peers &= bit ? m : ~m;
            }
            if (!valid) peers = 0;
            const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
            const uint32_t cnt = (uint32_t)__popcll(peers);
            const bool leader = valid && rank == 0;
            if (leader) sc.wcnt[wave * 256 + d] = cnt;
            __syncthreads();
            if (valid) {
                uint32_t pre = 0;
                for (int w = 0; w < wave; ++w) pre += sc.wcnt[w * 256 + d];
                const uint32_t o2 = sc.off[d] + pre + rank;
                dk[o2] = key;
                dv[o2] = val;
            }
            __syncthreads();
            if (leader) {
                atomicAdd(&sc.off[d], cnt);
                sc.wcnt[wave * 256 + d] = 0;
            }
            __syncthreads();
        }
        uint32_t *t;
        t = sk, sk = dk, dk = t;
        t = sv, sv = dv, dv = t;
        first = !first;
    }
    return first;
}

// Bitonic sort of 64 * R keys held by one wave, R per lane: element e lives in
// lane e / R, register e % R. Stages with partner distance j >= R exchange with
// lane ^ (j / R) through cross-lane shuffles; stages with j < R compare two
// registers of the same lane. Fully unrolled so the keys stay in registers.
template <int R>
__device__ __forceinline__ void wave_bitonic(uint64_t (&key)[R]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 2; k <= 64 * R; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= R) {
                const int lx = j / R;
                const bool lower = (lane & lx) == 0;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const bool up = ((lane * R + r) & k) == 0;
                    const uint64_t other = __shfl_xor(key[r], lx, 64);
                    const bool take_min = (lower == up);
                    const uint64_t mn = key[r] < other ? key[r] : other;
                    const uint64_t mx = key[r] < other ? other : key[r];
                    key[r] = take_min ? mn : mx;
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if ((r & j) == 0) {
                        const bool up = ((lane * R + r) & k) == 0;
                        const uint64_t a = key[r], b = key[r + j];
                        const bool swap = (a > b) == up;
                        key[r] = swap ? b : a;
                        key[r + j] = swap ? a : b;
                    }
                }
            }
        }
    }
}

template <int R>
__device__ __forceinline__ void wave_sort_list(const uint32_t *sz, uint32_t *sk, uint64_t beg, uint32_t len) {
    const int lane = threadIdx.x & 63;
    uint64_t key[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t e = lane * R + r;
        key[r] = e < len ? (((uint64_t)sz[beg + e] << 32) | sk[beg + e]) : ~0ull;
    }
    wave_bitonic<R>(key);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t e = lane * R + r;
        if (e < len) sk[beg + e] = (uint32_t)key[r];
    }
}

// One wave per list: lists up to kWaveList pairs are sorted in registers by
// (depth bits, index); longer ones are queued for k_long_sort.
__global__ __launch_bounds__(kThreads) void k_list_sort(const uint32_t *__restrict__ sz, uint32_t *__restrict__ sk,
                                                        const uint64_t *__restrict__ offsets, uint64_t n_lists,
                                                        uint32_t *__restrict__ queue,
                                                        unsigned long long *__restrict__ counters) {
    const uint64_t l = (uint64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (l >= n_lists) return;
    const uint64_t beg = offsets[l], end = offsets[l + 1];
    if (end <= beg + 1) return;
    const uint32_t len = (uint32_t)(end - beg);
    if (len <= 64) {
        wave_sort_list<1>(sz, sk, beg, len);
    } else if (len <= (uint32_t)kWaveList) {
        wave_sort_list<4>(sz, sk, beg, len);
    } else if ((threadIdx.x & 63) == 0) {
        const int q = len <= (uint32_t)kLdsList1 ? 0 : len <= (uint32_t)kLdsList2 ? 1 : 2;
        queue[(uint64_t)q * n_lists + atomicAdd(&counters[CNT_QUEUE + q], 1ull)] = (uint32_t)l;
    }
}

// One wave sorts a queued list in LDS (CAP pairs at most) with a stable LSD
// radix sort on the depth bits, 8-bit digits, only the digits that vary.
// A single wave needs no barrier: its LDS operations take effect in program
// order, so the histogram, the scan and the rank-and-scatter of each 64-pair
// chunk are visible to all lanes in sequence.
template <int CAP>
__global__ __launch_bounds__(64) void k_wave_radix(const uint32_t *__restrict__ sz, uint32_t *__restrict__ sk,
                                                   const uint64_t *__restrict__ offsets,
                                                   const uint32_t *__restrict__ queue,
                                                   const unsigned long long *__restrict__ counters, int which) {
    __shared__ uint32_t ak[CAP], av[CAP], bk[CAP], bv[CAP];
    __shared__ uint32_t hist[256];
    const int lane = threadIdx.x;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint64_t n_q = counters[CNT_QUEUE + which];
    for (uint64_t q = blockIdx.x; q < n_q; q += gridDim.x) {
        const uint32_t l = queue[q];
        const uint64_t beg = offsets[l];
        const uint32_t len = (uint32_t)(offsets[l + 1] - beg);
        uint32_t o = 0u, a = 0xffffffffu;
        for (uint32_t i = lane; i < len; i += 64) {
            const uint32_t z = sz[beg + i];
            ak[i] = z;
            av[i] = sk[beg + i];
            o |= z;
            a &= z;
        }
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) {
            o |= __shfl_xor(o, m, 64);
            a &= __shfl_xor(a, m, 64);
        }
        const uint32_t vary = o ^ a;
        uint32_t *srk = ak, *srv = av, *dsk = bk, *dsv = bv;
        for (int shift = 0; shift < 32; shift += 8) {
            if (((vary >> shift) & 0xffu) == 0) continue;
#pragma unroll
            for (int h = 0; h < 4; ++h) hist[lane * 4 + h] = 0;
            for (uint32_t i = lane; i < len; i += 64) atomicAdd(&hist[(srk[i] >> shift) & 0xffu], 1u);
            // exclusive scan of the 256 counters: 4 per lane, then across lanes
            uint32_t c[4], sum = 0;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                c[h] = hist[lane * 4 + h];
                sum += c[h];
            }
            uint32_t incl = sum;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off, 64);
                if (lane >= off) incl += y;
            }
            uint32_t run = incl - sum;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                hist[lane * 4 + h] = run;
                run += c[h];
            }
            for (uint32_t c0 = 0; c0 < len; c0 += 64) {
                const uint32_t i = c0 + lane;
                const bool valid = i < len;
                const uint32_t key = valid ? srk[i] : 0u;
                const uint32_t val = valid ? srv[i] : 0u;
                const uint32_t d = (key >> shift) & 0xffu;
                uint64_t peers = __ballot(valid);
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const bool bit = (d >> b) & 1u;
                    const uint64_t m = __ballot(bit);
                    peers &= bit ? m : ~m;
                }
                if (!valid) peers = 0;
                const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
                const uint32_t base = valid ? hist[d] : 0u;
                if (valid && rank == 0) hist[d] = base + (uint32_t)__popcll(peers);
                if (valid) {
                    dsk[base + rank] = key;
                    dsv[base + rank] = val;
                }
            }
            uint32_t *t;
            t = srk, srk = dsk, dsk = t;
            t = srv, srv = dsv, dsv = t;
        }
        for (uint32_t i = lane; i < len; i += 64) sk[beg + i] = srv[i];
    }
}

// Lists longer than kLdsList2: one 256-thread block each, stable LSD radix
// sort in global memory (the pair arrays of the emission serve as scratch).
__global__ __launch_bounds__(kThreads) void k_long_sort(uint32_t *__restrict__ sz, uint32_t *__restrict__ sk,
                                                        uint32_t *__restrict__ tz, uint32_t *__restrict__ tk,
                                                        const uint64_t *__restrict__ offsets,
                                                        const uint32_t *__restrict__ queue,
                                                        const unsigned long long *__restrict__ counters) {
    __shared__ SortScratch sc;
    const uint64_t n_long = counters[CNT_QUEUE + 2];
    for (uint64_t q = blockIdx.x; q < n_long; q += gridDim.x) {
        const uint32_t l = queue[q];
        const uint64_t beg = offsets[l], end = offsets[l + 1];
        const uint32_t len = (uint32_t)(end - beg);
        const bool first = block_sort_zk(sz + beg, sk + beg, tz + beg, tk + beg, len, sc);
        if (!first)
            for (uint32_t i = threadIdx.x; i < len; i += kThreads) sk[beg + i] = tk[beg + i];
        __syncthreads();
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
                 const uint64_t *d_n) {
    const uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        launch_fill_u64(s, reinterpret_cast<unsigned long long *>(offsets), 1, 0ull);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kThreads), 0, s, count, n, d_n, tmp);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kThreads), 0, s, tmp, nb, offsets + n);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, count, n, d_n, tmp, offsets);
}

uint64_t bucket_blocks_max(uint64_t capacity, int n_poses) { return (capacity + kBP - 1) / kBP + (uint64_t)n_poses; }

void launch_bucket(hipStream_t s, const uint32_t *ptile, const uint32_t *pz, const uint32_t *pk,
                   const uint64_t *pair_off, int64_t n, int n_poses, uint64_t capacity, int n_tiles, int tile_bits,
                   uint32_t *block_base, uint32_t *cnt, uint32_t *total, uint64_t *offsets, uint64_t *scan_tmp,
                   uint32_t *sz, uint32_t *sk) {
    const uint64_t nbm = bucket_blocks_max(capacity, n_poses);
    const uint64_t n_lists = (uint64_t)n_poses * n_tiles;
    const unsigned lblocks = (unsigned)((n_lists + kThreads - 1) / kThreads);
    const size_t lds = (size_t)n_tiles * sizeof(uint32_t);
    hipLaunchKernelGGL(k_seg_blocks, dim3(1), dim3(kThreads), 0, s, pair_off, n, n_poses, capacity, block_base);
    hipLaunchKernelGGL(k_tile_count, dim3((unsigned)nbm), dim3(kThreads), lds, s, ptile, pair_off, n, n_poses,
                       capacity, block_base, n_tiles, cnt);
    hipLaunchKernelGGL(k_col_sum, dim3(lblocks), dim3(kThreads), 0, s, cnt, block_base, n_poses, n_tiles, total);
    launch_scan(s, total, n_lists, offsets, scan_tmp, nullptr);
    hipLaunchKernelGGL(k_col_prefix, dim3(lblocks), dim3(kThreads), 0, s, cnt, block_base, n_poses, n_tiles, offsets);
    hipLaunchKernelGGL(k_tile_scatter, dim3((unsigned)nbm), dim3(64), lds, s, ptile, pz, pk, pair_off, n, n_poses,
                       capacity, block_base, cnt, n_tiles, tile_bits, sz, sk);
}

void launch_list_sort(hipStream_t s, uint32_t *sz, uint32_t *sk, uint32_t *tz, uint32_t *tk, const uint64_t *offsets,
                      int n_tiles, int n_poses, uint32_t *queue, unsigned long long *counters) {
    const uint64_t n_lists = (uint64_t)n_tiles * n_poses;
    hipLaunchKernelGGL(k_list_sort, dim3((unsigned)((n_lists + 3) / 4)), dim3(kThreads), 0, s, sz, sk, offsets,
                       n_lists, queue, counters);
    hipLaunchKernelGGL(k_wave_radix<kLdsList1>, dim3(4096), dim3(64), 0, s, sz, sk, offsets, queue, counters, 0);
    hipLaunchKernelGGL(k_wave_radix<kLdsList2>, dim3(1024), dim3(64), 0, s, sz, sk, offsets, queue + n_lists,
                       counters, 1);
    hipLaunchKernelGGL(k_long_sort, dim3(1024), dim3(kThreads), 0, s, sz, sk, tz, tk, offsets, queue + 2 * n_lists,
                       counters);
}

}  // namespace gsr
