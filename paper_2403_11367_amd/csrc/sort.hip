// Ordering of the (Gaussian, tile) pairs of every pose (S2-S4).
//
// Paper: Sec. III-A - the Gaussians are sorted by depth and composited front to
// back. Per (pose, tile) the blend needs its Gaussians in ascending depth, with
// equal depths in ascending submap index (a total order).
//
// Depth does not depend on the tile, so the order is built in two stable sorts:
//   1. per pose, the visible Gaussians are sorted by their depth keys (float32
//      depth bits minus the near plane's, which order like the depths) with a
//      stable LSD radix sort of 9-bit digits: three passes, and a fourth only
//      when some key reaches 2^27 (a depth above about 13 km for a 0.2 m near
//      plane). Its input is in index order, so equal depths stay in index order;
//   2. the pairs are emitted in that order (geometry.hip) and a stable sort by
//      tile (two passes: buckets of 64 tiles, then tiles) buckets them into
//      per-(pose, tile) lists, which keeps the depth order inside every list.
// Every rank is computed from counts and prefix sums (no ordering by atomics),
// so the result does not depend on scheduling.
#include "internal.h"

namespace gsr {

namespace {

constexpr int kThreads = 256;

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

// Exclusive scan of block_sums[0 .. nb) in place, nb = min(*d_nb, nb_max) (nb_max
// without d_nb), total to *out_total. One block of kBigThreads, kBigItems
// consecutive entries per thread per round.
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
        // loads clamped into range rather than under a branch, so that all of a
        // thread's loads are in flight at once
        uint64_t v[kBigItems], sum = 0;
#pragma unroll
        for (int k = 0; k < kBigItems; ++k) {
            const uint64_t x = block_sums[min(i0 + k, nb - 1)];
            v[k] = i0 + k < nb ? x : 0;
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

// Lanes of the wave whose `key` (its low kBits bits) equals this lane's, among
// the lanes with `valid`; 0 when not valid. Per bit: the ballot of the bit, and
// this lane's bit as a 0 / all-ones word s, so that the lanes agreeing with it
// are ~(ballot ^ s) in each 32-bit half (a few VALU operations per bit instead
// of 64-bit selects).
template <int kBits>
__device__ __forceinline__ uint64_t match_peers(uint32_t key, bool valid) {
    const uint64_t v = __ballot(valid);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
#pragma unroll
    for (int b = 0; b < kBits; ++b) {
        const uint32_t s = (uint32_t)((int32_t)(key << (31 - b)) >> 31);
        const uint64_t m = __ballot(s != 0u);
        lo &= ~((uint32_t)m ^ s);
        hi &= ~((uint32_t)(m >> 32) ^ s);
    }
    return valid ? ((uint64_t)hi << 32 | lo) : 0ull;
}

// ---- per-pose depth sort: stable LSD radix sort of the visible Gaussians ----
// Keys are float32 depth bits minus the near plane's (depths are above a
// non-negative near plane, so positive, and order like their bits); values are
// record slots (pose * n + submap index), which within a pose order like the
// indices. A pose's elements are
// cut into radix blocks of kRB; per pass every block counts its digits, one
// block per pose scans the counts in (digit, block) order into each block's
// output position for its first element of every digit, and the block writes
// its elements there in order. The passes read dense per-pose segments
// [vbase[p], vbase[p+1]): the preprocess's 64-slot regions (visible entries
// packed at the front of each) are compacted into them first, in slot order.
// (Passes over the sparse regions themselves cost 2.4x the blocks of a dense
// pass; the compaction is cheaper than that difference.)
constexpr int kRBWaves = 4;                // waves per radix block
constexpr int kRBThreads = 64 * kRBWaves;
constexpr int kRBWave = 1024;              // elements per wave, contiguous
constexpr int kRB = kRBWaves * kRBWave;    // elements per radix block
constexpr int kRBChunks = kRBWave / 64;    // 64-element chunks per wave
constexpr int kDigitBits = 9;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kKeyPasses = 4;              // 4 x 9 bits cover any 32-bit key
constexpr int kNarrowPasses = kNarrowKeyBits / kDigitBits;  // enough when every key is below 2^27
static_assert(kNarrowPasses * kDigitBits == kNarrowKeyBits && kKeyPasses * kDigitBits >= 32, "digit split");

// Whether pass `pass` runs: the passes past the narrow ones only when the
// preprocess flagged a key of 2^27 or more.
__device__ __forceinline__ bool radix_pass_runs(int pass, const unsigned long long *wide) {
    return pass < kNarrowPasses || *wide != 0ull;
}

struct RadixSrc {
    const uint32_t *keys, *vals;
    const uint32_t *vbase;  // segment starts, P + 1 entries
};

// Element `c * 64 + lane` of wave `wave`'s share of radix block (p, j): returns
// whether it exists and sets its position in keys / vals.
__device__ __forceinline__ bool radix_elem(const RadixSrc &src, int p, uint32_t j, int wave, int c, int lane,
                                           uint64_t &idx) {
    const uint64_t i = (uint64_t)src.vbase[p] + (uint64_t)j * kRB + (uint64_t)wave * kRBWave + (uint64_t)c * 64 + lane;
    idx = i;
    return i < (uint64_t)src.vbase[p + 1];
}

// cnt[(p * nbp + j) * kDigits + digit] = elements of radix block (p, j) with that
// digit of pass `pass`.
__global__ __launch_bounds__(kRBThreads) void k_radix_count(RadixSrc src, int pass, uint32_t nbp,
                                                          const unsigned long long *__restrict__ wide,
                                                          uint32_t *__restrict__ cnt) {
    __shared__ uint32_t s_h[kRBWaves][kDigits];  // per wave, so only a wave's own lanes meet at a counter
    if (!radix_pass_runs(pass, wide)) return;
    const int p = blockIdx.y;
    const uint32_t j = blockIdx.x;
    if ((uint64_t)src.vbase[p] + (uint64_t)j * kRB >= src.vbase[p + 1]) return;  // empty block
    const int shift = kDigitBits * pass;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < kRBWaves * kDigits; i += kRBThreads) (&s_h[0][0])[i] = 0;
    // every chunk's key is loaded before the first count, so the loads overlap
    uint32_t key[kRBChunks];
    uint32_t vmask = 0;
#pragma unroll
    for (int c = 0; c < kRBChunks; ++c) {
        uint64_t idx = 0;
        const bool valid = radix_elem(src, p, j, wave, c, lane, idx);
        key[c] = valid ? src.keys[idx] : 0u;
        vmask |= (uint32_t)valid << c;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kRBChunks; ++c)
        if ((vmask >> c) & 1u) atomicAdd(&s_h[wave][(key[c] >> shift) & (kDigits - 1)], 1u);
    __syncthreads();
    for (int d = threadIdx.x; d < kDigits; d += kRBThreads) {
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < kRBWaves; ++w) t += s_h[w][d];
        cnt[((uint64_t)p * nbp + j) * kDigits + d] = t;
    }
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

// Offsets of one segment's blocks per key, by a block of kKeys kGroups threads: cnt[j * K +
// k] (block j < nb of the segment, key k < K <= kKeys) are its blocks' key counts;
// off[j * K + k] <- the position, relative to the segment's first element, of
// block j's first element with key k (keys in order, blocks in order within a
// key); off may be cnt. Returns to thread k < K of the first group the start of
// key k's run (relative), and to every thread the segment's total in *all. The
// blocks are split over the kGroups groups of kKeys threads (thread = key), which
// sum their share, 8 blocks per step with the loads in flight together, and
// then write it from their prefix: a chain of nb / (8 kGroups) dependent loads
// instead of nb / 8 (for segments of many blocks).
template <int kKeys, int kGroups>
__device__ uint32_t seg_key_offsets(const uint32_t *cnt, uint32_t *off, uint32_t nb, int K,
                                    uint32_t (*s_part)[kKeys] /*[kGroups][kKeys]*/,
                                    uint32_t *s_wave /*[kKeys / 64]*/, uint32_t *all) {
    constexpr int kWaves = kKeys / 64;
    const int g = threadIdx.x / kKeys, k = threadIdx.x % kKeys;
    const uint32_t per = (nb + kGroups - 1) / kGroups;
    const uint32_t j0 = min(nb, g * per), j1 = min(nb, j0 + per);
    uint32_t tot = 0;
    if (k < K) {
        for (uint32_t j = j0; j < j1; j += 8) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = cnt[(uint64_t)min(j + u, j1 - 1) * K + k];
#pragma unroll
            for (int u = 0; u < 8; ++u) tot += j + u < j1 ? v[u] : 0u;
        }
    }
    s_part[g][k] = tot;
    __syncthreads();
    // key totals, scanned over the keys by the first kKeys threads
    uint32_t key_tot = 0;
    if (g == 0) {
#pragma unroll
        for (int h = 0; h < kGroups; ++h) key_tot += s_part[h][k];
    }
    uint32_t inc = key_tot;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (g == 0 && lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) total += s_wave[w];
    uint32_t start = 0;
    if (g == 0) {
        start = inc - key_tot;
        for (int w = 0; w < wave; ++w) start += s_wave[w];
        // each group's first position per key
        uint32_t run = start;
#pragma unroll
        for (int h = 0; h < kGroups; ++h) {
            const uint32_t x = s_part[h][k];
            s_part[h][k] = run;
            run += x;
        }
    }
    __syncthreads();
    if (k < K) {
        uint32_t run = s_part[g][k];
        for (uint32_t j = j0; j < j1; j += 8) {
            uint32_t v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = cnt[(uint64_t)min(j + u, j1 - 1) * K + k];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (j + u < j1) {
                    off[(uint64_t)(j + u) * K + k] = run;
                    run += v[u];
                }
        }
    }
    *all = total;
    return start;
}

// Per pose (one block): off[(p * nbp + j) * kDigits + d] = position, relative to
// the pose's first element, of radix block j's first element with digit d
// (digits in order, blocks in order within a digit).
constexpr int kOffGroups = 1024 / kDigits;  // radix blocks per pose: tens to hundreds
__global__ __launch_bounds__(kDigits * kOffGroups) void k_radix_offsets(const uint32_t *__restrict__ cnt, uint32_t nbp,
                                                                       const uint32_t *__restrict__ vbase, int pass,
                                                                       const unsigned long long *__restrict__ wide,
                                                                       uint32_t *__restrict__ off) {
    __shared__ uint32_t s_part[kOffGroups][kDigits];
    __shared__ uint32_t s_wave[kDigits / 64];
    if (!radix_pass_runs(pass, wide)) return;
    const int p = blockIdx.x;
    const uint32_t nb = (uint32_t)(((uint64_t)vbase[p + 1] - vbase[p] + kRB - 1) / kRB);
    uint32_t all = 0;
    (void)seg_key_offsets<kDigits, kOffGroups>(cnt + (uint64_t)p * nbp * kDigits, off + (uint64_t)p * nbp * kDigits,
                                               nb, kDigits, s_part, s_wave, &all);
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

// Compaction of the preprocess's region layout (per pose, regions of 64 slots,
// each holding its visible entries at the front, popcount(vmask) of them) into one dense
// run per pose, in slot order, so that every radix pass works on dense blocks.
// Per pose (one block): reg_off[p * n_regions + r] = entries of the pose's
// regions before r; nv[p] = the pose's total.
template <int kWaves>
__device__ uint32_t block_exclusive_scan_waves(uint32_t x, uint32_t *s_wave, uint32_t *total);

constexpr int kRegionThreads = 1024;  // about 8 regions per thread at 500k Gaussians
__global__ __launch_bounds__(kRegionThreads) void k_region_offsets(const uint64_t *__restrict__ vmask,
                                                                   int64_t n_regions, uint32_t *__restrict__ reg_off,
                                                                   uint32_t *__restrict__ nv) {
    __shared__ uint32_t s_wave[kRegionThreads / 64];
    const int p = blockIdx.x;
    const uint64_t *vc = vmask + (int64_t)p * n_regions;
    uint32_t *ro = reg_off + (int64_t)p * n_regions;
    const int64_t per = (n_regions + kRegionThreads - 1) / kRegionThreads;  // consecutive regions per thread
    const int64_t r0 = (int64_t)threadIdx.x * per, r1 = min(r0 + per, n_regions);
    // 8 regions per step, the loads in flight together (clamped, not under a branch)
    uint32_t sum = 0;
    for (int64_t r = r0; r < r1; r += 8) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = (uint32_t)__popcll(vc[min(r + u, r1 - 1)]);
#pragma unroll
        for (int u = 0; u < 8; ++u) sum += r + u < r1 ? v[u] : 0u;
    }
    uint32_t all = 0;
    uint32_t run = block_exclusive_scan_waves<kRegionThreads / 64>(sum, s_wave, &all);
    for (int64_t r = r0; r < r1; r += 8) {
        uint32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = (uint32_t)__popcll(vc[min(r + u, r1 - 1)]);
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (r + u < r1) {
                ro[r + u] = run;
                run += v[u];
            }
    }
    if (threadIdx.x == 0) nv[p] = all;
}

// Each wave takes kCompactRegions consecutive (pose, region) pairs; a region's
// entries go to vbase[p] + reg_off[..] onward. Lane i first loads region i's
// count and destination, so that the wave's copies do not wait on each other.
// (4 regions per wave measured fastest: 2, 8, 16 and 32 were 3-13% slower.)
constexpr int kCompactRegions = 4;
__global__ __launch_bounds__(kThreads) void k_compact(const uint64_t *__restrict__ vmask, int64_t n, int P,
                                                      const uint32_t *__restrict__ reg_off,
                                                      const uint32_t *__restrict__ vbase,
                                                      const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
                                                      uint32_t *__restrict__ kout, uint32_t *__restrict__ vout) {
    const int64_t n_regions = (n + 63) >> 6;
    const int64_t total = (int64_t)P * n_regions;
    const int64_t w0 = ((int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6)) * kCompactRegions;
    const int lane = threadIdx.x & 63;
    // lane i < kCompactRegions: region w0 + i's count, source and destination
    uint32_t my_cnt = 0;
    uint64_t my_src = 0, my_dst = 0;
    if (lane < kCompactRegions && w0 + lane < total) {
        const int64_t w = w0 + lane;
        const int p = (int)(w / n_regions);
        const int64_t r = w - (int64_t)p * n_regions;
        my_cnt = (uint32_t)__popcll(vmask[w]);
        my_src = (uint64_t)p * (uint64_t)n + ((uint64_t)r << 6);
        my_dst = (uint64_t)vbase[p] + reg_off[w];
    }
    // every region's entries are loaded before the first store, so the wave's
    // loads (two per region) are in flight together instead of one memory
    // latency per region
    uint32_t kv[kCompactRegions], vv[kCompactRegions];
#pragma unroll
    for (int i = 0; i < kCompactRegions; ++i) {
        const uint32_t cnt = (uint32_t)__shfl((int)my_cnt, i, 64);
        const uint64_t src = (uint64_t)__shfl((long long)my_src, i, 64);
        kv[i] = 0u;
        vv[i] = 0u;
        if ((uint32_t)lane < cnt) {
            kv[i] = kin[src + lane];
            vv[i] = vin[src + lane];
        }
    }
#pragma unroll
    for (int i = 0; i < kCompactRegions; ++i) {
        const uint32_t cnt = (uint32_t)__shfl((int)my_cnt, i, 64);
        const uint64_t dst = (uint64_t)__shfl((long long)my_dst, i, 64);
        if ((uint32_t)lane < cnt) {
            kout[dst + lane] = kv[i];
            vout[dst + lane] = vv[i];
        }
    }
}

// Exclusive scan of one uint32 per thread across a block of kWaves waves; *total gets the sum.
template <int kWaves>
__device__ uint32_t block_exclusive_scan_waves(uint32_t x, uint32_t *s_wave /*[kWaves]*/, uint32_t *total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) s_wave[wave] = inc;
    __syncthreads();
    uint32_t add = 0, sum = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t v = s_wave[w];
        if (w < wave) add += v;
        sum += v;
    }
    *total = sum;
    __syncthreads();
    return add + inc - x;
}

// Stable scatter of radix block (p, j). Each wave walks its share 64 elements at
// a time: lanes with equal digits are matched with ballots and ranked in lane
// order; the group's leader adds the group size to a per-wave, per-digit LDS
// counter and the value it returns (the wave's earlier elements with that
// digit) is broadcast to the group. One wave's LDS operations complete in
// program order, so the counters carry the order across chunks without a
// barrier, and the chunks' atomics need not wait for each other. The block then
// lays its elements out in LDS in output order (digits in order, waves in order
// within a digit) and writes them from there, so consecutive threads store
// consecutive positions of a digit's run (whole cache lines where the runs are
// long) instead of 64 lanes storing to 64 runs. The last pass (the third, or
// the fourth when it runs) does not write the keys: vout gets the sorted record
// slots and kout their tile counts, the input of the pair emission. LDS: the
// per-wave counters (8 KB, later the digits' output deltas) and the staging
// arrays (32 KB), 40 KB, so that 4 blocks share a compute unit.
__global__ __launch_bounds__(kRBThreads) void k_radix_scatter(RadixSrc src, int pass, uint32_t nbp, int n_poses,
                                                            const uint32_t *__restrict__ off,
                                                            const unsigned long long *__restrict__ wide,
                                                            uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                            const uint2 *__restrict__ rect, int64_t n,
                                                            bool packed, uint32_t slot0) {
    __shared__ uint32_t s_cnt[kRBWaves][kDigits];
    __shared__ uint32_t s_key[kRB], s_val[kRB];  // the block's elements in output order
    uint32_t *s_wave = s_key;                    // the scan's wave totals, before the staging
    uint32_t *s_delta = s_cnt[0];                // after the staging: the digits' output deltas
    if (!radix_pass_runs(pass, wide)) return;
    const bool last = pass == kKeyPasses - 1 || (pass == kNarrowPasses - 1 && *wide == 0ull);
    const int shift = kDigitBits * pass;
    // Workgroups go to the XCDs round robin by linear id; the mapping below puts
    // every block of pose p on XCD p % 8, in order, so the partial cache lines
    // that neighbouring blocks write at the ends of a digit's runs meet in one
    // L2 before they are written back. The grid has n_pose_slots = P rounded up
    // to 8 rows of nbp blocks.
    const uint32_t lin = blockIdx.y * nbp + blockIdx.x;
    const uint32_t xcd = lin % kXcdCount, slot = lin / kXcdCount;
    const int p = (int)(xcd + kXcdCount * (slot / nbp));
    const uint32_t j = slot % nbp;
    if (p >= n_poses) return;
    const uint32_t pose_base = src.vbase[p];
    if ((uint64_t)pose_base + (uint64_t)j * kRB >= src.vbase[p + 1]) return;  // empty block
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
        const uint32_t d = (key[c] >> shift) & (kDigits - 1);
        const uint64_t peers = match_peers<kDigitBits>(d, valid);
        const uint32_t r = (uint32_t)__popcll(peers & lt_mask);
        uint32_t old = 0;
        if (valid && r == 0) old = atomicAdd(&s_cnt[wave][d], (uint32_t)__popcll(peers));
        const int leader = (int)__builtin_ctzll(peers | (1ull << 63));
        const uint32_t base = (uint32_t)__shfl((int)old, leader, 64);
        rnk[c] = valid ? base + r : 0xffffffffu;
    }
    __syncthreads();
    // Block-local order: digit d's elements go to [ls[d], ls[d] + tot[d]) of the
    // staging arrays, wave by wave; s_cnt[w][d] <- wave w's first slot there, and
    // delta[d] = (output position of the block's first digit-d element) - ls[d].
    // Thread t takes digits 2t and 2t + 1.
    static_assert(kDigits == 2 * kRBThreads, "two digits per thread");
    const int d0 = 2 * threadIdx.x;
    uint32_t tot0 = 0, tot1 = 0;
#pragma unroll
    for (int w = 0; w < kRBWaves; ++w) {
        tot0 += s_cnt[w][d0];
        tot1 += s_cnt[w][d0 + 1];
    }
    uint32_t all = 0;
    const uint32_t ls0 = block_exclusive_scan_waves<kRBWaves>(tot0 + tot1, s_wave, &all), ls1 = ls0 + tot0;
    {
        uint32_t run0 = ls0, run1 = ls1;
#pragma unroll
        for (int w = 0; w < kRBWaves; ++w) {
            const uint32_t c0 = s_cnt[w][d0], c1 = s_cnt[w][d0 + 1];
            s_cnt[w][d0] = run0;
            s_cnt[w][d0 + 1] = run1;
            run0 += c0;
            run1 += c1;
        }
    }
    const uint32_t *o = off + ((uint64_t)p * nbp + j) * kDigits + d0;
    const uint32_t delta0 = pose_base + o[0] - ls0, delta1 = pose_base + o[1] - ls1;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kRBChunks; ++c) {
        if (rnk[c] == 0xffffffffu) continue;
        const uint32_t slot = s_cnt[wave][(key[c] >> shift) & (kDigits - 1)] + rnk[c];
        s_key[slot] = key[c];
        s_val[slot] = val[c];
    }
    __syncthreads();
    s_delta[d0] = delta0;  // (the counters are no longer read)
    s_delta[d0 + 1] = delta1;
    __syncthreads();
    // consecutive threads write consecutive positions of each digit's run
    for (uint32_t i = threadIdx.x; i < all; i += kRBThreads) {
        const uint32_t k = s_key[i], v = s_val[i];
        const uint32_t pos = s_delta[(k >> shift) & (kDigits - 1)] + i;
        if (last) {
            if (packed) {  // (index within the pose) | (tile count << kPackIndexBits)
                vout[pos] = slot0 + (uint32_t)((uint64_t)p * (uint64_t)n) + (v & ((1u << kPackIndexBits) - 1u));
                kout[pos] = v >> kPackIndexBits;
            } else {
                // values are record slots (pose * n + index); the tile count from the rectangle
                const uint2 r = rect[v];
                vout[pos] = v;
                kout[pos] = ((r.x >> 16) - (r.x & 0xffffu) + 1u) * ((r.y >> 16) - (r.y & 0xffffu) + 1u);
            }
        } else {
            kout[pos] = k;
            vout[pos] = v;
        }
    }
}

// ---- tile bucketing: a stable sort of the pairs by tile, per pose ----
// The pairs of pose p occupy [pseg[p], pseg[p+1]) of the emission arrays, in
// front-to-back order. They are sorted by tile in two stable passes of one
// segmented counting sort:
//   A. segments = poses, key = coarse bucket (tile >> 6: 64 consecutive tiles);
//   B. segments = (pose, bucket) ranges of A's output, key = tile & 63.
// A pass cuts every segment into blocks of kCB pairs. Each block counts its
// pairs per key; one block per segment scans the counts in (key, block) order,
// which gives every block the position of its first pair of each key and gives
// the segment the start of each key's run (A: the buckets, B: the tile lists,
// written as the list offsets); each block then writes its pairs in order.
// Both passes keep the emission order among equal keys, so every list is in
// front-to-back order. A block writes runs of about kCB / keys pairs (A: 33
// buckets, B: 64 tiles at 1408x376), so the scattered stores fill whole cache
// lines, and no block holds more than kCB pairs however skewed the lists are.
constexpr int kFineBits = 6;
constexpr int kFine = 1 << kFineBits;               // tiles per coarse bucket
constexpr int kMaxKeys = 256;                       // keys per pass
constexpr int kCBWaves = 4;
constexpr int kCBThreads = 64 * kCBWaves;
constexpr int kCBWave = 1024;                       // pairs per wave, contiguous
constexpr int kCB = kCBWaves * kCBWave;             // pairs per block
constexpr int kCBChunks = kCBWave / 64;

// A pass: segment i is [seg[i], seg[i+1]) of the input arrays; the key of a
// pair is (tile >> shift) & mask, one of n_keys.
struct SegPass {
    const uint64_t *seg;
    int n_seg;
    int shift;
    uint32_t mask;
    int n_keys;
};

// block_base[i] = sum over j < i of ceil(len(j) / kCB), for i in [0, n_seg], and
// bseg[gb] = the segment of block gb for gb < block_base[n_seg]. One block; each
// thread takes a run of consecutive segments, 8 at a time with the loads in
// flight together.
constexpr int kSegBlkThreads = 1024;
__global__ __launch_bounds__(kSegBlkThreads) void k_seg_blocks(const uint64_t *__restrict__ seg, int n_seg,
                                                               uint32_t *__restrict__ block_base,
                                                               uint32_t *__restrict__ bseg) {
    __shared__ uint32_t s_wave[kSegBlkThreads / 64];
    const int per = (n_seg + kSegBlkThreads - 1) / kSegBlkThreads;
    const int i0 = min(n_seg, (int)threadIdx.x * per), i1 = min(n_seg, i0 + per);
    uint32_t sum = 0;
    for (int c = i0; c < i1; c += 8) {
        uint64_t a[9];
#pragma unroll
        for (int u = 0; u < 9; ++u) a[u] = seg[min(c + u, n_seg)];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (c + u < i1) sum += (uint32_t)((a[u + 1] - a[u] + kCB - 1) / kCB);
    }
    uint32_t all = 0;
    uint32_t run = block_exclusive_scan_waves<kSegBlkThreads / 64>(sum, s_wave, &all);
    for (int c = i0; c < i1; c += 8) {
        uint64_t a[9];
#pragma unroll
        for (int u = 0; u < 9; ++u) a[u] = seg[min(c + u, n_seg)];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (c + u < i1) {
                const uint32_t nb = (uint32_t)((a[u + 1] - a[u] + kCB - 1) / kCB);
                block_base[c + u] = run;
                // many short segments: every thread maps its own segments' blocks
                if (n_seg > kSegBlkThreads / 4)
                    for (uint32_t j = 0; j < nb; ++j) bseg[run + j] = (uint32_t)(c + u);
                run += nb;
            }
    }
    if (threadIdx.x == 0) block_base[n_seg] = all;
    if (n_seg <= kSegBlkThreads / 4) {
        // few long segments: a wave maps one segment at a time, 64 blocks per store
        // (the block's own stores of block_base are visible after the barrier)
        __syncthreads();
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int i = wave; i < n_seg; i += kSegBlkThreads / 64) {
            const uint32_t b0 = block_base[i], b1 = block_base[i + 1];
            for (uint32_t gb = b0 + lane; gb < b1; gb += 64) bseg[gb] = (uint32_t)i;
        }
    }
}

// Segment of block gb; -1 past the last block.
__device__ __forceinline__ int block_segment(const uint32_t *block_base, const uint32_t *bseg, int n_seg,
                                             uint32_t gb) {
    return gb < block_base[n_seg] ? (int)bseg[gb] : -1;
}

// Loads block gb's pairs: wave w holds pairs w * kCBWave + 64 c + lane of the
// block, the tile in the low 16 bits of tr[c] (0xffff past the segment's end,
// tiles are below kMaxTilesPerPose) and, with vals, the index in val[c].
__device__ __forceinline__ void seg_load(const SegPass &ps, const uint32_t *block_base, int i, uint32_t gb,
                                         const uint16_t *tiles, const uint32_t *vals, uint32_t *tr, uint32_t *val) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t b0 = ps.seg[i] + (uint64_t)(gb - block_base[i]) * kCB + (uint64_t)wave * kCBWave;
    const uint64_t end = ps.seg[i + 1];
    const uint32_t n = (uint32_t)min<uint64_t>(kCBWave, end > b0 ? end - b0 : 0);  // the wave's pairs
    const uint16_t *t = tiles + b0;
    const uint32_t *v = vals ? vals + b0 : nullptr;
#pragma unroll
    for (int c = 0; c < kCBChunks; ++c) {
        const uint32_t j = (uint32_t)(c * 64 + lane);
        const bool valid = j < n;
        tr[c] = valid ? (uint32_t)t[j] : 0xffffu;
        if (vals) val[c] = valid ? v[j] : 0u;
    }
}

// cnt[gb * n_keys + k] = pairs of block gb with key k.
__global__ __launch_bounds__(kCBThreads) void k_seg_count(SegPass ps, const uint32_t *__restrict__ block_base,
                                                          const uint32_t *__restrict__ bseg,
                                                          const uint16_t *__restrict__ tiles,
                                                          uint32_t *__restrict__ cnt) {
    __shared__ uint32_t s_h[kCBWaves][kMaxKeys];  // per wave, so only a wave's own lanes meet at a counter
    const uint32_t gb = blockIdx.x;
    const int i = block_segment(block_base, bseg, ps.n_seg, gb);
    if (i < 0) return;
    const int wave = threadIdx.x >> 6;
    for (int k = threadIdx.x; k < kCBWaves * kMaxKeys; k += kCBThreads) (&s_h[0][0])[k] = 0;
    uint32_t tr[kCBChunks];
    seg_load(ps, block_base, i, gb, tiles, nullptr, tr, nullptr);
    __syncthreads();
    // Runs of equal keys in lane order (a Gaussian's tiles of one row mostly share
    // a bucket) are counted by their first lane, which adds the run's length: far
    // fewer lanes meet at one LDS counter than with one atomic per pair.
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < kCBChunks; ++c) {
        const bool valid = tr[c] != 0xffffu;
        const uint32_t key = valid ? (tr[c] >> ps.shift) & ps.mask : 0xffffffffu;
        const uint32_t prev = (uint32_t)__shfl_up((int)key, 1, 64);
        const bool head = valid && (lane == 0 || prev != key);
        const uint64_t heads = __ballot(head) | __ballot(!valid);  // a run also ends before an invalid lane
        if (head) {
            const uint64_t after = lane == 63 ? 0ull : heads >> (lane + 1);
            const uint32_t len = after ? (uint32_t)__builtin_ctzll(after) + 1u : (uint32_t)(64 - lane);
            atomicAdd(&s_h[wave][key], len);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < ps.n_keys; k += kCBThreads) {
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < kCBWaves; ++w) t += s_h[w][k];
        cnt[(uint64_t)gb * ps.n_keys + k] = t;
    }
}

// One block per segment: cnt[gb][k] <- position, relative to the segment's first
// pair, of block gb's first pair with key k (keys in order, blocks in order within
// a key). The start of key k's run (absolute) goes to
// starts[(i / per_row) * row + (i % per_row) * n_keys + k] where that column is
// below `row`; the block of the last segment also writes
// starts[(n_seg / per_row) * row] = seg[n_seg].
template <int kGroups>
__global__ __launch_bounds__(256 * kGroups) void k_seg_offsets(SegPass ps, uint32_t *__restrict__ cnt,
                                                               const uint32_t *__restrict__ block_base, int per_row,
                                                               int row, uint64_t *__restrict__ starts) {
    __shared__ uint32_t s_part[kGroups][kMaxKeys];
    __shared__ uint32_t s_wave[kMaxKeys / 64];
    const int i = blockIdx.x;
    const uint32_t g0 = block_base[i], g1 = block_base[i + 1];
    uint32_t all = 0;
    uint32_t *c = cnt + (uint64_t)g0 * ps.n_keys;
    const uint32_t start = seg_key_offsets<kMaxKeys, kGroups>(c, c, g1 - g0, ps.n_keys, s_part, s_wave, &all);
    const int k = threadIdx.x;  // (first group: thread = key)
    const int col = (i % per_row) * ps.n_keys + k;
    if (k < ps.n_keys && col < row) starts[(uint64_t)(i / per_row) * row + col] = ps.seg[i] + start;
    if (k == 0 && i == ps.n_seg - 1) starts[(uint64_t)(ps.n_seg / per_row) * row] = ps.seg[ps.n_seg];
}

// Scatter of block gb. Each wave ranks its pairs 64 at a time: lanes with equal
// keys are matched with ballots and ranked in lane order; the group's leader
// adds the group size to a per-wave, per-key LDS counter, and the value it
// returns (the wave's earlier pairs with that key) is broadcast to the group.
// One wave's LDS operations complete in program order, so the counters carry
// the order across chunks without a barrier. The block then lays its pairs out
// in LDS in output order and writes them from there, so consecutive threads
// store consecutive positions of a key's run. out_tiles may be null (the last
// pass).
template <int kBits>
__global__ __launch_bounds__(kCBThreads) void k_seg_scatter(SegPass ps, const uint32_t *__restrict__ block_base,
                                                            const uint32_t *__restrict__ bseg,
                                                            const uint32_t *__restrict__ offs,
                                                            const uint16_t *__restrict__ tiles,
                                                            const uint32_t *__restrict__ vals,
                                                            uint16_t *__restrict__ out_tiles,
                                                            uint32_t *__restrict__ out_vals) {
    __shared__ uint32_t s_cnt[kCBWaves][kMaxKeys];
    __shared__ uint32_t s_delta[kMaxKeys];
    __shared__ uint16_t s_tile[kCB];  // the block's pairs in output order
    __shared__ uint32_t s_val[kCB];
    __shared__ uint32_t s_wave[kCBWaves];
    const uint32_t gb = blockIdx.x;
    const int i = block_segment(block_base, bseg, ps.n_seg, gb);
    if (i < 0) return;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = threadIdx.x; j < kCBWaves * kMaxKeys; j += kCBThreads) (&s_cnt[0][0])[j] = 0;
    __syncthreads();
    const uint64_t lt_mask = lane ? (~0ull >> (64 - lane)) : 0ull;
    // tr[c]: tile in the low 16 bits, then the pair's rank among the wave's pairs
    // with its key in the high 16 (below kCBWave)
    uint32_t tr[kCBChunks], val[kCBChunks];
    seg_load(ps, block_base, i, gb, tiles, vals, tr, val);
#pragma unroll
    for (int c = 0; c < kCBChunks; ++c) {
        const bool valid = tr[c] != 0xffffu;
        const uint32_t key = valid ? (tr[c] >> ps.shift) & ps.mask : 0u;
        const uint64_t peers = match_peers<kBits>(key, valid);
        const uint32_t r = (uint32_t)__popcll(peers & lt_mask);
        uint32_t old = 0;
        if (valid && r == 0) old = atomicAdd(&s_cnt[wave][key], (uint32_t)__popcll(peers));
        const int leader = (int)__builtin_ctzll(peers | (1ull << 63));
        const uint32_t base = (uint32_t)__shfl((int)old, leader, 64);
        tr[c] |= (base + r) << 16;
    }
    __syncthreads();
    // Block-local order: key k's pairs go to [ls[k], ls[k] + tot[k]) of the
    // staging arrays, wave by wave; s_cnt[w][k] <- wave w's first slot there, and
    // s_delta[k] = (position of the block's first key-k pair in the segment) - ls[k].
    const int k = threadIdx.x;
    uint32_t tot = 0;
    if (k < ps.n_keys) {
#pragma unroll
        for (int w = 0; w < kCBWaves; ++w) tot += s_cnt[w][k];
    }
    uint32_t all = 0;
    const uint32_t ls = block_exclusive_scan_waves<kCBWaves>(tot, s_wave, &all);
    if (k < ps.n_keys) {
        uint32_t run = ls;
#pragma unroll
        for (int w = 0; w < kCBWaves; ++w) {
            const uint32_t x = s_cnt[w][k];
            s_cnt[w][k] = run;
            run += x;
        }
        s_delta[k] = offs[(uint64_t)gb * ps.n_keys + k] - ls;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kCBChunks; ++c) {
        const uint32_t tile = tr[c] & 0xffffu;
        if (tile == 0xffffu) continue;
        const uint32_t slot = s_cnt[wave][(tile >> ps.shift) & ps.mask] + (tr[c] >> 16);
        s_tile[slot] = (uint16_t)tile;
        s_val[slot] = val[c];
    }
    __syncthreads();
    // consecutive threads write consecutive positions of each key's run
    const uint64_t base = ps.seg[i];
    uint32_t *ov = out_vals + base;
    uint16_t *ot = out_tiles ? out_tiles + base : nullptr;
    for (uint32_t e = threadIdx.x; e < all; e += kCBThreads) {
        const uint32_t tile = s_tile[e];
        const uint32_t pos = s_delta[(tile >> ps.shift) & ps.mask] + e;
        if (ot) ot[pos] = (uint16_t)tile;
        ov[pos] = s_val[e];
    }
}

// One segmented pass: counts, offsets (run starts to `starts`), scatter.
void launch_seg_pass(hipStream_t s, const SegPass &ps, uint64_t n_blocks, uint32_t *block_base, uint32_t *bseg,
                     uint32_t *cnt, int per_row, int row, uint64_t *starts, const uint16_t *tiles,
                     const uint32_t *vals, uint16_t *out_tiles, uint32_t *out_vals) {
    int bits = 0;
    while ((1 << bits) < ps.n_keys) ++bits;
    hipLaunchKernelGGL(k_seg_blocks, dim3(1), dim3(kSegBlkThreads), 0, s, ps.seg, ps.n_seg, block_base, bseg);
    // few segments (the poses) of many blocks each: the offsets split each segment's
    // blocks over four thread groups
    const bool few_long = ps.n_seg <= 256;
    switch (bits) {
#define GSR_SEG(B)                                                                                                 \
    case B:                                                                                                        \
        hipLaunchKernelGGL(k_seg_count, dim3((unsigned)n_blocks), dim3(kCBThreads), 0, s, ps, block_base, bseg,     \
                           tiles, cnt);                                                                            \
        if (few_long)                                                                                              \
            hipLaunchKernelGGL(k_seg_offsets<4>, dim3((unsigned)ps.n_seg), dim3(1024), 0, s, ps, cnt, block_base,   \
                               per_row, row, starts);                                                              \
        else                                                                                                       \
            hipLaunchKernelGGL(k_seg_offsets<1>, dim3((unsigned)ps.n_seg), dim3(256), 0, s, ps, cnt, block_base,    \
                               per_row, row, starts);                                                              \
        hipLaunchKernelGGL(k_seg_scatter<B>, dim3((unsigned)n_blocks), dim3(kCBThreads), 0, s, ps, block_base, bseg, \
                           cnt, tiles, vals, out_tiles, out_vals);                                                 \
        break;
        GSR_SEG(0) GSR_SEG(1) GSR_SEG(2) GSR_SEG(3) GSR_SEG(4) GSR_SEG(5) GSR_SEG(6) GSR_SEG(7) GSR_SEG(8)
#undef GSR_SEG
        default: break;  // at most kMaxKeys keys
    }
}

// keep_off[l] = kept states of lists j < l (one per kKeepRecords records beyond
// the first kKeepRecords of a list), l in [0, n_lists]. One block.
constexpr int kKeepThreads = 1024;
__global__ __launch_bounds__(kKeepThreads) void k_keep_offsets(const uint64_t *__restrict__ offsets,
                                                               uint64_t capacity, uint32_t n_lists,
                                                               uint32_t *__restrict__ keep_off) {
    __shared__ uint32_t s_wave[kKeepThreads / 64];
    // kept states of a list [b, e): one per whole kKeepRecords before its last record
    auto kept = [&](uint64_t b, uint64_t e) -> uint32_t {
        b = min(b, capacity);
        e = min(e, capacity);
        return e > b + kKeepRecords ? (uint32_t)((e - b - 1) / kKeepRecords) : 0u;
    };
    // thread t: consecutive entries [l0, l1) of keep_off[0 .. n_lists], 8 lists per
    // step with the loads in flight together (clamped, not under a branch)
    const uint32_t per = (n_lists + 1 + kKeepThreads - 1) / kKeepThreads;
    const uint32_t l0 = min(n_lists + 1, threadIdx.x * per), l1 = min(l0 + per, n_lists + 1);
    uint32_t sum = 0;
    for (uint32_t l = l0; l < l1; l += 8) {
        uint64_t o[9];
#pragma unroll
        for (int u = 0; u < 9; ++u) o[u] = offsets[min(l + u, n_lists)];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (l + u < l1 && l + u < n_lists) sum += kept(o[u], o[u + 1]);
    }
    uint32_t all = 0;
    uint32_t run = block_exclusive_scan_waves<kKeepThreads / 64>(sum, s_wave, &all);
    for (uint32_t l = l0; l < l1; l += 8) {
        uint64_t o[9];
#pragma unroll
        for (int u = 0; u < 9; ++u) o[u] = offsets[min(l + u, n_lists)];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (l + u < l1) {
                keep_off[l + u] = run;
                if (l + u < n_lists) run += kept(o[u], o[u + 1]);
            }
    }
}

__global__ __launch_bounds__(kThreads) void k_keep_items(const uint32_t *__restrict__ keep_off, uint32_t n_lists,
                                                         uint32_t *__restrict__ items) {
    const uint32_t l = blockIdx.x * kThreads + threadIdx.x;
    if (l >= n_lists) return;
    const uint32_t first = l + keep_off[l], count = 1 + keep_off[l + 1] - keep_off[l];
    for (uint32_t j = 0; j < count; ++j) items[first + j] = l;
}

}  // namespace

void launch_keep_offsets(hipStream_t s, const uint64_t *offsets, uint64_t capacity, uint32_t n_lists,
                         uint32_t *keep_off) {
    hipLaunchKernelGGL(k_keep_offsets, dim3(1), dim3(kKeepThreads), 0, s, offsets, capacity, n_lists, keep_off);
}

void launch_keep_items(hipStream_t s, const uint32_t *keep_off, uint32_t n_lists, uint32_t *items) {
    if (n_lists == 0) return;
    hipLaunchKernelGGL(k_keep_items, dim3((n_lists + kThreads - 1) / kThreads), dim3(kThreads), 0, s, keep_off,
                       n_lists, items);
}

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

void launch_block_scan(hipStream_t s, uint64_t *sums, uint64_t nb_max, const uint64_t *d_nb, uint64_t *total) {
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kBigThreads), 0, s, sums, nb_max, d_nb, total);
}

uint64_t radix_blocks_per_pose(int64_t n) { return std::max<uint64_t>(1, ((uint64_t)n + kRB - 1) / kRB); }

uint64_t radix_count_elems(int64_t n, int n_poses) {
    return (uint64_t)n_poses * kDigits * radix_blocks_per_pose(n);
}

void launch_depth_sort(hipStream_t s, int64_t n, int n_poses, const uint64_t *vmask, const uint2 *rect,
                       uint32_t slot0, bool packed, const unsigned long long *wide, uint32_t *ka, uint32_t *va,
                       uint32_t *kb, uint32_t *vb, uint32_t *rcnt, uint32_t *roff, uint32_t *nv, uint32_t *vbase) {
    const uint32_t nbp = (uint32_t)radix_blocks_per_pose(n);
    const int64_t n_regions = (n + 63) >> 6;
    const dim3 grid(nbp, (unsigned)n_poses);
    const dim3 sgrid(nbp, (unsigned)((n_poses + kXcdCount - 1) / kXcdCount * kXcdCount));  // see k_radix_scatter
    // Compaction: regions in (kb, vb) -> dense (ka, va), in slot order. roff holds
    // the region offsets (P * n_regions <= radix_count_elems) until pass 0 writes
    // its digit offsets there.
    hipLaunchKernelGGL(k_region_offsets, dim3((unsigned)n_poses), dim3(kRegionThreads), 0, s, vmask, n_regions, roff,
                       nv);
    hipLaunchKernelGGL(k_pose_bases, dim3(1), dim3(kThreads), 0, s, nv, n_poses, vbase);
    const uint64_t n_waves = (uint64_t)n_poses * (uint64_t)n_regions;  // 0 for an empty submap
    if (n_waves > 0)
        hipLaunchKernelGGL(k_compact,
                           dim3((unsigned)((n_waves + kCompactRegions * (kThreads / 64) - 1) /
                                           (kCompactRegions * (kThreads / 64)))),
                           dim3(kThreads), 0, s, vmask, n, n_poses, roff, vbase, kb, vb, ka, va);
    // dense passes: (ka, va) -> (kb, vb) -> (ka, va) -> (kb, vb = tile counts, slots),
    // or with the fourth pass -> (ka, va = tile counts, slots); a pass that does
    // not run returns at once
    static_assert(kKeyPasses == kNarrowPasses + 1, "one optional pass");
    const uint32_t *kin = ka, *vin = va;
    for (int pass = 0; pass < kKeyPasses; ++pass) {
        RadixSrc src{kin, vin, vbase};
        hipLaunchKernelGGL(k_radix_count, grid, dim3(kRBThreads), 0, s, src, pass, nbp, wide, rcnt);
        hipLaunchKernelGGL(k_radix_offsets, dim3((unsigned)n_poses), dim3(kDigits * kOffGroups), 0, s, rcnt, nbp,
                           vbase, pass, wide, roff);
        uint32_t *ko = (pass & 1) ? ka : kb, *vo = (pass & 1) ? va : vb;
        hipLaunchKernelGGL(k_radix_scatter, sgrid, dim3(kRBThreads), 0, s, src, pass, nbp, n_poses, roff, wide, ko,
                           vo, rect, n, packed, slot0);
        kin = ko;
        vin = vo;
    }
}

int bucket_coarse(int n_tiles) { return (n_tiles + kFine - 1) / kFine; }

uint64_t bucket_blocks_max(uint64_t capacity, int n_poses, int n_tiles) {
    // pass B has the most segments (poses x buckets), each with one partial block at most
    return (capacity + kCB - 1) / kCB + (uint64_t)n_poses * bucket_coarse(n_tiles);
}

uint64_t bucket_count_elems(uint64_t capacity, int n_poses, int n_tiles) {
    return bucket_blocks_max(capacity, n_poses, n_tiles) * std::max(bucket_coarse(n_tiles), kFine);
}

void launch_bucket(hipStream_t s, const uint16_t *ptile, const uint32_t *pk, const uint64_t *pseg, int n_poses,
                   uint64_t capacity, int n_tiles, uint32_t *block_base, uint32_t *bseg, uint32_t *cnt,
                   uint64_t *cstart, uint16_t *ctile, uint32_t *cval, uint64_t *offsets, uint32_t *sk) {
    if (n_poses <= 0) return;
    const int n_coarse = bucket_coarse(n_tiles);
    const uint64_t nbm = bucket_blocks_max(capacity, n_poses, n_tiles);
    // A: poses -> buckets; cstart[p * n_coarse + b] = first pair of bucket (p, b), cstart[P * n_coarse] = pseg[P]
    const SegPass a{pseg, n_poses, kFineBits, 0xffffu, n_coarse};
    launch_seg_pass(s, a, nbm, block_base, bseg, cnt, 1, n_coarse, cstart, ptile, pk, ctile, cval);
    // B: buckets -> tiles; offsets[p * n_tiles + t] = first pair of list (p, t), offsets[P * n_tiles] = pseg[P]
    const SegPass b{cstart, n_poses * n_coarse, 0, (uint32_t)(kFine - 1), kFine};
    launch_seg_pass(s, b, nbm, block_base, bseg, cnt, n_coarse, n_tiles, offsets, ctile, cval, nullptr, sk);
}

}  // namespace gsr
