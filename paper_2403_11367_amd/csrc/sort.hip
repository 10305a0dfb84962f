// Pair ordering: the (pose, tile) counts are turned into list offsets by an
// exclusive scan, pairs are scattered into their tile's list (geometry.hip),
// and every list is then sorted by its 64-bit key (depth bits << 32 | submap
// index). The result is, per (pose, tile), the front-to-back order that
// Eq. 1 and Eq. 5 composite in (Sec. III-A: Gaussians "sorted by depth"), with
// equal depths ordered by submap index.
//
// Bucketing by tile is a one-digit counting sort; the in-list order comes from
// a bitonic network in LDS for lists up to kMidSortCap pairs and from an LSD
// radix sort (8-bit digits, stable block-level multisplit) in global memory
// beyond that.
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

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const uint32_t *__restrict__ count, uint64_t n,
                                                          uint64_t *__restrict__ block_sums) {
    __shared__ uint64_t s_wave[4];
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

__global__ __launch_bounds__(kThreads) void k_scan_apply(const uint32_t *__restrict__ count, uint64_t n,
                                                         const uint64_t *__restrict__ block_prefix,
                                                         uint64_t *__restrict__ offsets) {
    __shared__ uint64_t s_wave[4];
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

// Bitonic sort of s[0..n) ascending, n a power of two, by a 256-thread block.
__device__ void bitonic_lds(uint64_t *s, int n) {
    for (int k = 2; k <= n; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < (n >> 1); i += kThreads) {
                const int lo = 2 * j * (i / j) + (i % j);
                const int hi = lo + j;
                const bool up = (lo & k) == 0;
                const uint64_t a = s[lo], b = s[hi];
                if ((a > b) == up) {
                    s[lo] = b;
                    s[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

__device__ int pow2_ceil(int x) {
    int n = 1;
    while (n < x) n <<= 1;
    return n;
}

// Stable scatter of src[beg, end) by the 8-bit digit at `shift` into dst, one
// 256-thread block, in chunks of 256 elements taken in order. s_off[d] holds
// the next output position of digit d and is advanced; s_wcnt (4 x 256) must
// be zero on entry and is zero on exit. Within a chunk each wave finds the
// lanes that share its digit with 8 ballots, so equal digits keep their input
// order (lanes, then waves, then chunks).
template <typename K, bool kVals>
__device__ void stable_scatter(const K *src, const uint32_t *src_v, K *dst, uint32_t *dst_v, uint64_t beg,
                               uint64_t end, int shift, uint32_t *s_off, uint32_t *s_wcnt) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (uint64_t c0 = beg; c0 < end; c0 += kThreads) {
        const uint64_t i = c0 + tid;
        const bool valid = i < end;
        const K key = valid ? src[i] : K(0);
        uint32_t val = 0;
        if (kVals && valid) val = src_v[i];
        const uint32_t d = (uint32_t)((key >> shift) & 0xff);
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
        if (leader) s_wcnt[wave * 256 + d] = cnt;
        __syncthreads();
        if (valid) {
            uint32_t pre = 0;
            for (int w = 0; w < wave; ++w) pre += s_wcnt[w * 256 + d];
            const uint64_t o = (uint64_t)s_off[d] + pre + rank;
            dst[o] = key;
            if (kVals) dst_v[o] = val;
        }
        __syncthreads();
        if (leader) {
            atomicAdd(&s_off[d], cnt);
            s_wcnt[wave * 256 + d] = 0;
        }
        __syncthreads();
    }
}

// Exclusive scan of a 256-entry LDS array in place (256 threads); s_tmp[4].
__device__ void scan256(uint32_t *a, uint32_t *s_tmp) {
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

// Replace the low 32 bits (submap index) of sorted pairs by the Gaussian's
// internal position (the blend gathers screen records by that position).
__device__ __forceinline__ uint64_t to_internal(uint64_t key, const uint32_t *inv_perm) {
    return (key & 0xffffffff00000000ull) | inv_perm[(uint32_t)key];
}

// Lists of length <= kSmallSortCap are sorted here; longer ones are queued.
__global__ __launch_bounds__(kThreads) void k_tile_sort(uint64_t *__restrict__ pairs,
                                                        const uint64_t *__restrict__ offsets, int n_tiles,
                                                        uint64_t capacity, const uint32_t *__restrict__ inv_perm,
                                                        uint32_t *__restrict__ long_list,
                                                        unsigned long long *__restrict__ counters) {
    __shared__ uint64_t s[kSmallSortCap];
    const uint64_t list = (uint64_t)blockIdx.y * n_tiles + blockIdx.x;
    const uint64_t beg = offsets[list];
    const uint64_t end = min(offsets[list + 1], capacity);
    if (end <= beg) return;
    if (end - beg > (uint64_t)kSmallSortCap) {
        if (threadIdx.x == 0) {
            const unsigned long long slot = atomicAdd(&counters[CNT_LONG_TILES], 1ull);
            long_list[slot] = (uint32_t)list;
        }
        return;
    }
    const int len = (int)(end - beg);
    const int n = pow2_ceil(len);
    for (int i = threadIdx.x; i < n; i += kThreads) s[i] = i < len ? pairs[beg + i] : ~0ull;
    __syncthreads();
    bitonic_lds(s, n);
    for (int i = threadIdx.x; i < len; i += kThreads) pairs[beg + i] = to_internal(s[i], inv_perm);
}

// Stable LSD radix sort of keys[0..len) (8-bit digits, only digits that vary),
// ping-ponging with tmp; the result ends in keys. One 256-thread block.
__device__ void radix_sort_global(uint64_t *keys, uint64_t *tmp, uint64_t len, uint32_t *s_off /*[256]*/,
                                  uint32_t *s_wcnt /*[4][256]*/, uint32_t *s_tmp /*[4]*/,
                                  unsigned long long *s_red /*[2]*/) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_red[0] = 0ull;
        s_red[1] = ~0ull;
    }
    for (int i = tid; i < 4 * 256; i += kThreads) s_wcnt[i] = 0;
    __syncthreads();
    unsigned long long o = 0ull, a = ~0ull;
    for (uint64_t i = tid; i < len; i += kThreads) {
        o |= keys[i];
        a &= keys[i];
    }
    atomicOr(&s_red[0], o);
    atomicAnd(&s_red[1], a);
    __syncthreads();
    const uint64_t vary = s_red[0] ^ s_red[1];
    uint64_t *src = keys, *dst = tmp;
    for (int shift = 0; shift < 64; shift += 8) {
        if (((vary >> shift) & 0xffull) == 0) continue;
        s_off[tid] = 0;
        __syncthreads();
        for (uint64_t i = tid; i < len; i += kThreads) atomicAdd(&s_off[(src[i] >> shift) & 0xff], 1u);
        __syncthreads();
        scan256(s_off, s_tmp);
        stable_scatter<uint64_t, false>(src, nullptr, dst, nullptr, 0, len, shift, s_off, s_wcnt);
        uint64_t *t = src;
        src = dst;
        dst = t;
    }
    if (src != keys) {
        for (uint64_t i = tid; i < len; i += kThreads) keys[i] = src[i];
    }
    __syncthreads();
}

// Queued long lists: a fixed grid walks the queue. Lists up to kMidSortCap are
// sorted in LDS, longer ones by the global-memory radix sort.
__global__ __launch_bounds__(kThreads) void k_long_sort(uint64_t *__restrict__ pairs, uint64_t *__restrict__ tmp,
                                                        const uint64_t *__restrict__ offsets, uint64_t capacity,
                                                        const uint32_t *__restrict__ inv_perm,
                                                        const uint32_t *__restrict__ long_list,
                                                        const unsigned long long *__restrict__ counters) {
    __shared__ uint64_t s[kMidSortCap];
    const uint64_t n_long = counters[CNT_LONG_TILES];
    for (uint64_t q = blockIdx.x; q < n_long; q += gridDim.x) {
        const uint32_t list = long_list[q];
        const uint64_t beg = offsets[list];
        const uint64_t end = min(offsets[list + 1], capacity);
        const uint64_t len = end - beg;
        if (len <= (uint64_t)kMidSortCap) {
            const int n = pow2_ceil((int)len);
            for (int i = threadIdx.x; i < n; i += kThreads) s[i] = (uint64_t)i < len ? pairs[beg + i] : ~0ull;
            __syncthreads();
            bitonic_lds(s, n);
            for (int i = threadIdx.x; (uint64_t)i < len; i += kThreads) pairs[beg + i] = to_internal(s[i], inv_perm);
            __syncthreads();
        } else {
            uint32_t *s32 = reinterpret_cast<uint32_t *>(s);
            radix_sort_global(pairs + beg, tmp + beg, len, s32, s32 + 256, s32 + 256 + 1024,
                              reinterpret_cast<unsigned long long *>(s32 + 256 + 1024 + 8));
            for (uint64_t i = threadIdx.x; i < len; i += kThreads) pairs[beg + i] = to_internal(pairs[beg + i], inv_perm);
            __syncthreads();
        }
    }
}

// ---- device-wide stable LSD radix sort of (uint32 key, uint32 value) ----
constexpr int kRsItems = 16;
constexpr int kRsTile = kThreads * kRsItems;  // keys per block and pass

__global__ __launch_bounds__(kThreads) void k_rs_hist(const uint32_t *__restrict__ keys, uint64_t n, int shift,
                                                      int nb, uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_h[256];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t beg = (uint64_t)blockIdx.x * kRsTile;
    const uint64_t end = min(beg + kRsTile, n);
    for (uint64_t i = beg + threadIdx.x; i < end; i += kThreads) atomicAdd(&s_h[(keys[i] >> shift) & 0xff], 1u);
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = s_h[threadIdx.x];  // digit-major
}

__global__ __launch_bounds__(kThreads) void k_rs_scatter(const uint32_t *__restrict__ keys,
                                                         const uint32_t *__restrict__ vals,
                                                         uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
                                                         uint64_t n, int shift, int nb,
                                                         const uint64_t *__restrict__ offsets) {
    __shared__ uint32_t s_off[256];
    __shared__ uint32_t s_wcnt[4 * 256];
    for (int i = threadIdx.x; i < 4 * 256; i += kThreads) s_wcnt[i] = 0;
    s_off[threadIdx.x] = (uint32_t)offsets[(uint64_t)threadIdx.x * nb + blockIdx.x];
    __syncthreads();
    const uint64_t beg = (uint64_t)blockIdx.x * kRsTile;
    const uint64_t end = min(beg + kRsTile, n);
    stable_scatter<uint32_t, true>(keys, vals, keys_out, vals_out, beg, end, shift, s_off, s_wcnt);
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

void launch_scan(hipStream_t s, const uint32_t *count, uint64_t n, uint64_t *offsets, uint64_t *tmp) {
    const uint64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 0) {
        launch_fill_u64(s, reinterpret_cast<unsigned long long *>(offsets), 1, 0ull);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kThreads), 0, s, count, n, tmp);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kThreads), 0, s, tmp, nb, offsets + n);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, count, n, tmp, offsets);
}

void launch_tile_sort(hipStream_t s, uint64_t *pairs, uint64_t *pairs_tmp, const uint64_t *offsets, int n_tiles,
                      int n_poses, uint64_t capacity, const uint32_t *inv_perm, uint32_t *long_list,
                      unsigned long long *counters) {
    if (n_tiles <= 0 || n_poses <= 0) return;
    hipLaunchKernelGGL(k_tile_sort, dim3((unsigned)n_tiles, (unsigned)n_poses), dim3(kThreads), 0, s, pairs,
                       offsets, n_tiles, capacity, inv_perm, long_list, counters);
    hipLaunchKernelGGL(k_long_sort, dim3(1024), dim3(kThreads), 0, s, pairs, pairs_tmp, offsets, capacity,
                       inv_perm, long_list, counters);
}

uint64_t radix_tmp_elems(uint64_t n) {
    const uint64_t nb = (n + kRsTile - 1) / kRsTile;
    return 256 * nb / 2 + 1 + (256 * nb + 1) + scan_tmp_elems(256 * nb);  // u64 units
}

void launch_radix_sort_u32(hipStream_t s, uint32_t *keys, uint32_t *vals, uint32_t *keys_tmp, uint32_t *vals_tmp,
                           uint64_t n, int bits, uint64_t *tmp) {
    if (n <= 1) return;
    const uint64_t nb = (n + kRsTile - 1) / kRsTile;
    uint32_t *hist = reinterpret_cast<uint32_t *>(tmp);
    uint64_t *offs = tmp + 256 * nb / 2 + 1;
    uint64_t *stmp = offs + 256 * nb + 1;
    uint32_t *ks = keys, *vs = vals, *kd = keys_tmp, *vd = vals_tmp;
    const int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        const int shift = 8 * p;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nb), dim3(kThreads), 0, s, ks, n, shift, (int)nb, hist);
        launch_scan(s, hist, 256 * nb, offs, stmp);
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nb), dim3(kThreads), 0, s, ks, vs, kd, vd, n, shift,
                           (int)nb, offs);
        std::swap(ks, kd);
        std::swap(vs, vd);
    }
    if (ks != keys) {
        (void)hipMemcpyAsync(keys, ks, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
        (void)hipMemcpyAsync(vals, vs, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, s);
    }
}

}  // namespace gsr
