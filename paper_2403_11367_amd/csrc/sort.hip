// Ordering of the (Gaussian, tile) pairs of every pose (S2-S4).
//
// Paper: Sec. III-A - the Gaussians are sorted by depth and composited front to
// back. Per (pose, tile) the blend needs its Gaussians in ascending depth, with
// equal depths in ascending submap index (a total order).
//
// Everything here is built on one primitive, a device-wide stable LSD radix
// sort with 8-bit digits (k_rs_hist -> exclusive scan -> k_rs_scatter per
// digit). Stability is what carries the order through:
//   1. visible (pose, Gaussian) entries are compacted in (pose, index) order;
//   2. they are radix-sorted by (pose, depth bits): ties keep index order;
//   3. each entry emits one pair per tile it touches, in that depth order;
//   4. the pairs are radix-sorted by (pose * T + tile): within a tile they keep
//      depth order;
//   5. each list's [start, end) is found by binary search in the sorted keys.
// No atomics, so the result is deterministic run to run.
#include "internal.h"

namespace gsr {

namespace {

constexpr int kThreads = 256;
constexpr int kScanItems = 8;  // per thread
constexpr int kScanTile = kThreads * kScanItems;
constexpr int kRsItems = 16;
constexpr int kRsTile = kThreads * kRsItems;  // keys per block and pass

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

__device__ __forceinline__ uint64_t dev_count(const uint64_t *d_n, uint64_t n_max) {
    return d_n ? min(*d_n, n_max) : n_max;
}

// Per-block digit histogram, stored digit-major: hist[d * nb + block].
template <typename K>
__global__ __launch_bounds__(kThreads) void k_rs_hist(const K *__restrict__ keys, const uint64_t *__restrict__ d_n,
                                                      uint64_t n_max, int shift, int nb, uint32_t *__restrict__ hist) {
    __shared__ uint32_t s_h[256];
    s_h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t n = dev_count(d_n, n_max);
    const uint64_t beg = (uint64_t)blockIdx.x * kRsTile;
    const uint64_t end = min(beg + kRsTile, n);
    for (uint64_t i = beg + threadIdx.x; i < end; i += kThreads) atomicAdd(&s_h[(keys[i] >> shift) & 0xff], 1u);
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nb + blockIdx.x] = s_h[threadIdx.x];
}

// Stable scatter of one block's keys by the digit at `shift`. The block walks
// its range in chunks of 256 in order; within a chunk each wave finds the
// lanes sharing its digit with 8 ballots, and per-wave counts in LDS order the
// waves, so equal digits keep their input order. s_off[d] starts at the
// block's global offset for digit d (from the scanned histogram).
template <typename K>
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const K *__restrict__ keys, const uint32_t *__restrict__ vals,
                                                         K *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
                                                         const uint64_t *__restrict__ d_n, uint64_t n_max, int shift,
                                                         int nb, const uint64_t *__restrict__ offsets) {
    __shared__ unsigned long long s_off[256];
    __shared__ uint32_t s_wcnt[4 * 256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < 4 * 256; i += kThreads) s_wcnt[i] = 0;
    s_off[tid] = offsets[(uint64_t)tid * nb + blockIdx.x];
    __syncthreads();
    const uint64_t n = dev_count(d_n, n_max);
    const uint64_t beg = (uint64_t)blockIdx.x * kRsTile;
    const uint64_t end = min(beg + kRsTile, n);
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (uint64_t c0 = beg; c0 < end; c0 += kThreads) {
        const uint64_t i = c0 + tid;
        const bool valid = i < end;
        const K key = valid ? keys[i] : K(0);
        const uint32_t val = valid ? vals[i] : 0u;
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
            const uint64_t o = s_off[d] + pre + rank;
            keys_out[o] = key;
            vals_out[o] = val;
        }
        __syncthreads();
        if (leader) {
            atomicAdd(&s_off[d], (unsigned long long)cnt);
            s_wcnt[wave * 256 + d] = 0;
        }
        __syncthreads();
    }
}

__global__ void k_copy_u32(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, const uint64_t *d_n,
                           uint64_t n_max) {
    const uint64_t n = dev_count(d_n, n_max);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void k_copy_u64(const uint64_t *__restrict__ src, uint64_t *__restrict__ dst, const uint64_t *d_n,
                           uint64_t n_max) {
    const uint64_t n = dev_count(d_n, n_max);
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// [start, end) of list t (0 <= t < n_lists) in keys[0, n) sorted ascending:
// offsets[t] = lower_bound(t); offsets[n_lists] = n.
__global__ void k_ranges(const uint32_t *__restrict__ keys, const uint64_t *__restrict__ d_n, uint64_t n_max,
                         uint64_t n_lists, uint64_t *__restrict__ offsets) {
    const uint64_t n = dev_count(d_n, n_max);
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t <= n_lists;
         t += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t lo = 0, hi = n;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if ((uint64_t)keys[mid] < t)
                lo = mid + 1;
            else
                hi = mid;
        }
        offsets[t] = t == n_lists ? n : lo;
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

uint64_t radix_tmp_elems(uint64_t n_max) {
    const uint64_t nb = std::max<uint64_t>(1, (n_max + kRsTile - 1) / kRsTile);
    return (256 * nb + 1) / 2 + 1 + (256 * nb + 1) + scan_tmp_elems(256 * nb);  // uint64 units
}

template <typename K>
void launch_radix_sort(hipStream_t s, K *keys, uint32_t *vals, K *keys_tmp, uint32_t *vals_tmp, uint64_t n_max,
                       const uint64_t *d_n, int begin_bit, int end_bit, uint64_t *tmp) {
    if (n_max == 0 || end_bit <= begin_bit) return;
    const uint64_t nb = (n_max + kRsTile - 1) / kRsTile;
    uint32_t *hist = reinterpret_cast<uint32_t *>(tmp);
    uint64_t *offs = tmp + (256 * nb + 1) / 2 + 1;
    uint64_t *stmp = offs + 256 * nb + 1;
    K *ks = keys, *kd = keys_tmp;
    uint32_t *vs = vals, *vd = vals_tmp;
    for (int shift = begin_bit; shift < end_bit; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist<K>, dim3((unsigned)nb), dim3(kThreads), 0, s, ks, d_n, n_max, shift, (int)nb,
                           hist);
        launch_scan(s, hist, 256 * nb, offs, stmp, nullptr);
        hipLaunchKernelGGL(k_rs_scatter<K>, dim3((unsigned)nb), dim3(kThreads), 0, s, ks, vs, kd, vd, d_n, n_max,
                           shift, (int)nb, offs);
        std::swap(ks, kd);
        std::swap(vs, vd);
    }
    if (ks != keys) {
        const unsigned blocks = (unsigned)std::min<uint64_t>((n_max + kThreads - 1) / kThreads, 4096);
        if (sizeof(K) == 8)
            hipLaunchKernelGGL(k_copy_u64, dim3(blocks), dim3(kThreads), 0, s, (const uint64_t *)ks,
                               (uint64_t *)keys, d_n, n_max);
        else
            hipLaunchKernelGGL(k_copy_u32, dim3(blocks), dim3(kThreads), 0, s, (const uint32_t *)ks,
                               (uint32_t *)keys, d_n, n_max);
        hipLaunchKernelGGL(k_copy_u32, dim3(blocks), dim3(kThreads), 0, s, vs, vals, d_n, n_max);
    }
}

template void launch_radix_sort<uint32_t>(hipStream_t, uint32_t *, uint32_t *, uint32_t *, uint32_t *, uint64_t,
                                          const uint64_t *, int, int, uint64_t *);
template void launch_radix_sort<uint64_t>(hipStream_t, uint64_t *, uint32_t *, uint64_t *, uint32_t *, uint64_t,
                                          const uint64_t *, int, int, uint64_t *);

void launch_ranges(hipStream_t s, const uint32_t *keys, const uint64_t *d_n, uint64_t n_max, uint64_t n_lists,
                   uint64_t *offsets) {
    const unsigned blocks = (unsigned)std::min<uint64_t>((n_lists + 1 + kThreads - 1) / kThreads, 4096);
    hipLaunchKernelGGL(k_ranges, dim3(blocks), dim3(kThreads), 0, s, keys, d_n, n_max, n_lists, offsets);
}

}  // namespace gsr
