// Front-to-back compositing of colour and depth per tile (S5): 16x16 tiles by
// default, 32x8 and 8x32 as options.
//
// Paper: Sec. III-A, Eq. 1 and Eq. 5 with the footprint of Eq. 2:
//   C(x) = sum_i c_i a_i T_i,  D(x) = sum_i z_i a_i T_i,  T_i = prod_{j<i} (1 - a_j),
//   a_i = min(alpha_max, o_i exp(-d_i^2 / 2)) where d_i^2 <= cutoff and a_i >= alpha_min,
// over the depth-sorted list of the tile. A pixel stops after the layer that
// takes T below t_min (that layer counts).
//
// One 256-thread block per (tile, pose); wave w owns pixel rows 4w..4w+3 of the
// tile (a 16x4 band), one pixel per lane, and the band is split into four 4x4
// quarters (lanes 16q..16q+15). The block walks the tile's list in chunks of
// 252 records: every thread but the last of each wave stages one record in LDS
// (the conic as two scaled square-root factors, log2 of the opacity, and one
// log2 threshold that folds the cutoff and the alpha floor) and writes which
// (band, quarter) cells its support ellipse overlaps; each wave ballots its
// band's marks into one 64-bit mask per (quarter, 64-record group). A wave walks
// its four quarters side by side: step i takes the i-th record of every
// quarter (a quarter with fewer reads a record that cannot contribute; the
// per-step slots are laid out in LDS once per chunk), so a chunk costs the
// longest of the four walks rather than their union. Each pixel still sees its
// records in list order. A wave stops when all of its pixels have stopped; the
// block stops loading when all waves have.
//
// The backward of the compositing (k_blend_backward) runs the same walk: with
// w_i = a_i T_i and S_i the colour behind layer i (the final colour minus the
// colour up to and including it), dC/da_i = c_i T_i - S_i / (1 - a_i),
// dC/dc_i = w_i, dD/dz_i = w_i; dL/da_i takes these dotted with the image
// gradients, so one running sum of g.c w serves all four channels. Each visit's
// gradients with respect to the record's (u, v, conic, opacity, colour, depth)
// are summed over the quarter's 16 lanes, which all visit the same record, and
// added to the record's LDS accumulator; at the end of a chunk every staged
// record's sums go to global memory with one atomic add per value.
#include "blend_common.h"

namespace gsr {

namespace {

constexpr int kThreads = 256;
// Records staged per wave and chunk: 63 (lane 63 idle; a chunk of 252), 31 or 15
// (chunks of 124 or 60, for earlier exits on short lists). A template parameter.
template <bool B>
struct BoolTag {
    static constexpr bool value = B;
};
constexpr int kDummy = 255;             // LDS slot (wave 3, lane 63) of a record that never contributes

// Kept compositing state: for every tile list longer than kKeepRecords, each
// pixel's T and colour and depth sums just before list positions kKeepRecords,
// 2 kKeepRecords, ... (a multiple of the 252-record chunk). cp_off[list] is the
// index of the list's first kept state (an exclusive prefix over the lists);
// state [index][5][256]: T, r, g, b, depth per tile pixel (thread index).
struct KeepIo {
    const uint32_t *cp_off;
    float *state;
};

// Inputs and output of the backward walk, per launch (pose 0 = the launch's first).
// Block b walks segment s of list items[b] (s = b - list - cp_off[list]): the
// records from s kKeepRecords to the next kept state or the list's end, starting
// from kept state s (s > 0) or from T = 1 (s = 0).
struct GradIo {
    const float *img_rgb, *img_depth;  // the forward's images [P, 3, H, W], [P, H, W]
    const float *g_rgb, *g_depth;      // dL/d(images), same layouts
    float *gscreen;                    // [P, n, 10] screen-space gradients, accumulated
    const uint32_t *cp_off;            // kept states per list, as in KeepIo (all 0: none kept)
    const float *state;
    const uint32_t *items;             // list of each block
    uint32_t n_lists;
};

// Sums of the 10 values over each lane's 16-lane DPP row (one quarter): after
// rotations by 8, 4, 2 and 1 within the row (v += row_ror(v)) every lane holds
// its row's totals. All 64 lanes must be active. Written out because the
// compiler leaves a separate DPP move (and a zeroing move) in front of some of
// the adds; stage by stage across the 10 values, every DPP read comes 9
// instructions after the write it reads, and the leading s_nop covers the
// two wait states a DPP read needs after the compiler's last VALU write.
__device__ __forceinline__ void quarter_sums(float (&v)[kScreenGrads]) {
    static_assert(kScreenGrads == 10, "one operand per value");
    asm volatile(
        "s_nop 1\n"
        "v_add_f32_dpp %0, %0, %0 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %1, %1, %1 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %2, %2, %2 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %3, %3, %3 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %4, %4, %4 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %5, %5, %5 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %6, %6, %6 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %7, %7, %7 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %8, %8, %8 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %9, %9, %9 row_ror:8 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %0, %0, %0 row_ror:4 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %1, %1, %1 row_ror:4 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %2, %2, %2 row_ror:4 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %3, %3, %3 row_ror:4 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %4, %4, %4 row_ror:4 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %5, %5, %5 row_ror:4 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %6, %6, %6 row_ror:4 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %7, %7, %7 row_ror:4 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %8, %8, %8 row_ror:4 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %9, %9, %9 row_ror:4 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %0, %0, %0 row_ror:2 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %1, %1, %1 row_ror:2 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %2, %2, %2 row_ror:2 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %3, %3, %3 row_ror:2 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %4, %4, %4 row_ror:2 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %5, %5, %5 row_ror:2 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %6, %6, %6 row_ror:2 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %7, %7, %7 row_ror:2 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %8, %8, %8 row_ror:2 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %9, %9, %9 row_ror:2 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %0, %0, %0 row_ror:1 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %1, %1, %1 row_ror:1 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %2, %2, %2 row_ror:1 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %3, %3, %3 row_ror:1 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %4, %4, %4 row_ror:1 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %5, %5, %5 row_ror:1 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %6, %6, %6 row_ror:1 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %7, %7, %7 row_ror:1 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %8, %8, %8 row_ror:1 row_mask:0xf bank_mask:0xf\n"
        "v_add_f32_dpp %9, %9, %9 row_ror:1 row_mask:0xf bank_mask:0xf\n"
        : "+v"(v[0]), "+v"(v[1]), "+v"(v[2]), "+v"(v[3]), "+v"(v[4]), "+v"(v[5]), "+v"(v[6]), "+v"(v[7]),
          "+v"(v[8]), "+v"(v[9]));
}

// The compositing of one (tile, pose) by the whole block, or (kGrad) its
// backward: the same walk, so the same pixels visit the same records in the
// same order and recompute the forward's T bit for bit.
template <int kTW, bool kCount, int kStage, bool kGrad = false, bool kKeep = false>
__device__ __forceinline__ void blend_tile(int tile, int pose, const float4 *__restrict__ records, int64_t n,
                                           const uint32_t *__restrict__ pairs,
                                           const uint64_t *__restrict__ offsets, uint64_t capacity, int width,
                                           int height, int tiles_x, int n_tiles, const BlendConsts &k,
                                           float *__restrict__ out_rgb, float *__restrict__ out_depth,
                                           float *__restrict__ out_t, unsigned long long *__restrict__ counters,
                                           const GradIo &gio = GradIo{}, const KeepIo &keep = KeepIo{},
                                           uint32_t seg = 0) {
    static_assert(!kKeep || (kStage == 63 && !kGrad), "kept states are written by the 252-record forward");
    // slot = staging thread; the backward adds a fourth quad (A, B, C, u - tile centre x)
    constexpr int kQuads = kGrad ? 4 : 3;
    constexpr uint32_t kSlotBytes = 16u * kQuads;
    __shared__ float4 s_rec[kThreads * kQuads];
    // backward: the gradients of each staged record summed over the chunk's
    // quarter visits, [value][slot], flushed to global memory once per chunk
    __shared__ float s_acc[kGrad ? kScreenGrads : 1][kGrad ? kThreads : 1];
    // (band, quarter) cells of the record in each slot: the forward keeps them in
    // the unused last word of the colour quad (s2.w), the backward here
    __shared__ uint16_t s_cells[kGrad ? kThreads : 1];
    // per wave, quarter and step: slot of the record the quarter visits
    // per wave, quarter and step: LDS byte offset of the record the quarter
    // visits (steps 0..253: a walk has at most 252 steps and reads 2 ahead)
    constexpr int kSlotCap = 254;
    __shared__ __attribute__((aligned(16))) uint16_t s_slots[4][4][kSlotCap];
    __shared__ uint32_t s_live[4];   // per wave: any pixel still live after the chunk
    __shared__ uint32_t s_clamp[4];  // per wave: a staged record whose alpha may reach alpha_max

    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int quarter = lane >> 4;
    // tile of kTW x kTH pixels; wave w owns rows kBH w .. kBH w + kBH - 1 (a band of 64
    // pixels), split into four cells of kCW x kBH (16 lanes each, row-major inside)
    constexpr int kTH = kThreads / kTW, kBH = 64 / kTW, kCW = kTW / 4;
    static_assert(kTW == 8 || kTW == 16 || kTW == 32, "8x32, 16x16 or 32x8 tiles");
    const int pi = tx * kTW + quarter * kCW + ((lane & 15) % kCW);
    const int pj = ty * kTH + wave * kBH + ((lane & 15) / kCW);
    const bool in_image = pi < width && pj < height;
    const int row0 = ty * kTH, col0 = tx * kTW;
    // pixel centre relative to the tile centre (col0 + kTW / 2, row0 + kTH / 2), exact
    const float xc = (float)(pi - col0) - (0.5f * (float)kTW - 0.5f);
    const float yc = (float)(pj - row0) - (0.5f * (float)kTH - 0.5f);

    const uint64_t list = (uint64_t)pose * n_tiles + tile;
    const uint64_t beg = offsets[list];
    const uint64_t end = min(offsets[list + 1], capacity);
    // the walk's range: the whole list, or (backward) one kept-state segment of it
    uint64_t lbeg = beg, lend = end;
    if constexpr (kGrad) {
        lbeg = beg + (uint64_t)seg * kKeepRecords;
        if (seg < gio.cp_off[list + 1] - gio.cp_off[list]) lend = lbeg + kKeepRecords;
    }
    const float4 *rec_pose = records + (int64_t)pose * n * 3;

    if (tid == kDummy) {  // this thread never stages a record
        const float inf = __builtin_inff();
        s_rec[kDummy * kQuads + 0] = make_float4(0.f, 0.f, 0.f, 0.f);
        s_rec[kDummy * kQuads + 1] = make_float4(0.f, inf, 0.f, 0.f);
        s_rec[kDummy * kQuads + 2] = make_float4(0.f, 0.f, 0.f, 0.f);
    }

    // A pixel is live (still compositing) while T >= t_min: T never increases and
    // stops changing once the pixel has stopped, so no separate flag is kept.
    float T = in_image ? 1.f : 0.f, cr = 0.f, cg = 0.f, cb = 0.f, dep = 0.f;
    unsigned n_contrib = 0, n_visits = 0;  // only with kCount
    const char *s_rec_bytes = reinterpret_cast<const char *>(s_rec);

    // backward: the loss gradients of the pixel's colour and depth (g), the
    // g-weighted final colour and depth, and the g-weighted colour and depth up to
    // the current layer (s_front, accumulated as the forward accumulates colour)
    float gr = 0.f, gg = 0.f, gb = 0.f, gd = 0.f, g_fin = 0.f, s_front = 0.f;
    float *gpose = nullptr;
    if constexpr (kGrad) {
        const int64_t hw = (int64_t)width * height;
        const int64_t pix = in_image ? (int64_t)pj * width + pi : 0;
        const int64_t prgb = (int64_t)pose * 3 * hw + pix, pd = (int64_t)pose * hw + pix;
        gr = gio.g_rgb[prgb];
        gg = gio.g_rgb[prgb + hw];
        gb = gio.g_rgb[prgb + 2 * hw];
        gd = gio.g_depth[pd];
        g_fin = gr * gio.img_rgb[prgb] + gg * gio.img_rgb[prgb + hw] + gb * gio.img_rgb[prgb + 2 * hw] +
                gd * gio.img_depth[pd];
        gpose = gio.gscreen + (int64_t)pose * n * kScreenGrads;
        if (seg > 0) {
            // the forward's state before this segment, bit for bit
            const float *st = gio.state + (size_t)(gio.cp_off[list] + seg - 1) * 5 * kThreads;
            T = st[tid];
            s_front = gr * st[kThreads + tid] + gg * st[2 * kThreads + tid] + gb * st[3 * kThreads + tid] +
                      gd * st[4 * kThreads + tid];
        }
    }
    // forward with kept states: writes state s (s >= 1) of this list
    uint32_t kept = 0;  // states written
    auto keep_state = [&](uint32_t s_index) {
        float *st = keep.state + (size_t)(keep.cp_off[list] + s_index - 1) * 5 * kThreads;
        st[tid] = T;
        st[kThreads + tid] = cr;
        st[2 * kThreads + tid] = cg;
        st[3 * kThreads + tid] = cb;
        st[4 * kThreads + tid] = dep;
    };

    if constexpr (kGrad) {
#pragma unroll
        for (int j = 0; j < kScreenGrads; ++j) s_acc[j][tid] = 0.f;
    }
    uint32_t staged_g = 0xffffffffu;  // backward: Gaussian this thread staged in the current chunk

    for (uint64_t c0 = lbeg; c0 < lend; c0 += 4 * kStage) {
        if constexpr (kKeep) {
            // chunks are 252 records and kKeepRecords a multiple of that
            if (c0 != beg && (c0 - beg) % kKeepRecords == 0) keep_state(++kept);
        }
        // stage one record per thread (lanes 0..62 of every wave)
        const uint64_t kk = c0 + (uint64_t)wave * kStage + lane;
        uint32_t cells = 0;  // bit 4 * band + quarter
        bool may_clamp = false;  // o exp(-d^2/2) can reach alpha_max (o near or above it)
        if (lane < kStage && kk < lend) {
            const uint32_t g = pairs[kk];
            if constexpr (kGrad) staged_g = g;
            const float4 *r = rec_pose + (int64_t)g * 3;
            const float4 q0 = r[0], q1 = r[1], q2 = r[2];
            // 2^p2 <= 2^log2(o) ~ o (hardware log2 and exp2: a few ulp), so below this
            // bound the clamp at alpha_max never acts
            may_clamp = q1.y > k.alpha_max * 0.9999f;
            const uint32_t rx = __float_as_uint(q2.z), ry = __float_as_uint(q2.w);
            const int j0 = (int)(ry & 0xffffu) - row0, j1 = (int)(ry >> 16) - row0;
            // Cells are (band, quarter) pixel blocks. The support ellipse
            // E = {d^2 <= cutoff} meets a cell iff the x-extent of E within the
            // band's rows overlaps the quarter's columns (E is convex). With
            // dx = x - u, dy = y - v: the chord of E at height dy spans
            // (-B dy -+ sqrt(A R2 - det dy^2)) / A; its right end is concave in dy
            // and peaks at dy = -(B / C) dxm with value dxm = sqrt(R2 C / det)
            // (the left end mirrors it), so over a band the extreme is either that
            // peak or the chord at the nearer band edge. R2 carries a margin that
            // covers float32 rounding, so the test never drops a contributing cell.
            const float A = q0.z, B = q0.w, C = q1.x;
            // d^2 as a sum of squares (stage_record): a needle-thin footprint loses
            // about sqrt(A C / det) times less to rounding than the expanded form
            const float det = conic_det(A, B, C);
            const float iA = __builtin_amdgcn_rcpf(A), idet = __builtin_amdgcn_rcpf(det);
            const float u_rel = q0.x - (float)col0, v_rel = q0.y - (float)row0;
            // from the tile centre
            const float uc = q0.x - (float)(col0 + kTW / 2), vc = q0.y - (float)(row0 + kTH / 2);
            stage_record(q0, q1, q2, det, uc, vc, k, s_rec[tid * kQuads + 0], s_rec[tid * kQuads + 1],
                         s_rec[tid * kQuads + 2]);
            if constexpr (kGrad) s_rec[tid * kQuads + 3] = make_float4(A, B, C, uc);
            const float R2 = k.cull_r2;
            // hardware reciprocal and square root (about 1 ulp) for the overlap test:
            // the margin in R2 covers them
            const float ryv = __builtin_amdgcn_sqrtf(R2 * A * idet);
            const float dxm = __builtin_amdgcn_sqrtf(R2 * C * idet);
            const float dys = -B * __builtin_amdgcn_rcpf(C) * dxm;  // dy of the rightmost point of E
            if (det > 0.f && __builtin_isfinite(ryv) && __builtin_isfinite(dxm) && __builtin_isfinite(dys)) {
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    if (!(j0 <= kBH * b + kBH - 1 && j1 >= kBH * b)) continue;
                    // (all finite here; the clamps are medians)
                    const float ylo = max_finite(((float)(kBH * b) + 0.5f) - v_rel, -ryv);
                    const float yhi = min_finite(((float)(kBH * b + kBH) - 0.5f) - v_rel, ryv);
                    if (!(ylo <= yhi)) continue;
                    const float yr = __builtin_amdgcn_fmed3f(dys, ylo, yhi);   // where the right end peaks in the band
                    const float yl = __builtin_amdgcn_fmed3f(-dys, ylo, yhi);  // where the left end bottoms
                    const float xr = (-B * yr + __builtin_amdgcn_sqrtf(max_finite(A * R2 - det * yr * yr, 0.f))) * iA;
                    const float xl = (-B * yl - __builtin_amdgcn_sqrtf(max_finite(A * R2 - det * yl * yl, 0.f))) * iA;
                    const float x_hi = u_rel + xr + 1e-3f, x_lo = u_rel + xl - 1e-3f;  // tile-relative
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (x_hi >= (float)(kCW * q) + 0.5f && x_lo <= (float)(kCW * q + kCW) - 0.5f)
                            cells |= 1u << (4 * b + q);
                }
            } else {
                // fall back to the pixel rectangle
                const int i0 = (int)(rx & 0xffffu) - col0, i1 = (int)(rx >> 16) - col0;
#pragma unroll
                for (int b = 0; b < 4; ++b)
#pragma unroll
                    for (int q = 0; q < 4; ++q)
                        if (j0 <= kBH * b + kBH - 1 && j1 >= kBH * b && i0 <= kCW * q + kCW - 1 && i1 >= kCW * q)
                            cells |= 1u << (4 * b + q);
            }
        }
        // 0 for a thread without a record (the dummy's colour quad is all 0)
        if constexpr (kGrad)
            s_cells[tid] = (uint16_t)cells;
        else
            reinterpret_cast<uint32_t *>(&s_rec[tid * kQuads + 2])[3] = cells;
        {
            const bool wave_clamp = __ballot(may_clamp) != 0;
            if (lane == 0) s_clamp[wave] = wave_clamp;
        }
        __syncthreads();
        // read here, rewritten only after the end-of-chunk barrier
        const bool clamp_chunk = kGrad || (s_clamp[0] | s_clamp[1] | s_clamp[2] | s_clamp[3]) != 0;

        const uint32_t n_left = (uint32_t)min<uint64_t>(lend - c0, 4 * kStage);
        const uint32_t n_groups = (n_left + kStage - 1) / kStage;  // 64-record groups staged
        uint64_t lm = __ballot(!(T < k.t_min));  // live lanes
        if (lm != 0) {
            // Step i visits the i-th record (in list order) of every quarter that
            // overlaps it, or the dummy slot when the quarter has fewer. The record
            // in slot 64 g + l is entered by lane l at its rank in each quarter's
            // walk; every lane then reads its own quarter's slots. One wave: its
            // LDS accesses complete in program order.
            // (16-byte stores: a wave's four lists are 127 of them)
            uint4 *slots128 = reinterpret_cast<uint4 *>(&s_slots[wave][0][0]);
            constexpr uint32_t kDummyPair = kDummy * kSlotBytes * 0x00010001u;
            static_assert(kDummy * kSlotBytes < 65536u && (4 * kSlotCap * 2) % 16 == 0, "16-bit offsets, whole pieces");
            const uint4 dummy4 = make_uint4(kDummyPair, kDummyPair, kDummyPair, kDummyPair);
#pragma unroll
            for (int e = 0; e < (4 * kSlotCap / 8 + 63) / 64; ++e)
                if (e * 64 + lane < 4 * kSlotCap / 8) slots128[e * 64 + lane] = dummy4;
            // Group by group (lane l: the record in slot 64 g + l), each quarter's
            // walk grows by the group's records that overlap the quarter's cell.
            uint32_t run[4] = {0u, 0u, 0u, 0u};
            for (uint32_t grp = 0; grp < n_groups; ++grp) {
                uint32_t cw;  // this band's 4 marks
                if constexpr (kGrad)
                    cw = s_cells[grp * 64 + lane];
                else
                    cw = reinterpret_cast<const uint32_t *>(&s_rec[(grp * 64 + lane) * kQuads + 2])[3];
                cw >>= 4 * wave;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (((lm >> (16 * q)) & 0xffffull) == 0) continue;  // no live pixel in the quarter
                    const uint64_t m = __ballot((cw >> q) & 1u);
                    const uint32_t rank =
                        __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    if (__builtin_amdgcn_inverse_ballot_w64(m))
                        s_slots[wave][q][run[q] + rank] = (uint16_t)((grp * 64 + lane) * kSlotBytes);
                    run[q] += (uint32_t)__popcll(m);
                }
            }
            // (uniform: every run is a sum of ballot counts)
            const uint32_t steps = __builtin_amdgcn_readfirstlane(max(max(run[0], run[1]), max(run[2], run[3])));
            // Software pipeline, unrolled twice so the two register sets alternate:
            // the slots and geometry of step i + 1 are read during step i.
            auto load = [&](uint32_t o, float4 &ra, float4 &rb) {
                ra = *reinterpret_cast<const float4 *>(s_rec_bytes + o);
                rb = *reinterpret_cast<const float4 *>(s_rec_bytes + o + 16);
            };
            // The walk, with (kClamp) or without the clamp of alpha at alpha_max: a
            // chunk none of whose records can reach alpha_max skips it (exactly: the
            // clamp is then the identity).
            auto walk = [&](auto clamp_tag) {
                constexpr bool kClamp = decltype(clamp_tag)::value;
                // one step on a staged record: lanes outside the live mask lm take nothing
                auto step = [&](uint32_t o, const float4 &ra, const float4 &rb) {
                    const float p2 = footprint_p2(ra, rb, xc, yc);
                    const bool ok = __builtin_amdgcn_inverse_ballot_w64(lm) && p2 >= rb.y;
                    if (kCount) {
                        n_contrib += ok;
                        ++n_visits;
                    }
                    if constexpr (!kGrad) {
                        // Without a branch: w = 0 where the pixel does not take this
                        // record, and fma(c, 0, x) = x, T - 0 = T exactly (the sums are
                        // finite and never -0), so every pixel's result is unchanged.
                        const float4 c = *reinterpret_cast<const float4 *>(s_rec_bytes + o + 32);
                        const float e = __builtin_amdgcn_exp2f(p2);
                        const float al = kClamp ? clamp_alpha(e, k.alpha_max) : e;
                        const float w = ok ? al * T : 0.f;
                        cr = __builtin_fmaf(c.x, w, cr);
                        cg = __builtin_fmaf(c.y, w, cg);
                        cb = __builtin_fmaf(c.z, w, cb);
                        dep = __builtin_fmaf(rb.w, w, dep);
                        T -= w;
                    } else {
                        // Screen-space gradients of this pixel for this record (u, v,
                        // A, B, C, opacity, r, g, b, z), without a branch: the weight and
                        // dL/dalpha are zero where the pixel does not take the record (and
                        // dL/dalpha where alpha is clamped at alpha_max, a constant), so
                        // those lanes add zeros and keep T unchanged, exactly as the
                        // forward does.
                        float gv[kScreenGrads];
                        {
                            const float4 c = *reinterpret_cast<const float4 *>(s_rec_bytes + o + 32);
                            const float4 e = *reinterpret_cast<const float4 *>(s_rec_bytes + o + 48);
                            const float gexp = __builtin_amdgcn_exp2f(p2);
                            const float al = clamp_alpha(gexp, k.alpha_max);
                            const float w = ok ? al * T : 0.f;
                            // dL/dalpha = g.c T - g.(what this layer hides) / (1 - alpha), with
                            // g.(hidden) = g.(final) - g.(up to and including this layer)
                            const float gc = gr * c.x + gg * c.y + gb * c.z + gd * rb.w;
                            s_front = __builtin_fmaf(gc, w, s_front);
                            const float inv = __builtin_amdgcn_rcpf(1.f - al);
                            const float dla = gc * T - (g_fin - s_front) * inv;
                            // alpha = o exp(-d^2/2): dalpha/do = alpha / o, dalpha/d(d^2) = -alpha / 2
                            const float dla_f = (ok && gexp < k.alpha_max) ? dla : 0.f;
                            // (u - xc, v - yc) of the record: e.w and c.w
                            const float dx = xc - e.w, dy = yc - c.w;
                            const float gd2 = -0.5f * dla_f * al;
                            gv[0] = -2.f * gd2 * (e.x * dx + e.y * dy);
                            gv[1] = -2.f * gd2 * (e.y * dx + e.z * dy);
                            gv[2] = gd2 * dx * dx;
                            gv[3] = 2.f * gd2 * dx * dy;
                            gv[4] = gd2 * dy * dy;
                            gv[5] = dla_f * al * __builtin_amdgcn_exp2f(-rb.z);  // 1 / o = 2^-log2(o)
                            gv[6] = gr * w;
                            gv[7] = gg * w;
                            gv[8] = gb * w;
                            gv[9] = gd * w;
                            T -= w;
                        }
                        // any lane of the quarter contributing (every lane of a quarter visits the same record)
                        const uint64_t okm = __ballot(ok);
                        if (okm != 0) {
                            quarter_sums(gv);
                            if ((lane & 15) == 0 && ((okm >> (16 * quarter)) & 0xffffull) != 0) {
                                const uint32_t slot = o / kSlotBytes;
#pragma unroll
                                for (int j = 0; j < kScreenGrads; ++j) atomicAdd(&s_acc[j][slot], gv[j]);
                            }
                        }
                    }
                    lm = __ballot(!(T < k.t_min));
                };
                const uint16_t *sp = &s_slots[wave][quarter][0];  // this lane's quarter; sp[j]: step i + j
                float4 a0, b0, a1, b1;
                uint32_t o0 = sp[0], o1;
                load(o0, a0, b0);
                uint32_t o_next = sp[1];
                // Steps go in pairs, and the wave's exit is checked after each pair: a
                // pixel that stops in the first step of a pair is masked in the second
                // (lm is updated every step), and a step past a quarter's walk reads the
                // dummy record (every slot list is dummy-filled), so the extra step of an
                // odd count changes nothing. The walk ends at the longest quarter's
                // count, or when no pixel of the wave is live. (Checking every step, and
                // shortening the walk when a quarter's pixels have all stopped, cost more
                // in scalar instructions than they saved.)
                // i < steps <= 252 with i even, so every slot read, at most i + 3,
                // stays below kSlotCap
                for (uint32_t i = 0; i < steps; i += 2, sp += 2) {
                    o1 = o_next;  // step i + 1
                    load(o1, a1, b1);
                    const uint32_t oa = sp[2], ob = sp[3];  // steps i + 2, i + 3
                    step(o0, a0, b0);
                    o0 = oa;
                    load(o0, a0, b0);
                    o_next = ob;
                    step(o1, a1, b1);
                    if (lm == 0) break;
                }
            };
            if (clamp_chunk)
                walk(BoolTag<true>{});
            else if constexpr (!kGrad)
                walk(BoolTag<false>{});
        }
        // any live pixel in the block (each wave's flag is read after the barrier and
        // rewritten only after the next chunk's barrier)
        {
            const bool wave_live = __ballot(!(T < k.t_min)) != 0;
            if (lane == 0) s_live[wave] = wave_live;
        }
        __syncthreads();
        const bool live = (s_live[0] | s_live[1] | s_live[2] | s_live[3]) != 0;
        if constexpr (kGrad) {
            // every wave is done with the chunk: add each staged record's sums once
            if (staged_g != 0xffffffffu) {
                float *dst = gpose + (int64_t)staged_g * kScreenGrads;
#pragma unroll
                for (int j = 0; j < kScreenGrads; ++j) {
                    const float v = s_acc[j][tid];
                    if (v != 0.f) atomicAdd(dst + j, v);
                    s_acc[j][tid] = 0.f;
                }
                staged_g = 0xffffffffu;
            }
        }
        if (!live) break;
    }
    if constexpr (kKeep) {
        // states past an early stop equal the final state (nothing changes after it)
        const uint32_t n_kept = keep.cp_off[list + 1] - keep.cp_off[list];
        while (kept < n_kept) keep_state(++kept);
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

    if (!kGrad && in_image) {
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

template <int kTW, bool kCount, int kStage>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_blend(
    const float4 *__restrict__ records, int64_t n, const uint32_t *__restrict__ pairs,
    const uint64_t *__restrict__ offsets, uint64_t capacity, int width, int height, int tiles_x, int n_tiles,
    BlendConsts k, float *__restrict__ out_rgb, float *__restrict__ out_depth, float *__restrict__ out_t,
    unsigned long long *__restrict__ counters) {
    blend_tile<kTW, kCount, kStage>(blockIdx.x, blockIdx.y, records, n, pairs, offsets, capacity, width, height,
                                    tiles_x, n_tiles, k, out_rgb, out_depth, out_t, counters);
}

// Persistent variant: a fixed number of blocks take (pose, tile) items, pose
// major, from a work queue (*queue starts at 0) until it passes n_items; every
// block leaves once it draws an item past the end.
template <int kTW, bool kCount, int kStage>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_blend_queue(
    const float4 *__restrict__ records, int64_t n, const uint32_t *__restrict__ pairs,
    const uint64_t *__restrict__ offsets, uint64_t capacity, int width, int height, int tiles_x, int n_tiles,
    BlendConsts k, float *__restrict__ out_rgb, float *__restrict__ out_depth, float *__restrict__ out_t,
    unsigned long long *__restrict__ counters, unsigned int n_items, unsigned int *__restrict__ queue) {
    __shared__ unsigned int s_item;
    for (;;) {
        __syncthreads();  // the previous item is done with LDS and with s_item
        if (threadIdx.x == 0) s_item = atomicAdd(queue, 1u);
        __syncthreads();
        const unsigned int item = s_item;
        if (item >= n_items) break;
        blend_tile<kTW, kCount, kStage>((int)(item % (unsigned)n_tiles), (int)(item / (unsigned)n_tiles), records, n,
                                        pairs, offsets, capacity, width, height, tiles_x, n_tiles, k, out_rgb,
                                        out_depth, out_t, counters);
    }
}

template <int kTW, bool kCount, int kStage>
void launch_blend_t(hipStream_t s, const float4 *records, int64_t n, int n_poses, const uint32_t *pairs,
                    const uint64_t *offsets, uint64_t capacity, const Camera &cam, const TileGrid &tg,
                    const BlendConsts &bc, float *rgb, float *depth, float *tfinal, unsigned long long *counters,
                    int persistent_blocks, unsigned int *queue) {
    if (persistent_blocks > 0) {
        const unsigned n_items = (unsigned)tg.n_tiles * (unsigned)n_poses;
        const unsigned blocks = std::min<unsigned>((unsigned)persistent_blocks, n_items);
        launch_fill_u32(s, queue, 1, 0u);
        hipLaunchKernelGGL((k_blend_queue<kTW, kCount, kStage>), dim3(blocks), dim3(kThreads), 0, s, records, n, pairs,
                           offsets, capacity, cam.width, cam.height, tg.tiles_x, tg.n_tiles, bc, rgb, depth, tfinal,
                           counters, n_items, queue);
        return;
    }
    hipLaunchKernelGGL((k_blend<kTW, kCount, kStage>), dim3((unsigned)tg.n_tiles, (unsigned)n_poses), dim3(kThreads),
                       0, s, records, n, pairs, offsets, capacity, cam.width, cam.height, tg.tiles_x, tg.n_tiles, bc,
                       rgb, depth, tfinal, counters);
}

// The forward that also keeps the compositing state of long lists (chunks of 252).
// Held to 64 registers like the plain forward (8 waves per SIMD; left to itself
// the compiler takes 73 and 6 waves).
template <int kTW>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8))) void k_blend_keep(
    const float4 *__restrict__ records, int64_t n, const uint32_t *__restrict__ pairs,
    const uint64_t *__restrict__ offsets, uint64_t capacity, int width, int height, int tiles_x, int n_tiles,
    BlendConsts k, float *__restrict__ out_rgb, float *__restrict__ out_depth, float *__restrict__ out_t,
    KeepIo keep) {
    blend_tile<kTW, false, 63, false, true>(blockIdx.x, blockIdx.y, records, n, pairs, offsets, capacity, width,
                                            height, tiles_x, n_tiles, k, out_rgb, out_depth, out_t, nullptr, GradIo{},
                                            keep);
}

// Backward of the compositing: one 256-thread block per (list, kept-state
// segment), the forward's walk (chunks of 252 records).
template <int kTW>
__global__ __launch_bounds__(kThreads) void k_blend_backward(
    const float4 *__restrict__ records, int64_t n, const uint32_t *__restrict__ pairs,
    const uint64_t *__restrict__ offsets, uint64_t capacity, int width, int height, int tiles_x, int n_tiles,
    BlendConsts k, GradIo gio) {
    const uint32_t b = blockIdx.x;
    if (b >= gio.n_lists + gio.cp_off[gio.n_lists]) return;  // the grid is an upper bound
    const uint32_t list = gio.items[b];
    const uint32_t seg = b - list - gio.cp_off[list];
    blend_tile<kTW, false, 63, true>((int)(list % (uint32_t)n_tiles), (int)(list / (uint32_t)n_tiles), records, n,
                                     pairs, offsets, capacity, width, height, tiles_x, n_tiles, k, nullptr, nullptr,
                                     nullptr, nullptr, gio, KeepIo{}, seg);
}

template <int kTW>
void launch_blend_w(hipStream_t s, const float4 *records, int64_t n, int n_poses, const uint32_t *pairs,
                    const uint64_t *offsets, uint64_t capacity, const Camera &cam, const BlendConsts &bc,
                    const TileGrid &tg, float *rgb, float *depth, float *tfinal, bool count_evals,
                    unsigned long long *counters, int persistent_blocks, unsigned int *queue, int chunk,
                    const uint32_t *keep_off, float *keep_state) {
    if (keep_off) {
        hipLaunchKernelGGL(k_blend_keep<kTW>, dim3((unsigned)tg.n_tiles, (unsigned)n_poses), dim3(kThreads), 0, s,
                           records, n, pairs, offsets, capacity, cam.width, cam.height, tg.tiles_x, tg.n_tiles, bc,
                           rgb, depth, tfinal, KeepIo{keep_off, keep_state});
        return;
    }
#define GSR_BLEND(C, S)                                                                                             \
    launch_blend_t<kTW, C, S>(s, records, n, n_poses, pairs, offsets, capacity, cam, tg, bc, rgb, depth, tfinal,    \
                              counters, persistent_blocks, queue)
    if (chunk == 124) {
        if (count_evals) GSR_BLEND(true, 31); else GSR_BLEND(false, 31);
    } else if (chunk == 60) {
        if (count_evals) GSR_BLEND(true, 15); else GSR_BLEND(false, 15);
    } else {
        if (count_evals) GSR_BLEND(true, 63); else GSR_BLEND(false, 63);
    }
#undef GSR_BLEND
}

}  // namespace

bool blend_tile_supported(int tile_w, int tile_h) {
    return (tile_w == 16 && tile_h == 16) || (tile_w == 32 && tile_h == 8) || (tile_w == 8 && tile_h == 32);
}

void launch_blend_backward(hipStream_t s, const float4 *records, int64_t n, int n_poses, const uint32_t *pairs,
                           const uint64_t *offsets, uint64_t capacity, const Camera &cam, const Consts &k,
                           const TileGrid &tg, const float *img_rgb, const float *img_depth, const float *g_rgb,
                           const float *g_depth, float *gscreen, const uint32_t *keep_off, const float *keep_state,
                           const uint32_t *items, uint64_t max_blocks) {
    const uint32_t n_lists = (uint32_t)tg.n_tiles * (uint32_t)n_poses;
    const GradIo gio{img_rgb, img_depth, g_rgb, g_depth, gscreen, keep_off, keep_state, items, n_lists};
    if (max_blocks == 0) return;
#define GSR_BWD(W)                                                                                                  \
    hipLaunchKernelGGL(k_blend_backward<W>, dim3((unsigned)max_blocks), dim3(kThreads), 0, s, records, n, pairs,     \
                       offsets, capacity, cam.width, cam.height, tg.tiles_x, tg.n_tiles, blend_consts(k), gio)
    if (tg.tile_w == 32)
        GSR_BWD(32);
    else if (tg.tile_w == 8)
        GSR_BWD(8);
    else
        GSR_BWD(16);
#undef GSR_BWD
}

bool blend_chunk_supported(int chunk) { return chunk == 0 || chunk == 252 || chunk == 124 || chunk == 60; }

void launch_blend(hipStream_t s, const float4 *records, int64_t n, int n_poses, const uint32_t *pairs,
                  const uint64_t *offsets, uint64_t capacity, const Camera &cam, const Consts &k,
                  const TileGrid &tg, float *rgb, float *depth, float *tfinal, bool count_evals,
                  unsigned long long *counters, int persistent_blocks, unsigned int *queue, int chunk,
                  const uint32_t *keep_off, float *keep_state) {
    const BlendConsts bc = blend_consts(k);
#define GSR_BLEND_W(W)                                                                                              \
    launch_blend_w<W>(s, records, n, n_poses, pairs, offsets, capacity, cam, bc, tg, rgb, depth, tfinal, count_evals, \
                      counters, persistent_blocks, queue, chunk, keep_off, keep_state)
    if (tg.tile_w == 32)
        GSR_BLEND_W(32);
    else if (tg.tile_w == 8)
        GSR_BLEND_W(8);
    else
        GSR_BLEND_W(16);
#undef GSR_BLEND_W
}

}  // namespace gsr
