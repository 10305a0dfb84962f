// Submap retrieval on the host (gsr_crop).
//
// Paper: Sec. III-B2 stores the map in a 2D voxel grid, each voxel keyed by a
// unique hash ID, and builds a KD-tree over the voxel centres to find the voxels
// within a range of a camera; Sec. III-C1 retrieves the submap around the raw
// (e.g. GPS) prior pose this way. Cells here are `cell` metres wide, keyed by
// (floor(x / cell), floor(y / cell)); a cell is kept when its centre lies
// within `radius` of the prior (px, py); all its Gaussians come with it. The
// kept Gaussians are listed in Morton order of their `voxel`-metre 3D voxels
// (the paper stores the map in 1 m voxels), ties by ascending index, so that
// Gaussians close in the submap order are close in space; voxel <= 0 keeps
// ascending index order. This runs once per query, off the timed GPU path.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <unordered_map>
#include <vector>

#include "gsr.h"

namespace {

struct Cell {
    double cx, cy;
    std::vector<int64_t> members;
};

// 2D KD-tree over cell centres, stored implicitly: node i of a subarray is its
// median on the split axis.
struct KdTree {
    std::vector<int> order;  // cell ids in tree layout
    const std::vector<Cell> *cells = nullptr;

    void build(int lo, int hi, int axis) {
        if (hi - lo <= 1) return;
        const int mid = (lo + hi) / 2;
        std::nth_element(order.begin() + lo, order.begin() + mid, order.begin() + hi, [&](int a, int b) {
            const Cell &ca = (*cells)[a], &cb = (*cells)[b];
            return axis == 0 ? ca.cx < cb.cx : ca.cy < cb.cy;
        });
        build(lo, mid, axis ^ 1);
        build(mid + 1, hi, axis ^ 1);
    }

    void query(int lo, int hi, int axis, double px, double py, double r2, std::vector<int> &out) const {
        if (hi <= lo) return;
        const int mid = (lo + hi) / 2;
        const Cell &c = (*cells)[order[mid]];
        const double dx = c.cx - px, dy = c.cy - py;
        if (dx * dx + dy * dy <= r2) out.push_back(order[mid]);
        const double split = axis == 0 ? dx : dy;  // signed distance to the split line
        // left half holds coordinates <= the median, right half >= the median
        if (split >= 0.0 || split * split <= r2) query(lo, mid, axis ^ 1, px, py, r2, out);
        if (split <= 0.0 || split * split <= r2) query(mid + 1, hi, axis ^ 1, px, py, r2, out);
    }
};

}  // namespace

// Morton code of a 3D voxel: v = floor(coord / voxel) + 2^20 clamped to
// [0, 2^21 - 1] (0 if not finite); bit b of x, y, z goes to code bit 3b, 3b + 1, 3b + 2.
static uint64_t voxel_code(const float *m, double voxel) {
    uint64_t code = 0;
    for (int a = 0; a < 3; ++a) {
        double v = std::floor((double)m[a] / voxel) + (double)(1 << 20);
        v = std::isfinite(v) ? std::min(std::max(v, 0.0), (double)((1 << 21) - 1)) : 0.0;
        const uint64_t q = (uint64_t)v;
        for (int b = 0; b < 21; ++b) code |= ((q >> b) & 1ull) << (3 * b + a);
    }
    return code;
}

extern "C" int gsr_crop(const float *means, int64_t n, double cell, double px, double py, double radius,
                        double voxel, int64_t *idx, int64_t cap, int64_t *n_out) {
    if (!n_out) return GSR_EINVAL;
    *n_out = 0;
    if (n < 0 || (n > 0 && !means) || !(cell > 0.0) || !(radius >= 0.0) || !std::isfinite(px) ||
        !std::isfinite(py) || cap < 0 || (cap > 0 && !idx))
        return GSR_EINVAL;
    // voxel hash: cell id (ix, iy) -> dense cell number
    std::unordered_map<uint64_t, int> hash;
    std::vector<Cell> cells;
    hash.reserve(1024);
    for (int64_t i = 0; i < n; ++i) {
        const double x = means[i * 3 + 0], y = means[i * 3 + 1];
        if (!std::isfinite(x) || !std::isfinite(y)) continue;
        const double fx = std::floor(x / cell), fy = std::floor(y / cell);
        if (std::fabs(fx) > 2e9 || std::fabs(fy) > 2e9) continue;
        const int64_t ix = (int64_t)fx, iy = (int64_t)fy;
        const uint64_t key = ((uint64_t)(uint32_t)(int32_t)ix << 32) | (uint32_t)(int32_t)iy;
        auto it = hash.find(key);
        int id;
        if (it == hash.end()) {
            id = (int)cells.size();
            hash.emplace(key, id);
            cells.push_back(Cell{((double)ix + 0.5) * cell, ((double)iy + 0.5) * cell, {}});
        } else {
            id = it->second;
        }
        cells[id].members.push_back(i);
    }
    KdTree tree;
    tree.cells = &cells;
    tree.order.resize(cells.size());
    for (size_t i = 0; i < cells.size(); ++i) tree.order[i] = (int)i;
    tree.build(0, (int)cells.size(), 0);
    std::vector<int> hit;
    tree.query(0, (int)cells.size(), 0, px, py, radius * radius, hit);
    std::vector<int64_t> sel;
    for (int c : hit) sel.insert(sel.end(), cells[c].members.begin(), cells[c].members.end());
    std::sort(sel.begin(), sel.end());
    if (voxel > 0.0) {
        std::vector<std::pair<uint64_t, int64_t>> keyed(sel.size());
        for (size_t i = 0; i < sel.size(); ++i) keyed[i] = {voxel_code(means + sel[i] * 3, voxel), sel[i]};
        std::sort(keyed.begin(), keyed.end());
        for (size_t i = 0; i < sel.size(); ++i) sel[i] = keyed[i].second;
    }
    *n_out = (int64_t)sel.size();
    if ((int64_t)sel.size() > cap) return GSR_EINVAL;
    std::copy(sel.begin(), sel.end(), idx);
    return GSR_OK;
}
