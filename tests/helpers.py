"""Shared helpers for the GPU parity tests: upload seeded scenes, run the HIP
path through the C ABI, run the oracle on the same inputs, compare."""
from __future__ import annotations

import sys

import numpy as np

from oracle import blend, gaussians, keys, project, search

# parity bar (float32 render vs float64 oracle on identical float32 records),
# on every pixel: against the oracle's result, or where the oracle flags a
# decision within float32 error of its threshold, against one of the pixel's
# outcomes with those decisions taken either way
TOL_RGB = 1e-4       # abs
TOL_DEPTH = 1e-4     # abs (or relative to max(1, depth) where a test says so)
TOL_T = 1e-4         # abs, final transmittance
TOL_NCC = 1e-4       # abs


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, dev="cuda"):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), device=dev)


def camera(cam):
    from paper_2403_11367_amd import Camera
    return Camera(cam.width, cam.height, cam.fx, cam.fy, cam.cx, cam.cy)


def load(ctx, g, index=None):
    arrs = [to_dev(a.astype(np.float32)) for a in g.arrays()]
    idx = None if index is None else to_dev(np.asarray(index, np.int64))
    return ctx.load_submap(*arrs, index=idx)


def gpu_render(ctx, sm, cam, poses, cfg=None):
    import torch
    rgb, dep, tf = ctx.render(sm, camera(cam), to_dev(poses.astype(np.float32)), cfg, with_tfinal=True)
    torch.cuda.synchronize()
    return rgb.cpu().numpy(), dep.cpu().numpy(), tf.cpu().numpy()


def gpu_buffers(ctx):
    """Records, tile counts, list offsets and the sorted pair list (submap indices);
    check_pairs rebuilds the keys from the offsets and the records' depth bits."""
    from paper_2403_11367_amd import BUF_NTILES, BUF_OFFSETS, BUF_PAIRS, BUF_RECORDS
    recs = ctx.debug_buffer(BUF_RECORDS)
    return recs, ctx.debug_buffer(BUF_NTILES), ctx.debug_buffer(BUF_OFFSETS), (recs, ctx.debug_buffer(BUF_PAIRS))


def oracle_pose(prep, pose, cam, tile=(16, 16)):
    """(Render, ScreenRecords, sorted keys, sorted values, ranges) for one pose."""
    return search.render_pose(prep, pose, cam, tile, with_pairs=True)


def check_records(rec_gpu, nt_gpu, rec, n, p):
    """Bit-exact screen records and tile counts of pose p against the oracle."""
    r = rec_gpu.reshape(-1, n, 12)[p]
    nt = nt_gpu.reshape(-1, n)[p]
    vis = nt > 0
    assert np.array_equal(vis, rec.visible), f"visibility differs at {np.nonzero(vis != rec.visible)[0][:10]}"
    v = rec.visible
    for col, ref in ((0, rec.u), (1, rec.v), (2, rec.conic[:, 0]), (3, rec.conic[:, 1]), (4, rec.conic[:, 2]),
                     (9, rec.z), (5, rec.opacity), (6, rec.rgb[:, 0]), (7, rec.rgb[:, 1]), (8, rec.rgb[:, 2])):
        a = r[v, col].view(np.uint32)
        b = ref[v].astype(np.float32).view(np.uint32)
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, f"record column {col} differs for {bad.size} Gaussians, first {np.nonzero(v)[0][bad[:5]]}"
    rx = r[v, 10].view(np.uint32)
    ry = r[v, 11].view(np.uint32)
    got = np.stack([rx & 0xFFFF, rx >> 16, ry & 0xFFFF, ry >> 16], 1).astype(np.int64)
    assert np.array_equal(got, rec.rect[v])
    assert np.array_equal(nt[v].astype(np.int64), rec.n_tiles[v])


def check_pairs(off_gpu, pairs_gpu, ks, vs, rng, p, n_tiles):
    """Bit-exact keys and sorted order of pose p against the oracle's lexsort.
    The GPU key of a pair is rebuilt as (tile << 32) | depth bits of its record."""
    recs, vals = pairs_gpu
    lo, hi = int(off_gpu[p * n_tiles]), int(off_gpu[(p + 1) * n_tiles])
    seg = vals[lo:hi].astype(np.int64)
    starts = off_gpu[p * n_tiles:(p + 1) * n_tiles].astype(np.int64) - lo
    ends = off_gpu[p * n_tiles + 1:(p + 1) * n_tiles + 1].astype(np.int64) - lo
    assert np.array_equal(starts, rng[:, 0]) and np.array_equal(ends, rng[:, 1]), "tile ranges differ"
    assert seg.size == vs.size
    assert np.array_equal(seg.astype(np.uint32), vs), "sort order differs"
    tile_of = np.repeat(np.arange(n_tiles, dtype=np.uint64), (ends - starts))
    n_total = recs.size // 12
    n_g = n_total // ((off_gpu.size - 1) // n_tiles)
    z = recs.reshape(-1, n_g, 12)[p][seg, 9].view(np.uint32).astype(np.uint64)
    gkeys = (tile_of << np.uint64(32)) | z
    assert np.array_equal(gkeys, ks), "keys differ"


def compare_render(rgb, dep, tf, ref, label="", tol_depth=TOL_DEPTH, depth_rel=False):
    """GPU image vs oracle Render, every pixel held to the bars: unflagged pixels
    against the oracle's result, flagged ones against the nearest of their
    outcomes (``oracle.blend.outcomes``). depth_rel: the depth bar is
    tol_depth x max(1, depth) per pixel."""
    def depth_bar(d):
        return tol_depth * (np.maximum(1.0, np.abs(d)) if depth_rel else 1.0)

    e_rgb = np.abs(rgb - ref.rgb).max(axis=0)
    e_dep = np.abs(dep - ref.depth)
    e_t = np.abs(tf - ref.t_final)
    match = (e_rgb <= TOL_RGB) & (e_dep <= depth_bar(ref.depth)) & (e_t <= TOL_T)
    flag = ref.flag
    bad = ~match & ~flag
    if bad.any():
        j, i = np.argwhere(bad)[0]
        raise AssertionError(f"{label}: {int(bad.sum())} unflagged pixels off the bars, first ({i}, {j}): "
                             f"gpu rgb {rgb[:, j, i]} depth {dep[j, i]} T {tf[j, i]}, oracle rgb "
                             f"{ref.rgb[:, j, i]} depth {ref.depth[j, i]} T {ref.t_final[j, i]}")
    n_alt = 0
    for j, i in np.argwhere(~match & flag):
        outs = blend.outcomes(ref, int(i), int(j))
        got = np.array([rgb[0, j, i], rgb[1, j, i], rgb[2, j, i], dep[j, i], tf[j, i]])
        ok = ((np.abs(outs[:, :3] - got[:3]).max(axis=1) <= TOL_RGB)
              & (np.abs(outs[:, 3] - got[3]) <= depth_bar(outs[:, 3]))
              & (np.abs(outs[:, 4] - got[4]) <= TOL_T))
        assert ok.any(), (f"{label}: flagged pixel ({i}, {j}) matches none of its {outs.shape[0]} outcomes: "
                          f"gpu {got}, outcomes {outs}")
        n_alt += 1
    m = match & ~flag
    say(f"  {label}: max|drgb| {e_rgb[m].max() if m.any() else 0.0:.2e} "
        f"max|ddepth| {e_dep[m].max() if m.any() else 0.0:.2e} max|dT| {e_t[m].max() if m.any() else 0.0:.2e} "
        f"flagged {int(flag.sum())}/{flag.size}, matched through another outcome {n_alt}")


def prep(g):
    return search.prepare(g)


__all__ = ["blend", "gaussians", "keys", "project"]
