"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.py.

This module only draws random numbers and builds camera poses. It holds none
of the rendering or scoring arithmetic (no quaternion normalisation, no
projection, no compositing, no correlation); both sides of every comparison
receive the identical float32 arrays produced here.

Distributions follow the relocalisation setting of the paper: a 3D Gaussian
map (Sec. III-A: mean, per-axis scale, rotation quaternion [w, x, y, z], RGB
colour, opacity; Sec. III-B2: RGB only, no spherical harmonics), a pinhole
camera with intrinsics K and world-to-camera poses W_t (Sec. III-A), and a
grid of candidate poses around a prior (Sec. III-C1, Sec. IV-A). KITTI-360 is
not available here; the street-corridor layout of ``config1`` stands in for
its LiDAR-initialised maps (Sec. III-B1).

Conventions: world z is up; camera axes are OpenCV (x right, y down, z
forward); a pose is the world-to-camera matrix [R | t] (3x4, row-major).
Scales are linear (exp of the drawn log-scale) and opacities are post-sigmoid,
computed once here in float64 and rounded to float32.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

__all__ = [
    "Camera", "Gaussians", "Scene", "config0", "config1", "tiny_scene",
    "random_images", "pose_from_center", "yaw_grid_poses", "digest",
]


@dataclasses.dataclass(frozen=True)
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float


@dataclasses.dataclass
class Gaussians:
    means: np.ndarray    # [N,3] f32, world metres
    scales: np.ndarray   # [N,3] f32, linear, > 0
    quats: np.ndarray    # [N,4] f32, (w, x, y, z), not necessarily unit length
    opacity: np.ndarray  # [N]   f32, in (0, 1)
    rgb: np.ndarray      # [N,3] f32

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    def take(self, idx: np.ndarray) -> "Gaussians":
        return Gaussians(self.means[idx], self.scales[idx], self.quats[idx],
                         self.opacity[idx], self.rgb[idx])

    def arrays(self):
        return (self.means, self.scales, self.quats, self.opacity, self.rgb)


@dataclasses.dataclass
class Scene:
    name: str
    gaussians: Gaussians
    camera: Camera
    tile: tuple            # (tile_w, tile_h)
    poses: np.ndarray      # [P,3,4] f32 candidate world-to-camera poses
    hidden_pose: np.ndarray  # [3,4] f32
    query_noise: np.ndarray  # [3,H,W] f32, added to the render at hidden_pose
    prior_center: np.ndarray  # [3] f64, camera centre of the prior pose
    crop_cell: float = 0.0    # 2D voxel cell edge (m); 0 = no crop
    crop_radius: float = 0.0  # crop radius around the prior (m)
    crop_voxel: float = 1.0   # fine voxel (m) whose Morton order orders the submap
    hidden_offset: tuple = (0.0, 0.0, 0.0)  # hidden pose - prior: (dx m, dy m, dyaw degrees)
    camera_axes: np.ndarray | None = None   # camera axes (rows) in world, before the yaw


def offset_poses(scene: "Scene", offsets) -> np.ndarray:
    """Poses of the scene's camera at (dx m, dy m, dyaw degrees) from its prior; float32 [P,3,4]."""
    out = [pose_from_center(np.asarray(scene.prior_center) + np.array([dx, dy, 0.0]), scene.camera_axes,
                            np.deg2rad(dyaw)) for dx, dy, dyaw in offsets]
    return _f32(np.stack(out))


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _sigmoid64(x: np.ndarray) -> np.ndarray:
    return 1.0 / (1.0 + np.exp(-x))


def _rot_z(yaw: float) -> np.ndarray:
    c, s = np.cos(yaw), np.sin(yaw)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def pose_from_center(center, cam_axes_world: np.ndarray, yaw: float = 0.0) -> np.ndarray:
    """World-to-camera [R|t] (float64) for a camera at ``center``.

    ``cam_axes_world`` holds the camera's x, y, z axes as rows, in world
    coordinates, before the extra rotation ``yaw`` about world z.
    """
    r_c2w = _rot_z(yaw) @ np.asarray(cam_axes_world, dtype=np.float64).T
    r_w2c = r_c2w.T
    t = -r_w2c @ np.asarray(center, dtype=np.float64)
    return np.concatenate([r_w2c, t[:, None]], axis=1)


def yaw_grid_poses(center, cam_axes_world, dxs, dys, dyaws_deg) -> np.ndarray:
    """Candidate grid, x-offset slowest then y then yaw; float32 [P,3,4]."""
    out = []
    for dx in dxs:
        for dy in dys:
            for dyaw in dyaws_deg:
                c = np.asarray(center, dtype=np.float64) + np.array([dx, dy, 0.0])
                out.append(pose_from_center(c, cam_axes_world, np.deg2rad(dyaw)))
    return _f32(np.stack(out))


# camera looking along world +y, level (x_c = +x, y_c = -z, z_c = +y)
AXES_ALONG_Y = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, -1.0], [0.0, 1.0, 0.0]])
# camera looking along world +x, level (x_c = -y, y_c = -z, z_c = +x)
AXES_ALONG_X = np.array([[0.0, -1.0, 0.0], [0.0, 0.0, -1.0], [1.0, 0.0, 0.0]])


def config0() -> Scene:
    """Tiny scene: 4,096 Gaussians in a 20x20x5 m box, 128x96 camera, 16 poses.

    Draw order (seed 0): means, log-scales, quaternion components, opacity
    logits, colours. Candidates: 4x4 grid over world-x offset in
    linspace(-1, 1, 4) m and yaw in linspace(-5, 5, 4) degrees around the
    reference camera at (0, -16, 2.5) looking along +y. Hidden pose offset
    from seed 100; query noise N(0, 0.02) per channel from seed 101.
    """
    rng = np.random.default_rng(0)
    n = 4096
    means = rng.uniform([-10.0, -10.0, 0.0], [10.0, 10.0, 5.0], size=(n, 3))
    log_s = rng.normal(-2.0, 0.5, size=(n, 3))
    quats = rng.normal(0.0, 1.0, size=(n, 4))
    logit = rng.normal(0.0, 1.0, size=n)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    g = Gaussians(_f32(means), _f32(np.exp(log_s)), _f32(quats),
                  _f32(_sigmoid64(logit)), _f32(rgb))
    cam = Camera(128, 96, 100.0, 100.0, 64.0, 48.0)
    center = np.array([0.0, -16.0, 2.5])
    poses = yaw_grid_poses(center, AXES_ALONG_Y, np.linspace(-1, 1, 4), [0.0],
                           np.linspace(-5, 5, 4))
    hr = np.random.default_rng(100)
    hdx = hr.uniform(-1.0, 1.0)
    hyaw = hr.uniform(-5.0, 5.0)
    hidden = _f32(pose_from_center(center + np.array([hdx, 0.0, 0.0]), AXES_ALONG_Y,
                                   np.deg2rad(hyaw)))
    noise = _f32(np.random.default_rng(101).normal(0.0, 0.02, size=(3, cam.height, cam.width)))
    return Scene("config0", g, cam, (16, 16), poses, hidden, noise, center,
                 hidden_offset=(hdx, 0.0, hyaw), camera_axes=AXES_ALONG_Y)


def _quat_mul(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ], axis=-1)


def corridor_map(n: int, seed: int, length: float = 200.0) -> Gaussians:
    """LiDAR-like street corridor: 60% ground, 2 x 20% facades at y = +-8 m.

    Flat disks: in-plane log-scales N(-2.5, 0.4), normal log-scale N(-4, 0.3);
    the disk normal is the plane normal with a uniform spin about it.
    Colours U[0,1]^3, opacity sigmoid(N(1, 1)).
    Draw order: ground xyz, facade+ xyz, facade- xyz, log-scales, spins,
    colours, opacity logits.
    """
    rng = np.random.default_rng(seed)
    n_g = (n * 6) // 10
    n_f = (n - n_g) // 2
    n_f2 = n - n_g - n_f
    gx = rng.uniform(0.0, length, n_g)
    gy = rng.uniform(-8.0, 8.0, n_g)
    gz = rng.normal(0.0, 0.05, n_g)
    f1x = rng.uniform(0.0, length, n_f)
    f1y = 8.0 + rng.normal(0.0, 0.05, n_f)
    f1z = rng.uniform(0.0, 12.0, n_f)
    f2x = rng.uniform(0.0, length, n_f2)
    f2y = -8.0 + rng.normal(0.0, 0.05, n_f2)
    f2z = rng.uniform(0.0, 12.0, n_f2)
    means = np.concatenate([np.stack([gx, gy, gz], 1), np.stack([f1x, f1y, f1z], 1),
                            np.stack([f2x, f2y, f2z], 1)])
    inplane = rng.normal(-2.5, 0.4, size=(n, 2))
    normal = rng.normal(-4.0, 0.3, size=(n, 1))
    log_s = np.concatenate([inplane, normal], axis=1)
    spin = rng.uniform(0.0, 2.0 * np.pi, n)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    logit = rng.normal(1.0, 1.0, n)
    # spin about the local normal (local z)
    q_spin = np.stack([np.cos(spin / 2), np.zeros(n), np.zeros(n), np.sin(spin / 2)], 1)
    # facades: local z (normal) -> world y, by a -90 degree turn about x
    h = np.deg2rad(-90.0) / 2
    q_fac = np.array([np.cos(h), np.sin(h), 0.0, 0.0])
    quats = q_spin.copy()
    quats[n_g:] = _quat_mul(np.broadcast_to(q_fac, (n - n_g, 4)), q_spin[n_g:])
    return Gaussians(_f32(means), _f32(np.exp(log_s)), _f32(quats),
                     _f32(_sigmoid64(logit)), _f32(rgb))


def config1_camera() -> Camera:
    """1408x376 pinhole, f = 552 px, principal point at the image centre."""
    return Camera(1408, 376, 552.0, 552.0, 704.0, 188.0)


def config1(n: int = 1_000_000) -> Scene:
    """Driving-scale scene: corridor map (seed 1), 1408x376 camera, 64 poses.

    Prior / reference camera at (100, 0, 1.5) looking along +x, level. The
    submap is the 2D-voxel (10 m cells) crop of 50 m radius around it.
    Candidates: 4x4x4 grid, dx, dy in {-1.5,-0.5,0.5,1.5} m and yaw in
    {-7.5,-2.5,2.5,7.5} degrees. Hidden pose uniform over the grid extent
    (seed 10); query noise N(0, 0.02) (seed 11), added to a render of the full
    map at the hidden pose.
    """
    g = corridor_map(n, seed=1)
    cam = config1_camera()
    center = np.array([100.0, 0.0, 1.5])
    steps = [-1.5, -0.5, 0.5, 1.5]
    poses = yaw_grid_poses(center, AXES_ALONG_X, steps, steps, [-7.5, -2.5, 2.5, 7.5])
    hr = np.random.default_rng(10)
    hdx, hdy = hr.uniform(-1.5, 1.5, 2)
    hyaw = hr.uniform(-7.5, 7.5)
    hidden = _f32(pose_from_center(center + np.array([hdx, hdy, 0.0]), AXES_ALONG_X,
                                   np.deg2rad(hyaw)))
    noise = _f32(np.random.default_rng(11).normal(0.0, 0.02, size=(3, cam.height, cam.width)))
    return Scene("config1", g, cam, (16, 16), poses, hidden, noise, center,
                 crop_cell=10.0, crop_radius=50.0, hidden_offset=(hdx, hdy, hyaw), camera_axes=AXES_ALONG_X)


def tiny_scene(seed: int, n: int = 64, width: int = 64, height: int = 48,
               n_poses: int = 2, log_scale_mean: float = -1.5,
               depth_range=(2.0, 8.0), opacity_logit_mean: float = 0.0) -> Scene:
    """Small random scene in front of a camera at the origin looking along +y.

    Used for brute-force comparisons and ragged-size edge cases.
    """
    rng = np.random.default_rng(seed)
    y = rng.uniform(depth_range[0], depth_range[1], n)
    x = rng.uniform(-0.6, 0.6, n) * y
    z = rng.uniform(-0.45, 0.45, n) * y
    means = np.stack([x, y, z], 1)
    log_s = rng.normal(log_scale_mean, 0.5, size=(n, 3))
    quats = rng.normal(0.0, 1.0, size=(n, 4))
    logit = rng.normal(opacity_logit_mean, 1.0, n)
    rgb = rng.uniform(0.0, 1.0, size=(n, 3))
    g = Gaussians(_f32(means), _f32(np.exp(log_s)), _f32(quats),
                  _f32(_sigmoid64(logit)), _f32(rgb))
    f = 0.8 * width
    cam = Camera(width, height, f, f, width / 2.0, height / 2.0)
    center = np.zeros(3)
    yaws = np.linspace(-3.0, 3.0, n_poses) if n_poses > 1 else [0.0]
    poses = yaw_grid_poses(center, AXES_ALONG_Y, [0.0], [0.0], yaws)
    noise = _f32(rng.normal(0.0, 0.02, size=(3, height, width)))
    return Scene(f"tiny{seed}", g, cam, (16, 16), poses, poses[0].copy(), noise, center)


def search_order(seed: int, n: int) -> np.ndarray:
    """A seeded random visiting order of n candidates (int32 permutation)."""
    return np.random.default_rng(seed).permutation(n).astype(np.int32)


def scorer_params(seed: int) -> np.ndarray:
    """Initial parameters of the learned scorer (flat float32, the layout of the
    scorer's parameter vector): He-normal weights, zero biases.
    Shapes: per conv layer (2->32->64->64->128->128) W[co][3][3][ci], b[co];
    then fc1 W[128][128], b[128]; fc2 W[128], b[1]."""
    rng = np.random.default_rng(seed)
    chans = [2, 32, 64, 64, 128, 128]
    parts = []
    for ci, co in zip(chans[:-1], chans[1:]):
        parts += [rng.normal(0.0, np.sqrt(2.0 / (9 * ci)), (co, 3, 3, ci)), np.zeros(co)]
    parts += [rng.normal(0.0, np.sqrt(2.0 / 128), (128, 128)), np.zeros(128),
              rng.normal(0.0, np.sqrt(2.0 / 128), 128), np.zeros(1)]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


def random_images(seed: int, n: int, height: int, width: int, channels: int = 3) -> np.ndarray:
    """Smooth-plus-noise float32 images [n, channels, H, W] for NCC checks."""
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.linspace(0, 1, height), np.linspace(0, 1, width), indexing="ij")
    out = np.empty((n, channels, height, width), dtype=np.float32)
    for i in range(n):
        fx, fy, ph = rng.uniform(1, 6), rng.uniform(1, 6), rng.uniform(0, 2 * np.pi)
        base = 0.5 + 0.3 * np.sin(2 * np.pi * (fx * xx + fy * yy) + ph)
        for c in range(channels):
            out[i, c] = (base * rng.uniform(0.5, 1.5) + rng.normal(0, 0.1, base.shape)).astype(np.float32)
    return out


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


# ---- learned-scorer workload: 1024 candidates per query ----
SCORER_DX = [-3.5, -2.5, -1.5, -0.5, 0.5, 1.5, 2.5, 3.5]          # metres (world x)
SCORER_DY = SCORER_DX                                              # metres (world y)
SCORER_DYAW = [-37.5 + 5.0 * i for i in range(16)]                 # degrees
SCORER_TRAIN_MAPS = (401, 402, 403, 404)                           # 4 maps x 49 queries = 196
SCORER_EVAL_MAPS = (501, 502)                                      # 2 maps x 50 queries = 100
SCORER_QUERIES_PER_TRAIN_MAP = 49
SCORER_QUERIES_PER_EVAL_MAP = 50
SCORER_FACTOR = 4                                                  # low resolution = 1/4 in each direction


@dataclasses.dataclass
class ScorerQuery:
    prior: np.ndarray     # camera centre of the prior (x, y, z), float64
    poses: np.ndarray     # [1024, 3, 4] float32 candidate grid around the prior
    hidden: np.ndarray    # [3, 4] float32 true pose
    noise: np.ndarray     # [3, H, W] float32 query noise


def scorer_query(seed: int, cam: Camera) -> ScorerQuery:
    """One query of the learned-scorer workload on a corridor map: prior camera at
    x ~ U(60, 140), y ~ U(-1.5, 1.5), height 1.5 m, looking along +x; candidates
    8 dx x 8 dy x 16 dyaw (SCORER_* steps; x slowest, then y, then yaw); hidden
    pose uniform over the grid's extent; query noise N(0, 0.02) per channel.
    Draw order: prior x, prior y, hidden dx, dy, dyaw, noise."""
    rng = np.random.default_rng(seed)
    prior = np.array([rng.uniform(60.0, 140.0), rng.uniform(-1.5, 1.5), 1.5])
    poses = yaw_grid_poses(prior, AXES_ALONG_X, SCORER_DX, SCORER_DY, SCORER_DYAW)
    hdx, hdy = rng.uniform(SCORER_DX[0], SCORER_DX[-1], 2)
    hyaw = rng.uniform(SCORER_DYAW[0], SCORER_DYAW[-1])
    hidden = _f32(pose_from_center(prior + np.array([hdx, hdy, 0.0]), AXES_ALONG_X, np.deg2rad(hyaw)))
    noise = _f32(rng.normal(0.0, 0.02, size=(3, cam.height, cam.width)))
    return ScorerQuery(prior, poses, hidden, noise)


def scorer_query_seed(map_seed: int, i: int) -> int:
    return map_seed * 1000 + i


def low_res_camera(cam: Camera, f: int) -> Camera:
    """The camera with its image reduced f times (focal lengths and principal point / f)."""
    return Camera(cam.width // f, cam.height // f, cam.fx / f, cam.fy / f, cam.cx / f, cam.cy / f)


# ---- batched queries: 8 corridor maps of uneven size, 32 candidates each ----
BATCH_MAP_SEEDS = tuple(range(200, 208))
BATCH_DX = [-1.5, -0.5, 0.5, 1.5]
BATCH_DYAW = [-2.5, 2.5]


@dataclasses.dataclass
class BatchQuery:
    seed: int
    n: int                # Gaussians of the map
    gaussians: Gaussians
    poses: np.ndarray     # [32, 3, 4] float32
    hidden: np.ndarray    # [3, 4] float32
    noise: np.ndarray     # [3, H, W] float32


def batch_query(seed: int, cam: Camera) -> BatchQuery:
    """One query of the batched workload: a corridor map (config-1 layout) of
    N = round(exp(U(ln 2e5, ln 2e6))) Gaussians (drawn from seed * 10), its own
    map seed, the prior of config 1 at (100, 0, 1.5) looking along +x, candidates
    4 dx x 4 dy x 2 dyaw (BATCH_* steps), hidden pose uniform over the grid's
    extent (seed * 10 + 1), query noise N(0, 0.02) (seed * 10 + 2)."""
    n = int(round(np.exp(np.random.default_rng(seed * 10).uniform(np.log(2e5), np.log(2e6)))))
    g = corridor_map(n, seed=seed)
    center = np.array([100.0, 0.0, 1.5])
    poses = yaw_grid_poses(center, AXES_ALONG_X, BATCH_DX, BATCH_DX, BATCH_DYAW)
    hr = np.random.default_rng(seed * 10 + 1)
    hdx, hdy = hr.uniform(BATCH_DX[0], BATCH_DX[-1], 2)
    hyaw = hr.uniform(BATCH_DYAW[0], BATCH_DYAW[-1])
    hidden = _f32(pose_from_center(center + np.array([hdx, hdy, 0.0]), AXES_ALONG_X, np.deg2rad(hyaw)))
    noise = _f32(np.random.default_rng(seed * 10 + 2).normal(0.0, 0.02, size=(3, cam.height, cam.width)))
    return BatchQuery(seed, n, g, poses, hidden, noise)


# ---- map training: perturbed corridor map, views along the corridor ----
def training_views(seed: int, n: int, length: float = 200.0) -> np.ndarray:
    """n camera poses along a corridor of the given length: centre x ~ U(0.2 L,
    0.8 L), y ~ U(-3, 3), height 1.5 m, looking along +x with yaw U(-15, 15)
    degrees; float32 [n, 3, 4]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        c = np.array([rng.uniform(0.2 * length, 0.8 * length), rng.uniform(-3.0, 3.0), 1.5])
        out.append(pose_from_center(c, AXES_ALONG_X, np.deg2rad(rng.uniform(-15.0, 15.0))))
    return _f32(np.stack(out))


@dataclasses.dataclass
class TrainingMap:
    gt: Gaussians          # ground truth (renders it are the targets)
    means: np.ndarray      # initial parameters, float32
    log_scales: np.ndarray
    quats: np.ndarray
    logits: np.ndarray
    rgb: np.ndarray


def training_map(n: int = 500_000, seed: int = 3, perturb_seed: int = 32, length: float = 200.0) -> TrainingMap:
    """Ground-truth corridor map (seed 3) and the initial map of a training run: the
    ground truth perturbed (perturb_seed) by N(0, 0.05) m on the means, N(0, 0.2) on
    the log-scales, N(0, 0.05) on the quaternion components, N(0, 0.5) on the
    opacity logits and N(0, 0.1) on the colours (clipped to [0, 1]). Draw order:
    means, log-scales, quaternions, logits, colours."""
    gt = corridor_map(n, seed=seed, length=length)
    rng = np.random.default_rng(perturb_seed)
    f = lambda a: np.asarray(a, np.float64)  # noqa: E731
    op = f(gt.opacity)
    means = f(gt.means) + rng.normal(0.0, 0.05, (n, 3))
    log_s = np.log(f(gt.scales)) + rng.normal(0.0, 0.2, (n, 3))
    quats = f(gt.quats) + rng.normal(0.0, 0.05, (n, 4))
    logits = np.log(op / (1.0 - op)) + rng.normal(0.0, 0.5, n)
    rgb = np.clip(f(gt.rgb) + rng.normal(0.0, 0.1, (n, 3)), 0.0, 1.0)
    return TrainingMap(gt, _f32(means), _f32(log_s), _f32(quats), _f32(logits), _f32(rgb))
