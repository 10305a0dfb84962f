"""ctypes binding of libgsr (include/gsr.h, include/gsr_scorer.h): argument marshalling only.

Every computation runs in the HIP library; this module checks tensor
devices, dtypes and shapes, passes ``data_ptr()`` and the current torch
stream, and turns status codes into exceptions. PyTorch is used for device
memory and streams only. If ``libgsr.so`` has not been built, importing this
module raises ``ImportError``: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import weakref
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GSR_LIB selects another build of the library (the host-sanitised one in the CPU tests)
LIB_PATH = os.environ.get("GSR_LIB") or os.path.join(_HERE, "libgsr.so")

GSR_OK = 0
STATUS = {0: "GSR_OK", -1: "GSR_EINVAL", -2: "GSR_ENOMEM", -3: "GSR_EHIP", -4: "GSR_ENODEV",
          -5: "GSR_EOVERFLOW", -6: "GSR_EUNSUPPORTED", -7: "GSR_EDEVICE"}
BUF_RECORDS, BUF_NTILES, BUF_OFFSETS, BUF_PAIRS = 0, 1, 2, 3
RENDER_COUNT_EVALS = 1
RENDER_KEEP_STATE = 2  # keep long lists' compositing states for gsr_render_backward
RENDER_RETRY_OVERFLOW = 4  # with a fixed capacity: re-render exactly after an overflow

# every symbol declared in include/gsr.h and include/gsr_scorer.h
EXPORTS = [
    "gsr_create", "gsr_destroy", "gsr_set_stream", "gsr_set_profiling", "gsr_default_cfg",
    "gsr_submap_load", "gsr_submap_load_host", "gsr_submap_free", "gsr_submap_size", "gsr_set_workspace_limit", "gsr_render", "gsr_render_multi",
    "gsr_render_backward", "gsr_ncc", "gsr_ncc_noalloc",
    "gsr_topk", "gsr_search", "gsr_capture_begin", "gsr_capture_end", "gsr_graph_launch", "gsr_graph_destroy",
    "gsr_sync", "gsr_get_stats", "gsr_debug_size", "gsr_debug_copy", "gsr_crop",
    "gsr_status_string", "gsr_last_error",
    "gsr_scorer_param_count", "gsr_scorer_create", "gsr_scorer_destroy", "gsr_scorer_set_params",
    "gsr_scorer_get_params", "gsr_pool_grey", "gsr_scorer_inputs", "gsr_scorer_forward", "gsr_scorer_backward",
    "gsr_scorer_adamw", "gsr_scorer_train_step", "gsr_search_pruned",
]


class GsrError(RuntimeError):
    def __init__(self, status: int, message: str = ""):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {message}")


class CameraC(C.Structure):
    _fields_ = [("width", C.c_int32), ("height", C.c_int32), ("fx", C.c_float), ("fy", C.c_float),
                ("cx", C.c_float), ("cy", C.c_float)]


class RenderCfg(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("eps_dilate", C.c_float),
                ("z_near", C.c_float), ("jac_clamp", C.c_float), ("cutoff_d2", C.c_float),
                ("alpha_min", C.c_float), ("alpha_max", C.c_float), ("t_min", C.c_float),
                ("flags", C.c_int32), ("pair_capacity", C.c_int64), ("pose_groups", C.c_int32),
                ("blend_blocks_per_cu", C.c_int32), ("blend_chunk", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_submap", C.c_int64), ("n_poses", C.c_int64), ("n_visible", C.c_int64),
                ("n_pairs", C.c_int64), ("pair_capacity", C.c_int64),
                ("evals_contrib", C.c_int64), ("evals_lanes", C.c_int64),
                ("overflow", C.c_int32), ("bad_index", C.c_int32),
                ("n_profiled_renders", C.c_int32), ("n_profiled_ncc", C.c_int32),
                ("ms_preprocess", C.c_float), ("ms_sort", C.c_float), ("ms_blend", C.c_float),
                ("ms_ncc", C.c_float), ("ms_render", C.c_float), ("n_groups", C.c_int32),
                ("render_serial", C.c_int64), ("n_culled_nonfinite", C.c_int64), ("workspace_bytes", C.c_int64),
                ("overflow_retried", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class AdamW(C.Structure):
    _fields_ = [("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("weight_decay", C.c_float)]


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2403_11367_amd.build`")
    # torch first: its HIP runtime has the soname libgsr links against, so the
    # library then binds to that same runtime (one runtime per process, sharing
    # torch's streams and allocations); loaded the other way round, the process
    # would hold two HIP runtimes
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P, I, I32, I64, F, D = C.c_void_p, C.c_int, C.c_int32, C.c_int64, C.c_float, C.c_double
    sig = {
        "gsr_create": (I, [C.POINTER(P), I, P]),
        "gsr_destroy": (I, [P]),
        "gsr_set_stream": (I, [P, P]),
        "gsr_set_profiling": (I, [P, I]),
        "gsr_default_cfg": (I, [C.POINTER(RenderCfg)]),
        "gsr_submap_load": (I, [P, I64, P, P, P, P, P, P, I64, C.POINTER(P)]),
        "gsr_submap_load_host": (I, [P, I64, P, P, P, P, P, P, I64, C.POINTER(P)]),
        "gsr_set_workspace_limit": (I, [P, I64]),
        "gsr_submap_free": (I, [P]),
        "gsr_submap_size": (I64, [P]),
        "gsr_render": (I, [P, P, C.POINTER(CameraC), P, I32, C.POINTER(RenderCfg), P, P, P]),
        "gsr_render_multi": (I, [P, P, P, I32, C.POINTER(CameraC), P, C.POINTER(RenderCfg), P, P, P]),
        "gsr_render_backward": (I, [P, P, P, P, P, I32, P, P, P, P, P, P, P, P, P]),
        "gsr_capture_begin": (I, [P]),
        "gsr_capture_end": (I, [P, C.POINTER(P)]),
        "gsr_graph_launch": (I, [P]),
        "gsr_graph_destroy": (I, [P]),
        "gsr_ncc": (I, [P, P, P, I32, I32, I32, P]),
        "gsr_ncc_noalloc": (I, [P, P, P, I32, I32, I32, P]),
        "gsr_topk": (I, [P, P, I32, I32, P]),
        "gsr_search": (I, [P, P, C.POINTER(CameraC), P, I32, P, I32, I32, F, P, C.POINTER(RenderCfg), P,
                           C.POINTER(I32), C.POINTER(F), C.POINTER(I32)]),
        "gsr_sync": (I, [P]),
        "gsr_get_stats": (I, [P, C.POINTER(Stats)]),
        "gsr_debug_size": (I, [P, I, C.POINTER(I64)]),
        "gsr_debug_copy": (I, [P, I, P, I64]),
        "gsr_crop": (I, [P, I64, D, D, D, D, D, P, I64, C.POINTER(I64)]),
        "gsr_status_string": (C.c_char_p, [I]),
        "gsr_last_error": (C.c_char_p, [P]),
        "gsr_scorer_param_count": (I64, []),
        "gsr_scorer_create": (I, [P, I32, I32, I32, C.POINTER(P)]),
        "gsr_scorer_destroy": (I, [P]),
        "gsr_scorer_set_params": (I, [P, P]),
        "gsr_scorer_get_params": (I, [P, P]),
        "gsr_pool_grey": (I, [P, P, I32, I32, I32, I32, P]),
        "gsr_scorer_inputs": (I, [P, P, I32, P, P]),
        "gsr_scorer_forward": (I, [P, P, I32, P]),
        "gsr_scorer_backward": (I, [P, P, P, I32, P, P]),
        "gsr_scorer_adamw": (I, [P, P, C.POINTER(AdamW)]),
        "gsr_scorer_train_step": (I, [P, P, P, I32, C.POINTER(AdamW), P]),
        "gsr_search_pruned": (I, [P, P, P, C.POINTER(CameraC), C.POINTER(CameraC), P, I32, I32, P, I32,
                                  C.POINTER(RenderCfg), P, P, P, C.POINTER(I32), C.POINTER(F)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()


def default_cfg(**overrides) -> RenderCfg:
    cfg = RenderCfg()
    LIB.gsr_default_cfg(C.byref(cfg))
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


def crop(means: np.ndarray, cell: float, center_xy: Sequence[float], radius: float,
         voxel: float = 1.0) -> np.ndarray:
    """Indices (int64) of the Gaussians in cells within `radius` of the prior, in Morton
    order of their `voxel`-metre voxels (ascending index if voxel <= 0)."""
    m = np.ascontiguousarray(means, dtype=np.float32)
    n = m.shape[0]
    out = np.empty(max(n, 1), dtype=np.int64)
    cnt = C.c_int64(0)
    rc = LIB.gsr_crop(m.ctypes.data, n, float(cell), float(center_xy[0]), float(center_xy[1]),
                      float(radius), float(voxel), out.ctypes.data, out.size, C.byref(cnt))
    if rc != GSR_OK:
        raise GsrError(rc, "gsr_crop")
    return out[: cnt.value].copy()


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float

    def c(self) -> CameraC:
        return CameraC(self.width, self.height, self.fx, self.fy, self.cx, self.cy)


def _torch():
    import torch
    return torch


def _dev_f32(t, name, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


class Submap:
    def __init__(self, ctx: "Context", handle: C.c_void_p):
        self.ctx = ctx
        self.handle = handle

    @property
    def n(self) -> int:
        return int(LIB.gsr_submap_size(self.handle))

    def free(self):
        if self.handle:
            LIB.gsr_submap_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Graph:
    """A captured sequence of library calls (gsr_graph); launch() replays it on the
    context's current torch stream."""

    def __init__(self, ctx: "Context", handle: C.c_void_p):
        self.ctx = ctx
        self.handle = handle

    def launch(self):
        self.ctx._bind_stream()
        self.ctx._check(LIB.gsr_graph_launch(self.handle), "gsr_graph_launch")

    def close(self):
        if self.handle:
            LIB.gsr_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """One GPU context; every call enqueues on the current torch stream of its device."""

    def __init__(self, device: int = 0):
        torch = _torch()
        self.device = int(device)
        self.handle = C.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        rc = LIB.gsr_create(C.byref(self.handle), self.device, C.c_void_p(stream))
        if rc != GSR_OK:
            raise GsrError(rc, "gsr_create")
        self._children = weakref.WeakSet()  # scorers and graphs: destroyed before the context

    def _check(self, rc: int, what: str):
        if rc != GSR_OK:
            msg = LIB.gsr_last_error(self.handle)
            raise GsrError(rc, f"{what}: {msg.decode() if msg else ''}")

    def _bind_stream(self):
        s = _torch().cuda.current_stream(self.device).cuda_stream
        self._check(LIB.gsr_set_stream(self.handle, C.c_void_p(s)), "gsr_set_stream")

    def close(self):
        if self.handle:
            for child in list(getattr(self, "_children", ())):
                child.close()
            LIB.gsr_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_profiling(self, on: bool):
        self._check(LIB.gsr_set_profiling(self.handle, int(bool(on))), "gsr_set_profiling")

    def load_submap(self, means, scales, quats, opacity, rgb, index=None,
                    into: Optional[Submap] = None) -> Submap:
        torch = _torch()
        n = means.shape[0]
        _dev_f32(means, "means", (n, 3))
        _dev_f32(scales, "scales", (n, 3))
        _dev_f32(quats, "quats", (n, 4))
        _dev_f32(opacity, "opacity", (n,))
        _dev_f32(rgb, "rgb", (n, 3))
        if index is not None:
            if index.dtype != torch.int64 or index.device.type != "cuda" or index.dim() != 1 \
                    or not index.is_contiguous():
                raise TypeError("index must be a contiguous 1-D int64 CUDA tensor")
            n_sel, iptr = index.shape[0], index.data_ptr()
        else:
            n_sel, iptr = n, None
        self._bind_stream()
        reuse = into is not None and bool(into.handle)
        h = C.c_void_p(into.handle.value) if reuse else C.c_void_p()
        rc = LIB.gsr_submap_load(self.handle, n, means.data_ptr(), scales.data_ptr(), quats.data_ptr(),
                                 opacity.data_ptr(), rgb.data_ptr(), iptr, n_sel, C.byref(h))
        self._check(rc, "gsr_submap_load")
        if reuse and h.value == into.handle.value:
            return into  # refilled in place
        if reuse:
            into.handle = None  # the library freed it when it allocated a larger one
        return Submap(self, h)

    def load_submap_host(self, means, scales, quats, opacity, rgb, index=None,
                         into: Optional[Submap] = None) -> Submap:
        """gsr_submap_load_host: the same from host (numpy) arrays; returns once packed."""
        arrs = [np.ascontiguousarray(a, dtype=np.float32) for a in (means, scales, quats, opacity, rgb)]
        n = arrs[0].shape[0]
        for a, w, name in zip(arrs, (3, 3, 4, None, 3), ("means", "scales", "quats", "opacity", "rgb")):
            if a.shape != ((n, w) if w else (n,)):
                raise ValueError(f"{name} has shape {a.shape}")
        idx = None if index is None else np.ascontiguousarray(index, dtype=np.int64)
        n_sel = n if idx is None else idx.shape[0]
        reuse = into is not None and bool(into.handle)
        h = C.c_void_p(into.handle.value) if reuse else C.c_void_p()
        self._bind_stream()
        rc = LIB.gsr_submap_load_host(self.handle, n, *[a.ctypes.data for a in arrs],
                                      None if idx is None else idx.ctypes.data, n_sel, C.byref(h))
        self._check(rc, "gsr_submap_load_host")
        if reuse and h.value == into.handle.value:
            return into
        if reuse:
            into.handle = None
        return Submap(self, h)

    def set_workspace_limit(self, nbytes: int):
        """gsr_set_workspace_limit: cap the context workspace (0 = no cap)."""
        self._check(LIB.gsr_set_workspace_limit(self.handle, int(nbytes)), "gsr_set_workspace_limit")

    def render(self, submap: Submap, camera: Camera, poses, cfg: Optional[RenderCfg] = None,
               rgb=None, depth=None, tfinal=None, with_tfinal: bool = False):
        torch = _torch()
        P = poses.shape[0]
        _dev_f32(poses, "poses", (P, 3, 4))
        H, W = camera.height, camera.width
        dev = poses.device
        if rgb is None:
            rgb = torch.empty((P, 3, H, W), dtype=torch.float32, device=dev)
        if depth is None:
            depth = torch.empty((P, H, W), dtype=torch.float32, device=dev)
        if with_tfinal and tfinal is None:
            tfinal = torch.empty((P, H, W), dtype=torch.float32, device=dev)
        _dev_f32(rgb, "rgb", (P, 3, H, W))
        _dev_f32(depth, "depth", (P, H, W))
        if tfinal is not None:
            _dev_f32(tfinal, "tfinal", (P, H, W))
        self._bind_stream()
        cam = camera.c()
        rc = LIB.gsr_render(self.handle, submap.handle, C.byref(cam), poses.data_ptr(), P,
                            C.byref(cfg) if cfg is not None else None, rgb.data_ptr(), depth.data_ptr(),
                            tfinal.data_ptr() if tfinal is not None else None)
        self._check(rc, "gsr_render")
        return (rgb, depth, tfinal) if tfinal is not None else (rgb, depth)

    def render_multi(self, submaps: Sequence[Submap], poses_per_submap: Sequence[int], camera: Camera, poses,
                     cfg: Optional[RenderCfg] = None, rgb=None, depth=None, tfinal=None, with_tfinal: bool = False):
        """One render of several queries (gsr_render_multi): submap q at poses_per_submap[q]
        consecutive poses of `poses`. Same outputs as gsr_render per submap."""
        torch = _torch()
        P = poses.shape[0]
        counts = np.ascontiguousarray(poses_per_submap, dtype=np.int32)
        if counts.ndim != 1 or counts.size != len(submaps) or int(counts.sum()) != P:
            raise ValueError("poses_per_submap must give one count per submap, summing to the pose count")
        _dev_f32(poses, "poses", (P, 3, 4))
        H, W = camera.height, camera.width
        dev = poses.device
        if rgb is None:
            rgb = torch.empty((P, 3, H, W), dtype=torch.float32, device=dev)
        if depth is None:
            depth = torch.empty((P, H, W), dtype=torch.float32, device=dev)
        if with_tfinal and tfinal is None:
            tfinal = torch.empty((P, H, W), dtype=torch.float32, device=dev)
        _dev_f32(rgb, "rgb", (P, 3, H, W))
        _dev_f32(depth, "depth", (P, H, W))
        if tfinal is not None:
            _dev_f32(tfinal, "tfinal", (P, H, W))
        handles = (C.c_void_p * len(submaps))(*[sm.handle.value if isinstance(sm.handle, C.c_void_p) else sm.handle
                                                for sm in submaps])
        self._bind_stream()
        cam = camera.c()
        rc = LIB.gsr_render_multi(self.handle, handles, counts.ctypes.data, len(submaps), C.byref(cam),
                                  poses.data_ptr(), C.byref(cfg) if cfg is not None else None, rgb.data_ptr(),
                                  depth.data_ptr(), tfinal.data_ptr() if tfinal is not None else None)
        self._check(rc, "gsr_render_multi")
        return (rgb, depth, tfinal) if tfinal is not None else (rgb, depth)

    def render_backward(self, submap: Submap, scales, quats, poses, rgb, depth, grad_rgb, grad_depth):
        """Gradients (means, scales, quats, opacity, rgb) of a loss through the last
        render of `submap` at `poses` (gsr_render_backward), given dL/drgb and dL/ddepth."""
        torch = _torch()
        n = submap.n
        P = poses.shape[0]
        _dev_f32(scales, "scales", (n, 3))
        _dev_f32(quats, "quats", (n, 4))
        _dev_f32(poses, "poses", (P, 3, 4))
        H, W = rgb.shape[2], rgb.shape[3]
        for t, nm, sh in ((rgb, "rgb", (P, 3, H, W)), (depth, "depth", (P, H, W)), (grad_rgb, "grad_rgb", (P, 3, H, W)),
                          (grad_depth, "grad_depth", (P, H, W))):
            _dev_f32(t, nm, sh)
        dev = scales.device
        out = [torch.empty(sh, dtype=torch.float32, device=dev) for sh in ((n, 3), (n, 3), (n, 4), (n,), (n, 3))]
        self._bind_stream()
        rc = LIB.gsr_render_backward(self.handle, submap.handle, scales.data_ptr(), quats.data_ptr(), poses.data_ptr(),
                                     P, rgb.data_ptr(), depth.data_ptr(), grad_rgb.data_ptr(), grad_depth.data_ptr(),
                                     *[o.data_ptr() for o in out])
        self._check(rc, "gsr_render_backward")
        return tuple(out)

    def capture_begin(self):
        """Start recording this context's calls into a HIP graph (gsr_capture_begin).
        The current torch stream must not be the default stream."""
        self._bind_stream()
        self._check(LIB.gsr_capture_begin(self.handle), "gsr_capture_begin")

    def capture_end(self) -> "Graph":
        g = C.c_void_p()
        self._check(LIB.gsr_capture_end(self.handle, C.byref(g)), "gsr_capture_end")
        graph = Graph(self, g)
        self._children.add(graph)
        return graph

    def ncc(self, query, renders, scores=None):
        torch = _torch()
        P, _, H, W = renders.shape
        _dev_f32(query, "query", (3, H, W))
        _dev_f32(renders, "renders", (P, 3, H, W))
        if scores is None:
            scores = torch.empty((P,), dtype=torch.float32, device=renders.device)
        _dev_f32(scores, "scores", (P,))
        self._bind_stream()
        self._check(LIB.gsr_ncc(self.handle, query.data_ptr(), renders.data_ptr(), P, H, W,
                                scores.data_ptr()), "gsr_ncc")
        return scores

    def ncc_noalloc(self, query, renders, scores):
        """gsr_ncc_noalloc: NCC into the caller's `scores` [P] with the library's
        static scratch (no allocation anywhere in the call)."""
        P, _, H, W = renders.shape
        _dev_f32(query, "query", (3, H, W))
        _dev_f32(renders, "renders", (P, 3, H, W))
        _dev_f32(scores, "scores", (P,))
        self._bind_stream()
        self._check(LIB.gsr_ncc_noalloc(self.handle, query.data_ptr(), renders.data_ptr(), P, H, W,
                                        scores.data_ptr()), "gsr_ncc_noalloc")
        return scores

    def topk(self, scores, k: int = 1, out=None):
        torch = _torch()
        P = scores.shape[0]
        _dev_f32(scores, "scores", (P,))
        if out is None:
            out = torch.empty((k,), dtype=torch.int32, device=scores.device)
        if out.dtype != torch.int32 or out.shape != (k,) or out.device.type != "cuda":
            raise TypeError("out must be an int32 CUDA tensor of shape (k,)")
        self._bind_stream()
        self._check(LIB.gsr_topk(self.handle, scores.data_ptr(), P, k, out.data_ptr()), "gsr_topk")
        return out

    def search(self, submap: Submap, camera: Camera, poses, order, batch: int, max_eval: int,
               threshold: float, query, cfg: Optional[RenderCfg] = None, scores=None):
        """Random-order search with an early stop (gsr_search). Returns
        (best candidate, its NCC, candidates scored, scores tensor)."""
        torch = _torch()
        P = poses.shape[0]
        _dev_f32(poses, "poses", (P, 3, 4))
        _dev_f32(query, "query", (3, camera.height, camera.width))
        order = np.ascontiguousarray(order, dtype=np.int32)
        if order.shape != (P,):
            raise ValueError("order must hold one entry per candidate")
        if scores is None:
            scores = torch.full((P,), float("nan"), dtype=torch.float32, device=poses.device)
        _dev_f32(scores, "scores", (P,))
        self._bind_stream()
        cam = camera.c()
        best, score, n = C.c_int32(0), C.c_float(0), C.c_int32(0)
        rc = LIB.gsr_search(self.handle, submap.handle, C.byref(cam), poses.data_ptr(), P,
                            order.ctypes.data, batch, max_eval, threshold, query.data_ptr(),
                            C.byref(cfg) if cfg is not None else None, scores.data_ptr(),
                            C.byref(best), C.byref(score), C.byref(n))
        self._check(rc, "gsr_search")
        return best.value, score.value, n.value, scores

    def sync(self):
        self._check(LIB.gsr_sync(self.handle), "gsr_sync")

    def stats(self) -> dict:
        st = Stats()
        self._check(LIB.gsr_get_stats(self.handle, C.byref(st)), "gsr_get_stats")
        return st.as_dict()

    def debug_buffer(self, which: int) -> np.ndarray:
        nb = C.c_int64(0)
        self._check(LIB.gsr_debug_size(self.handle, which, C.byref(nb)), "gsr_debug_size")
        dt = {BUF_RECORDS: np.float32, BUF_NTILES: np.uint32, BUF_OFFSETS: np.uint64,
              BUF_PAIRS: np.uint32}[which]
        out = np.empty(nb.value // np.dtype(dt).itemsize, dtype=dt)
        if out.size:
            self._check(LIB.gsr_debug_copy(self.handle, which, out.ctypes.data, nb.value), "gsr_debug_copy")
        return out

    def search_pruned(self, submap: Submap, camera: Camera, camera_low: Camera, poses, query, k: int,
                      scorer: Optional["Scorer"] = None, batch: int = 0, cfg: Optional[RenderCfg] = None):
        """Pruned search (gsr_search_pruned): predict every candidate's score at low
        resolution (scorer, or low-resolution NCC if scorer is None), keep the k best,
        decide among them by full-resolution NCC. Returns (best candidate, its NCC,
        predicted scores [P], kept candidates [k], their NCC [k])."""
        torch = _torch()
        P = poses.shape[0]
        _dev_f32(poses, "poses", (P, 3, 4))
        _dev_f32(query, "query", (3, camera.height, camera.width))
        dev = poses.device
        pred = torch.empty((P,), dtype=torch.float32, device=dev)
        top = torch.empty((k,), dtype=torch.int32, device=dev)
        ncc = torch.empty((k,), dtype=torch.float32, device=dev)
        self._bind_stream()
        cam, caml = camera.c(), camera_low.c()
        best, score = C.c_int32(0), C.c_float(0)
        rc = LIB.gsr_search_pruned(self.handle, scorer.handle if scorer is not None else None, submap.handle,
                                   C.byref(cam), C.byref(caml), poses.data_ptr(), P, batch, query.data_ptr(), k,
                                   C.byref(cfg) if cfg is not None else None, pred.data_ptr(), top.data_ptr(),
                                   ncc.data_ptr(), C.byref(best), C.byref(score))
        self._check(rc, "gsr_search_pruned")
        return best.value, score.value, pred, top, ncc

    def pool_grey(self, rgb, factor: int, out=None):
        """factor x factor mean pool of the grey of rgb [n, 3, H, W] -> [n, H/f, W/f]."""
        torch = _torch()
        n, _, H, W = rgb.shape
        _dev_f32(rgb, "rgb", (n, 3, H, W))
        if out is None:
            out = torch.empty((n, H // factor, W // factor), dtype=torch.float32, device=rgb.device)
        _dev_f32(out, "out", (n, H // factor, W // factor))
        self._bind_stream()
        self._check(LIB.gsr_pool_grey(self.handle, rgb.data_ptr(), n, H, W, factor, out.data_ptr()), "gsr_pool_grey")
        return out


def _dev_bf16_bits(t, name, shape):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype not in (torch.int16, torch.bfloat16):
        raise TypeError(f"{name} must be a CUDA int16 or bfloat16 tensor (bfloat16 bits)")
    if not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be contiguous with shape {tuple(shape)}")
    return t


class Scorer:
    """Learned candidate scorer (include/gsr_scorer.h) on a context: inputs of
    height x width, batches of up to max_batch candidates."""

    def __init__(self, ctx: Context, height: int, width: int, max_batch: int):
        self.ctx = ctx
        self.height, self.width, self.max_batch = int(height), int(width), int(max_batch)
        self.handle = C.c_void_p()
        ctx._bind_stream()
        ctx._check(LIB.gsr_scorer_create(ctx.handle, self.height, self.width, self.max_batch,
                                         C.byref(self.handle)), "gsr_scorer_create")
        self.n_params = int(LIB.gsr_scorer_param_count())
        ctx._children.add(self)

    def close(self):
        if self.handle:
            LIB.gsr_scorer_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _x(self, x):
        n = x.shape[0]
        return _dev_bf16_bits(x, "x", (n, self.height, self.width, 2)), n

    def set_params(self, params):
        _dev_f32(params, "params", (self.n_params,))
        self.ctx._bind_stream()
        self.ctx._check(LIB.gsr_scorer_set_params(self.handle, params.data_ptr()), "gsr_scorer_set_params")

    def get_params(self, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty((self.n_params,), dtype=torch.float32, device=f"cuda:{self.ctx.device}")
        _dev_f32(out, "out", (self.n_params,))
        self.ctx._bind_stream()
        self.ctx._check(LIB.gsr_scorer_get_params(self.handle, out.data_ptr()), "gsr_scorer_get_params")
        return out

    def inputs(self, renders, query_grey, out=None):
        """Network inputs [n, h, w, 2] (bfloat16) from renders [n, 3, h, w] and the pooled query [h, w]."""
        torch = _torch()
        n = renders.shape[0]
        _dev_f32(renders, "renders", (n, 3, self.height, self.width))
        _dev_f32(query_grey, "query_grey", (self.height, self.width))
        if out is None:
            out = torch.empty((n, self.height, self.width, 2), dtype=torch.bfloat16, device=renders.device)
        _dev_bf16_bits(out, "out", (n, self.height, self.width, 2))
        self.ctx._bind_stream()
        self.ctx._check(LIB.gsr_scorer_inputs(self.handle, renders.data_ptr(), n, query_grey.data_ptr(),
                                              out.data_ptr()), "gsr_scorer_inputs")
        return out

    def forward(self, x, scores=None):
        torch = _torch()
        x, n = self._x(x)
        if scores is None:
            scores = torch.empty((n,), dtype=torch.float32, device=x.device)
        _dev_f32(scores, "scores", (n,))
        self.ctx._bind_stream()
        self.ctx._check(LIB.gsr_scorer_forward(self.handle, x.data_ptr(), n, scores.data_ptr()), "gsr_scorer_forward")
        return scores

    def backward(self, x, labels, grads=None, loss=None):
        """(loss [1], gradient [n_params]) of the mean squared error at the current parameters."""
        torch = _torch()
        x, n = self._x(x)
        _dev_f32(labels, "labels", (n,))
        if grads is None:
            grads = torch.empty((self.n_params,), dtype=torch.float32, device=x.device)
        if loss is None:
            loss = torch.empty((1,), dtype=torch.float32, device=x.device)
        _dev_f32(grads, "grads", (self.n_params,))
        _dev_f32(loss, "loss", (1,))
        self.ctx._bind_stream()
        self.ctx._check(LIB.gsr_scorer_backward(self.handle, x.data_ptr(), labels.data_ptr(), n, loss.data_ptr(),
                                                grads.data_ptr()), "gsr_scorer_backward")
        return loss, grads

    @staticmethod
    def adamw_cfg(lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=1e-4) -> AdamW:
        return AdamW(lr, beta1, beta2, eps, weight_decay)

    def adamw(self, grads, opt: AdamW):
        _dev_f32(grads, "grads", (self.n_params,))
        self.ctx._bind_stream()
        self.ctx._check(LIB.gsr_scorer_adamw(self.handle, grads.data_ptr(), C.byref(opt)), "gsr_scorer_adamw")

    def train_step(self, x, labels, opt: AdamW, loss=None):
        torch = _torch()
        x, n = self._x(x)
        _dev_f32(labels, "labels", (n,))
        if loss is None:
            loss = torch.empty((1,), dtype=torch.float32, device=x.device)
        _dev_f32(loss, "loss", (1,))
        self.ctx._bind_stream()
        self.ctx._check(LIB.gsr_scorer_train_step(self.handle, x.data_ptr(), labels.data_ptr(), n, C.byref(opt),
                                                  loss.data_ptr()), "gsr_scorer_train_step")
        return loss
