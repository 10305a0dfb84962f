"""MI355X-native render + NCC hot path of 3DGS-ReLoc (arXiv 2403.11367).

The compute runs in ``libgsr.so`` (hand-written HIP kernels for gfx950 behind
the C ABI in ``include/gsr.h``); ``gsr`` is its ctypes binding and
``reloc`` the small driver of Sec. III-C1 (crop -> load -> render -> NCC ->
select). Build the library with ``python -m paper_2403_11367_amd.build``.
"""
from .gsr import (BUF_NTILES, BUF_OFFSETS, BUF_PAIRS, BUF_RECORDS, Camera, Context, GsrError,  # noqa: F401
                  RenderCfg, Submap, crop, default_cfg)
