"""MI355X-native render + NCC hot path of 3DGS-ReLoc (arXiv 2403.11367).

The compute runs in ``libgsr.so`` (hand-written HIP kernels for gfx950 behind
the C ABI in ``include/gsr.h``); ``gsr`` is its ctypes binding and
``reloc`` the small driver of Sec. III-C1 (crop -> load -> render -> NCC ->
select). Build the library with ``python -m paper_2403_11367_amd.build``.

The binding is imported on first use of one of its names, so that the build
module can run before the library exists; using the package without a built
library raises ImportError.
"""
_BINDING = ("BUF_NTILES", "BUF_OFFSETS", "BUF_PAIRS", "BUF_RECORDS", "Camera", "Context", "GsrError",
            "RenderCfg", "Scorer", "Submap", "crop", "default_cfg")

__all__ = list(_BINDING)


def __getattr__(name):
    if name in _BINDING:
        from . import gsr
        return getattr(gsr, name)
    raise AttributeError(f"module {__name__!r} has no attribute {name!r}")
