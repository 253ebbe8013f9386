"""Asymmetric bidirectional optical flow stitching on MI355X (gfx950).

Bidirectional coarse-to-fine flow and the asymmetric warp-and-blend of
Meng & Liu (arXiv 2006.01201, Section III.C) as hand-written HIP kernels
behind a C ABI (``include/abf.h``, ``libabf.so``). ``Plan`` (in ``api``)
is the torch-facing wrapper; ``_abi`` is the raw ctypes binding; ``synth``
generates seeded synthetic inputs.
"""
__all__ = ["Plan", "Params", "synth"]


def __getattr__(name):
    if name in ("Plan", "Params", "Batch"):
        from . import api

        return getattr(api, name)
    raise AttributeError(name)
