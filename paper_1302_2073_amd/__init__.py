"""MI355X (gfx950) implementation of pROST's per-frame hot path.

Seidel, Hage, Kleinsteuber, "pROST: A Smoothed lp-norm Robust Online
Subspace Tracking Method for Realtime Background Subtraction in Video",
arXiv:1302.2073.  The kernels live in libprost.so (csrc/), reached through
the C ABI of include/prost.h; this package only marshals arguments.
"""
from . import _lib  # noqa: F401

__all__ = ["Tracker", "BatchTracker", "make_params", "roc_counts", "Ingest", "resample_rgb8", "mask_upsample"]


def __getattr__(name):
    if name in ("Tracker", "BatchTracker", "make_params", "bf16_bits", "bf16_to_f64", "roc_counts",
                "quality_measures"):
        from . import tracker
        return getattr(tracker, name)
    if name in ("Ingest", "resample_rgb8", "mask_upsample"):
        from . import ingest
        return getattr(ingest, name)
    raise AttributeError(name)
