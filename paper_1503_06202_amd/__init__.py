"""MI355X (gfx950) correlator X-engine.

For every frequency channel of a frame of 4+4-bit offset-binary complex
samples, the engine integrates the pairwise products of all inputs over the
upper triangle including the autocorrelations (Sec. I; Sec. IV-C, "Full
Correlation"; Eq. (1)), exactly, as int32 (re, im).

The work runs in ``libxeng.so``: HIP kernels for gfx950 behind the C ABI of
``include/xeng.h``.  This package marshals torch device tensors and streams
into that ABI (``engine``), tunes batched plans (``tune``) and runs the
streaming request loop (``stream``).
"""
from .engine import BatchPlan, Plan, XengError, correlate, num_baselines, vis_shape  # noqa: F401

__all__ = ["Plan", "BatchPlan", "XengError", "correlate", "num_baselines", "vis_shape"]
