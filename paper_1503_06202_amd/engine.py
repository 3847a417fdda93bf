"""Python face of the X-engine: plans over torch device tensors.

torch provides device memory and streams; the correlation itself runs in
``libxeng.so`` (HIP kernels for gfx950) through the C ABI of
``include/xeng.h``.  There is no CPU path: without the library, or without a
GPU, calls raise.

Layouts (Sec. II-A footnote for the sample code; Eq. (1) for the baseline
count):
  samples  uint8  [T][F][N], high nibble = Re + 8, low nibble = Im + 8
  vis      int32  [F][N(N+1)/2][2], row-major upper triangle, (re, im)
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence, Tuple

import torch

from . import _lib
from ._lib import XengError  # noqa: F401

FORMS = {"i8": _lib.XENG_FORM_I8, "f8": _lib.XENG_FORM_F8}


def num_baselines(N: int) -> int:
    """N(N+1)/2: all pairs of inputs including autocorrelations (Eq. (1))."""
    return N * (N + 1) // 2


def vis_shape(N: int, F: int) -> Tuple[int, int, int]:
    return (F, num_baselines(N), 2)


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _check_samples(samples: torch.Tensor) -> Tuple[int, int, int]:
    if samples.dtype != torch.uint8 or samples.dim() != 3:
        raise ValueError("samples must be a uint8 tensor [T][F][N]")
    if not samples.is_cuda:
        raise ValueError("samples must be on the GPU")
    if not samples.is_contiguous():
        raise ValueError("samples must be contiguous")
    T, F, N = samples.shape
    return int(T), int(F), int(N)


def _check_vis(vis: torch.Tensor, N: int, F: int, device) -> None:
    if vis.dtype != torch.int32 or tuple(vis.shape) != vis_shape(N, F):
        raise ValueError(f"vis must be int32 {vis_shape(N, F)}")
    if not vis.is_cuda or not vis.is_contiguous() or vis.device != device:
        raise ValueError("vis must be a contiguous tensor on the samples' GPU")


class Plan:
    """A correlation plan for frames of N inputs, F channels, T <= T_max samples.

    ``form`` is "i8" (int8 MFMA, int32 accumulators) or "f8" (FP8 e4m3 MFMA,
    f32 partial sums flushed to int32 every <= 32768 samples).  With
    ``accumulate`` the frame's sums are added to ``vis``.  With ``gates`` > 0
    the plan can also gate the output into up to that many buffers
    (``correlate_gated``); with ``flagged`` it can correlate frames with
    invalid samples and count the valid pairs (``correlate_flagged``); with
    ``beams`` > 0 it is a beamformer for that many beams (``set_weights``,
    ``beamform``).
    """

    def __init__(self, N: int, F: int, T_max: int, form: str = "i8", accumulate: bool = False,
                 split_t: int = 0, kernel: int = 0, gates: int = 0, flagged: bool = False,
                 beams: int = 0):
        if form not in FORMS:
            raise ValueError(f"form must be one of {sorted(FORMS)}")
        if (gates > 0) + bool(flagged) + (beams > 0) > 1:
            raise ValueError("a plan is gated, flagged or a beamformer, not several")
        self.N, self.F, self.T_max, self.form, self.accumulate = N, F, T_max, form, accumulate
        self.gates, self.flagged, self.beams = gates, flagged, beams
        flags = FORMS[form] | (_lib.XENG_ACCUMULATE if accumulate else 0)
        h = ctypes.c_void_p()
        if beams:
            if form != "i8" or accumulate:
                raise ValueError("a beamformer plan takes no form or accumulate option")
            _lib.check(_lib.lib().xeng_plan_beams(ctypes.byref(h), int(N), int(F), int(T_max),
                                                  int(beams), 0), "xeng_plan_beams")
        elif flagged:
            _lib.check(_lib.lib().xeng_plan_flagged(ctypes.byref(h), int(N), int(F), int(T_max),
                                                    flags), "xeng_plan_flagged")
        elif gates:
            _lib.check(_lib.lib().xeng_plan_gated(ctypes.byref(h), int(N), int(F), int(T_max),
                                                  int(gates), flags), "xeng_plan_gated")
        else:
            _lib.check(_lib.lib().xeng_plan(ctypes.byref(h), int(N), int(F), int(T_max), flags),
                       "xeng_plan")
        self._h = h
        if split_t or kernel:
            self.set_tuning(split_t, kernel)

    @property
    def handle(self) -> int:
        return self._h.value

    def set_tuning(self, split_t: int = 0, kernel: int = 0) -> None:
        """split_t: time slices per tile (0 = automatic); kernel: 0 automatic,
        1 = 128 x 128 tiles, 2 = 128 x 256 tiles (needs N % 16 == 0), 3 / 4 =
        128 x 128 tiles with split / common wave roles in diagonal tiles, 5 =
        the channel kernel (one workgroup per channel and time slice; int8,
        N <= 256; other plans use 1)."""
        _lib.check(_lib.lib().xeng_plan_set_tuning(self._h, int(split_t), int(kernel)),
                   "xeng_plan_set_tuning")

    def correlate(self, samples: torch.Tensor, vis: Optional[torch.Tensor] = None,
                  stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """Visibilities of ``samples`` [T][F][N] (asynchronous on ``stream``)."""
        T, F, N = _check_samples(samples)
        if vis is None:
            if self.accumulate:
                raise ValueError("an accumulating plan needs the vis to add into")
            vis = torch.empty(vis_shape(N, F), dtype=torch.int32, device=samples.device)
        else:
            _check_vis(vis, N, F, samples.device)
        rc = _lib.lib().xeng_correlate(self._h, samples.data_ptr(), N, F, T, vis.data_ptr(),
                                       _stream_handle(stream))
        _lib.check(rc, "xeng_correlate", self._h.value)
        return vis

    def set_delays(self, delays, D_max: int = 0) -> None:
        """Shift input n by delays[n] samples (one value per 16-input group;
        None turns shifting off).  The D_max rows before each samples tensor
        passed to this plan must hold the history: pass a view that starts
        D_max rows into a buffer of [history; frame]."""
        import numpy as np

        if delays is None:
            _lib.check(_lib.lib().xeng_plan_set_delays(self._h, None, 0), "xeng_plan_set_delays")
            return
        d = np.ascontiguousarray(np.asarray(delays, dtype=np.int32))
        if d.shape != (self.N,):
            raise ValueError("delays must hold one int per input")
        _lib.check(_lib.lib().xeng_plan_set_delays(
            self._h, d.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(D_max)),
            "xeng_plan_set_delays", self._h.value)

    def correlate_gated(self, samples: torch.Tensor, gate, G: int,
                        vis: Optional[torch.Tensor] = None,
                        stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """Gated visibilities [G][F][B][2]: ``gate`` (host, one int per sample)
        picks each sample's buffer; values outside 0..G-1 drop the sample."""
        import numpy as np

        T, F, N = _check_samples(samples)
        g = np.ascontiguousarray(np.asarray(gate, dtype=np.int32))
        if g.shape != (T,):
            raise ValueError("gate must hold one int per time sample")
        shape = (int(G),) + vis_shape(N, F)
        if vis is None:
            if self.accumulate:
                raise ValueError("an accumulating plan needs the vis to add into")
            vis = torch.empty(shape, dtype=torch.int32, device=samples.device)
        elif (vis.dtype != torch.int32 or tuple(vis.shape) != shape or not vis.is_cuda
              or not vis.is_contiguous() or vis.device != samples.device):
            raise ValueError(f"vis must be a contiguous int32 {shape} tensor on the samples' GPU")
        rc = _lib.lib().xeng_correlate_gated(
            self._h, samples.data_ptr(), N, F, T,
            g.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(G), vis.data_ptr(),
            _stream_handle(stream))
        _lib.check(rc, "xeng_correlate_gated", self._h.value)
        return vis

    def correlate_flagged(self, samples: torch.Tensor, flags: torch.Tensor,
                          vis: Optional[torch.Tensor] = None, counts: Optional[torch.Tensor] = None,
                          stream: Optional[torch.cuda.Stream] = None):
        """Visibilities and valid-pair counts of a frame with invalid samples.

        ``flags`` is a device int32/uint32-sized tensor [T][F][ceil(N/32)] of
        flag words (bit i % 32 of word i // 32 set = sample invalid).  Flagged
        samples of ``samples`` are set to 0x88 in place.  Returns ``(vis,
        counts)``: int32 [F][B][2] and int32 [F][B].
        """
        T, F, N = _check_samples(samples)
        W = (N + 31) // 32
        if (flags.dtype not in (torch.int32, torch.uint32) or tuple(flags.shape) != (T, F, W)
                or not flags.is_cuda or not flags.is_contiguous()
                or flags.device != samples.device):
            raise ValueError(f"flags must be a contiguous 32-bit tensor {(T, F, W)} on the "
                             "samples' GPU")
        if vis is None or counts is None:
            if self.accumulate:
                raise ValueError("an accumulating plan needs the vis and counts to add into")
        if vis is None:
            vis = torch.empty(vis_shape(N, F), dtype=torch.int32, device=samples.device)
        else:
            _check_vis(vis, N, F, samples.device)
        cshape = (F, num_baselines(N))
        if counts is None:
            counts = torch.empty(cshape, dtype=torch.int32, device=samples.device)
        elif (counts.dtype != torch.int32 or tuple(counts.shape) != cshape or not counts.is_cuda
              or not counts.is_contiguous() or counts.device != samples.device):
            raise ValueError(f"counts must be a contiguous int32 {cshape} tensor on the "
                             "samples' GPU")
        rc = _lib.lib().xeng_correlate_flagged(self._h, samples.data_ptr(), flags.data_ptr(), N, F,
                                               T, vis.data_ptr(), counts.data_ptr(),
                                               _stream_handle(stream))
        _lib.check(rc, "xeng_correlate_flagged", self._h.value)
        return vis, counts

    def normalize(self, vis: torch.Tensor, counts: torch.Tensor, scale: float,
                  out: Optional[torch.Tensor] = None,
                  stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """Renormalised visibilities float32 [F][B][2]: vis * scale / counts
        (float64, rounded once), 0 where counts == 0."""
        N, F = self.N, self.F
        _check_vis(vis, N, F, vis.device)
        cshape = (F, num_baselines(N))
        if (counts.dtype != torch.int32 or tuple(counts.shape) != cshape or not counts.is_cuda
                or not counts.is_contiguous() or counts.device != vis.device):
            raise ValueError(f"counts must be a contiguous int32 {cshape} tensor on vis's GPU")
        if out is None:
            out = torch.empty(vis_shape(N, F), dtype=torch.float32, device=vis.device)
        elif (out.dtype != torch.float32 or tuple(out.shape) != vis_shape(N, F)
              or not out.is_cuda or not out.is_contiguous() or out.device != vis.device):
            raise ValueError(f"out must be a contiguous float32 {vis_shape(N, F)} tensor")
        rc = _lib.lib().xeng_normalize(self._h, vis.data_ptr(), counts.data_ptr(), float(scale),
                                       out.data_ptr(), _stream_handle(stream))
        _lib.check(rc, "xeng_normalize", self._h.value)
        return out

    def set_weights(self, weights) -> None:
        """Beam weights, int8 [F][B][N][2] (re, im) in -127..127, applied
        without a conjugate (host array; copied to the device)."""
        import numpy as np

        w = np.ascontiguousarray(np.asarray(weights, dtype=np.int8))
        if w.shape != (self.F, self.beams, self.N, 2):
            raise ValueError(f"weights must be int8 {(self.F, self.beams, self.N, 2)}")
        _lib.check(_lib.lib().xeng_beam_set_weights(
            self._h, w.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))), "xeng_beam_set_weights",
            self._h.value)

    def beamform(self, samples: torch.Tensor, out: Optional[torch.Tensor] = None,
                 stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
        """Beams int32 [T][F][B][2]: y = sum_n w[f][b][n] x[t][f][n]."""
        T, F, N = _check_samples(samples)
        shape = (T, F, self.beams, 2)
        if out is None:
            out = torch.empty(shape, dtype=torch.int32, device=samples.device)
        elif (out.dtype != torch.int32 or tuple(out.shape) != shape or not out.is_cuda
              or not out.is_contiguous() or out.device != samples.device):
            raise ValueError(f"out must be a contiguous int32 {shape} tensor on the samples' GPU")
        rc = _lib.lib().xeng_beamform(self._h, samples.data_ptr(), N, F, T, out.data_ptr(),
                                      _stream_handle(stream))
        _lib.check(rc, "xeng_beamform", self._h.value)
        return out

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().xeng_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def correlate(samples: torch.Tensor, form: str = "i8", vis: Optional[torch.Tensor] = None,
              accumulate: bool = False, split_t: int = 0, kernel: int = 0,
              stream: Optional[torch.cuda.Stream] = None) -> torch.Tensor:
    """One-shot correlation of a frame (plans, runs and frees a plan)."""
    T, F, N = _check_samples(samples)
    with Plan(N, F, T, form=form, accumulate=accumulate, split_t=split_t, kernel=kernel) as p:
        return p.correlate(samples, vis, stream)


def correlate_batch_noalloc(instances: Sequence[Tuple[int, int, int]],
                            samples: Sequence[Optional[torch.Tensor]],
                            vis: Sequence[Optional[torch.Tensor]], form: str = "i8",
                            accumulate: bool = False, split_t: Optional[Sequence[int]] = None,
                            shared_vis: bool = False,
                            stream: Optional[torch.cuda.Stream] = None) -> None:
    """The batched form without a plan (``xeng_correlate_batch_noalloc``): the
    library allocates nothing and queues kernels only, for callers that cannot
    allocate.  Calls that overlap on one GPU share its fixed workspace and
    race: keep them on one stream."""
    if form not in FORMS:
        raise ValueError(f"form must be one of {sorted(FORMS)}")
    inst = [tuple(map(int, x)) for x in instances]
    n = len(inst)
    splits = list(split_t) if split_t is not None else [0] * n
    if len(splits) != n:
        raise ValueError("one split_t per instance")
    arr = (_lib.XengInstance * max(1, n))()
    for k, ((N, F, T), sp) in enumerate(zip(inst, splits)):
        arr[k] = _lib.XengInstance(N, F, T, int(sp))
    sp_arr, vp_arr = _pointer_arrays(inst, samples, vis)
    flags = FORMS[form] | (_lib.XENG_ACCUMULATE if accumulate else 0)
    if shared_vis:
        flags |= _lib.XENG_SHARED_VIS
    rc = _lib.lib().xeng_correlate_batch_noalloc(arr, n, flags, sp_arr, vp_arr,
                                                 _stream_handle(stream))
    _lib.check(rc, "xeng_correlate_batch_noalloc")


def _pointer_arrays(instances, samples, vis):
    """Device pointer arrays of a batch; a None sample tensor skips that instance."""
    n = len(instances)
    if len(samples) != n or len(vis) != n:
        raise ValueError(f"need {n} sample and vis entries")
    sp = (ctypes.c_void_p * max(1, n))()
    vp = (ctypes.c_void_p * max(1, n))()
    for k, (N, F, T) in enumerate(instances):
        if samples[k] is None:
            continue
        Ts, Fs, Ns = _check_samples(samples[k])
        if (Ts, Fs, Ns) != (T, F, N):
            raise ValueError(f"instance {k}: samples shape {(Ts, Fs, Ns)} != planned {(T, F, N)}")
        if vis[k] is None:
            raise ValueError(f"instance {k} is active and needs its vis")
        _check_vis(vis[k], N, F, samples[k].device)
        sp[k] = samples[k].data_ptr()
        vp[k] = vis[k].data_ptr()
    return sp, vp


class BatchPlan:
    """Many independent (N, F, T) instances correlated by one persistent launch."""

    def __init__(self, instances: Sequence[Tuple[int, int, int]], form: str = "i8",
                 accumulate: bool = False, split_t: Optional[Sequence[int]] = None,
                 shared_vis: bool = False):
        if form not in FORMS:
            raise ValueError(f"form must be one of {sorted(FORMS)}")
        self.instances: List[Tuple[int, int, int]] = [tuple(map(int, x)) for x in instances]
        self.form, self.accumulate = form, accumulate
        n = len(self.instances)
        splits = list(split_t) if split_t is not None else [0] * n
        if len(splits) != n:
            raise ValueError("one split_t per instance")
        arr = (_lib.XengInstance * max(1, n))()
        for k, ((N, F, T), s) in enumerate(zip(self.instances, splits)):
            arr[k] = _lib.XengInstance(N, F, T, int(s))
        flags = FORMS[form] | (_lib.XENG_ACCUMULATE if accumulate else 0)
        if shared_vis:
            flags |= _lib.XENG_SHARED_VIS
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().xeng_plan_batch(ctypes.byref(h), arr, n, flags), "xeng_plan_batch")
        self._h = h
        self._keep = None

    def _arrays(self, samples: Sequence[Optional[torch.Tensor]],
                vis: Sequence[Optional[torch.Tensor]]):
        """Pointer arrays; a None sample tensor skips that instance this call."""
        return _pointer_arrays(self.instances, samples, vis)

    def correlate(self, samples: Sequence[Optional[torch.Tensor]],
                  vis: Sequence[Optional[torch.Tensor]],
                  stream: Optional[torch.cuda.Stream] = None, graph: bool = False) -> None:
        """Correlate the active instances (samples[k] not None) in one launch.

        With ``graph`` the launch replays a HIP graph captured on first use.
        """
        sp, vp = self._arrays(samples, vis)
        fn = _lib.lib().xeng_correlate_batch_graph if graph else _lib.lib().xeng_correlate_batch
        rc = fn(self._h, sp, vp, _stream_handle(stream))
        _lib.check(rc, "xeng_correlate_batch", self._h.value)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().xeng_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
