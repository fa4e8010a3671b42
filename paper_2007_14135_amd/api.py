"""Thin Python layer over the C ABI: argument marshalling only.

Device buffers are torch tensors on the current HIP device (torch is used for memory and
streams only); every step of the estimation runs in libnssdoa's kernels.
"""

from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _abi


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return int(t.data_ptr())


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Options:
    """Tunables of nssdoa_options (defaults as documented in the header)."""

    def __init__(self, jacobi_tol=1e-15, max_sweeps=30, refine_halfwidth=4, lowq_tau=2e-3,
                 extra_candidates=4):
        self.c = _abi.Options(jacobi_tol, max_sweeps, refine_halfwidth, lowq_tau, extra_candidates, 0)


class Plan:
    """Array geometries (positions in wavelengths, shape (M, 3)) and azimuth scan grids."""

    def __init__(self, arrays: Sequence[np.ndarray], grids: Sequence[tuple], options: Optional[Options] = None):
        lib = _abi.load()
        self._pos = [np.ascontiguousarray(a, dtype=np.float64).reshape(-1, 3) for a in arrays]
        arr = (_abi.Array * len(self._pos))()
        for i, p in enumerate(self._pos):
            arr[i] = _abi.Array(p.shape[0], 0, p.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        grd = (_abi.Grid * len(grids))()
        for i, g in enumerate(grids):
            start, step, L = g[0], g[1], g[2]
            circ = g[3] if len(g) > 3 else 0
            grd[i] = _abi.Grid(float(start), float(step), int(L), int(circ))
        h = ctypes.c_void_p()
        opt = ctypes.byref(options.c) if options is not None else None
        _abi.check(lib.nssdoa_plan_create(ctypes.byref(h), arr, len(self._pos), grd, len(grids), opt),
                   "nssdoa_plan_create")
        self.handle = h
        self.M = [p.shape[0] for p in self._pos]
        self.grids = [tuple(g) for g in grids]

    def close(self):
        if self.handle:
            _abi.check(_abi.load().nssdoa_plan_destroy(self.handle), "nssdoa_plan_destroy")
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                _abi.load().nssdoa_plan_destroy(self.handle)
        except Exception:
            pass


class Batch:
    """A validated, scheduled set of frames for one algorithm and scan precision.

    ``frames`` is a sequence of (array_id, grid_id, N, D, x_off, ldx, spec_off) tuples.
    """

    def __init__(self, plan: Plan, alg: str, prec: str, frames: Sequence[tuple], max_D: int):
        lib = _abi.load()
        fr = (_abi.Frame * len(frames))()
        for i, f in enumerate(frames):
            fr[i] = _abi.Frame(*[int(v) for v in f])
        h = ctypes.c_void_p()
        _abi.check(lib.nssdoa_batch_create(ctypes.byref(h), plan.handle, _abi.ALGS[alg], _abi.PRECS[prec],
                                           fr, len(frames), int(max_D)), "nssdoa_batch_create")
        self.handle = h
        self.plan = plan
        self.alg, self.prec = alg, prec
        self.n_frames = len(frames)
        self.max_D = int(max_D)
        self.frames = [tuple(int(v) for v in f) for f in frames]

    def close(self):
        if self.handle:
            _abi.check(_abi.load().nssdoa_batch_destroy(self.handle), "nssdoa_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                _abi.load().nssdoa_batch_destroy(self.handle)
        except Exception:
            pass

    def workspace_size(self) -> int:
        n = ctypes.c_size_t()
        _abi.check(_abi.load().nssdoa_workspace_size(self.handle, ctypes.byref(n)), "nssdoa_workspace_size")
        return int(n.value)

    def workspace_offset(self, item: int, frame: int) -> int:
        n = ctypes.c_size_t()
        _abi.check(_abi.load().nssdoa_workspace_offset(self.handle, int(item), int(frame), ctypes.byref(n)),
                   "nssdoa_workspace_offset")
        return int(n.value)

    def estimate(self, X, spectrum, peaks, npeaks, status, workspace, stream=None) -> None:
        """Enqueue Steps 1-6 on ``stream`` (default: torch's current stream).

        X is a real tensor viewing interleaved complex values (float32 for c64, float64 for
        c128); its complex element count is numel // 2."""
        lib = _abi.load()
        ws_bytes = workspace.numel() * workspace.element_size()
        x_elems = X.numel() // 2
        s_elems = spectrum.numel() if spectrum is not None else 0
        _abi.check(lib.nssdoa_estimate(self.handle, _ptr(X), x_elems, _ptr(spectrum), s_elems, _ptr(peaks),
                                       _ptr(npeaks), _ptr(status), _ptr(workspace), ws_bytes,
                                       _stream_handle(stream)),
                   "nssdoa_estimate")

    def set_timing(self, enable: bool) -> None:
        _abi.check(_abi.load().nssdoa_set_timing(self.handle, 1 if enable else 0), "nssdoa_set_timing")

    def stage_time(self, stage: str):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _abi.check(_abi.load().nssdoa_stage_time(self.handle, _abi.STAGES[stage], ctypes.byref(ms), ctypes.byref(n)),
                   "nssdoa_stage_time")
        return float(ms.value), int(n.value)


def decode_peaks(peaks_host_bytes: np.ndarray, n_frames: int, max_D: int) -> np.ndarray:
    """View a host copy of the peaks buffer as a structured (n_frames, max_D) array."""
    return np.frombuffer(np.ascontiguousarray(peaks_host_bytes).tobytes(), dtype=_abi.PEAK_DTYPE).reshape(n_frames, max_D)
