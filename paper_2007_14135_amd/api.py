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

    def __init__(self, eig_tol=1e-15, eig_max_iter=30, refine_halfwidth=4, lowq_tau=5e-4,
                 extra_candidates=4, scan_rows=0, eig_method="auto", c64_scan="split3"):
        m = _abi.EIG_METHODS.get(eig_method, eig_method) if isinstance(eig_method, str) else int(eig_method)
        if isinstance(m, str):
            raise ValueError("eig_method must be one of %s" % sorted(_abi.EIG_METHODS))
        k = _abi.C64_SCANS.get(c64_scan, c64_scan) if isinstance(c64_scan, str) else int(c64_scan)
        if isinstance(k, str):
            raise ValueError("c64_scan must be one of %s" % sorted(_abi.C64_SCANS))
        self.c = _abi.Options(eig_tol, eig_max_iter, refine_halfwidth, lowq_tau, extra_candidates, scan_rows, m, k)


def grid_points(g: tuple) -> int:
    """Grid points of a grid tuple: L, or L * n_polar for a 2-D grid."""
    return int(g[2]) * (int(g[6]) if len(g) > 4 and int(g[6]) > 0 else 1)


class Plan:
    """Array geometries (positions in wavelengths, shape (M, 3)) and scan grids: (start, step, L,
    circular) for azimuth grids, (start, step, L, circular, polar_start, polar_step, n_polar) for
    azimuth x polar-angle grids."""

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
            if len(g) > 4:     # 2-D: (start, step, L, circular, polar_start, polar_step, n_polar)
                grd[i] = _abi.Grid(float(start), float(step), int(L), int(circ), float(g[4]), float(g[5]), int(g[6]), 0)
            else:
                grd[i] = _abi.Grid(float(start), float(step), int(L), int(circ), 0.0, 0.0, 0, 0)
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

    def estimate_noalloc(self, X, spectrum, peaks, npeaks, status, stream=None) -> None:
        """nssdoa_estimate on the library's own per-device workspace array (no allocation)."""
        lib = _abi.load()
        s_elems = spectrum.numel() if spectrum is not None else 0
        _abi.check(lib.nssdoa_estimate_noalloc(self.handle, _ptr(X), X.numel() // 2, _ptr(spectrum), s_elems,
                                               _ptr(peaks), _ptr(npeaks), _ptr(status), _stream_handle(stream)),
                   "nssdoa_estimate_noalloc")

    def features(self, workspace, feats, stream=None) -> None:
        """Proposal features (device float [n_frames][M(M+1)]) of the covariances the last estimate
        on this workspace computed."""
        _abi.check(_abi.load().nssdoa_features(self.handle, _ptr(workspace), workspace.numel() * workspace.element_size(),
                                               _ptr(feats), int(feats.shape[1]), _stream_handle(stream)),
                   "nssdoa_features")

    def scan_form(self, form: str, workspace, spectrum, stream=None) -> None:
        """Rescan the frames of the last estimate on this workspace with an alternative Step-5 form
        (plain FP32, no FP64 re-evaluation): 'factored', 'quadratic' or 'complement'."""
        _abi.check(_abi.load().nssdoa_scan_form(self.handle, _abi.SCAN_FORMS[form], _ptr(workspace),
                                                workspace.numel() * workspace.element_size(), _ptr(spectrum),
                                                spectrum.numel(), _stream_handle(stream)),
                   "nssdoa_scan_form")

    def windowed_workspace_size(self, mlp: Optional["MLP"] = None) -> int:
        n = ctypes.c_size_t()
        _abi.check(_abi.load().nssdoa_windowed_workspace_size(self.handle, mlp.handle if mlp is not None else None,
                                                              ctypes.byref(n)), "nssdoa_windowed_workspace_size")
        return int(n.value)

    def estimate_windowed(self, X, scores, topk: int, half_window_deg: float, score_threshold: float,
                          spectrum, peaks, npeaks, status, workspace, stream=None,
                          window_floor: float = float("-inf"), local_max_bins: bool = False) -> None:
        """Windowed estimation with caller scores (device float [n_frames][n_bins])."""
        lib = _abi.load()
        ws_bytes = workspace.numel() * workspace.element_size()
        s_elems = spectrum.numel() if spectrum is not None else 0
        _abi.check(lib.nssdoa_estimate_windowed(self.handle, _ptr(X), X.numel() // 2, _ptr(scores),
                                                int(scores.shape[1]), int(topk), float(half_window_deg),
                                                float(score_threshold), float(window_floor),
                                                int(bool(local_max_bins)), _ptr(spectrum),
                                                s_elems, _ptr(peaks),
                                                _ptr(npeaks), _ptr(status), _ptr(workspace), ws_bytes,
                                                _stream_handle(stream)),
                   "nssdoa_estimate_windowed")

    def estimate_learned(self, mlp: "MLP", X, topk: int, half_window_deg: float, fallback_score: float,
                         spectrum, peaks, npeaks, status, workspace, stream=None, window_score: float = 0.0,
                         local_max_bins: bool = False) -> None:
        """Windowed estimation with the learned proposal network."""
        lib = _abi.load()
        ws_bytes = workspace.numel() * workspace.element_size()
        s_elems = spectrum.numel() if spectrum is not None else 0
        _abi.check(lib.nssdoa_estimate_learned(self.handle, mlp.handle, _ptr(X), X.numel() // 2, int(topk),
                                               float(half_window_deg), float(fallback_score), float(window_score),
                                               int(bool(local_max_bins)), _ptr(spectrum),
                                               s_elems, _ptr(peaks), _ptr(npeaks), _ptr(status), _ptr(workspace),
                                               ws_bytes, _stream_handle(stream)),
                   "nssdoa_estimate_learned")

    def graph(self, X, spectrum, peaks, npeaks, status, workspace) -> "Graph":
        """Capture one nssdoa_estimate on these buffers into a replayable graph."""
        return Graph(self, X, spectrum, peaks, npeaks, status, workspace)

    def set_timing(self, enable) -> None:
        """True: time every stage; False: off; a list of stage names: only those."""
        if isinstance(enable, (list, tuple, set)):
            mask = 0
            for name in enable:
                mask |= 1 << _abi.STAGES[name]
        else:
            mask = -1 if enable else 0
        _abi.check(_abi.load().nssdoa_set_timing(self.handle, mask), "nssdoa_set_timing")

    def stage_time(self, stage: str):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _abi.check(_abi.load().nssdoa_stage_time(self.handle, _abi.STAGES[stage], ctypes.byref(ms), ctypes.byref(n)),
                   "nssdoa_stage_time")
        return float(ms.value), int(n.value)


def noalloc_workspace_limit() -> int:
    """Bytes of the workspace array nssdoa_estimate_noalloc uses."""
    n = ctypes.c_size_t()
    _abi.check(_abi.load().nssdoa_noalloc_workspace_limit(ctypes.byref(n)), "nssdoa_noalloc_workspace_limit")
    return int(n.value)


class Graph:
    """nssdoa_graph: a captured nssdoa_estimate launched as one graph."""

    def __init__(self, batch: Batch, X, spectrum, peaks, npeaks, status, workspace):
        lib = _abi.load()
        h = ctypes.c_void_p()
        ws_bytes = workspace.numel() * workspace.element_size()
        s_elems = spectrum.numel() if spectrum is not None else 0
        _abi.check(lib.nssdoa_graph_create(ctypes.byref(h), batch.handle, _ptr(X), X.numel() // 2, _ptr(spectrum),
                                           s_elems, _ptr(peaks), _ptr(npeaks), _ptr(status), _ptr(workspace),
                                           ws_bytes), "nssdoa_graph_create")
        self.handle = h
        self.batch = batch          # the batch must outlive the graph

    def launch(self, stream=None) -> None:
        _abi.check(_abi.load().nssdoa_graph_launch(self.handle, _stream_handle(stream)), "nssdoa_graph_launch")

    def close(self):
        if self.handle:
            _abi.check(_abi.load().nssdoa_graph_destroy(self.handle), "nssdoa_graph_destroy")
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                _abi.load().nssdoa_graph_destroy(self.handle)
        except Exception:
            pass


class Pipeline:
    """nssdoa_pipeline: batches of host snapshots copied in, estimated and copied out on `depth`
    slots.  Host buffers are tensors (pinned for overlapping copies); a submission's buffers must
    stay untouched until wait(ticket) returns."""

    def __init__(self, batch: Batch, depth: int):
        h = ctypes.c_void_p()
        _abi.check(_abi.load().nssdoa_pipeline_create(ctypes.byref(h), batch.handle, int(depth)),
                   "nssdoa_pipeline_create")
        self.handle = h
        self.batch = batch

    def submit(self, X_host, peaks_host, npeaks_host, status_host, spectrum_host=None) -> int:
        t = ctypes.c_int64()
        _abi.check(_abi.load().nssdoa_pipeline_submit(self.handle, _ptr(X_host), _ptr(spectrum_host), _ptr(peaks_host),
                                                      _ptr(npeaks_host), _ptr(status_host), ctypes.byref(t)),
                   "nssdoa_pipeline_submit")
        return int(t.value)

    def wait(self, ticket: int) -> None:
        _abi.check(_abi.load().nssdoa_pipeline_wait(self.handle, int(ticket)), "nssdoa_pipeline_wait")

    def close(self):
        if self.handle:
            _abi.check(_abi.load().nssdoa_pipeline_destroy(self.handle), "nssdoa_pipeline_destroy")
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                _abi.load().nssdoa_pipeline_destroy(self.handle)
        except Exception:
            pass


def decode_peaks(peaks_host_bytes: np.ndarray, n_frames: int, max_D: int) -> np.ndarray:
    """View a host copy of the peaks buffer as a structured (n_frames, max_D) array."""
    return np.frombuffer(np.ascontiguousarray(peaks_host_bytes).tobytes(), dtype=_abi.PEAK_DTYPE).reshape(n_frames, max_D)


class MLP:
    """The proposal network object (nssdoa_mlp): parameters, Adam state, activations on device."""

    HEADER_WORDS = 8

    def __init__(self, n_in: int, width: int, n_out: int, max_batch: int):
        lib = _abi.load()
        h = ctypes.c_void_p()
        _abi.check(lib.nssdoa_mlp_create(ctypes.byref(h), int(n_in), int(width), int(n_out), int(max_batch)),
                   "nssdoa_mlp_create")
        self.handle = h
        self.sizes = (int(n_in), int(width), int(n_out))
        self.max_batch = int(max_batch)
        n = ctypes.c_size_t()
        _abi.check(lib.nssdoa_mlp_param_count(h, ctypes.byref(n)), "nssdoa_mlp_param_count")
        self.n_params = int(n.value)

    def close(self):
        if self.handle:
            _abi.check(_abi.load().nssdoa_mlp_destroy(self.handle), "nssdoa_mlp_destroy")
            self.handle = None

    def __del__(self):
        try:
            if getattr(self, "handle", None):
                _abi.load().nssdoa_mlp_destroy(self.handle)
        except Exception:
            pass

    def save(self) -> bytes:
        lib = _abi.load()
        n = ctypes.c_size_t()
        _abi.check(lib.nssdoa_mlp_save(self.handle, None, ctypes.byref(n)), "nssdoa_mlp_save")
        buf = ctypes.create_string_buffer(n.value)
        _abi.check(lib.nssdoa_mlp_save(self.handle, buf, ctypes.byref(n)), "nssdoa_mlp_save")
        return buf.raw

    def load(self, blob: bytes) -> None:
        _abi.check(_abi.load().nssdoa_mlp_load(self.handle, blob, len(blob)), "nssdoa_mlp_load")

    def load_params(self, flat_params: np.ndarray, step: int = 0, m=None, v=None) -> None:
        """Load FP32 parameters (in the C ABI order) and optional Adam moments."""
        p = np.ascontiguousarray(flat_params, dtype=np.float32)
        assert p.size == self.n_params
        z = np.zeros_like(p)
        mm = z if m is None else np.ascontiguousarray(m, dtype=np.float32)
        vv = z if v is None else np.ascontiguousarray(v, dtype=np.float32)
        hdr = np.array([0x50434c4d, 1, self.sizes[0], self.sizes[1], self.sizes[2], int(step), 0, 0], dtype=np.int32)
        self.load(hdr.tobytes() + p.tobytes() + mm.tobytes() + vv.tobytes())

    def state(self):
        """(params, m, v, step) as host arrays."""
        raw = self.save()
        hdr = np.frombuffer(raw[:32], dtype=np.int32)
        f = np.frombuffer(raw[32:], dtype=np.float32)
        n = self.n_params
        return f[:n].copy(), f[n:2 * n].copy(), f[2 * n:].copy(), int(hdr[5])

    def forward(self, feats, logits, stream=None) -> None:
        _abi.check(_abi.load().nssdoa_mlp_forward(self.handle, _ptr(feats), int(feats.shape[0]), _ptr(logits),
                                                  _stream_handle(stream)), "nssdoa_mlp_forward")

    def train_step(self, feats, targets, lr: float, loss, stream=None) -> None:
        _abi.check(_abi.load().nssdoa_mlp_train_step(self.handle, _ptr(feats), _ptr(targets), int(feats.shape[0]),
                                                     float(lr), _ptr(loss), _stream_handle(stream)),
                   "nssdoa_mlp_train_step")

    def gradients(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        _abi.check(_abi.load().nssdoa_mlp_gradients(self.handle, out.ctypes.data_as(ctypes.c_void_p), out.size),
                   "nssdoa_mlp_gradients")
        return out


def flatten_params(params) -> np.ndarray:
    """[(W1, b1), (W2, b2), (W3, b3)] -> one vector in the C ABI order."""
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in params])


def unflatten_params(flat: np.ndarray, sizes):
    out, o = [], 0
    for fin, fout in zip(sizes[:-1], sizes[1:]):
        W = flat[o:o + fin * fout].reshape(fout, fin)
        o += fin * fout
        b = flat[o:o + fout]
        o += fout
        out.append((W, b))
    return out
