"""Convenience wrapper: allocate the device buffers of one batch with torch and run it.

Still marshalling only: the buffers are torch tensors, the work is nssdoa_estimate.
"""

from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

from . import _abi
from .api import Batch, Options, Plan, decode_peaks, grid_points


@dataclasses.dataclass
class DeviceBatch:
    plan: Plan
    batch: Batch
    X: object            # torch tensor (flat complex64/complex128 viewed as float)
    spectrum: object     # torch tensor or None
    peaks: object        # torch uint8 tensor, n * max_D * 32 bytes
    npeaks: object       # torch int32
    status: object       # torch int32 (uint32 bits)
    workspace: object    # torch uint8
    spec_len: List[int]
    spec_off: List[int]

    def run(self, stream=None):
        self.batch.estimate(self.X, self.spectrum, self.peaks, self.npeaks, self.status, self.workspace, stream)

    def run_noalloc(self, stream=None):
        """The same estimate on the library's per-device workspace array (no allocation)."""
        self.batch.estimate_noalloc(self.X, self.spectrum, self.peaks, self.npeaks, self.status, stream)

    def capture(self):
        """A graph of nssdoa_estimate on this batch's buffers (replay with .launch(stream))."""
        return self.batch.graph(self.X, self.spectrum, self.peaks, self.npeaks, self.status, self.workspace)

    def _windowed_workspace(self, mlp=None):
        import torch
        need = self.batch.windowed_workspace_size(mlp)
        if self.workspace.numel() < need:
            self.workspace = torch.empty(need, dtype=torch.uint8, device=self.workspace.device)

    def run_windowed(self, scores, topk: int, half_window_deg: float, score_threshold: float, stream=None,
                     window_floor: float = float("-inf"), local_max_bins: bool = False):
        """Windowed estimation with caller scores (device float tensor [n_frames][n_bins])."""
        self._windowed_workspace()
        self.batch.estimate_windowed(self.X, scores, topk, half_window_deg, score_threshold, self.spectrum,
                                     self.peaks, self.npeaks, self.status, self.workspace, stream,
                                     window_floor=window_floor, local_max_bins=local_max_bins)

    def run_learned(self, mlp, topk: int, half_window_deg: float, fallback_score: float, stream=None,
                    window_score: float = 0.0, local_max_bins: bool = False):
        """Windowed estimation with the learned proposal network."""
        self._windowed_workspace(mlp)
        self.batch.estimate_learned(mlp, self.X, topk, half_window_deg, fallback_score, self.spectrum,
                                    self.peaks, self.npeaks, self.status, self.workspace, stream,
                                    window_score=window_score, local_max_bins=local_max_bins)

    def host_results(self):
        import torch
        torch.cuda.synchronize()
        n, mD = self.batch.n_frames, self.batch.max_D
        pk = decode_peaks(self.peaks.cpu().numpy(), n, mD)
        out = dict(peaks=pk, npeaks=self.npeaks.cpu().numpy().copy(),
                   status=self.status.cpu().numpy().astype(np.uint32))
        if self.spectrum is not None:
            s = self.spectrum.cpu().numpy()
            out["spectra"] = [s[o:o + L].copy() for o, L in zip(self.spec_off, self.spec_len)]
        return out

    def workspace_array(self, item: int, frame: int, count: int, dtype) -> np.ndarray:
        """Host copy of `count` elements of a workspace item (after run + synchronize)."""
        off = self.batch.workspace_offset(item, frame)
        nbytes = count * np.dtype(dtype).itemsize
        raw = self.workspace[off:off + nbytes].cpu().numpy()
        return np.frombuffer(raw.tobytes(), dtype=dtype).copy()


def prepare(arrays: Sequence[np.ndarray], grids: Sequence[tuple], frames: Sequence[tuple],
            X_flat: np.ndarray, alg: str, prec: str, max_D: int, *, with_spectrum: bool = True,
            options: Optional[Options] = None, device: str = "cuda", X_device=None) -> DeviceBatch:
    """Create plan and batch, upload X, allocate outputs.  frames: (array_id, grid_id, N, D,
    x_off, ldx) tuples; spectrum offsets are assigned here, frame after frame."""
    import torch

    plan = Plan(arrays, grids, options)
    spec_off, spec_len, full = [], [], []
    off = 0
    for f in frames:
        L = grid_points(grids[f[1]])
        spec_off.append(off)
        spec_len.append(L)
        full.append(tuple(f[:6]) + (off,))
        off += L
    batch = Batch(plan, alg, prec, full, max_D)
    sdt = torch.float64 if prec == "c128" else torch.float32
    if X_device is not None:
        X = X_device                               # snapshots already on the device
    elif prec == "c128":
        X = torch.from_numpy(np.ascontiguousarray(X_flat, dtype=np.complex128).view(np.float64)).to(device)
    else:
        X = torch.from_numpy(np.ascontiguousarray(X_flat, dtype=np.complex64).view(np.float32)).to(device)
    spectrum = torch.empty(off, dtype=sdt, device=device) if with_spectrum else None
    n = len(frames)
    peaks = torch.empty(n * max_D * _abi.PEAK_DTYPE.itemsize, dtype=torch.uint8, device=device)
    npeaks = torch.empty(n, dtype=torch.int32, device=device)
    status = torch.empty(n, dtype=torch.int32, device=device)
    ws = torch.empty(batch.workspace_size(), dtype=torch.uint8, device=device)
    return DeviceBatch(plan, batch, X, spectrum, peaks, npeaks, status, ws, spec_len, spec_off)
