"""Autotuner of the matrix-core scan's work-item size (nssdoa_options.scan_rows).

A scan work item is one chunk of stacked noise-subspace rows times 256 grid angles: larger chunks
reuse each steering tile over more frames, smaller ones give more work items to spread over the
256 compute units and a shorter tail.  The best size depends on the batch (frames per group, rows
per frame, grid lengths), so it is measured: for every candidate the batch is scheduled with that
size and the scan stage of nssdoa_estimate is timed with HIP events on the launch stream
(nssdoa_stage_time); the fastest candidate wins.  Choices are cached in a JSON file keyed by the
device, the algorithm, the scan precision and a signature of the batch's shape, so a workload is
tuned once per device.
"""

from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Iterable, Optional, Sequence, Tuple

import numpy as np

# Revision of the scan kernels the cached choices were measured on; changing the kernels makes
# old entries miss.
KERNEL_REV = "scan-8"

CANDIDATES = {"c64": (64, 96, 128, 160, 192, 256, 320, 384, 512),
              "c64-split16": (128, 192, 256, 384, 512, 640, 768, 896, 1024),
              "c64-split3": (128, 192, 256, 384, 512, 640, 768, 896, 1024),
              "bf16": (512, 1024, 2048, 4096, 8192, 16384),
              "f16": (512, 1024, 2048, 4096, 8192, 16384)}


def signature(arrays: Sequence[np.ndarray], grids: Sequence[tuple], frames: Sequence[tuple], alg: str,
              prec: str, kernel: str = "split3") -> str:
    """A digest of what the scan schedule depends on: per (array, grid) group its M, its L and
    the multiset of noise-subspace ranks K of its frames, plus the algorithm, the precision and
    the C64 scan kernel."""
    groups: Dict[Tuple[int, int], list] = {}
    for f in frames:
        a, g, D = int(f[0]), int(f[1]), int(f[3])
        M = int(np.asarray(arrays[a]).reshape(-1, 3).shape[0])
        K = M - D if alg in ("music", "ev") else 1
        groups.setdefault((a, g), []).append(K)
    desc = []
    for (a, g), ks in sorted(groups.items()):
        M = int(np.asarray(arrays[a]).reshape(-1, 3).shape[0])
        desc.append((M, int(grids[g][2]), tuple(np.bincount(ks).tolist())))
    key = (KERNEL_REV, alg, prec, desc) if prec != "c64" else (KERNEL_REV, alg, prec, kernel, desc)
    return hashlib.sha1(repr(key).encode()).hexdigest()[:20]


def choose(timings: Dict[int, float]) -> int:
    """The fastest candidate; ties go to the smaller work item."""
    return min(timings, key=lambda c: (timings[c], c))


class Cache:
    """{device: {signature: {"scan_rows": n, "timings_ms": {...}}}} in a JSON file."""

    def __init__(self, path: Optional[str]):
        self.path = path
        self.data = {}
        if path and os.path.exists(path):
            with open(path) as fh:
                self.data = json.load(fh)

    def get(self, device: str, sig: str) -> Optional[int]:
        e = self.data.get(device, {}).get(sig)
        return int(e["scan_rows"]) if e else None

    def put(self, device: str, sig: str, rows: int, timings: Dict[int, float]) -> None:
        self.data.setdefault(device, {})[sig] = {"scan_rows": int(rows),
                                                 "timings_ms": {str(k): float(v) for k, v in timings.items()}}
        if self.path:
            tmp = self.path + ".tmp"
            with open(tmp, "w") as fh:
                json.dump(self.data, fh, indent=1, sort_keys=True)
            os.replace(tmp, self.path)


def device_name() -> str:
    """Architecture and compute-unit count of the current device (the tuning depends on these)."""
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return "%s/%dCU" % (getattr(p, "gcnArchName", "?").split(":")[0], p.multi_processor_count)


def tune(arrays, grids, frames, X_flat, alg: str, prec: str, max_D: int, *, candidates: Optional[Iterable[int]] = None,
         cache_path: Optional[str] = None, reps: int = 5, options=None, log=None) -> Tuple[int, Dict[int, float]]:
    """Best scan_rows for this batch (from the cache when present) and the measured timings."""
    import torch
    from .api import Options
    from .runner import prepare
    if prec == "c128":
        return 0, {}
    dev = device_name()
    kernel = {0: "split3", 1: "fp32", 2: "split16"}[0 if options is None else int(options.c.c64_scan)]
    sig = signature(arrays, grids, frames, alg, prec, kernel)
    cache = Cache(cache_path)
    hit = cache.get(dev, sig)
    if hit is not None:
        return hit, {}
    timings = {}
    X_dev = None
    for rows in (candidates or CANDIDATES["c64-" + kernel if prec == "c64" and kernel != "fp32" else prec]):
        if options is None:
            opt = Options(scan_rows=int(rows))
        else:
            c = options.c
            opt = Options(c.eig_tol, c.eig_max_iter, c.refine_halfwidth, c.lowq_tau, c.extra_candidates, int(rows),
                          c.eig_method, c.c64_scan)
        db = prepare(arrays, grids, frames, X_flat, alg, prec, max_D, with_spectrum=False, options=opt, X_device=X_dev)
        X_dev = db.X
        db.run()
        torch.cuda.synchronize()
        db.batch.set_timing(["scan"])
        for _ in range(reps):
            db.run()
        ms, n = db.batch.stage_time("scan")
        db.batch.set_timing(False)
        timings[int(rows)] = ms / max(n, 1)
        if log:
            log("scan_rows %5d: scan %.4f ms" % (rows, timings[int(rows)]))
        del db
    best = choose(timings)
    cache.put(dev, sig, best, timings)
    return best, timings
