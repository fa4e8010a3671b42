"""Throughput benchmark of the DOA hot path on one MI355X.

One step = one nssdoa_estimate call over the whole batch: covariance, FP64 eigensolve and
noise-subspace matrix, FP32-accuracy matrix-core spectrum scan (by default FP16 split operands of
three parts, which reproduce every FP32 operand, with FP32 accumulation; --c64-scan fp32 for FP32
operands, split16 for two parts), FP64 low-Q re-evaluation and peak
selection, for 256 synthetic frames of the 16-element workload (N = 4096 snapshots, D = 4,
18000-point grid at 0.01 deg), MUSIC.  Snapshots are resident in HBM before the timed region.

The timed steps keep --streams whole batches in flight (step k on stream k mod S, each stream
with its own copy of the snapshots, its own workspace and outputs), as a serving loop would; a
second, single-stream pass gives the latency of one batch and times the scan kernel alone.

Prints one JSON line with the throughput (spectrum points/s), the same step with the other C64
scan kernels for comparison, the roofline position of the scan kernel (timed live with HIP events on the launch stream; HBM traffic from the committed
counter summary while the kernel source is unchanged), the FP64 oracle's throughput on the host
cores over a bounded sample of the same frames, and, when trained proposal weights are present,
the learned-proposal workload (8192 frames, 0.001 deg grid) run by the learned path and by the
full scan on the same GPU.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP16_MFMA_TFLOPS = 2516.6
PEAK_HBM_GBS = 8000.0
METRIC = "MUSIC spectrum points/s & frames/s at ≤0.01° peak err, learned vs full scan"
WEIGHTS = os.path.join(ROOT, "paper_2007_14135_amd", "weights", "proposal_ula16.npy")
# the scan kernels and the host code that orders their work items (the counter summary holds a
# digest of both)
SCAN_SRC = [os.path.join(ROOT, "paper_2007_14135_amd", "csrc", f) for f in ("scan_f32.hip", "api.hip")]
PMC_SUMMARY = {"split16": os.path.join(ROOT, "profiles", "scan_split16_c2_music_pmc.txt"),
               "fp32": os.path.join(ROOT, "profiles", "scan_f32_c2_music_pmc.txt"),
               "split3": os.path.join(ROOT, "profiles", "scan_split3_c2_music_pmc.txt")}
SCAN_KERNEL = {"split16": "scan_split16_kernel<16, 2>", "fp32": "scan_f32_kernel<16>",
               "split3": "scan_split16_kernel<16, 3>"}
MFMA_PRODUCTS = {"split16": 3.0, "fp32": 1.0, "split3": 6.0}   # matrix-core products per FP32-accuracy product
SCAN_DESC = {"fp32": "FP32 operands, FP32 accumulation",
             "split16": "FP16 split operands of two parts (22-bit operands), FP32 accumulation",
             "split3": "FP16 split operands of three parts (33-bit operands, every FP32 operand reproduced), "
                       "six products per FP32-accuracy product, FP32 accumulation"}
STAGE_KERNEL = {"covariance": "cov_mfma_kernel<float2, 1>", "eigen": "evd_ql_kernel", "scan": None}
TUNE_CACHE = os.path.join(ROOT, "paper_2007_14135_amd", "tuning", "autotune_cache.json")
PEAK_FP64_TFLOPS = 78.6
LEARNED_WINDOW_SCORE = 0.05  # windows beyond a frame's first D bins need sigmoid(logit) >= this
HOST_WORKERS = 16          # host processes: the CPU share of one GPU on the measurement machine


def _oracle_worker(args):
    """Generate the frames (untimed), then time the oracle on them `repeats` times."""
    config, idx, alg, repeats = args
    from threadpoolctl import threadpool_limits
    import oracle
    from synth import make_frame
    with threadpool_limits(1):
        frames = [make_frame(config, i) for i in idx]
        t0 = time.perf_counter()
        out = []
        for r in range(repeats):
            for fr in frames:
                est = oracle.estimate(fr.X, fr.pos, fr.D, fr.grid, alg)
                if r == 0:
                    out.append((est.peaks.tolist(), est.angles[est.peaks].tolist()))
        busy = time.perf_counter() - t0
    return busy, out


def cpu_baseline(config, frame_ids, alg, L, repeats):
    import multiprocessing as mp
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(cores, HOST_WORKERS, len(frame_ids)))
    chunks = [frame_ids[i::workers] for i in range(workers)]
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_oracle_worker, [(config, c, alg, repeats) for c in chunks])
    wall = max(r[0] for r in res)           # the slowest worker bounds the parallel run
    cpu_s = sum(r[0] for r in res)
    peaks = {}
    for c, r in zip(chunks, res):
        for i, pk in zip(c, r[1]):
            peaks[i] = pk
    value = repeats * len(frame_ids) * L / wall
    return dict(value=value, unit="points/s", cores=workers, kind="oracle",
                host_cores_in_affinity=cores, cpu_model=cpu_model(),
                sample="all %d frames of the workload, %d passes, FP64 numpy/LAPACK oracle, covariance to peaks, "
                       "one process per core with BLAS threads = 1 (%d worker processes: the host CPU share of "
                       "one GPU; %d cores in this process's affinity); %.1f s of CPU work in %.1f s"
                       % (len(frame_ids), repeats, workers, cores, cpu_s, wall)), peaks


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _frames_worker(args):
    config, idx = args
    from threadpoolctl import threadpool_limits
    from synth import make_frame
    with threadpool_limits(1):
        return [make_frame(config, i) for i in idx]


def make_frames_parallel(config, n):
    """Frames 0..n-1 of a configuration, drawn by a fork pool (before the GPU is touched)."""
    import multiprocessing as mp
    from synth.frames import pack_frames
    workers = max(1, min(len(os.sched_getaffinity(0)), HOST_WORKERS))
    step = 256
    jobs = [(config, list(range(s, min(n, s + step)))) for s in range(0, n, step)]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_frames_worker, jobs)
    frames = [fr for p in parts for fr in p]
    return pack_frames(frames, dtype=np.complex64)


def scan_traffic(scan_rows, kernel):
    """HBM bytes per scan launch from the committed counter summary, or None when the summary is
    missing or was taken on another version of the scan kernel or another work-item size."""
    try:
        kv = {}
        with open(PMC_SUMMARY[kernel]) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        h = hashlib.sha256()
        for path in SCAN_SRC:
            with open(path, "rb") as fh:
                h.update(fh.read())
        sha = h.hexdigest()
        if kv.get("source_sha256") != sha or int(kv.get("scan_rows", -1)) != scan_rows:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def _timed(run, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        run()
    ev1.record(stream)
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def learned_leg(fs, steps, warmup):
    """The learned-proposal workload by the learned path and by the full scan."""
    import torch
    import paper_2007_14135_amd as nd
    from paper_2007_14135_amd.runner import prepare
    params = np.load(WEIGHTS, allow_pickle=False)
    net = nd.MLP(272, 512, 180, max_batch=8192)
    net.load_params(params)
    fr0 = fs.frames[0]
    F, L = len(fs), fr0.grid_L
    frames = [(0, 0, fr.N, fr.D, int(fs.x_off[f]), int(fs.ld[f])) for f, fr in enumerate(fs.frames)]
    db = prepare([fr0.pos], [(fr0.grid_start, fr0.grid_step, L, 0)], frames, fs.X_flat, "music", "c64", 4,
                 with_spectrum=False, device="cuda:0")
    stream = torch.cuda.current_stream()
    db._windowed_workspace(net)
    ms_full = _timed(lambda: db.run(stream), steps, warmup, stream)
    full = db.host_results()
    ms_learned = _timed(lambda: db.run_learned(net, 6, 1.0, 0.5, stream, window_score=LEARNED_WINDOW_SCORE, local_max_bins=True),
                        steps * 4, warmup, stream)
    learned = db.host_results()
    # honest ablation: a non-learned proposer on the device (MUSIC at 1 deg through the library, its
    # peaks' bins scored 1 by a scatter, then the same windowed search of the fine grid)
    coarse = prepare([fr0.pos], [(-89.5, 1.0, 180, 0)], frames, fs.X_flat, "music", "c64", 4, with_spectrum=False,
                     device="cuda:0", X_device=db.X)
    scores = torch.zeros(F, 180, dtype=torch.float32, device="cuda:0")
    cidx = coarse.peaks.view(torch.int32).view(F, coarse.batch.max_D, 8)[:, :, 0]

    def coarse_run():
        coarse.run(stream)
        scores.zero_()
        scores.scatter_(1, cidx.clamp(min=0).long(), (cidx >= 0).float())
        db.run_windowed(scores, 6, 1.0, 0.5, stream, window_floor=0.5)

    ms_coarse = _timed(coarse_run, steps * 4, warmup, stream)
    coarse_res = db.host_results()
    del coarse
    db.batch.set_timing(True)                      # stage breakdown: a separate, untimed pass
    for _ in range(3):
        db.run_learned(net, 6, 1.0, 0.5, stream, window_score=LEARNED_WINDOW_SCORE, local_max_bins=True)
    stages = {s: db.batch.stage_time(s) for s in ("covariance", "eigen", "proposal", "scan", "peaks")}
    db.batch.set_timing(False)
    fallback = (learned["status"] & nd.ST_FALLBACK_USED) != 0
    miss_coarse = 0
    for f in range(F):
        nf, nc = int(full["npeaks"][f]), int(coarse_res["npeaks"][f])
        a_full = np.sort(full["peaks"][f]["angle_deg"][:nf])
        a_c = np.sort(coarse_res["peaks"][f]["angle_deg"][:nc])
        if nf != nc or (nf and np.max(np.abs(a_full - a_c)) > 0.01 + 1e-9):
            miss_coarse += 1
    miss = 0
    # RMSE over the sources of frames that report D peaks, matched in sorted order
    sq = {"full": [0.0, 0], "learned": [0.0, 0]}
    for f, fr in enumerate(fs.frames):
        nf, nl = int(full["npeaks"][f]), int(learned["npeaks"][f])
        a_full = np.sort(full["peaks"][f]["angle_deg"][:nf])
        a_learned = np.sort(learned["peaks"][f]["angle_deg"][:nl])
        if nf != nl or (nf and np.max(np.abs(a_full - a_learned)) > 0.01 + 1e-9):
            miss += 1
        truth = np.sort(fr.angles_deg)
        for key, a in (("full", a_full), ("learned", a_learned)):
            if len(a) == len(truth):
                sq[key][0] += float(np.sum((a - truth) ** 2))
                sq[key][1] += len(truth)
    return {
        "workload": "ULA M=16, D U{1..4}, SNR U[-5,20] dB, N log-U[256,4096] complex64, %d frames, "
                    "grid [-90,90) at 0.001 deg (L=%d), MUSIC; learned: windows of +-1 deg around the 6 best "
                    "local maxima of the network's bin scores (beyond the first D only those scoring >= %.2f), "
                    "full-grid fallback below score 0.5 or "
                    "when the windows hold fewer than D peaks" % (F, L, LEARNED_WINDOW_SCORE),
        "frames": F,
        "frames_per_s_full": F / (ms_full / 1e3),
        "frames_per_s_learned": F / (ms_learned / 1e3),
        "gain": ms_full / ms_learned,
        "ms_per_batch_full": ms_full,
        "ms_per_batch_learned": ms_learned,
        "full_grid_equiv_points_per_s_learned": F * L / (ms_learned / 1e3),
        "points_per_s_full": F * L / (ms_full / 1e3),
        "miss_rate_vs_full": miss / F,
        "fallback_rate": float(np.mean(fallback)),
        "rmse_deg_vs_truth_full": math.sqrt(sq["full"][0] / max(sq["full"][1], 1)),
        "rmse_deg_vs_truth_learned": math.sqrt(sq["learned"][0] / max(sq["learned"][1], 1)),
        "learned_stage_ms": {k: v[0] / max(v[1], 1) for k, v in stages.items()},
        "coarse_music_proposer": {
            "how": "MUSIC at 1 deg through the library, its peaks' bins as scores (device scatter), then the "
                   "same windowed search; everything on the device",
            "ms_per_batch": ms_coarse, "frames_per_s": F / (ms_coarse / 1e3), "miss_rate_vs_full": miss_coarse / F,
            "fallback_rate": float(np.mean((coarse_res["status"] & nd.ST_FALLBACK_USED) != 0)),
            "learned_gain_over_it": ms_coarse / ms_learned},
    }


def stage_rooflines(stage_ms, frames, alg, prec_scan_peak):
    """Each stage of one step against the roofline of the unit it is bound by, with its own
    algorithmic work (per frame f: covariance 8 M N bytes of complex64 snapshots read, eigensolve
    12 M^3 FP64 flops, scan 8 M K L flops, peak search 4 L bytes of spectrum read)."""
    cov_b = sum(8.0 * fr.M * fr.N for fr in frames)
    eig_f = sum(12.0 * fr.M ** 3 for fr in frames)
    scan_f = sum(8.0 * fr.M * (fr.M - fr.D if alg in ("music", "ev") else 1) * fr.grid_L for fr in frames)
    peak_b = sum(4.0 * fr.grid_L for fr in frames)
    out = {}
    for name, work, unit, peak, bound, scale in (
            ("covariance", cov_b, "GB/s", PEAK_HBM_GBS, "hbm", 1e9),
            ("eigen", eig_f, "TFLOP/s", PEAK_FP64_TFLOPS, "alu", 1e12),
            ("scan", scan_f, "TFLOP/s", prec_scan_peak, "mfma", 1e12),
            ("peaks", peak_b, "GB/s", PEAK_HBM_GBS, "hbm", 1e9)):
        ms = stage_ms.get(name)
        if not ms:
            continue
        ach = work / (ms / 1e3) / scale
        out[name] = {"ms": ms, "bound": bound, "work_per_launch": work, "achieved": ach, "peak": peak, "unit": unit,
                     "frac": ach / peak}
    return out


def _oracle_peaks_worker(args):
    """FP64 oracle over frames of a configuration: (index, peak angles, spectrum or None)."""
    config, idx, alg, keep_spectrum = args
    from threadpoolctl import threadpool_limits
    import oracle
    from synth import make_frame
    out = []
    with threadpool_limits(1):
        for i in idx:
            fr = make_frame(config, i)
            est = oracle.estimate(fr.X, fr.pos, fr.D, fr.grid, alg)
            out.append((i, sorted(est.angles[est.peaks].tolist()), est.P if i in keep_spectrum else None))
    return out


def oracle_peaks_parallel(config, n, alg, keep_spectrum=()):
    import multiprocessing as mp
    workers = max(1, min(len(os.sched_getaffinity(0)), HOST_WORKERS, n))
    jobs = [(config, list(range(w, n, workers)), alg, tuple(keep_spectrum)) for w in range(workers)]
    with mp.get_context("fork").Pool(workers) as pool:
        parts = pool.map(_oracle_peaks_worker, jobs)
    peaks, spectra = {}, {}
    for part in parts:
        for i, pk, P in part:
            peaks[i] = pk
            if P is not None:
                spectra[i] = P
    return peaks, spectra


def _peak_errors(res, n_frames, opeaks):
    worst, mism = 0.0, 0
    for i in range(n_frames):
        n = int(res["npeaks"][i])
        g = sorted(res["peaks"][i]["angle_deg"][:n].tolist())
        o = opeaks[i]
        if len(g) != len(o):
            mism += 1
            continue
        if n:
            worst = max(worst, max(abs(a - b) for a, b in zip(g, o)))
    return worst, mism


def c1_leg(fs1, steps, warmup):
    """The FP64 single-frame workload: latency of one estimate call per algorithm (eager call and
    replay of the captured graph), and the peaks against the oracle."""
    import torch
    import oracle
    from paper_2007_14135_amd.runner import prepare
    fr = fs1.frames[0]
    stream = torch.cuda.current_stream()
    out = {"workload": "ULA M=8, D=2, N=1024 complex128 snapshots, 10 dB, one frame, grid [-90,90) at 0.1 deg "
                       "(L=1800), FP64 throughout", "us_per_frame": {}, "us_per_frame_graph": {},
           "peak_err_deg_vs_oracle": {}}
    for alg in ("phd", "music", "ev", "mn"):
        db = prepare([fr.pos], [(fr.grid_start, fr.grid_step, fr.grid_L, 0)],
                     [(0, 0, fr.N, fr.D, int(fs1.x_off[0]), int(fs1.ld[0]))], fs1.X_flat, alg, "c128", fr.D,
                     device="cuda:0")
        out["us_per_frame"][alg] = 1e3 * _timed(lambda: db.run(stream), steps, warmup, stream)
        g = db.capture()
        out["us_per_frame_graph"][alg] = 1e3 * _timed(lambda: g.launch(stream), steps, warmup, stream)
        res = db.host_results()
        est = oracle.estimate(fr.X, fr.pos, fr.D, fr.grid, alg)
        err, mism = _peak_errors(res, 1, {0: sorted(est.angles[est.peaks].tolist())})
        out["peak_err_deg_vs_oracle"][alg] = err if not mism else None
        g.close()
        del db
    return out


PAPER_TABLE10_MS = {1: 0.438, 30: 0.647, 60: 0.812, 90: 0.924}   # MUSIC end to end, GTX 1660 Ti, float32


def c6_leg(fs6, steps, warmup):
    """The paper's own experiment (Section 5, Tables 8 and 10): 8-element UCA of radius 0.5 lambda,
    two sources at 15 dB, MUSIC over azimuth 0:1:359 deg x 1, 30, 60 or 90 polar angles, FP32-accuracy
    scan (complex64) with FP64 eigensolve and peak refinement.  Per grid: the latency of one frame
    (eager call and graph replay), the throughput of a batch of frames, and the peaks against the
    oracle."""
    import torch
    import oracle
    from synth import EL_GRIDS_2D
    from paper_2007_14135_amd.runner import prepare
    stream = torch.cuda.current_stream()
    fr0 = fs6.frames[0]
    F = len(fs6)
    frames = [(0, 0, fr.N, fr.D, int(fs6.x_off[f]), int(fs6.ld[f])) for f, fr in enumerate(fs6.frames)]
    out = {"workload": "UCA M=8 radius 0.5 lambda, D=2 uncorrelated sources at 15 dB (azimuth U[0,330] deg >= 30 "
                       "deg apart, polar angle U[60,90] deg), N=1024 complex64 snapshots; MUSIC over azimuth 0:1:359 "
                       "deg (circular) x n_polar polar angles at 1 deg; FP32-accuracy scan, FP64 eigensolve and peaks",
           "batch_frames": F, "grids": {}}
    for n_el, el in sorted(EL_GRIDS_2D.items()):
        grid = (fr0.grid_start, fr0.grid_step, fr0.grid_L, 1) + tuple(el)
        one = prepare([fr0.pos], [grid], frames[:1], fs6.X_flat, "music", "c64", 2, device="cuda:0")
        us = 1e3 * _timed(lambda: one.run(stream), steps, warmup, stream)
        g = one.capture()
        us_g = 1e3 * _timed(lambda: g.launch(stream), steps, warmup, stream)
        g.close()
        del one
        db = prepare([fr0.pos], [grid], frames, fs6.X_flat, "music", "c64", 2, device="cuda:0")
        ms_b = _timed(lambda: db.run(stream), max(10, steps // 10), warmup, stream)
        res = db.host_results()
        err, mism = 0.0, 0
        for f in range(min(F, 16)):
            fr = fs6.frames[f]
            est = oracle.estimate_2d(fr.X, fr.pos, fr.D, fr.grid, el, "music", circular_az=True)
            n = int(res["npeaks"][f])
            got = sorted(zip(res["peaks"][f]["angle_deg"][:n].tolist(), res["peaks"][f]["polar_deg"][:n].tolist()))
            ref = sorted(map(tuple, est.peak_angles.tolist()))
            if len(got) != len(ref):
                mism += 1
                continue
            for a, b in zip(got, ref):
                err = max(err, abs(a[0] - b[0]), abs(a[1] - b[1]))
        pts = fr0.grid_L * el[2]
        out["grids"]["360x%d" % n_el] = {
            "points": pts, "us_per_frame": us, "us_per_frame_graph": us_g,
            "batch_ms": ms_b, "frames_per_s_batched": F / (ms_b / 1e3), "points_per_s_batched": F * pts / (ms_b / 1e3),
            "peak_err_deg_vs_oracle": err, "peak_count_mismatch_frames": mism, "oracle_frames_checked": min(F, 16),
            "paper_table10_ms_gtx1660ti_context": PAPER_TABLE10_MS[n_el]}
        del db
    return out


def streaming_leg(fs, db, n_batches=24, depth=3):
    """Snapshots that arrive in pinned host memory (the continuously working system of Section 5.3
    with the pinned buffers of Table 9's third step): each 256-frame batch copied in, estimated and
    its peaks copied out through a pipeline of `depth` slots.  Reported: the PCIe-inclusive rate,
    and the copy-in and estimate times of one batch alone (their maximum bounds the pipelined time
    per batch when they overlap)."""
    import time as _t
    import torch
    import paper_2007_14135_amd as nd
    F = len(fs)
    n_host = 4                                   # host batches cycled through (same frames)
    Xs = [torch.from_numpy(np.ascontiguousarray(fs.X_flat).view(np.float32).copy()).pin_memory()
          for _ in range(n_host)]
    outs = [(torch.empty(F * db.batch.max_D * 32, dtype=torch.uint8).pin_memory(),
             torch.empty(F, dtype=torch.int32).pin_memory(), torch.empty(F, dtype=torch.int32).pin_memory())
            for _ in range(n_host)]
    stream = torch.cuda.current_stream()
    # copy-in alone and estimate alone
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for k in range(8):
        db.X.copy_(Xs[k % n_host], non_blocking=True)
    ev1.record(stream)
    torch.cuda.synchronize()
    h2d_ms = ev0.elapsed_time(ev1) / 8
    comp_ms = _timed(lambda: db.run(stream), 20, 3, stream)
    pipe = nd.Pipeline(db.batch, depth)
    for k in range(depth):                       # warm the slots
        pipe.wait(pipe.submit(Xs[k % n_host], *outs[k % n_host]))
    t0 = _t.perf_counter()
    tickets = []
    for k in range(n_batches):
        if k >= n_host:
            pipe.wait(tickets[k - n_host])      # that host buffer's previous results are in
        tickets.append(pipe.submit(Xs[k % n_host], *outs[k % n_host]))
    for t in tickets[-n_host:]:
        pipe.wait(t)
    wall = _t.perf_counter() - t0
    pipe.close()
    ms = 1e3 * wall / n_batches
    same = all(np.array_equal(o[1].numpy(), outs[0][1].numpy()) for o in outs)
    x_bytes = Xs[0].numel() * 4
    return {"how": "256-frame batches in pinned host memory through nssdoa_pipeline (%d slots): copy-in, estimate, "
                   "copy-out of peaks; host wall clock over %d batches" % (depth, n_batches),
            "ms_per_batch": ms, "frames_per_s_pcie_inclusive": F / (ms / 1e3),
            "points_per_s_pcie_inclusive": F * fs.frames[0].grid_L / (ms / 1e3),
            "copy_in_ms_alone": h2d_ms, "copy_in_GBps": x_bytes / (h2d_ms / 1e3) / 1e9,
            "estimate_ms_alone": comp_ms, "overlap_bound_ms": max(h2d_ms, comp_ms),
            "results_equal_across_batches": bool(same)}


def scan_forms_leg(fs, db, opeaks_frames=8):
    """Alternative Step-5 forms on the benchmark batch (plain FP32 on the vector ALUs, no FP64
    re-evaluation): kernel time per form, and the largest relative error of Q against the oracle
    near the nulls (Q < 5e-4 ||B||_F^2) and elsewhere over the first frames."""
    import torch
    import oracle
    stream = torch.cuda.current_stream()
    db.run(stream)
    out = {"how": "nssdoa_scan_form after the estimate: factored ||B^H a||^2, Table 2's a^H C a, and the "
                  "complement ||a||^2 - ||E_s^H a||^2; FP32, every grid point, %d frames against the oracle"
                  % opeaks_frames}
    ests = [oracle.estimate(fr.X, fr.pos, fr.D, fr.grid, "music") for fr in fs.frames[:opeaks_frames]]
    for form in ("factored", "quadratic", "complement"):
        spec = torch.empty_like(db.spectrum)
        ms = _timed(lambda: db.batch.scan_form(form, db.workspace, spec, stream), 20, 2, stream)
        P = spec.cpu().numpy().astype(np.float64)
        low, rest = 0.0, 0.0
        for f, est in enumerate(ests):
            L = fs.frames[f].grid_L
            rel = np.abs(1.0 / P[db.spec_off[f]:db.spec_off[f] + L] - est.Q) / est.Q
            m = est.Q < 5e-4 * np.sum(np.abs(est.B) ** 2)
            low = max(low, float(rel[m].max()) if m.any() else 0.0)
            rest = max(rest, float(rel[~m].max()))
        out[form] = {"kernel_ms": ms, "max_rel_err_Q_near_nulls": low, "max_rel_err_Q_elsewhere": rest}
    return out


PAPER_TABLE7_MS = {8: {"matlab_svd": 0.018, "eigen_jacobisvd": 0.112, "cusolver_gesvdj": 390.279},
                   64: {"matlab_svd": 0.836, "eigen_jacobisvd": 29.910, "cusolver_gesvdj": 386.242},
                   512: {"matlab_svd": 64.283, "eigen_jacobisvd": 18651.0}}


def eigensolver_leg(sizes=(8, 16, 32, 64), n_batch=256):
    """The eigensolver study of Section 5.2 (Tables 6 and 7) for Step-2 on the covariances of the
    method's frames: each of the library's FP64 Hermitian solvers (bisection + inverse iteration,
    implicit QL, cyclic Jacobi) at M = 8..64, the latency of one matrix and the time per matrix in
    a batch (HIP events around the eigen stage, which also adds the chunk partial covariances and
    builds B), with the Eq. 5 residual ||R - U diag(lambda) U^H|| and ||U^H U - I|| of every matrix
    read back; host LAPACK (numpy eigh, one thread) beside it at 8, 64 and 512."""
    import time as _t
    import torch
    from threadpoolctl import threadpool_limits
    from paper_2007_14135_amd import WS_COV, WS_EVALS, WS_EVECS
    from paper_2007_14135_amd.api import Options
    from paper_2007_14135_amd.runner import prepare
    from synth import make_frames
    stream = torch.cuda.current_stream()
    out = {"how": "covariances of ULA frames (D = 4, N = 1024, SNR U[0,20] dB, 1 deg grid); eigen stage timed with "
                  "HIP events; residuals in FP64 on the host from the solver's own output; Frobenius norms relative "
                  "to ||R||_F", "gpu": {}, "host_lapack": {}, "paper_table7_ms_context": PAPER_TABLE7_MS}
    for M in sizes:
        fs = make_frames("c2", n_frames=n_batch, M=M, N=1024, grid_step=1.0, start=2000)
        fr0 = fs.frames[0]
        frames = [(0, 0, fr.N, fr.D, int(fs.x_off[f]), int(fs.ld[f])) for f, fr in enumerate(fs.frames)]
        for meth in (((("bisect", "auto"),) if M <= 16 else ()) + (("ql", "ql"), ("jacobi", "jacobi"))):
            name, opt = meth
            res_max = orth_max = 0.0
            times = {}
            for n in (1, n_batch):
                db = prepare([fr0.pos], [(fr0.grid_start, fr0.grid_step, fr0.grid_L, 0)], frames[:n], fs.X_flat,
                             "music", "c64", 4, options=Options(eig_method=opt), device="cuda:0")
                db.run(stream)
                db.batch.set_timing(["eigen"])
                for _ in range(20):
                    db.run(stream)
                ms, k = db.batch.stage_time("eigen")
                db.batch.set_timing(False)
                times[n] = ms / k
                if n == n_batch:
                    torch.cuda.synchronize()
                    for f in range(0, n, 8):
                        R = db.workspace_array(WS_COV, f, M * M, np.complex128).reshape(M, M)
                        lam = db.workspace_array(WS_EVALS, f, M, np.float64)
                        U = db.workspace_array(WS_EVECS, f, M * M, np.complex128).reshape(M, M)
                        res_max = max(res_max, float(np.linalg.norm(R - (U * lam) @ U.conj().T) / np.linalg.norm(R)))
                        orth_max = max(orth_max, float(np.linalg.norm(U.conj().T @ U - np.eye(M))))
                del db
            out["gpu"]["%s_M%d" % (name, M)] = {"ms_one_matrix": times[1], "us_per_matrix_in_batch_of_%d" % n_batch:
                                                1e3 * times[n_batch] / n_batch, "eq5_residual_rel_max": res_max,
                                                "orthogonality_max": orth_max}
    rng = np.random.default_rng(7)
    with threadpool_limits(1):
        for M in (8, 64, 512):
            Xh = (rng.standard_normal((M, 4 * M)) + 1j * rng.standard_normal((M, 4 * M))) / np.sqrt(2.0)
            R = Xh @ Xh.conj().T / (4 * M)
            reps = max(3, int(2000 / M))
            t0 = _t.perf_counter()
            for _ in range(reps):
                lam, U = np.linalg.eigh(R)
            ms = 1e3 * (_t.perf_counter() - t0) / reps
            out["host_lapack"]["M%d" % M] = {"ms_one_matrix": ms,
                                            "eq5_residual_rel": float(np.linalg.norm(R - (U * lam) @ U.conj().T)
                                                                      / np.linalg.norm(R))}
    return out


def c3_leg(fs3, steps, warmup, tune_cache, kernel):
    """The uneven workload: 4096 frames (M 8..64, ULA/UCA, uneven D, N, SNR, grid step) as one
    graph launch with the autotuned scan work-item size."""
    import torch
    from paper_2007_14135_amd import autotune
    from paper_2007_14135_amd.api import Options
    from paper_2007_14135_amd.runner import prepare
    arrays, grids, frames, amap, gmap = [], [], [], {}, {}
    for f, fr in enumerate(fs3.frames):
        ka = (fr.geometry, fr.M)
        if ka not in amap:
            amap[ka] = len(arrays)
            arrays.append(fr.pos)
        kg = fr.grid
        if kg not in gmap:
            gmap[kg] = len(grids)
            grids.append((fr.grid_start, fr.grid_step, fr.grid_L, 0))
        frames.append((amap[ka], gmap[kg], fr.N, fr.D, int(fs3.x_off[f]), int(fs3.ld[f])))
    max_D = max(fr.D for fr in fs3.frames)
    rows, _ = autotune.tune(arrays, grids, frames, fs3.X_flat, "music", "c64", max_D, cache_path=tune_cache or None,
                            options=Options(c64_scan=kernel))
    db = prepare(arrays, grids, frames, fs3.X_flat, "music", "c64", max_D, with_spectrum=False, device="cuda:0",
                 options=Options(scan_rows=rows, c64_scan=kernel))
    stream = torch.cuda.current_stream()
    g = db.capture()
    ms = _timed(lambda: g.launch(stream), steps, warmup, stream)
    res = db.host_results()
    db.batch.set_timing(True)
    for _ in range(3):
        db.run(stream)
    stages = {s: db.batch.stage_time(s) for s in ("covariance", "eigen", "scan", "peaks")}
    db.batch.set_timing(False)
    stage_ms = {k: v[0] / max(v[1], 1) for k, v in stages.items()}
    g.close()
    F = len(fs3)
    points = sum(fr.grid_L for fr in fs3.frames)
    peak = PEAK_FP32_MFMA_TFLOPS if kernel == "fp32" else PEAK_FP16_MFMA_TFLOPS
    return {"workload": "4096 uneven frames: M in {8,16,32,64}, ULA or UCA, D U{1..M/4}, N log-U[256,8192], "
                        "SNR U[-5,20] dB, grid step in {0.1,0.01,0.002} deg over [-90,90), MUSIC, complex64; one "
                        "graph launch, autotuned scan work items",
            "frames": F, "points": points, "snapshot_bytes": int(fs3.X_flat.nbytes), "c64_scan": kernel,
            "scan_rows": rows or 384, "ms_per_batch": ms, "frames_per_s": F / (ms / 1e3),
            "points_per_s": points / (ms / 1e3), "stage_ms": stage_ms,
            "stage_roofline": stage_rooflines(stage_ms, fs3.frames, "music", peak),
            "status_nonzero_frames": int(np.count_nonzero(res["status"] & 0x7))}


def c4_leg(fs4, steps, warmup, tune_cache, opeaks, ospectra):
    """The precision workload (64 frames, M=64, 180000-point grid) with the BF16 and the FP16
    scan: throughput, spectrum dB error against the FP64 oracle at every point of the frames the
    oracle's spectra were kept for, and the peak error in degrees on every frame."""
    import torch
    from paper_2007_14135_amd import autotune
    from paper_2007_14135_amd.runner import prepare
    fr0 = fs4.frames[0]
    arrays = [fr0.pos]
    grids = [(fr0.grid_start, fr0.grid_step, fr0.grid_L, 0)]
    frames = [(0, 0, fr.N, fr.D, int(fs4.x_off[f]), int(fs4.ld[f])) for f, fr in enumerate(fs4.frames)]
    stream = torch.cuda.current_stream()
    F, L = len(fs4), fr0.grid_L
    K = fr0.M - fr0.D
    out = {"workload": "ULA M=64, D=8 (gap >= 1 deg), N=16384 complex64 snapshots, 5 dB, 64 frames, grid "
                       "[-90,90) at 0.001 deg (L=180000), MUSIC; 16-bit matrix-core scan with FP32 accumulation, "
                       "FP64 eigensolve, FP64 re-evaluation of low-Q points and FP64 peak refinement",
           "frames": F}
    X_dev = None
    for prec in ("bf16", "f16"):
        rows, _ = autotune.tune(arrays, grids, frames, fs4.X_flat, "music", prec, fr0.D, cache_path=tune_cache or None)
        from paper_2007_14135_amd.api import Options
        db = prepare(arrays, grids, frames, fs4.X_flat, "music", prec, fr0.D, device="cuda:0", X_device=X_dev,
                     options=Options(scan_rows=rows))
        X_dev = db.X
        ms = _timed(lambda: db.run(stream), steps, warmup, stream)
        res = db.host_results()
        db.batch.set_timing(True)
        for _ in range(2):
            db.run(stream)
        stages = {s: db.batch.stage_time(s) for s in ("covariance", "eigen", "scan", "peaks")}
        db.batch.set_timing(False)
        stage_ms = {k: v[0] / max(v[1], 1) for k, v in stages.items()}
        err, mism = _peak_errors(res, F, opeaks)
        dbe = []
        for i, P in ospectra.items():
            dbe.append(np.abs(10.0 * np.log10(res["spectra"][i].astype(np.float64) / P)))
        dbe = np.concatenate(dbe) if dbe else np.zeros(1)
        scan_s = stage_ms["scan"] / 1e3
        out[prec] = {"scan_rows": rows, "ms_per_batch": ms, "frames_per_s": F / (ms / 1e3),
                     "points_per_s": F * L / (ms / 1e3), "stage_ms": stage_ms,
                     "scan_roofline": {"bound": "mfma", "achieved": 8.0 * fr0.M * K * L * F / scan_s / 1e12,
                                       "peak": PEAK_FP16_MFMA_TFLOPS, "unit": "TFLOP/s",
                                       "frac": 8.0 * fr0.M * K * L * F / scan_s / 1e12 / PEAK_FP16_MFMA_TFLOPS},
                     "db_err_vs_oracle": {"frames": sorted(ospectra), "median": float(np.median(dbe)),
                                          "p99": float(np.percentile(dbe, 99)), "max": float(dbe.max())},
                     "peak_err_deg_max_vs_oracle": err, "peak_count_mismatch_frames": mism,
                     "status_nonzero_frames": int(np.count_nonzero(res["status"]))}
        del db
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--alg", default="music", choices=["music", "ev", "mn", "phd"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-repeats", type=int, default=4, help="passes of the oracle over the 256 frames")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--learned-frames", type=int, default=8192)
    ap.add_argument("--no-tune", action="store_true", help="skip the scan autotuner (default work items)")
    ap.add_argument("--c64-scan", default="split3", choices=["split16", "fp32", "split3"],
                    help="matrix-core kernel of the complex64 scan (FP32 operands, or FP16 split operands of two or "
                         "three parts)")
    ap.add_argument("--no-c1", action="store_true", help="skip the FP64 single-frame latency leg")
    ap.add_argument("--no-c3", action="store_true", help="skip the 4096-frame uneven-batch leg")
    ap.add_argument("--no-c4", action="store_true", help="skip the 16-bit precision leg")
    ap.add_argument("--no-2d", action="store_true", help="skip the paper's 2-D (azimuth x polar angle) leg")
    ap.add_argument("--no-stream", action="store_true", help="skip the pinned-host streaming pipeline leg")
    ap.add_argument("--no-forms", action="store_true", help="skip the alternative scan-form ablation leg")
    ap.add_argument("--no-eig", action="store_true", help="skip the eigensolver study leg")
    ap.add_argument("--no-compare", action="store_true", help="skip the step with the other C64 scan kernel")
    ap.add_argument("--streams", type=int, default=4,
                    help="batches in flight: step k runs on stream k mod S with its own copy of the snapshots, "
                         "workspace and outputs (1 = one batch at a time)")
    ap.add_argument("--tune-cache", default=TUNE_CACHE, help="JSON cache of autotuner choices")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="finish with one device-to-device copy of this many MiB (the reference of the HBM "
                         "byte counters: a plain copy reads and writes exactly that much)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the path is per-frame data parallel and this build "
              "measures one GPU's share (see DESIGN.md for how it shards); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    # host work first, in fork pools, before anything touches the GPU
    from synth import make_frames
    fs = make_frames("c2")
    F = len(fs)
    fr0 = fs.frames[0]
    L, M, D = fr0.grid_L, fr0.M, fr0.D
    cb = opeaks = None
    if not args.no_cpu_baseline:
        cb, opeaks = cpu_baseline("c2", list(range(F)), args.alg, L, args.cpu_repeats)
    fs5 = None
    if not args.no_learned and os.path.exists(WEIGHTS):
        fs5 = make_frames_parallel("c5", args.learned_frames)
    fs1 = make_frames("c1") if not args.no_c1 else None
    fs6 = make_frames("c6", n_frames=256) if not args.no_2d else None
    fs3 = make_frames_parallel("c3", 4096) if not args.no_c3 else None
    fs4 = o4 = None
    if not args.no_c4:
        fs4 = make_frames_parallel("c4", 64)
        o4 = oracle_peaks_parallel("c4", 64, "music", keep_spectrum=(0, 21, 42, 63))

    import torch
    from paper_2007_14135_amd import autotune
    from paper_2007_14135_amd.api import Options
    from paper_2007_14135_amd.runner import prepare

    torch.cuda.set_device(0)
    arrays = [fr0.pos]
    grids = [(fr0.grid_start, fr0.grid_step, L, 0)]
    frames = [(0, 0, fr.N, fr.D, int(fs.x_off[f]), int(fs.ld[f])) for f, fr in enumerate(fs.frames)]
    rows, tune_ms = 0, {}
    if not args.no_tune:
        rows, tune_ms = autotune.tune(arrays, grids, frames, fs.X_flat, args.alg, "c64", D,
                                      cache_path=args.tune_cache or None,
                                      options=Options(c64_scan=args.c64_scan))
    db = prepare(arrays, grids, frames, fs.X_flat, args.alg, "c64", D, device="cuda:0",
                 options=Options(scan_rows=rows, c64_scan=args.c64_scan))
    stream = torch.cuda.current_stream()
    S = max(1, args.streams)

    def in_flight(kernel, rows_k, first):
        """S batches of the same frames, each with its own snapshot copy, workspace and outputs."""
        out = [first]
        for _ in range(S - 1):
            out.append(prepare(arrays, grids, frames, fs.X_flat, args.alg, "c64", D, device="cuda:0",
                               options=Options(scan_rows=rows_k, c64_scan=kernel), X_device=first.X.clone()))
        return out

    streams = [stream] + [torch.cuda.Stream() for _ in range(S - 1)]   # default priority

    def run_steps(batches, k_steps):
        fork = torch.cuda.Event()
        fork.record(stream)
        for s_ in streams[1:]:
            s_.wait_event(fork)
        for k in range(k_steps):
            batches[k % S].run(streams[k % S])
        for s_ in streams[1:]:
            stream.wait_stream(s_)

    dbs = in_flight(args.c64_scan, rows, db)
    run_steps(dbs, max(args.warmup, S))
    torch.cuda.synchronize()

    # timed region: K steps, step k on stream k mod S (whole batches in flight)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    t0 = time.perf_counter()
    run_steps(dbs, args.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    res = db.host_results()
    for extra in dbs[1:]:                         # every in-flight copy computed the same results
        r2 = extra.host_results()
        assert np.array_equal(r2["npeaks"], res["npeaks"]) and np.array_equal(r2["status"], res["status"])
    del dbs[1:]

    # one batch at a time: latency per step and the scan kernel's roofline (HIP events around
    # the scan launch on its stream, the GPU otherwise idle)
    db.batch.set_timing(["scan"])
    lat_ms = _timed(lambda: db.run(stream), args.steps, 1, stream)
    scan_ms, scan_n = db.batch.stage_time("scan")
    db.batch.set_timing(False)
    # stage breakdown from a separate, untimed pass (events around every stage)
    db.batch.set_timing(True)
    for _ in range(min(args.steps, 10)):
        db.run(stream)
    stages = {s: db.batch.stage_time(s) for s in ("covariance", "eigen", "scan", "peaks")}
    db.batch.set_timing(False)

    K = M - D if args.alg in ("music", "ev") else 1
    scan_flops = 8.0 * M * K * L * F                 # algorithmic, per launch (= per step)
    scan_avg_s = scan_ms / scan_n / 1e3
    achieved_tflops = scan_flops / scan_avg_s / 1e12
    points = F * L
    value = points / (ms_step / 1e3)
    split = args.c64_scan != "fp32"
    peak = PEAK_FP16_MFMA_TFLOPS if split else PEAK_FP32_MFMA_TFLOPS
    # matrix-core flops executed: a split forms each FP32-accuracy product from 3 or 6 FP16 products
    mfma_flops = scan_flops * MFMA_PRODUCTS[args.c64_scan]
    stage_ms = {k: v[0] / max(v[1], 1) for k, v in stages.items()}
    stage_roof = stage_rooflines(stage_ms, fs.frames, args.alg, peak)
    # the single-kernel stage that takes longest in one step (the peak stage is three kernels)
    dominant = max(("covariance", "eigen", "scan"), key=lambda k: stage_ms[k])

    # the same step with the other C64 scan kernels (their own tuned work items), for comparison
    other = None
    if not args.no_compare:
        other = {}
        for okern in [k for k in ("fp32", "split16", "split3") if k != args.c64_scan]:
            orows = 0
            if not args.no_tune:
                orows, _ = autotune.tune(arrays, grids, frames, fs.X_flat, args.alg, "c64", D,
                                         cache_path=args.tune_cache or None, options=Options(c64_scan=okern))
            db2 = prepare(arrays, grids, frames, fs.X_flat, args.alg, "c64", D, device="cuda:0",
                          options=Options(scan_rows=orows, c64_scan=okern), X_device=db.X)
            dbs2 = in_flight(okern, orows, db2)
            run_steps(dbs2, max(args.warmup, S))
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run_steps(dbs2, args.steps)
            e1.record(stream)
            torch.cuda.synchronize()
            oms = e0.elapsed_time(e1) / args.steps
            del dbs2[1:]
            olat = _timed(lambda: db2.run(stream), args.steps, 1, stream)
            db2.batch.set_timing(["scan"])
            for _ in range(min(args.steps, 10)):
                db2.run(stream)
            osc, osn = db2.batch.stage_time("scan")
            db2.batch.set_timing(False)
            o_avg = osc / max(osn, 1)
            o_peak = PEAK_FP32_MFMA_TFLOPS if okern == "fp32" else PEAK_FP16_MFMA_TFLOPS
            ores = db2.host_results()
            other[okern] = {"scan_rows": orows or 384, "value": points / (oms / 1e3), "ms_per_step": oms,
                            "latency_ms_one_batch": olat, "scan_kernel": SCAN_KERNEL[okern],
                            "scan_avg_launch_ms": o_avg,
                            "scan_roofline_frac": scan_flops / (o_avg / 1e3) / 1e12 / o_peak,
                            "scan_mfma_frac": scan_flops * MFMA_PRODUCTS[okern] / (o_avg / 1e3) / 1e12 / o_peak,
                            "scan_peak_tflops": o_peak,
                            "peaks_equal_headline": bool(np.array_equal(ores["npeaks"], res["npeaks"]) and all(
                                np.array_equal(ores["peaks"][i]["idx"][:n], res["peaks"][i]["idx"][:n])
                                for i, n in enumerate(res["npeaks"])))}
            del db2

    scan_roofline = {
        "kernel": SCAN_KERNEL[args.c64_scan],
        "bound": "mfma",
        "achieved": achieved_tflops,
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": achieved_tflops / peak,
        "traffic": scan_traffic(rows or 384, args.c64_scan) if args.alg == "music" else None,
        "algorithmic_flops_per_launch": scan_flops,
        "mfma_flops_per_launch": mfma_flops,
        "mfma_frac": mfma_flops / scan_avg_s / 1e12 / peak,
        "avg_launch_ms": scan_avg_s * 1e3,
    }
    if dominant == "scan":
        roofline = scan_roofline
    else:
        # another stage dominates: its own kernel against its own unit, the scan's figures beside
        sr = stage_roof[dominant]
        roofline = {"kernel": STAGE_KERNEL[dominant], "bound": sr["bound"], "achieved": sr["achieved"],
                    "peak": sr["peak"], "unit": sr["unit"], "frac": sr["frac"], "traffic": None,
                    "avg_launch_ms": sr["ms"], "scan": scan_roofline}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(args.warmup, S),
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16x2-split/f32-acc" if args.c64_scan == "split16" else "f32",
        "dtype_note": "complex64 snapshots; FP64 covariance accumulation, eigensolve, noise subspace and peak "
                      "refinement; scan: " + SCAN_DESC[args.c64_scan],
        "data": "synthetic",
        "frames_per_s": F / (ms_step / 1e3),
        "batches_in_flight": S,
        "latency_ms_one_batch": lat_ms,
        "value_one_batch_at_a_time": points / (lat_ms / 1e3),
        "config": {
            "workload": "ULA M=16, D=4, N=4096 complex64 snapshots, SNR U[0,20] dB, 256 frames, "
                        "grid [-90,90) at 0.01 deg (L=18000), %s; FP64 covariance/eigensolve/refinement, "
                        "FP32-accuracy matrix-core scan (%s)" % (args.alg.upper(), SCAN_DESC[args.c64_scan]),
            "frames": F, "M": M, "D": D, "N": fr0.N, "L": L, "alg": args.alg,
            "scan_rows": rows or 384, "c64_scan": args.c64_scan,
        },
        "autotune": {"knob": "scan_rows", "chosen": rows or 384,
                     "scan_ms_by_candidate": {str(k): v for k, v in tune_ms.items()}},
        "stage_ms": stage_ms,
        "stage_roofline": stage_roof,
        "dominant_kernel_stage": dominant,
        "roofline": roofline,
        "other_c64_scans": other,
        "host_wall_s": wall,
        "status_nonzero_frames": int(np.count_nonzero(res["status"])),
    }

    if cb is not None:
        out["cpu_baseline"] = cb
        # peak error of the GPU path vs the oracle on the same frames (degrees)
        worst, mism = 0.0, 0
        for i in range(F):
            oidx, oang = opeaks[i]
            n = int(res["npeaks"][i])
            gang = sorted(res["peaks"][i]["angle_deg"][:n].tolist())
            oang = sorted(oang)
            if len(gang) != len(oang):
                mism += 1
                continue
            worst = max(worst, max(abs(a - b) for a, b in zip(gang, oang)))
        out["peak_err_deg_max_vs_oracle"] = worst
        out["peak_count_mismatch_frames"] = mism
    if not args.no_stream:
        out["streaming_pcie"] = streaming_leg(fs, db)
    if not args.no_forms and args.alg == "music":
        out["scan_forms_ablation"] = scan_forms_leg(fs, db)
    if not args.no_eig:
        out["eigensolver_study"] = eigensolver_leg()
    if fs5 is not None:
        del db
        torch.cuda.empty_cache()
        out["learned_vs_full"] = learned_leg(fs5, 3, 1)
    if fs1 is not None:
        out["c1_fp64_single_frame"] = c1_leg(fs1, 200, 10)
    if fs6 is not None:
        out["paper_2d_uca8"] = c6_leg(fs6, 200, 10)
    if fs3 is not None:
        out["c3_uneven_batch"] = c3_leg(fs3, 5, 2, args.tune_cache, args.c64_scan)
        del fs3
        torch.cuda.empty_cache()
    if fs4 is not None:
        out["c4_precision"] = c4_leg(fs4, 5, 1, args.tune_cache, o4[0], o4[1])
        torch.cuda.empty_cache()
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = n
    print(json.dumps(out))


if __name__ == "__main__":
    main()
