"""Training of the learned proposal network on the GPU with the library's own kernels.

Data: frames of the learned-proposal workload (ULA M = 16 at half-wavelength spacing, D uniform in
1..4, SNR uniform in [-5, 20] dB, N log-uniform in [256, 4096], angles in [-70, 70] deg at least
5 deg apart) drawn by the seeded generator from frame indices that the evaluation batch never
uses (evaluation takes frames 0..8191; training starts at TRAIN_FIRST_FRAME).
Every quantity derived from the snapshots comes from the library, on the device, as the learned
path computes it at inference: per chunk of frames the snapshots go through nssdoa_estimate
(MUSIC at 0.1 deg: covariance, eigensolve, scan, peaks), then nssdoa_features reads the same
covariances.
Inputs: the covariance features, upper triangle i <= j of R M / trace(R) with real and imaginary
parts interleaved (272 values at M = 16).
Labels: multi-hot 1-degree bins (bin b covers [-90 + b, -89 + b) deg) of the D peaks of that MUSIC
scan (method-matched: the windows must contain the peaks the full scan would report).
Optimiser: Adam (beta 0.9 / 0.999, eps 1e-8) on mean binary cross-entropy in
nssdoa_mlp_train_step, minibatches in a seeded order, cosine learning-rate decay.  The blob of
nssdoa_mlp_save (parameters and Adam state) is written after every epoch; --resume continues
from one.

    python -m paper_2007_14135_amd.train --frames 1000000 --epochs 8 \\
        --out paper_2007_14135_amd/weights/proposal_ula16.npy
"""

from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

N_FEAT, WIDTH, N_BINS, M = 272, 512, 180, 16
TRAIN_FIRST_FRAME = 1_000_000
LABEL_GRID = (-90.0, 0.1, 1800)


def _generate(args):
    """Frames [start, start + count) of the learned-proposal workload: their snapshots packed back
    to back (complex64), per-frame offsets and snapshot counts, and source counts."""
    start, count = args
    from threadpoolctl import threadpool_limits
    from synth import make_frame
    from synth.frames import pack_frames
    with threadpool_limits(1):
        fs = pack_frames([make_frame("c5", start + k) for k in range(count)], dtype=np.complex64)
    N = np.array([fr.N for fr in fs.frames], dtype=np.int32)
    D = np.array([fr.D for fr in fs.frames], dtype=np.int32)
    return start, fs.X_flat, fs.x_off, N, D


def ula_positions(m: int) -> np.ndarray:
    pos = np.zeros((m, 3))
    pos[:, 0] = 0.5 * np.arange(m)
    return pos


def generate(first: int, n: int, workers: int, chunk: int = 1024, log=print):
    """Features and MUSIC bin labels of n frames: a fork pool draws the snapshots (before anything
    touches the GPU in this process's children), the library turns each chunk into features and
    labels on the device."""
    import torch
    from . import api, _abi
    plan = api.Plan([ula_positions(M)], [LABEL_GRID + (0,)])
    labels = np.zeros((n, N_BINS), dtype=np.float32)
    D_all = np.empty(n, dtype=np.int32)
    jobs = [(first + s, min(chunk, n - s)) for s in range(0, n, chunk)]
    t0 = time.time()
    done = 0
    with mp.get_context("fork").Pool(workers) as pool:     # forked before this process touches the GPU
        feats = torch.empty((n, N_FEAT), dtype=torch.float32, device="cuda")
        for start, X_flat, x_off, N, D in pool.imap_unordered(_generate, jobs):
            o, c = start - first, len(D)
            frames = [(0, 0, int(N[k]), int(D[k]), int(x_off[k]), int(N[k]), 0) for k in range(c)]
            b = api.Batch(plan, "music", "c64", frames, 4)
            X = torch.from_numpy(np.ascontiguousarray(X_flat).view(np.float32)).cuda()
            peaks = torch.empty(c * 4 * _abi.PEAK_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
            npk = torch.empty(c, dtype=torch.int32, device="cuda")
            st = torch.empty(c, dtype=torch.int32, device="cuda")
            ws = torch.empty(b.workspace_size(), dtype=torch.uint8, device="cuda")
            b.estimate(X, None, peaks, npk, st, ws)
            b.features(ws, feats[o:o + c])
            pk = api.decode_peaks(peaks.cpu().numpy(), c, 4)
            cnt = npk.cpu().numpy()
            for r in range(c):
                for j in range(int(cnt[r])):
                    a = float(pk[r, j]["angle_deg"])
                    labels[o + r, int(min(max(math.floor(a + 90.0), 0), N_BINS - 1))] = 1.0
            D_all[o:o + c] = D
            b.close()
            done += c
            if done % (chunk * 64) < chunk or done == n:
                log("features and labels of %d / %d frames (%.0f s)" % (done, n, time.time() - t0))
    plan.close()
    return feats, labels, D_all


def window_recall(logits: np.ndarray, labels: np.ndarray, topk: int = 6) -> float:
    """Fraction of label bins lying within one bin of one of the topk best bins (a +-1 deg window
    around a bin centre covers the neighbouring bins' centres)."""
    top = np.argsort(-logits, axis=1, kind="stable")[:, :topk]
    hit = tot = 0
    for r in range(len(labels)):
        lab = np.nonzero(labels[r])[0]
        tot += len(lab)
        hit += sum(1 for b in lab if np.min(np.abs(top[r] - b)) <= 1)
    return hit / max(tot, 1)


def train(args) -> dict:
    log = lambda s: print(s, flush=True)  # noqa: E731
    workers = args.workers or min(16, len(os.sched_getaffinity(0)))
    import torch
    from . import api
    Xd, labels, D = generate(args.first_frame, args.frames, workers, log=log)
    n_val = max(1024, args.frames // 100)
    n_tr = args.frames - n_val
    Yd = torch.from_numpy(labels).cuda()
    net = api.MLP(N_FEAT, WIDTH, N_BINS, max_batch=max(args.batch, 1024))
    if args.resume:
        with open(args.resume, "rb") as fh:
            net.load(fh.read())
    else:
        from .init import he_uniform
        net.load_params(he_uniform(args.seed, (N_FEAT, WIDTH, WIDTH, N_BINS)))
    steps_per_epoch = n_tr // args.batch
    total = steps_per_epoch * args.epochs
    step = net.state()[3]
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    history = []
    t0 = time.time()
    while step < total:
        epoch = step // steps_per_epoch
        perm = torch.from_numpy(np.random.default_rng(args.seed + 1 + epoch).permutation(n_tr)).cuda()
        acc, nacc = 0.0, 0
        for k in range(step % steps_per_epoch, steps_per_epoch):
            lr = args.lr_min + 0.5 * (args.lr - args.lr_min) * (1.0 + math.cos(math.pi * step / total))
            idx = perm[k * args.batch:(k + 1) * args.batch]
            net.train_step(Xd.index_select(0, idx), Yd.index_select(0, idx), lr, loss)
            step += 1
            if k % 64 == 0:
                acc += float(loss.item())
                nacc += 1
        val_logits = torch.empty(n_val, N_BINS, dtype=torch.float32, device="cuda")
        for s in range(0, n_val, 1024):
            e = min(n_val, s + 1024)
            net.forward(Xd[n_tr + s:n_tr + e], val_logits[s:e])
        vl = val_logits.cpu().numpy()
        vy = labels[n_tr:]
        z = vl.astype(np.float64)
        vloss = float(np.mean(np.maximum(z, 0) - z * vy + np.log1p(np.exp(-np.abs(z)))))
        rec = window_recall(vl, vy)
        fb = float(np.mean(vl.max(axis=1) < 0.0))
        history.append(dict(epoch=epoch + 1, train_loss=acc / max(nacc, 1), val_loss=vloss, val_recall6=rec,
                            val_fallback=fb, seconds=time.time() - t0))
        log("epoch %d: train loss %.5f  val loss %.5f  val recall@6 %.4f  fallback %.4f  (%.0f s)"
            % (epoch + 1, acc / max(nacc, 1), vloss, rec, fb, time.time() - t0))
        if args.checkpoint:
            with open(args.checkpoint, "wb") as fh:
                fh.write(net.save())
    params = net.state()[0]
    meta = dict(frames=args.frames, first_frame=args.first_frame, validation_frames=n_val, epochs=args.epochs,
                batch=args.batch, lr=args.lr, lr_min=args.lr_min, seed=args.seed, sizes=[N_FEAT, WIDTH, WIDTH, N_BINS],
                label_grid=list(LABEL_GRID), history=history)
    if args.out:
        os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
        np.save(args.out, params)
        with open(os.path.splitext(args.out)[0] + ".json", "w") as fh:
            json.dump(meta, fh, indent=1)
        log("wrote %s" % args.out)
    return meta


def main(argv=None):
    p = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    p.add_argument("--frames", type=int, default=1_000_000)
    p.add_argument("--first-frame", type=int, default=TRAIN_FIRST_FRAME)
    p.add_argument("--epochs", type=int, default=8)
    p.add_argument("--batch", type=int, default=1024)
    p.add_argument("--lr", type=float, default=1e-3)
    p.add_argument("--lr-min", type=float, default=5e-5)
    p.add_argument("--seed", type=int, default=20071413)
    p.add_argument("--workers", type=int, default=0)
    p.add_argument("--out", default="")
    p.add_argument("--checkpoint", default="")
    p.add_argument("--resume", default="")
    train(p.parse_args(argv))


if __name__ == "__main__":
    sys.exit(main())
