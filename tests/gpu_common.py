"""Helpers for the GPU parity tests: synthetic frames -> C-ABI inputs, and oracle comparisons."""

from __future__ import annotations

import numpy as np

import oracle

NEAR_TIE_REL = 1e-9      # FP64 values closer than this (relative) may order either way


def frameset_inputs(fs):
    """(arrays, grids, frames, X_flat) for a synth FrameSet: one array per distinct geometry and
    one grid per distinct (start, step, L)."""
    arrays, akey = [], {}
    grids, gkey = [], {}
    frames = []
    for f, fr in enumerate(fs.frames):
        ka = (fr.M, fr.pos.tobytes())
        if ka not in akey:
            akey[ka] = len(arrays)
            arrays.append(fr.pos)
        kg = (fr.grid_start, fr.grid_step, fr.grid_L)
        if kg not in gkey:
            gkey[kg] = len(grids)
            grids.append((fr.grid_start, fr.grid_step, fr.grid_L, 0))
        frames.append((akey[ka], gkey[kg], fr.N, fr.D, int(fs.x_off[f]), int(fs.ld[f])))
    return arrays, grids, frames, fs.X_flat


def oracle_frame(fr, alg, circular=False):
    return oracle.estimate(fr.X, fr.pos, fr.D, fr.grid, alg, circular=circular)


def spectrum_rel_err(P_gpu, est):
    P_gpu = np.asarray(P_gpu, dtype=np.float64)
    return np.abs(P_gpu - est.P) / np.abs(est.P)


def peaks_match(gpu_idx, est, D, tol=NEAR_TIE_REL):
    """True when the GPU's selected indices equal the oracle's, up to FP64 near-ties: a GPU index
    may replace an oracle index when it is the neighbour straddling the same maximum, or another
    oracle peak, and the two oracle values differ by less than `tol` relative."""
    gpu = [int(i) for i in gpu_idx if i >= 0]
    ref = [int(i) for i in est.peaks]
    if sorted(gpu) == sorted(ref):
        return True, 0
    if len(gpu) != len(ref):
        return False, 0
    P = est.P
    ties = 0
    unmatched_ref = [r for r in ref if r not in gpu]
    for g in [g for g in gpu if g not in ref]:
        ok = False
        for r in list(unmatched_ref):
            if abs(P[g] - P[r]) <= tol * abs(P[r]) and (abs(g - r) == 1 or g in set(est.all_peaks.tolist())):
                unmatched_ref.remove(r)
                ok = True
                break
        if not ok:
            return False, ties
        ties += 1
    return True, ties
