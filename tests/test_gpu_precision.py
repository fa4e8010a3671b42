"""GPU parity of the 16-bit (BF16 / FP16) matrix-core scans against the FP64 oracle.

Bound (derived from the arithmetic): operands rounded to 16 bits with FP32 accumulation give a
relative error of Q of about 2u sqrt(||B||_F^2 / Q); points with Q < tau ||B||_F^2 (tau = 2e-3)
are re-evaluated in FP64, so the worst remaining error is at Q = tau ||B||_F^2.  A numpy emulation
of the rounding on 64-element frames gives at most 0.071 dB (BF16, u = 2^-9) and 0.012 dB (FP16,
u = 2^-11); the gates below are twice that.  Peak indices must equal the oracle's (FP64 near-tie
rule) because candidates are re-picked from FP64 windows.
"""

import numpy as np
import pytest

from synth import make_frame, make_frames
from synth.frames import FrameSet, pack_frames
from gpu_common import frameset_inputs, oracle_frame, peaks_match

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DB_GATE = {"bf16": 0.15, "f16": 0.03}


def _run(fs, alg, prec, max_D):
    from paper_2007_14135_amd.runner import prepare
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    arrays, grids, frames, X = frameset_inputs(fs)
    db = prepare(arrays, grids, frames, X, alg, prec, max_D)
    print("run: %s %s frames=%d M=%s L=%s" % (alg, prec, len(fs), sorted({f.M for f in fs.frames}),
                                               sorted({f.grid_L for f in fs.frames})), flush=True)
    db.run()
    return db, db.host_results()


def _check(frames, res, idx, alg, prec):
    worst_db, worst_deg = 0.0, 0.0
    for f, i in enumerate(idx):
        fr = frames[f]
        est = oracle_frame(fr, alg)
        P = res["spectra"][i].astype(np.float64)
        db = np.abs(10.0 * np.log10(P / est.P))
        worst_db = max(worst_db, float(db.max()))
        assert db.max() <= DB_GATE[prec], (prec, alg, f, float(db.max()), int(np.argmax(db)))
        n = int(res["npeaks"][i])
        pk = res["peaks"][i]
        assert n == len(est.peaks)
        ok, _ = peaks_match(pk["idx"][:n], est, fr.D)
        assert ok, (prec, alg, f, pk["idx"][:n].tolist(), est.peaks.tolist())
        for r in range(n):
            j = int(pk["idx"][r])
            assert abs(pk["value"][r] - est.P[j]) <= 1e-8 * est.P[j]
        gdeg = np.sort(pk["angle_deg"][:n])
        worst_deg = max(worst_deg, float(np.max(np.abs(gdeg - np.sort(est.peak_angles)))) if n else 0.0)
    print("%s %s: max |dB error| %.4f, max peak error %.4f deg" % (prec, alg, worst_db, worst_deg), flush=True)


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_lp_scan_music_64_elements(prec):
    # 64-element frames of the precision workload at a 0.01 deg grid (71 angle tiles, ragged tail)
    fs = make_frames("c4", n_frames=4, N=4096, grid_step=0.01)
    db, res = _run(fs, "music", prec, 8)
    assert np.all(res["status"] == 0)
    _check(fs.frames, res, range(4), "music", prec)


@pytest.mark.parametrize("alg", ["ev", "mn", "phd"])
def test_lp_scan_other_methods_fp16(alg):
    fs = make_frames("c4", n_frames=2, N=4096, grid_step=0.01)
    db, res = _run(fs, alg, "f16", 8)
    _check(fs.frames, res, range(2), alg, "f16")


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_lp_scan_16_elements(prec):
    fs = make_frames("c2", n_frames=6, N=2048)
    db, res = _run(fs, "music", prec, 4)
    _check(fs.frames, res, range(6), "music", prec)


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_lp_scan_mixed_sizes(prec):
    frames = []
    for i in range(16):
        fr = make_frame("c3", i, N=512)
        if fr.grid_L > 18000:
            fr = make_frame("c3", i, N=512, grid_step=0.01)
        frames.append(fr)
    fs = pack_frames(frames, dtype=np.complex64)
    db, res = _run(fs, "music", prec, 16)
    _check(frames, res, range(16), "music", prec)


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_c4_full_precision_workload(prec):
    # The full precision workload: 64 frames, M=64, N=16384, L=180000 (0.001 deg).  Four frames
    # are compared point by point with the oracle; every frame must report 8 peaks, status 0.
    fs = make_frames("c4")
    db, res = _run(fs, "music", prec, 8)
    assert np.all(res["status"] == 0), res["status"]
    assert np.all(res["npeaks"] == 8)
    idx = [0, 21, 42, 63]
    _check([fs.frames[i] for i in idx], res, idx, "music", prec)
