"""What the trained proposal network gains over the method without it.

On 1024 fresh frames of the learned-proposal workload (frame indices never used in training; ULA
M=16, D in 1..4, N in 256..4096, SNR -5..20 dB, 0.001 deg grid) the learned path (windows of
+-1 deg around the 6 best local maxima of the network's scores, beyond the first D only those
scoring at least 0.05; full-grid fallback below score 0.5) is compared with the full scan on the
same GPU:
  * a miss is a frame whose peaks differ from the full scan's by more than 0.01 deg (or in
    number); the full scan itself is at parity with the FP64 oracle (test_gpu_parity);
  * the learned path must be faster than the full scan, with at most one missed frame in 1024
    (frames whose windows hold fewer than D peaks are searched again over the whole grid on the
    device, so a proposal that misses a source costs time, not accuracy);
  * without training (the same network at its initial weights) the windows are in the wrong
    places: the miss rate is far higher, or every frame falls back, so the gain is the network's;
  * a non-learned proposer run entirely on the device (the library's own MUSIC scan at 1 deg,
    its D peaks turned into bin scores by a scatter on the device, then the same windowed search
    with windows at those D bins only) is the honest ablation.  It never falls back, and the
    learned path does not beat it: 0.93x of its speed at 8192 frames, 0.64x at 1024 (the learned
    path's extra cost is its whole-grid fallbacks); the gate is no more misses than it, and at most
    twice its time.
"""

import os

import numpy as np
import pytest

from synth import make_frames

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2007_14135_amd", "weights", "proposal_ula16.npy")
ST_FALLBACK = 0x20
WINDOW_SCORE = 0.05


def _timed(fn, reps=3):
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _miss_rate(fs, ref, res):
    miss = 0
    for f in range(len(fs)):
        n0, n1 = int(ref["npeaks"][f]), int(res["npeaks"][f])
        a0 = np.sort(ref["peaks"][f]["angle_deg"][:n0])
        a1 = np.sort(res["peaks"][f]["angle_deg"][:n1])
        if n0 != n1 or (n0 and np.max(np.abs(a0 - a1)) > 0.01 + 1e-9):
            miss += 1
    return miss / len(fs)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2007_14135_amd as nd
    from paper_2007_14135_amd.runner import prepare
    assert os.path.exists(WEIGHTS), "trained weights missing: " + WEIGHTS
    fs = make_frames("c5", n_frames=1024)
    fr0 = fs.frames[0]
    frames = [(0, 0, fr.N, fr.D, int(fs.x_off[f]), int(fs.ld[f])) for f, fr in enumerate(fs.frames)]
    db = prepare([fr0.pos], [(fr0.grid_start, fr0.grid_step, fr0.grid_L, 0)], frames, fs.X_flat, "music",
                 "c64", 4, with_spectrum=False)
    trained = nd.MLP(272, 512, 180, max_batch=1024)
    trained.load_params(np.load(WEIGHTS, allow_pickle=False))
    db._windowed_workspace(trained)
    ms_full = _timed(lambda: db.run())
    full = db.host_results()
    return nd, fs, db, trained, full, ms_full


def test_trained_network_beats_the_full_scan(setup):
    nd, fs, db, trained, full, ms_full = setup
    ms = _timed(lambda: db.run_learned(trained, 6, 1.0, 0.5, window_score=WINDOW_SCORE, local_max_bins=True))
    res = db.host_results()
    miss = _miss_rate(fs, full, res)
    fb = float(np.mean((res["status"] & ST_FALLBACK) != 0))
    print("trained: %.3f ms vs full scan %.3f ms (gain %.2fx), miss rate %.4f, fallback %.4f"
          % (ms, ms_full, ms_full / ms, miss, fb), flush=True)
    assert miss * len(fs) <= 1
    assert ms < ms_full


def test_untrained_network_misses(setup):
    nd, fs, db, trained, full, ms_full = setup
    from paper_2007_14135_amd.init import he_uniform
    raw = nd.MLP(272, 512, 180, max_batch=1024)
    raw.load_params(he_uniform(1, (272, 512, 512, 180)))
    res = None
    ms = _timed(lambda: db.run_learned(raw, 6, 1.0, 0.5))
    res = db.host_results()
    miss = _miss_rate(fs, full, res)
    fb = float(np.mean((res["status"] & ST_FALLBACK) != 0))
    print("untrained: %.3f ms, miss rate %.4f, fallback %.4f" % (ms, miss, fb), flush=True)
    # either the windows miss (no fallback) or everything falls back (no gain): never both good
    assert miss > 0.2 or ms > 0.5 * ms_full


def coarse_proposer(fs, db):
    """The non-learned proposal, on the device: MUSIC at 1 deg (bin centres -89.5 + b) through the
    library, its peaks' bins scored 1 (others 0) by a scatter on the device, then the windowed
    search of the fine grid with those scores."""
    from paper_2007_14135_amd.runner import prepare
    fr0 = fs.frames[0]
    frames = [(0, 0, fr.N, fr.D, int(fs.x_off[f]), int(fs.ld[f])) for f, fr in enumerate(fs.frames)]
    coarse = prepare([fr0.pos], [(-89.5, 1.0, 180, 0)], frames, fs.X_flat, "music", "c64", 4, with_spectrum=False,
                     X_device=db.X)
    F = len(fs)
    scores = torch.zeros(F, 180, dtype=torch.float32, device="cuda")
    # peak records are 32 bytes: int32 idx, int32 reserved, double angle, double value, double polar
    idx = coarse.peaks.view(torch.int32).view(F, coarse.batch.max_D, 8)[:, :, 0]

    def run():
        coarse.run()
        scores.zero_()
        scores.scatter_(1, idx.clamp(min=0).long(), (idx >= 0).float())
        db.run_windowed(scores, 6, 1.0, 0.5, window_floor=0.5)

    return run


def test_coarse_scan_proposer_ablation(setup):
    nd, fs, db, trained, full, ms_full = setup
    run = coarse_proposer(fs, db)
    ms = _timed(run)
    res = db.host_results()
    miss = _miss_rate(fs, full, res)
    fb = float(np.mean((res["status"] & ST_FALLBACK) != 0))
    ms_l = _timed(lambda: db.run_learned(trained, 6, 1.0, 0.5, window_score=WINDOW_SCORE, local_max_bins=True))
    res_l = db.host_results()
    miss_l = _miss_rate(fs, full, res_l)
    print("coarse 1-deg MUSIC proposer (on the device): %.3f ms, miss rate %.4f, fallback %.4f; learned %.3f ms, "
          "miss rate %.4f" % (ms, miss, fb, ms_l, miss_l), flush=True)
    # the coarse MUSIC proposer is a strong baseline: it never falls back (its scores are exact
    # source bins), while the network sends its unsure frames (about 1-2 %) to whole-grid scans,
    # whose fixed cost weighs more on 1024 frames than on the 8192 of the workload; the gate here
    # is accuracy, with a regression bound on time (the benchmark reports the 8192-frame ratio)
    print("learned / coarse time: %.3f" % (ms_l / ms), flush=True)
    assert ms_l <= 2.0 * ms
    assert miss_l <= miss + 1.0 / len(fs)
