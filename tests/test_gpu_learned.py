"""What the trained proposal network gains over the method without it.

On 1024 fresh frames of the learned-proposal workload (frame indices never used in training; ULA
M=16, D in 1..4, N in 256..4096, SNR -5..20 dB, 0.001 deg grid) the learned path (6 windows of
+-1 deg, full-grid fallback below score 0.5) is compared with the full scan on the same GPU:
  * a miss is a frame whose peaks differ from the full scan's by more than 0.01 deg (or in
    number); the full scan itself is at parity with the FP64 oracle (test_gpu_parity);
  * the learned path must be faster than the full scan, with at most 3 % misses;
  * without training (the same network at its initial weights) the windows are in the wrong
    places: the miss rate is far higher, so the gain is the network's;
  * a non-learned proposer (the library's own MUSIC scan at 1 deg, its D peaks as windows) is
    reported beside it as the honest ablation.
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
    ms = _timed(lambda: db.run_learned(trained, 6, 1.0, 0.5))
    res = db.host_results()
    miss = _miss_rate(fs, full, res)
    fb = float(np.mean((res["status"] & ST_FALLBACK) != 0))
    print("trained: %.3f ms vs full scan %.3f ms (gain %.2fx), miss rate %.4f, fallback %.4f"
          % (ms, ms_full, ms_full / ms, miss, fb), flush=True)
    assert miss <= 0.03
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


def test_coarse_scan_proposer_ablation(setup):
    # non-learned proposal: the library's MUSIC at 1 deg (bin centres -89.5 + b), its D peaks
    # become the windows (score 1 at each peak's bin, 0 elsewhere)
    nd, fs, db, trained, full, ms_full = setup
    from paper_2007_14135_amd.runner import prepare
    fr0 = fs.frames[0]
    frames = [(0, 0, fr.N, fr.D, int(fs.x_off[f]), int(fs.ld[f])) for f, fr in enumerate(fs.frames)]
    coarse = prepare([fr0.pos], [(-89.5, 1.0, 180, 0)], frames, fs.X_flat, "music", "c64", 4, with_spectrum=False)
    coarse.X = db.X
    scores = torch.zeros(len(fs), 180, dtype=torch.float32, device="cuda")

    def propose_and_scan():
        coarse.run()
        torch.cuda.synchronize()
        r = coarse.host_results()
        s = np.zeros((len(fs), 180), dtype=np.float32)
        for f in range(len(fs)):
            for j in range(int(r["npeaks"][f])):
                s[f, int(r["peaks"][f]["idx"][j])] = 1.0
        scores.copy_(torch.from_numpy(s))
        db.run_windowed(scores, 6, 1.0, 0.5)

    ms = _timed(propose_and_scan, reps=2)
    res = db.host_results()
    miss = _miss_rate(fs, full, res)
    fb = float(np.mean((res["status"] & ST_FALLBACK) != 0))
    print("coarse 1-deg MUSIC proposer: %.3f ms (host round trip included), miss rate %.4f, fallback %.4f"
          % (ms, miss, fb), flush=True)
