"""The uneven batched workload at full size: 4096 independent frames with M in {8, 16, 32, 64},
ULA or UCA, D in 1..M/4, N log-uniform in [256, 8192], SNR -5..20 dB and grid steps of 0.1, 0.01
and 0.002 deg, estimated (MUSIC, FP32 matrix-core scan) by one graph launch.

Checked on every frame: status bits, peak counts, peaks inside the grid and in descending value
order.  Checked point by point against the FP64 oracle on one frame of every (M, grid step)
combination: spectrum within 1e-4 relative, peak indices identical (FP64 near-tie rule).
"""

import numpy as np
import pytest

from synth import make_frame
from synth.frames import pack_frames
from gpu_common import frameset_inputs, oracle_frame, peaks_match, spectrum_rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ST_NONFINITE, ST_NOCONV, ST_FEWER = 0x1, 0x2, 0x8


def test_uneven_4096_frames_one_graph_launch():
    from paper_2007_14135_amd.runner import prepare
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    frames = [make_frame("c3", i) for i in range(4096)]
    fs = pack_frames(frames, dtype=np.complex64)
    arrays, grids, fr_tab, X = frameset_inputs(fs)
    print("uneven batch: %d frames, %.2f GB of snapshots, %d arrays, %d grids, sum L = %d" % (
        len(frames), fs.X_flat.nbytes / 1e9, len(arrays), len(grids), sum(f.grid_L for f in frames)), flush=True)
    db = prepare(arrays, grids, fr_tab, X, "music", "c64", 16)
    g = db.capture()
    g.launch()
    res = db.host_results()
    st = res["status"]
    assert not np.any(st & (ST_NONFINITE | ST_NOCONV)), np.nonzero(st & (ST_NONFINITE | ST_NOCONV))[0][:10]
    for f, fr in enumerate(frames):
        n = int(res["npeaks"][f])
        assert 0 <= n <= fr.D
        assert bool(st[f] & ST_FEWER) == (n < fr.D)
        pk = res["peaks"][f]
        idx = pk["idx"][:n]
        assert np.all((idx > 0) & (idx < fr.grid_L - 1))
        assert np.all(np.diff(pk["value"][:n]) <= 0)
        assert np.all(pk["idx"][n:] == -1)
    # one frame of every (M, grid) combination against the oracle
    seen, worst, checked = set(), 0.0, 0
    for f, fr in enumerate(frames):
        key = (fr.M, fr.grid_L)
        if key in seen:
            continue
        seen.add(key)
        est = oracle_frame(fr, "music")
        err = spectrum_rel_err(res["spectra"][f], est)
        worst = max(worst, float(err.max()))
        assert err.max() <= 1e-4, (f, key, float(err.max()))
        n = int(res["npeaks"][f])
        assert n == len(est.peaks), (f, key)
        ok, _ = peaks_match(res["peaks"][f]["idx"][:n], est, fr.D)
        assert ok, (f, key, res["peaks"][f]["idx"][:n].tolist(), est.peaks.tolist())
        checked += 1
    print("uneven batch: %d frames checked against the oracle (every M x grid), max rel spectrum error %.3e"
          % (checked, worst), flush=True)
    g.close()
