"""The scan autotuner on the GPU: it measures every candidate, and a batch scheduled with the
chosen work-item size gives the same peaks as the default schedule (spectra within FP32
rounding: the size only moves frames' rows within the MFMA tiles)."""

import numpy as np
import pytest

from synth import make_frames
from gpu_common import frameset_inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_autotune_choice_keeps_results(tmp_path):
    from paper_2007_14135_amd import autotune
    from paper_2007_14135_amd.api import Options
    from paper_2007_14135_amd.runner import prepare
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fs = make_frames("c2", n_frames=32, N=1024)
    arrays, grids, frames, X = frameset_inputs(fs)
    cache = str(tmp_path / "tune.json")
    best, t = autotune.tune(arrays, grids, frames, X, "music", "c64", 4, candidates=(64, 128, 384, 1024),
                            cache_path=cache, reps=3)
    print("autotune: %s -> %d" % ({k: round(v, 4) for k, v in t.items()}, best), flush=True)
    assert best in (64, 128, 384, 1024) and set(t) == {64, 128, 384, 1024}
    again, t2 = autotune.tune(arrays, grids, frames, X, "music", "c64", 4, cache_path=cache)
    assert again == best and t2 == {}                      # from the cache
    ref = prepare(arrays, grids, frames, X, "music", "c64", 4)
    ref.run()
    r0 = ref.host_results()
    for rows in (64, 1024):
        db = prepare(arrays, grids, frames, X, "music", "c64", 4, options=Options(scan_rows=rows))
        db.run()
        r1 = db.host_results()
        assert np.array_equal(r0["npeaks"], r1["npeaks"])
        assert np.array_equal(r0["peaks"]["idx"], r1["peaks"]["idx"])
        for a, b in zip(r0["spectra"], r1["spectra"]):
            assert np.max(np.abs(a - b) / a) <= 2e-6
