"""nssdoa_estimate_noalloc against nssdoa_estimate, through the C ABI.

The no-allocation entry point runs the same kernels on the library's per-device workspace array,
so its outputs must equal nssdoa_estimate's bit for bit on the same inputs.  Two calls in a row,
the second on a smaller batch, check that nothing of the first call's contents in the shared
array leaks into the second; a batch whose workspace exceeds the array is rejected on the host.
"""

import numpy as np
import pytest

from synth import make_frames
from gpu_common import frameset_inputs, oracle_frame, peaks_match, spectrum_rel_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _prepare(fs, alg, prec, with_spectrum=True):
    from paper_2007_14135_amd.runner import prepare
    arrays, grids, frames, X = frameset_inputs(fs)
    return prepare(arrays, grids, frames, X, alg, prec, max(fr.D for fr in fs.frames), with_spectrum=with_spectrum)


def _outputs(db):
    torch.cuda.synchronize()
    out = dict(peaks=db.peaks.cpu().numpy().copy(), npeaks=db.npeaks.cpu().numpy().copy(),
               status=db.status.cpu().numpy().copy())
    if db.spectrum is not None:
        out["spectrum"] = db.spectrum.cpu().numpy().copy()
    return out


def _same(a, b, label):
    for k in a:
        assert a[k].dtype == b[k].dtype and a[k].shape == b[k].shape, (label, k)
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), (label, k)


def _fill(db):
    # outputs start from garbage, so stale values cannot pass for results
    db.peaks.fill_(0xA5)
    db.npeaks.fill_(-7)
    db.status.fill_(-1)
    if db.spectrum is not None:
        db.spectrum.fill_(float("nan"))


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_noalloc_equals_estimate_on_two_calls(prec):
    _need_gpu()
    print("noalloc: %s, 48 frames of the 16-element workload, then 6 smaller frames" % prec, flush=True)
    big = make_frames("c2", n_frames=48, N=2048, grid_step=0.02)
    small = make_frames("c2", n_frames=6, N=512, grid_step=0.05, start=100)
    if prec == "c128":
        big = make_frames("c1", n_frames=8, N=1024)
        small = make_frames("c1", n_frames=3, N=256, start=20)
    results = []
    for fs in (big, small):
        db = _prepare(fs, "music", prec)
        _fill(db)
        db.run_noalloc()
        got = _outputs(db)
        _fill(db)
        db.run()
        ref = _outputs(db)
        _same(got, ref, (prec, len(fs)))
        results.append((fs, got, db))
    # the smaller second call is also at parity with the oracle (sampled frames)
    fs, got, db = results[1]
    res = db.host_results()
    for f in range(len(fs)):
        fr = fs.frames[f]
        est = oracle_frame(fr, "music")
        rel = spectrum_rel_err(res["spectra"][f], est)
        assert rel.max() <= (1e-4 if prec == "c64" else 1e-9), (f, float(rel.max()))
        n = int(res["npeaks"][f])
        ok, _ = peaks_match(res["peaks"][f]["idx"][:n], est, fr.D)
        assert ok and n == len(est.peaks), f


def test_noalloc_without_caller_spectrum():
    _need_gpu()
    print("noalloc: spectrum kept in the workspace array", flush=True)
    fs = make_frames("c2", n_frames=16, N=1024, grid_step=0.05, start=300)
    db = _prepare(fs, "ev", "c64", with_spectrum=False)
    _fill(db)
    db.run_noalloc()
    got = _outputs(db)
    _fill(db)
    db.run()
    _same(got, _outputs(db), "no spectrum")


def test_noalloc_rejects_a_batch_beyond_the_array():
    _need_gpu()
    from paper_2007_14135_amd import _abi
    from paper_2007_14135_amd.api import noalloc_workspace_limit
    limit = noalloc_workspace_limit()
    assert limit == 64 << 20
    # 96 frames on a 0.001 deg grid with the spectrum in the workspace: 69 MB of it
    fs = make_frames("c2", n_frames=96, N=256, grid_step=0.001, start=500)
    db = _prepare(fs, "music", "c64", with_spectrum=False)
    assert db.batch.workspace_size() > limit
    _fill(db)
    with pytest.raises(_abi.NssdoaError) as ei:
        db.run_noalloc()
    assert ei.value.status == _abi.EINVAL
    assert "no-allocation workspace" in str(ei.value)
    torch.cuda.synchronize()
    assert np.all(db.npeaks.cpu().numpy() == -7)      # nothing was enqueued
