"""GPU parity of the 2-D (azimuth x polar angle) scans against the FP64 oracle, through the C ABI.

The paper's test scenario (Section 5): an 8-element UCA of radius 0.5 lambda, two uncorrelated
sources at 15 dB, scanned over azimuth 0:1:359 deg (circular) times 1, 30, 60 or 90 polar angles
(the 360 x {1, 30, 60, 90} grids of Tables 8 and 10).  Bars as for the 1-D scans: the FP32-accuracy
scan (complex64) within 1e-4 relative of oracle.estimate_2d at every grid point, the FP64 scan
(complex128) within 1e-9, and the selected peaks (row-major indices, azimuth and polar angle)
identical to the oracle's 8-neighbour rule up to FP64 near-ties.
"""

import numpy as np
import pytest

import oracle
from synth import EL_GRIDS_2D, make_frames
from synth.frames import pack_frames, make_frame

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

NEAR_TIE_REL = 1e-9


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run2d(fs, el, alg, prec, circular=1, extra_1d=None):
    """One batch of the frames of fs on the 2-D grid (azimuth of each frame's grid x el); with
    extra_1d, a second grid (a 1-D one) is added and the frames listed there use it."""
    from paper_2007_14135_amd.runner import prepare
    _need_gpu()
    fr0 = fs.frames[0]
    grids = [(fr0.grid_start, fr0.grid_step, fr0.grid_L, circular, el[0], el[1], el[2])]
    gid = [0] * len(fs)
    if extra_1d is not None:
        grids.append(extra_1d[0])
        for f in extra_1d[1]:
            gid[f] = 1
    frames = [(0, gid[f], fr.N, fr.D, int(fs.x_off[f]), int(fs.ld[f])) for f, fr in enumerate(fs.frames)]
    print("run2d: %s %s frames=%d grid=%s x %s" % (alg, prec, len(fs), fr0.grid, el), flush=True)
    db = prepare([fr0.pos], grids, frames, fs.X_flat, alg, prec, max(fr.D for fr in fs.frames))
    db.run()
    return db.host_results()


def _peaks_match_2d(got, est):
    ref = [int(i) for i in est.peaks]
    got = [int(i) for i in got]
    if sorted(got) == sorted(ref):
        return True
    if len(got) != len(ref):
        return False
    P = est.P.ravel()
    allp = set(est.all_peaks.tolist())
    for g in [g for g in got if g not in ref]:
        # a GPU peak may replace an oracle one only when both are oracle peaks of equal FP64 value
        if g not in allp or not any(abs(P[g] - P[r]) <= NEAR_TIE_REL * P[r] for r in ref if r not in got):
            return False
    return True


def _check(fs, res, el, alg, prec, circular=True, frames=None):
    tol = 1e-4 if prec == "c64" else 1e-9
    worst = 0.0
    for f in (range(len(fs)) if frames is None else frames):
        fr = fs.frames[f]
        est = oracle.estimate_2d(fr.X, fr.pos, fr.D, fr.grid, el, alg, circular_az=circular)
        P = np.asarray(res["spectra"][f], dtype=np.float64).reshape(est.P.shape)
        rel = np.abs(P - est.P) / est.P
        worst = max(worst, float(rel.max()))
        assert rel.max() <= tol, (alg, prec, el, f, float(rel.max()), int(np.argmax(rel)))
        n = int(res["npeaks"][f])
        pk = res["peaks"][f]
        assert n == len(est.peaks), (alg, prec, el, f, n, est.peaks.tolist())
        assert _peaks_match_2d(pk["idx"][:n], est), (alg, prec, el, f, pk["idx"][:n].tolist(), est.peaks.tolist())
        az, pol = est.angles
        for r in range(n):
            i = int(pk["idx"][r])
            assert pk["angle_deg"][r] == az[i % len(az)] and pk["polar_deg"][r] == pol[i // len(az)]
            assert abs(pk["value"][r] - est.P.ravel()[i]) <= 1e-8 * est.P.ravel()[i]
        assert np.all(pk["idx"][n:] == -1)
        expect = 0x8 if len(est.peaks) < fr.D else 0     # NSSDOA_ST_FEWER_PEAKS
        assert int(res["status"][f]) == expect, (f, int(res["status"][f]))
    print("%s %s %s: max rel spectrum error %.3e" % (alg, prec, el, worst), flush=True)


@pytest.mark.parametrize("n_el", [1, 30, 60, 90])
@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_paper_scenario_grids(n_el, prec):
    fs = make_frames("c6", n_frames=4)
    if prec == "c128":
        fs = pack_frames(fs.frames, dtype=np.complex128)
    el = EL_GRIDS_2D[n_el]
    res = _run2d(fs, el, "music", prec)
    _check(fs, res, el, "music", prec)


@pytest.mark.parametrize("alg", ["phd", "ev", "mn"])
def test_other_methods_on_the_largest_grid(alg):
    fs = make_frames("c6", n_frames=3, start=10)
    el = EL_GRIDS_2D[90]
    res = _run2d(fs, el, alg, "c64")
    _check(fs, res, el, alg, "c64")


def test_non_circular_azimuth_and_ragged_rows():
    # a sector that does not wrap, an azimuth count that is not a multiple of the 256-point items,
    # and polar angles ending in the horizontal plane, where a planar array's spectrum is
    # stationary in phi, so peaks can sit on the grid's last row
    frames = [make_frame("c6", 30 + i, grid_step=0.7) for i in range(3)]
    fs = pack_frames(frames, dtype=np.complex64)
    fr0 = fs.frames[0]
    assert fr0.grid_L % 256 != 0
    el = (70.0, 0.5, 41)
    res = _run2d(fs, el, "music", "c64", circular=0)
    _check(fs, res, el, "music", "c64", circular=False)


def test_mixed_1d_and_2d_frames_in_one_batch():
    # 2-D frames and 1-D frames of the same array share one batch; each follows its own grid
    from gpu_common import oracle_frame, peaks_match
    fs = make_frames("c6", n_frames=4, start=50)
    el = EL_GRIDS_2D[30]
    one_d = ((0.0, 0.25, 1440, 1), [1, 3])
    res = _run2d(fs, el, "music", "c64", extra_1d=one_d)
    _check(fs, res, el, "music", "c64", frames=[0, 2])
    for f in (1, 3):
        fr = fs.frames[f]
        est = oracle.estimate(fr.X, fr.pos, fr.D, (0.0, 0.25, 1440), "music", circular=True)
        rel = np.abs(res["spectra"][f] - est.P) / est.P
        assert rel.max() <= 1e-4, (f, float(rel.max()))
        n = int(res["npeaks"][f])
        ok, _ = peaks_match(res["peaks"][f]["idx"][:n], est, fr.D)
        assert ok and n == len(est.peaks)
        assert np.all(res["peaks"][f]["polar_deg"][:n] == 90.0)


def test_windowed_estimation_rejects_2d_grids():
    from paper_2007_14135_amd import _abi
    from paper_2007_14135_amd.runner import prepare
    _need_gpu()
    fs = make_frames("c6", n_frames=2, start=70)
    fr0 = fs.frames[0]
    grids = [(fr0.grid_start, fr0.grid_step, fr0.grid_L, 1) + EL_GRIDS_2D[30]]
    frames = [(0, 0, fr.N, fr.D, int(fs.x_off[f]), int(fs.ld[f])) for f, fr in enumerate(fs.frames)]
    db = prepare([fr0.pos], grids, frames, fs.X_flat, "music", "c64", 2)
    scores = torch.zeros(2, 180, dtype=torch.float32, device="cuda")
    with pytest.raises(_abi.NssdoaError) as e:
        db.run_windowed(scores, 6, 1.0, 0.5)
    assert e.value.status == _abi.EUNSUPPORTED
