"""GPU parity of the HIP path against the FP64 oracle, called through the C ABI.

Bars: covariance bit-exact for Gaussian-integer snapshots; eigen-pairs within FP64 rounding;
FP32 spectra within 1e-4 relative of the oracle at every grid point (after the library's FP64
re-evaluation of low-Q points); FP64 spectra within 1e-9; peak indices identical up to FP64
near-ties (relative 1e-9, see gpu_common).
"""

import sys

import numpy as np
import pytest

import oracle
from synth import make_frame, make_frames
from synth.frames import FrameSet, integer_snapshots, pack_frames, ula_positions, uca_positions, Frame
from gpu_common import frameset_inputs, oracle_frame, peaks_match, spectrum_rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(fs, alg, prec, max_D=None, with_spectrum=True, options=None):
    from paper_2007_14135_amd.runner import prepare
    _need_gpu()
    arrays, grids, frames, X = frameset_inputs(fs)
    if max_D is None:
        max_D = max(fr.D for fr in fs.frames)
    db = prepare(arrays, grids, frames, X, alg, prec, max_D, with_spectrum=with_spectrum, options=options)
    print("run: %s %s frames=%d M=%s L=%s" % (alg, prec, len(fs), sorted({f.M for f in fs.frames}),
                                               sorted({f.grid_L for f in fs.frames})), flush=True)
    db.run()
    return db, db.host_results()


def _check_frames(fs, res, alg, tol, peak_val_tol, label):
    worst, ties = 0.0, 0
    for f, fr in enumerate(fs.frames):
        est = oracle_frame(fr, alg)
        rel = spectrum_rel_err(res["spectra"][f], est)
        worst = max(worst, float(rel.max()))
        assert rel.max() <= tol, (label, f, float(rel.max()), int(np.argmax(rel)))
        n = int(res["npeaks"][f])
        pk = res["peaks"][f]
        assert n == len(est.peaks), (label, f, n, len(est.peaks))
        ok, t = peaks_match(pk["idx"][:n], est, fr.D)
        ties += t
        assert ok, (label, f, pk["idx"][:n].tolist(), est.peaks.tolist())
        for r in range(n):
            i = int(pk["idx"][r])
            assert abs(pk["value"][r] - est.P[i]) <= peak_val_tol * est.P[i], (label, f, r)
            assert pk["angle_deg"][r] == est.angles[i]
        assert np.all(pk["idx"][n:] == -1)
    print("%s: max rel spectrum error %.3e, near-ties %d" % (label, worst, ties), flush=True)
    return worst


def test_covariance_bit_exact_integer_snapshots():
    # Gaussian-integer snapshots: every partial sum is an exact integer in FP64, so R = S / N is
    # the correctly rounded quotient of exact integers; ragged N spans several LDS tiles/chunks.
    rng = np.random.default_rng(11)
    frames = []
    for i, (M, N) in enumerate([(8, 1000), (16, 4097), (16, 257), (32, 3000), (64, 1500), (8, 1)]):
        X = integer_snapshots(rng, M, N)
        frames.append(Frame(M=M, N=N, D=1, pos=ula_positions(M), geometry="ula", snr_db=0.0, sigma2=1.0,
                            angles_deg=np.zeros(1), grid_start=-90.0, grid_step=1.0, grid_L=180, X=X))
    fs = pack_frames(frames, dtype=np.complex64)
    db, res = _run(fs, "music", "c64")
    from paper_2007_14135_amd import WS_COV
    for f, fr in enumerate(frames):
        R = db.workspace_array(WS_COV, f, fr.M * fr.M, np.complex128).reshape(fr.M, fr.M)
        Xi = fr.X.astype(np.complex128)
        Sre = np.rint((Xi @ Xi.conj().T).real).astype(np.int64)
        Sim = np.rint((Xi @ Xi.conj().T).imag).astype(np.int64)
        exp = Sre.astype(np.float64) / fr.N + 1j * (Sim.astype(np.float64) / fr.N)
        assert np.array_equal(R, exp), (f, np.max(np.abs(R - exp)))


@pytest.mark.parametrize("sizes", [[(8, 1000), (16, 4097), (16, 257), (8, 1), (16, 63), (16, 64), (8, 65)],
                                   [(8, 1), (8, 4096), (8, 129), (8, 700)]])
def test_covariance_bit_exact_on_the_vector_kernel(sizes):
    # batches with M <= 16 (complex64) accumulate on the FP64 vector ALUs: the same exact sums
    rng = np.random.default_rng(12)
    frames = []
    for M, N in sizes:
        X = integer_snapshots(rng, M, N)
        frames.append(Frame(M=M, N=N, D=1, pos=ula_positions(M), geometry="ula", snr_db=0.0, sigma2=1.0,
                            angles_deg=np.zeros(1), grid_start=-90.0, grid_step=1.0, grid_L=180, X=X))
    fs = pack_frames(frames, dtype=np.complex64)
    db, res = _run(fs, "music", "c64")
    from paper_2007_14135_amd import WS_COV
    for f, fr in enumerate(frames):
        R = db.workspace_array(WS_COV, f, fr.M * fr.M, np.complex128).reshape(fr.M, fr.M)
        Xi = fr.X.astype(np.complex128)
        Sre = np.rint((Xi @ Xi.conj().T).real).astype(np.int64)
        Sim = np.rint((Xi @ Xi.conj().T).imag).astype(np.int64)
        exp = Sre.astype(np.float64) / fr.N + 1j * (Sim.astype(np.float64) / fr.N)
        assert np.array_equal(R, exp), (f, np.max(np.abs(R - exp)))


def test_eigendecomposition_matches_oracle():
    from paper_2007_14135_amd import WS_EVALS, WS_EVECS, WS_COV
    fs = make_frames("c2", n_frames=6, N=1024)
    db, res = _run(fs, "music", "c64")
    for f, fr in enumerate(fs.frames):
        M = fr.M
        R = db.workspace_array(WS_COV, f, M * M, np.complex128).reshape(M, M)
        lam = db.workspace_array(WS_EVALS, f, M, np.float64)
        U = db.workspace_array(WS_EVECS, f, M * M, np.complex128).reshape(M, M)
        Ro = oracle.covariance(fr.X)
        assert np.allclose(R, Ro, rtol=0, atol=1e-13 * np.abs(Ro).max())
        lo, Uo = oracle.eig_desc(Ro)
        assert np.all(np.diff(lam) <= 0)
        assert np.allclose(lam, lo, rtol=1e-11, atol=1e-13 * lo[0])
        assert np.linalg.norm(R - U @ np.diag(lam) @ U.conj().T) <= 1e-13 * np.linalg.norm(R)
        assert np.linalg.norm(U.conj().T @ U - np.eye(M)) <= 1e-13 * M
        D = fr.D
        Pn = U[:, D:] @ U[:, D:].conj().T
        Pno = Uo[:, D:] @ Uo[:, D:].conj().T
        assert np.abs(Pn - Pno).max() <= 1e-10
    assert np.all(res["status"] & 0x3 == 0)


def _custom_frame(X):
    M, N = X.shape
    return Frame(M=M, N=N, D=1, pos=ula_positions(M), geometry="ula", snr_db=0.0, sigma2=1.0,
                 angles_deg=np.zeros(1), grid_start=-90.0, grid_step=1.0, grid_L=180, X=X)


@pytest.mark.parametrize("M", [16, 32])
def test_covariance_matrix_core_bound_per_entry(M):
    # The matrix-core covariance forms Re R from Z Z^T - P - P^T (Z = Re x + Im x in FP64), whose
    # products can round: each entry may deviate from the FP64 oracle by at most 6u sqrt(R_ii R_jj)
    # beyond the accumulation's own rounding.  Checked per entry, normalised by sqrt(R_ii R_jj),
    # on ordinary frames, on rows 2^-8 .. 2^7 apart in scale, and on imaginary parts 2^-20 below
    # the real parts (where Z's sums round); a one-row-block and a two-row-block batch.
    from paper_2007_14135_amd import WS_COV
    rng = np.random.default_rng(21)
    frames = []
    for i in range(3):
        base = make_frame("c2", 40 + i, N=2048).X.astype(np.complex128)
        X = np.vstack([base, base[::-1] * np.exp(0.3j)])[:M] if M > 16 else base
        if i == 1:
            X = X * (2.0 ** (np.arange(M) % 16 - 8.0))[:, None]
        if i == 2:
            X = X.real + 1j * X.imag * 2.0 ** -20
        frames.append(_custom_frame(X.astype(np.complex64)))
    frames.append(_custom_frame((rng.standard_normal((M, 777)) + 1j * rng.standard_normal((M, 777))).astype(np.complex64)))
    fs = pack_frames(frames, dtype=np.complex64)
    db, res = _run(fs, "music", "c64")
    worst = 0.0
    for f, fr in enumerate(frames):
        R = db.workspace_array(WS_COV, f, M * M, np.complex128).reshape(M, M)
        Ro = oracle.covariance(fr.X)
        d = np.sqrt(np.outer(Ro.diagonal().real, Ro.diagonal().real))
        err = np.abs(R - Ro) / d
        worst = max(worst, float(err.max()))
        # 6u from Z's products plus the FP64 accumulation's rounding (observed 7.8e-16): 1e-14
        assert err.max() <= 1e-14, (f, float(err.max()))
        # the imaginary part comes from exact products alone: relative to its own scale
        im_scale = np.abs(Ro.imag).max()
        assert np.abs(R.imag - Ro.imag).max() <= 1e-13 * im_scale, f
    print("covariance M=%d: worst per-entry error %.2e of sqrt(R_ii R_jj)" % (M, worst), flush=True)


@pytest.mark.parametrize("method", ["auto", "ql", "jacobi"])
def test_eigensolvers_across_sizes_and_structures(method):
    # Both solvers against the oracle's LAPACK eigensolve for M = 2 .. 64 (odd, even, the
    # maximum), and on structures that stress the deflation logic: a scaled identity (T is
    # diagonal from the start), rank one (N = 1, a cluster of zero eigenvalues) and R = 0.
    from paper_2007_14135_amd import WS_EVALS, WS_EVECS, WS_COV
    from paper_2007_14135_amd.api import Options
    frames = [make_frame("c1", i, M=M, D=D, N=N) for i, (M, D, N) in enumerate(
        [(2, 1, 300), (3, 1, 500), (8, 3, 4096), (16, 4, 1000), (17, 5, 999), (32, 6, 2000), (64, 8, 3000)])]
    frames.append(_custom_frame(np.sqrt(12.0) * np.eye(12, dtype=np.complex128)))
    rng = np.random.default_rng(5)
    frames.append(_custom_frame((rng.standard_normal((16, 1)) + 1j * rng.standard_normal((16, 1)))))
    frames.append(_custom_frame(np.zeros((8, 40), dtype=np.complex128)))
    fs = pack_frames(frames, dtype=np.complex128)
    db, res = _run(fs, "music", "c128", max_D=8, options=Options(eig_method=method))
    assert np.all(res["status"] & 0x2 == 0), res["status"]
    for f, fr in enumerate(frames):
        M = fr.M
        R = db.workspace_array(WS_COV, f, M * M, np.complex128).reshape(M, M)
        lam = db.workspace_array(WS_EVALS, f, M, np.float64)
        U = db.workspace_array(WS_EVECS, f, M * M, np.complex128).reshape(M, M)
        lo, Uo = oracle.eig_desc(oracle.covariance(fr.X))
        scale = max(abs(lo[0]), 1e-300)
        assert np.all(np.diff(lam) <= 0), (method, f)
        assert np.allclose(lam, lo, rtol=1e-11, atol=1e-13 * scale), (method, f, np.abs(lam - lo).max() / scale)
        assert np.linalg.norm(R - U @ np.diag(lam) @ U.conj().T) <= 1e-13 * np.linalg.norm(R), (method, f)
        assert np.linalg.norm(U.conj().T @ U - np.eye(M)) <= 1e-13 * M, (method, f)
        if f < 7:   # the generated frames: a clear signal/noise gap at D
            D = fr.D
            Pn = U[:, D:] @ U[:, D:].conj().T
            Pno = Uo[:, D:] @ Uo[:, D:].conj().T
            assert np.abs(Pn - Pno).max() <= 1e-10, (method, f)


def test_eigensolver_iteration_limit_sets_status():
    # One QL iteration per eigenvalue (or one Jacobi sweep) is not enough for a 16-element
    # covariance: the frame is flagged and the call still completes.
    from paper_2007_14135_amd.api import Options
    from paper_2007_14135_amd import ST_EVD_NOT_CONVERGED
    fs = make_frames("c2", n_frames=2, N=1024, grid_step=0.1)
    for method in ("ql", "jacobi"):      # the bisection of "auto" (M <= 16) always completes
        db, res = _run(fs, "music", "c64", options=Options(eig_method=method, eig_max_iter=1))
        assert np.all(res["status"] & ST_EVD_NOT_CONVERGED), (method, res["status"])


@pytest.mark.parametrize("kernel", ["split16", "fp32", "split3"])
@pytest.mark.parametrize("alg", ["music", "ev", "mn", "phd"])
def test_c2_frames_fp32_scan_parity(alg, kernel):
    # 12 frames of the 16-element workload at its full 18000-point grid (71 angle tiles, ragged
    # last tile) and full 4096 snapshots, on the three C64 scan kernels (FP16 split of two parts,
    # FP32 operands, FP16 split of three parts).
    from paper_2007_14135_amd.api import Options
    fs = make_frames("c2", n_frames=12)
    db, res = _run(fs, alg, "c64", options=Options(c64_scan=kernel))
    assert np.all(res["status"] == 0), res["status"]
    _check_frames(fs, res, alg, 1e-4, 1e-8, "c2-%s-%s" % (alg, kernel))


@pytest.mark.parametrize("alg", ["music", "phd"])
def test_three_part_split_at_least_as_accurate_as_fp32_operands(alg):
    # the FP16 split of three parts against the FP32-operand kernel on the same 12 frames: the
    # relative spectrum error against the oracle at the points the scan writes unrefined (Q above
    # the FP64 re-evaluation threshold), worst case and 99th percentile
    from paper_2007_14135_amd.api import Options
    fs = make_frames("c2", n_frames=12, start=100)
    errs = {}
    for kernel in ("fp32", "split3"):
        db, res = _run(fs, alg, "c64", options=Options(c64_scan=kernel))
        e = []
        for f, fr in enumerate(fs.frames):
            est = oracle_frame(fr, alg)
            keep = est.Q >= 5e-4 * np.sum(np.abs(est.B) ** 2)
            e.append(spectrum_rel_err(res["spectra"][f], est)[keep])
        e = np.concatenate(e)
        errs[kernel] = (float(e.max()), float(np.percentile(e, 99)), float(e.mean()))
    print("unrefined points, relative error max / p99 / mean: FP32 operands %.2e / %.2e / %.2e, "
          "three-part split %.2e / %.2e / %.2e" % (errs["fp32"] + errs["split3"]), flush=True)
    assert errs["split3"][0] <= 1.25 * errs["fp32"][0]
    assert errs["split3"][1] <= 1.25 * errs["fp32"][1]
    assert errs["split3"][2] <= 1.25 * errs["fp32"][2]


@pytest.mark.parametrize("alg", ["phd", "music", "ev", "mn"])
def test_c1_fp64_parity(alg):
    fs = make_frames("c1")
    db, res = _run(fs, alg, "c128")
    assert res["status"][0] == 0
    _check_frames(fs, res, alg, 1e-9, 1e-9, "c1-" + alg)


@pytest.mark.parametrize("kernel", ["split16", "fp32", "split3"])
def test_uneven_frames_chunking_and_groups(kernel):
    # Mixed M, geometry, D and grid in one batch: several groups, several launches, ragged
    # row chunks (K varies, rows padded to 8), M-bucketed peak kernels; both C64 scan kernels.
    from paper_2007_14135_amd.api import Options
    frames = []
    for i in range(24):
        fr = make_frame("c3", i, N=512)
        if fr.grid_L > 18000:
            fr = make_frame("c3", i, N=512, grid_step=0.01)
        frames.append(fr)
    fs = pack_frames(frames, dtype=np.complex64)
    db, res = _run(fs, "music", "c64", max_D=16, options=Options(c64_scan=kernel))
    assert np.all(res["status"] & 0x7 == 0), res["status"]
    _check_frames(fs, res, "music", 1e-4, 1e-8, "c3-mixed-" + kernel)


def test_many_frames_one_group_multiple_chunks():
    frames = [make_frame("c5", i, N=700, grid_step=0.01) for i in range(40)]
    fs = pack_frames(frames, dtype=np.complex64)
    db, res = _run(fs, "ev", "c64", max_D=4)
    _check_frames(fs, res, "ev", 1e-4, 1e-8, "c5-like-ev")


@pytest.mark.parametrize("M,D", [(2, 1), (5, 2), (7, 6), (8, 7)])
def test_fp64_small_and_odd_arrays(M, D):
    frames = [make_frame("c1", 0, M=M, D=D, N=300)]
    fs = pack_frames(frames, dtype=np.complex128)
    for alg in ("music", "mn", "ev", "phd"):
        db, res = _run(fs, alg, "c128")
        _check_frames(fs, res, alg, 1e-9, 1e-9, "odd-%d-%d-%s" % (M, D, alg))


def test_D_equals_M_minus_1_fp32():
    frames = [make_frame("c2", i, M=8, D=7, N=2048, grid_step=0.1) for i in range(3)]
    fs = pack_frames(frames, dtype=np.complex64)
    db, res = _run(fs, "music", "c64", max_D=7)
    _check_frames(fs, res, "music", 1e-4, 1e-8, "D=M-1")


def test_nonfinite_input_flags_only_its_frame():
    frames = [make_frame("c2", i, N=512, grid_step=0.1) for i in range(3)]
    frames[1].X = frames[1].X.copy()
    frames[1].X[3, 17] = np.nan
    fs = pack_frames(frames, dtype=np.complex64)
    db, res = _run(fs, "music", "c64")
    from paper_2007_14135_amd import ST_NONFINITE_INPUT, ST_FEWER_PEAKS
    assert res["status"][1] & ST_NONFINITE_INPUT
    assert res["npeaks"][1] == 0 and np.all(res["peaks"][1]["idx"] == -1)
    assert np.all(np.isnan(res["spectra"][1]))
    for f in (0, 2):
        assert res["status"][f] == 0 and res["npeaks"][f] == frames[f].D


def test_single_snapshot_rank_one():
    # N = 1: R = x x^H has one nonzero eigenvalue; MUSIC's noise projector is still defined.
    frames = [make_frame("c1", 0, N=1, D=1)]
    fs = pack_frames(frames, dtype=np.complex128)
    db, res = _run(fs, "music", "c128")
    assert not (res["status"][0] & 0x2), "the eigensolver must converge on a singular R"
    est = oracle_frame(frames[0], "music")
    rel = spectrum_rel_err(res["spectra"][0], est)
    assert rel.max() <= 1e-9
    db, res = _run(fs, "ev", "c128")
    from paper_2007_14135_amd import ST_DEGENERATE
    assert res["status"][0] & ST_DEGENERATE


def test_circular_grid_fp64():
    # Full-circle azimuth grid with a circular array: the peak search wraps around.
    M = 8
    pos = uca_positions(M, 0.5)
    rng = np.random.default_rng(3)
    th = np.array([-170.0, 3.0, 120.5])
    A = np.exp(2j * np.pi * (np.outer(pos[:, 0], np.sin(np.deg2rad(th))) + np.outer(pos[:, 1], np.cos(np.deg2rad(th)))))
    N = 2000
    S = (rng.standard_normal((3, N)) + 1j * rng.standard_normal((3, N))) / np.sqrt(2)
    W = 0.05 * (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N)))
    fr = Frame(M=M, N=N, D=3, pos=pos, geometry="uca", snr_db=20, sigma2=0.005, angles_deg=th,
               grid_start=-180.0, grid_step=1.0, grid_L=360, X=(A @ S + W))
    fs = pack_frames([fr], dtype=np.complex128)
    from paper_2007_14135_amd.runner import prepare
    _need_gpu()
    arrays, grids, frames, X = frameset_inputs(fs)
    grids = [(g[0], g[1], g[2], 1) for g in grids]
    db = prepare(arrays, grids, frames, X, "music", "c128", 3)
    db.run()
    res = db.host_results()
    est = oracle.estimate(fr.X, fr.pos, fr.D, fr.grid, "music", circular=True)
    assert np.max(spectrum_rel_err(res["spectra"][0], est)) <= 1e-9
    ok, _ = peaks_match(res["peaks"][0]["idx"][:res["npeaks"][0]], est, 3)
    assert ok, (res["peaks"][0]["idx"], est.peaks)


def test_repeat_runs_bit_identical():
    fs = make_frames("c2", n_frames=8, N=2048)
    db, r1 = _run(fs, "music", "c64")
    db.run()
    r2 = db.host_results()
    for a, b in zip(r1["spectra"], r2["spectra"]):
        assert np.array_equal(a, b)
    assert np.array_equal(r1["peaks"], r2["peaks"])


def test_c2_full_batch_bench_configuration():
    # The benchmark's workload in the benchmark's launch configuration: 256 frames, N=4096,
    # L=18000, MUSIC, with the scan work-item size bench.py takes from the committed autotuner
    # cache for this batch.  Every frame is compared point by point with the oracle and must
    # report D peaks with status 0.
    import os
    from paper_2007_14135_amd import autotune
    from paper_2007_14135_amd.api import Options
    _need_gpu()
    fs = make_frames("c2")
    arrays, grids, frames, _ = frameset_inputs(fs)
    cache = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2007_14135_amd", "tuning",
                         "autotune_cache.json")
    rows = autotune.Cache(cache).get(autotune.device_name(), autotune.signature(arrays, grids, frames, "music", "c64"))
    print("bench configuration: scan_rows %s" % rows, flush=True)
    db, res = _run(fs, "music", "c64", options=Options(scan_rows=rows or 0))
    assert np.all(res["status"] == 0)
    assert np.all(res["npeaks"] == 4)
    for s in res["spectra"]:
        assert np.all(np.isfinite(s)) and np.all(s > 0)
    _check_frames(fs, res, "music", 1e-4, 1e-8, "c2-full-bench-configuration")
