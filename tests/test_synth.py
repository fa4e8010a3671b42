"""Checks of the seeded frame generator (Section 3.1 signal model) and its agreement with the oracle."""

import numpy as np
import pytest

from synth import CONFIGS, make_frame, make_frames
from synth.frames import integer_snapshots, uca_positions, ula_positions
import oracle


def test_reproducible_and_distinct():
    a = make_frame("c2", 3, N=256)
    b = make_frame("c2", 3, N=256)
    c = make_frame("c2", 4, N=256)
    assert np.array_equal(a.X, b.X) and np.array_equal(a.angles_deg, b.angles_deg)
    assert not np.array_equal(a.X, c.X)
    assert a.X.dtype == np.complex64
    assert make_frame("c1", 0, N=64).X.dtype == np.complex128


@pytest.mark.parametrize("cfg,lo,hi,gap", [("c1", -60, 60, 10), ("c2", -70, 70, 5),
                                           ("c3", -70, 70, 5), ("c4", -60, 60, 1), ("c5", -70, 70, 5)])
def test_angle_ranges_and_gaps(cfg, lo, hi, gap):
    for i in range(12):
        fr = make_frame(cfg, i, N=16)
        a = fr.angles_deg
        assert len(a) == fr.D
        assert np.all(a >= lo) and np.all(a <= hi)
        assert np.all(np.diff(a) >= gap)


def test_config_parameter_ranges():
    c1 = make_frame("c1", 0, N=16)
    assert (c1.M, c1.D, c1.grid_L, c1.grid_step, c1.snr_db) == (8, 2, 1800, 0.1, 10.0)
    c2 = make_frame("c2", 0, N=16)
    assert (c2.M, c2.D, c2.grid_L) == (16, 4, 18000) and 0 <= c2.snr_db <= 20
    c4 = make_frame("c4", 0, N=16)
    assert (c4.M, c4.D, c4.grid_L, c4.snr_db) == (64, 8, 180000, 5.0)
    seen_M, seen_geo, seen_L = set(), set(), set()
    for i in range(60):
        f = make_frame("c3", i, N=16)
        assert f.M in (8, 16, 32, 64) and 1 <= f.D <= f.M // 4 and -5 <= f.snr_db <= 20
        if f.geometry == "uca":
            assert np.allclose(np.hypot(f.pos[:, 0], f.pos[:, 1]), 0.5 * f.M / np.pi)
        seen_M.add(f.M); seen_geo.add(f.geometry); seen_L.add(f.grid_L)
    assert seen_M == {8, 16, 32, 64} and seen_geo == {"ula", "uca"} and seen_L == {1800, 18000, 90000}
    for i in range(40):
        rng_f = make_frame("c5", i, N=16)
        assert 1 <= rng_f.D <= 4 and rng_f.M == 16


def test_sample_moments_match_model():
    # diag(R) -> D + sigma^2 (unit-power sources plus noise); R -> A A^H + sigma^2 I at rate 1/sqrt(N)
    fr = make_frame("c2", 1)
    X = fr.X.astype(np.complex128)
    R = X @ X.conj().T / fr.N
    A = np.exp(2j * np.pi * np.outer(fr.pos[:, 0], np.sin(np.deg2rad(fr.angles_deg))))
    Rm = A @ A.conj().T + fr.sigma2 * np.eye(fr.M)
    scale = fr.D + fr.sigma2
    assert np.max(np.abs(R - Rm)) < 8 * scale / np.sqrt(fr.N)
    assert abs(np.mean(np.diag(R).real) - scale) < 6 * scale / np.sqrt(fr.N * fr.M)


def test_source_direction_convention_matches_oracle():
    # A source drawn at +theta must show up as a MUSIC peak at +theta, not -theta (mirror check).
    for i in range(4):
        fr = make_frame("c2", i, N=2048, grid_step=0.05)
        est = oracle.estimate(fr.X, fr.pos, fr.D, fr.grid, "music")
        got = np.sort(est.peak_angles)
        assert np.max(np.abs(got - fr.angles_deg)) < 0.5, (got, fr.angles_deg)


def test_pack_layout():
    fs = make_frames("c2", n_frames=3, N=100)
    for f, fr in enumerate(fs.frames):
        blk = fs.X_flat[fs.x_off[f]:fs.x_off[f] + fr.M * fr.N].reshape(fr.M, fr.N)
        assert np.array_equal(blk, fr.X)
        assert fs.x_off[f] % 64 == 0


def test_integer_snapshots_are_small_gaussian_integers():
    x = integer_snapshots(np.random.default_rng(0), 4, 50)
    assert np.all(np.abs(x.real) <= 7) and np.all(x.real == np.round(x.real))
