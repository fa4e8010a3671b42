"""Pins for the oracle's 2-D (azimuth x polar angle) spectrum and peak search.

* one polar-angle row at phi = 90 deg equals the azimuth-only spectrum (Eq. 2 with sin phi = 1);
* a planar array cannot tell phi from 180 - phi: its spectrum is mirror-symmetric about 90 deg;
* a uniform circular array maps onto itself under a rotation by 360/M deg: permuting the elements
  cyclically shifts the 2-D spectrum by that many degrees of azimuth;
* noise-free limit: with an exact covariance and sources on grid points, Q vanishes there and the
  D largest 2-D peaks are the sources' grid points (a non-planar array, so that the polar angle
  is identifiable on both sides);
* the 8-neighbour peak rule against a brute force written separately, on random grids with ties,
  and on hand-built cases (an edge row, the azimuth wrap, a two-point plateau, a mesa, a constant).
"""

import numpy as np
import pytest

import oracle
from oracle import (covariance, eig_desc, find_peaks_2d, grid_angles, noise_subspace_matrix, select_peaks_2d,
                    spectrum_factored, spectrum_factored_2d, steering)


def _uca(M, r):
    ang = 2 * np.pi * np.arange(M) / M
    return np.stack([r * np.cos(ang), r * np.sin(ang), np.zeros(M)], axis=1)


def _R(pos, th, ph, N, s2, seed):
    rng = np.random.default_rng(seed)
    A = np.stack([steering(pos, t, p) for t, p in zip(th, ph)], axis=1)
    D = A.shape[1]
    S = (rng.standard_normal((D, N)) + 1j * rng.standard_normal((D, N))) / np.sqrt(2)
    W = np.sqrt(s2) * (rng.standard_normal((len(pos), N)) + 1j * rng.standard_normal((len(pos), N))) / np.sqrt(2)
    return covariance(A @ S + W)


def test_horizontal_row_equals_azimuth_spectrum():
    pos = _uca(8, 0.5)
    R = _R(pos, [40.0, 200.0], [80.0, 70.0], 512, 0.03, 1)
    lam, U = eig_desc(R)
    B = noise_subspace_matrix("music", lam, U, 2)
    az = grid_angles(0.0, 1.0, 360)
    Q2, _ = spectrum_factored_2d(B, pos, az, [90.0])
    Q1, _ = spectrum_factored(B, pos, az)
    assert np.array_equal(Q2[0], Q1)


def test_planar_array_mirror_symmetry():
    pos = _uca(8, 0.5)
    R = _R(pos, [10.0, 130.0], [75.0, 62.0], 256, 0.1, 2)
    lam, U = eig_desc(R)
    B = noise_subspace_matrix("ev", lam, U, 2)
    az = grid_angles(0.0, 1.0, 360)
    Qa, _ = spectrum_factored_2d(B, pos, az, grid_angles(1.0, 1.0, 89))
    Qb, _ = spectrum_factored_2d(B, pos, az, 180.0 - grid_angles(1.0, 1.0, 89))
    assert np.allclose(Qa, Qb, rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("alg", ["music", "ev", "phd"])      # MN weights element 0, which a rotation moves
def test_uca_rotation_shifts_the_spectrum(alg):
    M = 8
    pos = _uca(M, 0.5)
    R = _R(pos, [33.0, 250.0], [71.0, 88.0], 400, 0.05, 3)
    az = grid_angles(0.0, 1.0, 360)
    el = grid_angles(61.0, 1.0, 30)
    lam, U = eig_desc(R)
    _, P = spectrum_factored_2d(noise_subspace_matrix(alg, lam, U, 2), pos, az, el)
    # element m -> m + 1 (R' = Pi R Pi^T) is the scene rotated by 360/M = 45 deg of azimuth
    perm = np.roll(np.arange(M), 1)
    Rp = R[np.ix_(perm, perm)]
    lam2, U2 = eig_desc(Rp)
    _, P2 = spectrum_factored_2d(noise_subspace_matrix(alg, lam2, U2, 2), pos, az, el)
    assert np.allclose(P2, np.roll(P, -45, axis=1), rtol=1e-9, atol=0)


def test_noise_free_limit_2d_peaks_at_the_sources():
    # a non-planar array (a UCA plus one element on the z axis) makes the polar angle identifiable
    pos = np.concatenate([_uca(8, 0.5), [[0.0, 0.0, 0.5]]])
    az = grid_angles(0.0, 1.0, 360)
    el = grid_angles(31.0, 1.0, 60)
    src = [(57, 40), (300, 12)]                       # (azimuth index, polar index)
    th = [az[i] for i, _ in src]
    ph = [el[j] for _, j in src]
    A = np.stack([steering(pos, t, p) for t, p in zip(th, ph)], axis=1)
    R = A @ A.conj().T + 0.2 * np.eye(len(pos))
    lam, U = eig_desc(R)
    for alg in ("music", "ev", "mn"):
        B = noise_subspace_matrix(alg, lam, U, 2)
        Q, P = spectrum_factored_2d(B, pos, az, el)
        for i, j in src:
            assert Q[j, i] < 1e-24
        sel = select_peaks_2d(P, find_peaks_2d(P, circular_az=True), 2)
        assert sorted(sel.tolist()) == sorted(j * 360 + i for i, j in src)


def _brute_peaks(P, circ):
    E, A = P.shape
    out = []
    for j in range(E):
        for i in range(A):
            p = j * A + i
            good, above = True, False
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    if dj == 0 and di == 0:
                        continue
                    jj, ii = j + dj, i + di
                    if circ:
                        ii %= A
                    if not (0 <= jj < E and 0 <= ii < A):
                        continue
                    q = jj * A + ii
                    if q < p and not P[j, i] > P[jj, ii]:
                        good = False
                    if q > p and not P[j, i] >= P[jj, ii]:
                        good = False
                    if P[j, i] > P[jj, ii]:
                        above = True
            if good and above:
                out.append(p)
    return out


@pytest.mark.parametrize("circ", [False, True])
def test_peak_rule_equals_brute_force_with_ties(circ):
    rng = np.random.default_rng(8)
    for trial in range(40):
        E, A = int(rng.integers(1, 6)), int(rng.integers(3, 9))
        P = rng.integers(0, 4, size=(E, A)).astype(float)       # many ties
        assert find_peaks_2d(P, circ).tolist() == _brute_peaks(P, circ), (trial, P)


def test_peak_rule_hand_built_cases():
    P = np.zeros((3, 6))
    P[0, 2] = 5.0                                     # on the first row: an edge peak
    assert find_peaks_2d(P).tolist() == [2]
    P = np.zeros((2, 6))
    P[1, 0] = 3.0
    P[1, 5] = 2.0                                     # neighbours across the azimuth wrap
    assert find_peaks_2d(P, circular_az=False).tolist() == [6, 11]
    assert find_peaks_2d(P, circular_az=True).tolist() == [6]
    P = np.zeros((3, 5))
    P[1, 1] = P[1, 2] = 4.0                           # a two-point plateau: its first point
    assert find_peaks_2d(P).tolist() == [6]
    P = np.ones((2, 3))                               # constant: no peak
    assert find_peaks_2d(P).tolist() == []
    P = np.zeros((4, 6))
    P[1:3, 2:4] = 1.0                                 # a 2 x 2 mesa: reported once, at its first point
    assert find_peaks_2d(P).tolist() == [8]


def test_estimate_2d_pairs_and_layout():
    from synth import EL_GRIDS_2D, make_frame
    fr = make_frame("c6", 0)
    est = oracle.estimate_2d(fr.X, fr.pos, fr.D, (0.0, 1.0, 360), EL_GRIDS_2D[30], "music", circular_az=True)
    assert est.P.shape == (30, 360) and len(est.peaks) == 2
    for k, l in enumerate(est.peaks):
        assert est.peak_angles[k, 0] == float(l % 360) and est.peak_angles[k, 1] == 61.0 + l // 360
    # the sources (at polar angles 60..90) are found within a few degrees of azimuth
    got = np.sort(est.peak_angles[:, 0])
    want = np.sort(fr.angles_deg)
    assert np.max(np.abs(got - want)) < 3.0, (got, want)
