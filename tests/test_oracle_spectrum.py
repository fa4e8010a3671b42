"""Pins for the oracle's pseudo-spectrum (Table 2 Step-5, Table 3 Step-4) and the whole pipeline."""

import mpmath
import numpy as np
import pytest

from oracle import (covariance, eig_desc, estimate, find_peaks, grid_angles, noise_subspace_matrix,
                    select_peaks, spectrum_factored, spectrum_quadratic_form, step4_matrix, steering)


def _ula(M):
    pos = np.zeros((M, 3))
    pos[:, 0] = 0.5 * np.arange(M)
    return pos


def _uca(M, r):
    ang = 2 * np.pi * np.arange(M) / M
    return np.stack([r * np.cos(ang), r * np.sin(ang), np.zeros(M)], axis=1)


def _noisy_R(pos, th, N, s2, seed):
    rng = np.random.default_rng(seed)
    M, D = len(pos), len(th)
    A = steering(pos, th).T
    S = (rng.standard_normal((D, N)) + 1j * rng.standard_normal((D, N))) / np.sqrt(2)
    W = np.sqrt(s2) * (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))) / np.sqrt(2)
    return covariance(A @ S + W)


@pytest.mark.parametrize("alg", ["phd", "music", "ev", "mn"])
def test_factored_equals_quadratic_form(alg):
    pos = _ula(8)
    R = _noisy_R(pos, [-20.0, 31.0], 512, 0.1, 5)
    lam, U = eig_desc(R)
    B = noise_subspace_matrix(alg, lam, U, 2)
    C = step4_matrix(alg, lam, U, 2)
    ang = grid_angles(-90, 0.1, 1800)
    Q, P = spectrum_factored(B, pos, ang)
    invP, P2 = spectrum_quadratic_form(C, pos, ang)
    assert np.allclose(Q, invP, rtol=1e-9, atol=0)
    assert np.allclose(P, P2, rtol=1e-9, atol=0)


@pytest.mark.parametrize("geom", ["ula", "uca"])
@pytest.mark.parametrize("alg", ["music", "ev", "mn", "phd"])
def test_noise_free_limit_peaks_at_true_angles(geom, alg):
    # Exact R = A A^H + s2 I with the true angles on grid points: Q vanishes there and, for the
    # subspace methods, the D largest peaks are exactly the true indices.
    M, step = 8, 0.1
    pos = _ula(M) if geom == "ula" else _uca(M, 0.5 * M / np.pi)
    idx = np.array([412, 1037])                      # -48.8 and 13.7 degrees
    ang = grid_angles(-90, step, 1800)
    th = ang[idx]
    A = steering(pos, th).T
    s2 = 0.2
    R = A @ A.conj().T + s2 * np.eye(M)
    lam, U = eig_desc(R)
    assert np.allclose(lam[2:], s2, atol=1e-12)
    B = noise_subspace_matrix(alg, lam, U, 2)
    Q, P = spectrum_factored(B, pos, ang)
    assert np.all(Q[idx] < 1e-25 * max(1.0, np.max(Q)))
    if alg != "phd":
        sel = select_peaks(P, find_peaks(P), 2)
        assert sorted(sel.tolist()) == sorted(idx.tolist())


def _haar_unitary(K, rng):
    Z = rng.standard_normal((K, K)) + 1j * rng.standard_normal((K, K))
    Qm, Rm = np.linalg.qr(Z)
    return Qm * (np.diag(Rm) / np.abs(np.diag(Rm)))[None, :]


def test_rotation_invariance_music_mn():
    rng = np.random.default_rng(21)
    pos = _ula(16)
    R = _noisy_R(pos, [-40.0, -5.0, 12.0, 50.0], 2048, 0.05, 9)
    lam, U = eig_desc(R)
    D = 4
    ang = grid_angles(-90, 0.05, 3600)
    Ur = U.copy()
    Ur[:, D:] = U[:, D:] @ _haar_unitary(16 - D, rng)
    for alg in ("music", "mn"):
        Q1, _ = spectrum_factored(noise_subspace_matrix(alg, lam, U, D), pos, ang)
        Q2, _ = spectrum_factored(noise_subspace_matrix(alg, lam, Ur, D), pos, ang)
        assert np.allclose(Q1, Q2, rtol=1e-10, atol=1e-14)


def test_cross_algorithm_identities_D_equals_M_minus_1():
    pos = _ula(6)
    R = _noisy_R(pos, [-50.0, -20.0, 0.0, 25.0, 60.0], 1024, 0.1, 4)
    lam, U = eig_desc(R)
    D = 5
    ang = grid_angles(-90, 0.1, 1800)
    P = {a: spectrum_factored(noise_subspace_matrix(a, lam, U, D), pos, ang)[1] for a in ("phd", "music", "ev", "mn")}
    emin = U[:, -1]
    assert np.allclose(P["music"], P["phd"], rtol=1e-10)
    assert np.allclose(P["ev"], lam[-1] * P["phd"], rtol=1e-10)
    assert np.allclose(P["mn"], abs(emin[0]) ** 2 * P["phd"], rtol=1e-10)


def test_ev_equals_sigma2_times_music_for_exact_R():
    pos = _ula(10)
    th = [-33.03, 8.017, 41.05]                       # off-grid: Q stays above the rounding floor
    A = steering(pos, th).T
    s2 = 0.37
    R = A @ np.diag([1.0, 2.0, 0.5]) @ A.conj().T + s2 * np.eye(10)
    lam, U = eig_desc(R)
    ang = grid_angles(-90, 0.1, 1800)
    Pm = spectrum_factored(noise_subspace_matrix("music", lam, U, 3), pos, ang)[1]
    Pe = spectrum_factored(noise_subspace_matrix("ev", lam, U, 3), pos, ang)[1]
    assert np.allclose(Pe, s2 * Pm, rtol=1e-10)


def test_music_complement_identity():
    pos = _ula(12)
    R = _noisy_R(pos, [-10.0, 22.0, 35.0], 700, 0.2, 13)
    lam, U = eig_desc(R)
    D = 3
    ang = grid_angles(-90, 0.1, 1800)
    Q, _ = spectrum_factored(noise_subspace_matrix("music", lam, U, D), pos, ang)
    a = steering(pos, ang)
    Qc = np.sum(np.abs(a) ** 2, axis=1) - np.sum(np.abs(a @ U[:, :D].conj()) ** 2, axis=1)
    assert np.allclose(Q, Qc, rtol=1e-8, atol=1e-12)


def test_mpmath_bruteforce_pipeline():
    # Whole path at 50 digits for a 3-element array: snapshots -> R -> eigenpairs -> C -> a^H C a.
    mpmath.mp.dps = 50
    rng = np.random.default_rng(77)
    M, N, D = 3, 9, 1
    pos = np.array([[0.0, 0.0, 0.0], [0.5, 0.1, 0.0], [1.1, -0.3, 0.0]])
    X = (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))).astype(np.complex128)
    Xm = mpmath.matrix([[mpmath.mpc(X[i, n].real, X[i, n].imag) for n in range(N)] for i in range(M)])
    Rm = (Xm * Xm.H) / N
    E, V = mpmath.eighe(Rm)
    order = sorted(range(M), key=lambda i: -E[i])
    lam = [E[i] for i in order]
    cols = [V[:, i] for i in order]

    def C_of(alg):
        if alg == "phd":
            e = cols[-1]
            return e * e.H
        En = cols[D:]
        if alg == "music":
            return sum((c * c.H for c in En), mpmath.zeros(M))
        if alg == "ev":
            return sum(((c / lam[D + k]) * c.H for k, c in enumerate(En)), mpmath.zeros(M))
        Pn = sum((c * c.H for c in En), mpmath.zeros(M))
        e1 = mpmath.matrix([1, 0, 0])
        lmb = 1 / (e1.H * Pn * e1)[0]
        v = Pn * e1 * lmb
        return v * v.H

    angs = [-71.3, -12.0, 0.0, 33.3, 80.9]
    for alg in ("phd", "music", "ev", "mn"):
        est = estimate(X, pos, D, (-90.0, 0.1, 1800), alg)
        Cm = C_of(alg)
        for t in angs:
            tr = mpmath.radians(t)
            a = mpmath.matrix([mpmath.expj(2 * mpmath.pi * (pos[m, 0] * mpmath.sin(tr) + pos[m, 1] * mpmath.cos(tr)))
                               for m in range(M)])
            Pmp = 1 / mpmath.re((a.H * Cm * a)[0])
            Q, P = spectrum_factored(est.B, pos, [t])
            assert abs(float(P[0]) - float(Pmp)) <= 1e-9 * abs(float(Pmp)), (alg, t)
