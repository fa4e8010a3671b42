"""Pins for the oracle's eigendecomposition (Table 2 Step-2) and noise-subspace matrices (Table 3)."""

import mpmath
import numpy as np
import pytest

from oracle import eig_desc, noise_subspace_matrix, step4_matrix, steering


def _model_R(pos, angles, p, sigma2):
    A = steering(pos, angles).T                     # (M, D)
    return A @ np.diag(np.asarray(p, dtype=float)) @ A.conj().T + sigma2 * np.eye(len(pos))


def _ula(M):
    pos = np.zeros((M, 3))
    pos[:, 0] = 0.5 * np.arange(M)
    return pos


@pytest.mark.parametrize("M", [4, 8, 16])
def test_eigenvalues_closed_form_one_source(M):
    # R = p a a^H + s2 I: eigenvalues s2 + p*M (once) and s2 (M-1 times), descending.
    p, s2 = 2.5, 0.1
    R = _model_R(_ula(M), [23.0], [p], s2)
    lam, U = eig_desc(R)
    assert abs(lam[0] - (s2 + p * M)) < 1e-12 * M
    assert np.allclose(lam[1:], s2, atol=1e-13)
    assert np.all(np.diff(lam) <= 1e-14)


@pytest.mark.parametrize("M,th", [(8, (-20.0, 7.0)), (16, (3.0, 5.0)), (6, (-60.0, 40.0))])
def test_eigenvalues_closed_form_two_equal_sources(M, th):
    # Equal powers p: signal eigenvalues s2 + p (M +- |a1^H a2|); the rest equal s2.
    p, s2 = 1.0, 0.05
    pos = _ula(M)
    R = _model_R(pos, th, [p, p], s2)
    a = steering(pos, th)
    c = abs(np.vdot(a[0], a[1]))
    lam, _ = eig_desc(R)
    assert np.allclose(lam[:2], [s2 + p * (M + c), s2 + p * (M - c)], rtol=1e-12, atol=1e-12)
    assert np.allclose(lam[2:], s2, atol=1e-12)


def test_eig_residual_and_orthonormality_eq5():
    rng = np.random.default_rng(3)
    for M in (2, 5, 8, 16, 64):
        Z = rng.standard_normal((M, 3 * M)) + 1j * rng.standard_normal((M, 3 * M))
        R = Z @ Z.conj().T / (3 * M)
        lam, U = eig_desc(R)
        res = np.linalg.norm(R - U @ np.diag(lam) @ U.conj().T)
        assert res <= 1e-13 * np.linalg.norm(R)
        assert np.linalg.norm(U.conj().T @ U - np.eye(M)) <= 1e-13 * M
        assert np.all(np.diff(lam) <= 0)


def test_eig_analytic_2x2():
    a, c, b = 3.0, -1.0, 1.5 - 2.0j
    R = np.array([[a, b], [np.conj(b), c]])
    lam, U = eig_desc(R)
    h = np.sqrt(((a - c) / 2) ** 2 + abs(b) ** 2)
    assert np.allclose(lam, [(a + c) / 2 + h, (a + c) / 2 - h], atol=1e-14)
    for k in range(2):
        assert np.allclose(R @ U[:, k], lam[k] * U[:, k], atol=1e-13)


@pytest.mark.parametrize("M", [2, 3, 4])
def test_eig_bruteforce_mpmath(M):
    # 50-digit Hermitian eigensolver: eigenvalues and eigenprojectors agree with the oracle.
    mpmath.mp.dps = 50
    rng = np.random.default_rng(100 + M)
    Z = rng.standard_normal((M, 2 * M)) + 1j * rng.standard_normal((M, 2 * M))
    R = Z @ Z.conj().T / (2 * M)
    Rm = mpmath.matrix([[mpmath.mpc(R[i, j].real, R[i, j].imag) for j in range(M)] for i in range(M)])
    E, Q = mpmath.eighe(Rm)
    ev = sorted([float(E[i]) for i in range(M)], reverse=True)
    lam, U = eig_desc(R)
    assert np.allclose(lam, ev, rtol=1e-13, atol=1e-14)
    order = sorted(range(M), key=lambda i: -float(E[i]))
    for k, i in enumerate(order):
        q = np.array([complex(Q[r, i]) for r in range(M)])
        P_mp = np.outer(q, q.conj())
        P_or = np.outer(U[:, k], U[:, k].conj())
        assert np.allclose(P_mp, P_or, atol=1e-12)


def _random_R(M, D, seed):
    rng = np.random.default_rng(seed)
    N = 4 * M
    pos = _ula(M)
    th = np.sort(rng.uniform(-60, 60, D))
    A = steering(pos, th).T
    S = (rng.standard_normal((D, N)) + 1j * rng.standard_normal((D, N))) / np.sqrt(2)
    W = 0.3 * (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))) / np.sqrt(2)
    X = A @ S + W
    return X @ X.conj().T / N


@pytest.mark.parametrize("M,D", [(8, 2), (16, 4), (5, 1)])
def test_nss_identities(M, D):
    R = _random_R(M, D, 11 * M + D)
    lam, U = eig_desc(R)
    Es, En = U[:, :D], U[:, D:]
    # MUSIC: E_n E_n^H = I - E_s E_s^H
    B = noise_subspace_matrix("music", lam, U, D)
    assert B.shape == (M, M - D)
    assert np.allclose(B @ B.conj().T, np.eye(M) - Es @ Es.conj().T, atol=1e-13)
    # EV: B B^H = E_n diag(1/lambda_n) E_n^H, and equals the Step-4 matrix as written
    Bev = noise_subspace_matrix("ev", lam, U, D)
    assert np.allclose(Bev @ Bev.conj().T, En @ np.diag(1 / lam[D:]) @ En.conj().T, atol=1e-12)
    assert np.allclose(Bev @ Bev.conj().T, step4_matrix("ev", lam, U, D), atol=1e-12)
    # MN: d_1 = 1, E_s^H d = 0, ||d||^2 = 1 / (P_n)_11
    d = noise_subspace_matrix("mn", lam, U, D)[:, 0]
    Pn11 = np.sum(np.abs(En[0, :]) ** 2)
    assert abs(d[0] - 1.0) < 1e-13
    assert np.allclose(Es.conj().T @ d, 0, atol=1e-12)
    assert abs(np.vdot(d, d).real - 1.0 / Pn11) < 1e-11 / Pn11
    # PHD: the eigenvector of the smallest eigenvalue
    e = noise_subspace_matrix("phd", lam, U, D)[:, 0]
    assert np.allclose(R @ e, lam.min() * e, atol=1e-12)
    for alg in ("phd", "music", "mn"):
        Bx = noise_subspace_matrix(alg, lam, U, D)
        assert np.allclose(Bx @ Bx.conj().T, step4_matrix(alg, lam, U, D), atol=1e-12)


def test_nss_rejects_unknown():
    lam, U = eig_desc(np.eye(3))
    with pytest.raises(ValueError):
        noise_subspace_matrix("capon", lam, U, 1)
