"""Pins for the oracle's steering vector (Eq. 2), scan grid and covariance (Eq. 3)."""

import numpy as np
import pytest

from oracle import covariance, grid_angles, steering


def test_steering_literal_values_eq2():
    # Eq. 2 with positions in wavelengths: a_m = exp(+j 2 pi (x sin(th) sin(phi) + y cos(th) sin(phi) + z cos(phi))).
    # Hand-evaluated: an element at x = 0.5 sees phase pi * sin(theta).
    pos = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0]])
    a30 = steering(pos, 30.0)
    assert np.allclose(a30, [1.0, 1j], atol=1e-15)          # exp(j pi/2) = +j (sign of Eq. 2)
    assert np.allclose(steering(pos, -30.0), [1.0, -1j], atol=1e-15)
    assert np.allclose(steering(pos, 90.0), [1.0, -1.0], atol=1e-15)
    assert np.allclose(steering(pos, 0.0), [1.0, 1.0], atol=1e-15)
    # y term carries cos(theta): y = 0.25 at broadside gives exp(j pi/2)
    posy = np.array([[0.0, 0.25, 0.0]])
    assert np.allclose(steering(posy, 0.0), [1j], atol=1e-15)
    assert np.allclose(steering(posy, 90.0), [1.0], atol=1e-15)
    # z term carries cos(phi): straight overhead (phi = 0) a z = 0.25 element sees j
    posz = np.array([[0.0, 0.0, 0.25]])
    assert np.allclose(steering(posz, 17.0, phi_deg=0.0), [1j], atol=1e-15)
    assert np.allclose(steering(posz, 17.0), [1.0], atol=1e-15)   # horizontal plane: no z term
    # x and y terms scale with sin(phi)
    assert np.allclose(steering(pos, 90.0, phi_deg=30.0), [1.0, 1j], atol=1e-15)


def test_steering_shapes_modulus_translation():
    rng = np.random.default_rng(1)
    pos = rng.uniform(-3, 3, size=(7, 3))
    th = np.linspace(-90, 89, 50)
    A = steering(pos, th)
    assert A.shape == (50, 7)
    assert np.allclose(np.abs(A), 1.0, atol=1e-14)
    # translating the array multiplies every steering vector by one common phase per direction
    shift = np.array([0.3, -1.1, 0.0])
    A2 = steering(pos + shift, th)
    ratio = A2 / A
    assert np.allclose(ratio, ratio[:, :1], atol=1e-12)


def test_grid_exact_values():
    for step, L in ((0.1, 1800), (0.01, 18000), (0.002, 90000), (0.001, 180000)):
        assert int(round(180.0 / step)) == L
        g = grid_angles(-90.0, step, L)
        assert g[0] == -90.0
        assert g[-1] < 90.0 and abs(g[-1] - (90.0 - step)) < 1e-9
        # each value is computed from its index, not accumulated
        assert g[L // 2] == -90.0 + step * (L // 2)


def _brute_cov(X):
    """Eq. 3 summed snapshot by snapshot with exact Python integers (for Gaussian-integer X)."""
    M, N = X.shape
    R = [[0j] * M for _ in range(M)]
    for n in range(N):
        for i in range(M):
            for j in range(M):
                xi = complex(int(X[i, n].real), int(X[i, n].imag))
                xj = complex(int(X[j, n].real), int(X[j, n].imag))
                R[i][j] += xi * xj.conjugate()
    return np.array(R) / N


def test_covariance_exact_integer_snapshots():
    rng = np.random.default_rng(7)
    M, N = 5, 37
    X = (rng.integers(-9, 10, (M, N)) + 1j * rng.integers(-9, 10, (M, N))).astype(np.complex64)
    R = covariance(X)
    Rb = _brute_cov(X)
    assert R.shape == (M, M)
    assert np.array_equal(R * N, Rb * N)          # integer sums are exact in float64
    assert np.array_equal(R, R.conj().T)           # Hermitian
    # 1/N normalisation (not 1/(N-1)): the diagonal is the mean power per element
    assert np.allclose(np.diag(R).real, np.mean(np.abs(X.astype(np.complex128)) ** 2, axis=1), rtol=0, atol=1e-12)


def test_covariance_rank_one_and_conjugation_side():
    x = np.array([[1 + 2j], [3 - 1j]])
    R = covariance(x)
    # R_ij = x_i conj(x_j): R_01 = (1+2j)(3+1j) = 1 + 7j
    assert R[0, 1] == 1 + 7j
    assert R[1, 0] == 1 - 7j
    assert R[0, 0] == 5 and R[1, 1] == 10
