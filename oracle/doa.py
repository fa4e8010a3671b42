"""FP64 oracle: covariance -> eigendecomposition -> noise subspace -> pseudo-spectrum -> peaks.

TEST INFRASTRUCTURE (see the package docstring).  Each function cites the part of the paper it
writes out.  Readings taken where the paper is silent are stated in the docstrings:

* Directions are azimuth theta in the horizontal plane (phi = 90 deg in Eq. 2) unless a polar
  angle is passed; positions are in wavelengths, so 2*pi/lambda * x becomes 2*pi * x.
* The scan grid is theta_l = start + l * step for l = 0..L-1, each value computed directly.
* The covariance divides by N (Eq. 3) with no mean removal or loading.
* "jsvd" of the Hermitian positive semi-definite covariance is its eigendecomposition with the
  eigenvalues in descending order (Table 2, Step-2).
* Peaks (Table 2, Step-6): a grid point is a peak when it rises above its left neighbour and
  the run of equal values it starts is followed by a strictly smaller value; the plateau is
  reported at its first index.  The two ends of a non-circular grid are never peaks.  Peaks are
  ranked by value, descending, ties to the lower index, and the first D are kept; fewer than D
  are returned when fewer exist.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

ALGS = ("phd", "music", "ev", "mn")
TINY_Q = 1e-300


def grid_angles(start: float, step: float, L: int) -> np.ndarray:
    """Scan angles in degrees: theta_l = start + l * step, each computed from l (Table 2, Step-5 AngleSer)."""
    return float(start) + float(step) * np.arange(int(L), dtype=np.float64)


def steering(pos: np.ndarray, theta_deg, phi_deg: Optional[float] = None) -> np.ndarray:
    """Steering vectors of Eq. 2, one row per direction: shape (..., M).

    a_m(theta, phi) = exp{ j 2 pi (x_m sin(theta) sin(phi) + y_m cos(theta) sin(phi) + z_m cos(phi)) }
    with positions in wavelengths.  ``phi_deg=None`` is the horizontal plane (sin phi = 1,
    cos phi = 0 exactly).
    """
    pos = np.asarray(pos, dtype=np.float64)
    th = np.deg2rad(np.asarray(theta_deg, dtype=np.float64))
    if phi_deg is None:
        sphi, cphi = 1.0, 0.0
    else:
        ph = np.deg2rad(float(phi_deg))
        sphi, cphi = np.sin(ph), np.cos(ph)
    cyc = (np.multiply.outer(np.sin(th) * sphi, pos[:, 0])
           + np.multiply.outer(np.cos(th) * sphi, pos[:, 1])
           + np.multiply.outer(np.full(np.shape(th), cphi), pos[:, 2]))
    return np.exp(2j * np.pi * cyc)


def covariance(X: np.ndarray) -> np.ndarray:
    """Sample covariance of Eq. 3 (Table 2, Step-1): R = X X^H / N for X of shape (M, N)."""
    X = np.asarray(X).astype(np.complex128)
    N = X.shape[1]
    return (X @ X.conj().T) / N


def eig_desc(R: np.ndarray):
    """Table 2, Step-2: eigenvalues (descending) and eigenvectors (columns) of Hermitian R.

    For a Hermitian positive semi-definite R the singular value decomposition the paper calls
    is its eigendecomposition; LAPACK's Hermitian solver is the library primitive here.
    """
    w, V = np.linalg.eigh(np.asarray(R, dtype=np.complex128))
    return w[::-1].copy(), V[:, ::-1].copy()


def noise_subspace_matrix(alg: str, lam: np.ndarray, U: np.ndarray, D: int) -> np.ndarray:
    """B with B B^H equal to the Step-4 matrix C of Table 3, so a^H C a = ||B^H a||^2.

    * PHD: e_min, the eigenvector of the smallest eigenvalue (C = e_min e_min^H).
    * MUSIC: E_n = the eigenvectors D+1..M (C = E_n E_n^H).
    * EV: E_n scaled column-wise by lambda^(-1/2), since C = E_n diag(1/lambda_n) E_n^H.
    * MN: valph = P_n e_1 / (e_1^H P_n e_1) with P_n = E_n E_n^H (C = valph valph^H).
    """
    lam = np.asarray(lam, dtype=np.float64)
    U = np.asarray(U, dtype=np.complex128)
    M = U.shape[0]
    if alg == "phd":
        return U[:, [int(np.argmin(lam))]].copy()
    En = U[:, D:]
    if alg == "music":
        return En.copy()
    if alg == "ev":
        return En * (1.0 / np.sqrt(lam[D:]))[None, :]
    if alg == "mn":
        Pn = En @ En.conj().T
        e1 = np.zeros(M, dtype=np.complex128)
        e1[0] = 1.0
        lmb = 1.0 / np.real(e1.conj() @ Pn @ e1)
        valph = Pn @ (lmb * e1)
        return valph[:, None]
    raise ValueError("unknown algorithm %r" % (alg,))


def step4_matrix(alg: str, lam: np.ndarray, U: np.ndarray, D: int) -> np.ndarray:
    """The Step-4 matrix C of Table 3, formed as written (used to cross-check the factored form)."""
    lam = np.asarray(lam, dtype=np.float64)
    U = np.asarray(U, dtype=np.complex128)
    M = U.shape[0]
    if alg == "phd":
        e = U[:, int(np.argmin(lam))]
        return np.outer(e, e.conj())
    En = U[:, D:]
    if alg == "music":
        return En @ En.conj().T
    if alg == "ev":
        Enw = En * (1.0 / lam[D:])[None, :]
        return Enw @ En.conj().T
    if alg == "mn":
        Pn = En @ En.conj().T
        e1 = np.zeros(M, dtype=np.complex128)
        e1[0] = 1.0
        lmb = 1.0 / np.real(e1.conj() @ Pn @ e1)
        valph = Pn @ (lmb * e1)
        return np.outer(valph, valph.conj())
    raise ValueError("unknown algorithm %r" % (alg,))


def spectrum_quadratic_form(C: np.ndarray, pos: np.ndarray, angles_deg, phi_deg=None):
    """Table 2, Step-5 as written: invP = a^H C a, P = 1/invP.  Returns (invP, P)."""
    A = steering(pos, angles_deg, phi_deg)
    invP = np.real(np.einsum("lm,mn,ln->l", A.conj(), C, A))
    return invP, 1.0 / invP


def spectrum_factored(B: np.ndarray, pos: np.ndarray, angles_deg, phi_deg=None):
    """Step-5 with C = B B^H: Q = ||B^H a||^2 (a sum of squares), P = 1/max(Q, 1e-300).

    Returns (Q, P).  Algebraically identical to the quadratic form; numerically it avoids the
    cancellation of a^H C a near the spectrum peaks.
    """
    A = steering(pos, angles_deg, phi_deg)
    T = A @ np.asarray(B, dtype=np.complex128).conj()      # (L, K): row l = (B^H a_l)^T
    Q = np.sum(T.real ** 2 + T.imag ** 2, axis=1)
    return Q, 1.0 / np.maximum(Q, TINY_Q)


def find_peaks(P: np.ndarray, circular: bool = False) -> np.ndarray:
    """Table 2, Step-6 findPeaks: indices of the local maxima of P, ascending.

    A point l is a peak when P[l] > P[l-1] and the first value after the run of values equal to
    P[l] is strictly smaller; the run (plateau) is reported at l.  On a non-circular grid
    index 0 and L-1 are never peaks and a run reaching the last index is not a peak.  On a
    circular grid neighbours wrap around and a constant spectrum has no peak.
    """
    P = np.asarray(P)
    L = len(P)
    out = []
    if L < 3:
        return np.zeros(0, dtype=np.int64)
    if not circular:
        l = 1
        while l < L - 1:
            if P[l] > P[l - 1]:
                r = l + 1
                while r < L and P[r] == P[l]:
                    r += 1
                if r < L and P[r] < P[l]:
                    out.append(l)
                l = r
            else:
                l += 1
    else:
        for l in range(L):
            if P[l] > P[(l - 1) % L]:
                r = l + 1
                steps = 0
                while P[r % L] == P[l] and steps < L:
                    r += 1
                    steps += 1
                if P[r % L] < P[l]:
                    out.append(l)
    return np.asarray(out, dtype=np.int64)


def select_peaks(P: np.ndarray, peaks: np.ndarray, D: int) -> np.ndarray:
    """Table 2, Step-6 PeakSelection: the D largest peaks by value, ties to the lower index."""
    peaks = [int(i) for i in peaks]
    peaks.sort(key=lambda i: (-float(P[i]), i))
    return np.asarray(peaks[:D], dtype=np.int64)


@dataclasses.dataclass
class Estimate:
    R: np.ndarray
    lam: np.ndarray
    U: np.ndarray
    B: np.ndarray
    angles: np.ndarray
    Q: np.ndarray
    P: np.ndarray
    peaks: np.ndarray        # selected indices, best first
    peak_angles: np.ndarray  # degrees
    all_peaks: np.ndarray    # every local maximum, ascending


def estimate(X: np.ndarray, pos: np.ndarray, D: int, grid, alg: str, *,
             circular: bool = False, phi_deg=None) -> Estimate:
    """Table 2, Steps 1-6 for one frame: X (M, N) -> spectrum and the D strongest peaks."""
    R = covariance(X)
    lam, U = eig_desc(R)
    B = noise_subspace_matrix(alg, lam, U, D)
    angles = grid_angles(*grid)
    Q, P = spectrum_factored(B, pos, angles, phi_deg)
    allp = find_peaks(P, circular)
    sel = select_peaks(P, allp, D)
    return Estimate(R, lam, U, B, angles, Q, P, sel, angles[sel], allp)


def estimate_windowed(X: np.ndarray, pos: np.ndarray, D: int, grid, alg: str, windows, *,
                      phi_deg=None) -> Estimate:
    """Steps 1-6 with the Step-5 scan and the Step-6 search restricted to index windows.

    Not part of the paper: the restriction used by proposal-driven (learned) estimation.
    ``windows`` is a list of disjoint half-open index ranges [l0, l1) of the grid.  Spectrum
    values outside every window are unknown, so each window is searched as a non-circular
    spectrum of its own (Step-6 findPeaks on P[l0:l1]: its end points are never peaks) and the
    peaks of all windows are ranked together (PeakSelection).  P holds NaN outside the windows.
    """
    R = covariance(X)
    lam, U = eig_desc(R)
    B = noise_subspace_matrix(alg, lam, U, D)
    angles = grid_angles(*grid)
    L = len(angles)
    Q = np.full(L, np.nan)
    P = np.full(L, np.nan)
    allp = []
    for l0, l1 in windows:
        if l1 <= l0:
            continue
        Qw, Pw = spectrum_factored(B, pos, angles[l0:l1], phi_deg)
        Q[l0:l1] = Qw
        P[l0:l1] = Pw
        allp.extend(int(i) + l0 for i in find_peaks(Pw, circular=False))
    allp = np.asarray(sorted(allp), dtype=np.int64)
    sel = select_peaks(P, allp, D)
    return Estimate(R, lam, U, B, angles, Q, P, sel, angles[sel], allp)


def spectrum_factored_2d(B: np.ndarray, pos: np.ndarray, az_deg, el_deg):
    """Step-5 over a 2-D grid of Eq. 2's angle pairs: Q[j, i] = ||B^H a(theta_i, phi_j)||^2 with
    theta the azimuth and phi the polar angle (phi = 90 deg is the horizontal plane), one row per
    polar angle.  Returns (Q, P) of shape (len(el_deg), len(az_deg)), P = 1/max(Q, 1e-300)."""
    rows = [spectrum_factored(B, pos, az_deg, float(ph))[0] for ph in np.atleast_1d(el_deg)]
    Q = np.asarray(rows, dtype=np.float64)
    return Q, 1.0 / np.maximum(Q, TINY_Q)


def find_peaks_2d(P: np.ndarray, circular_az: bool = False) -> np.ndarray:
    """Table 2 Step-6 findPeaks over a 2-D grid: linear (row-major) indices j * n_az + i of the
    points that exceed their 8 neighbours, ascending.

    Readings (the paper prints no rule): only neighbours inside the grid count, so edge rows and
    columns can hold peaks (a planar array's spectrum is mirror-symmetric about phi = 90 deg, where
    the paper's grids end); the azimuth axis wraps when circular, the polar axis never does.  Ties:
    a point must be strictly greater than every neighbour that precedes it in row-major order, at
    least equal to every neighbour that follows it, and strictly greater than at least one
    neighbour, so a plateau is reported at its first point and a constant patch not at all.
    """
    P = np.asarray(P, dtype=np.float64)
    E, A = P.shape
    lin = np.arange(E * A).reshape(E, A)
    ok = np.ones((E, A), dtype=bool)
    above_one = np.zeros((E, A), dtype=bool)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            if dj == 0 and di == 0:
                continue
            jj = np.arange(E)[:, None] + dj
            ii = np.arange(A)[None, :] + di
            if circular_az:
                ii = ii % A
            inside = (jj >= 0) & (jj < E) & (ii >= 0) & (ii < A)
            jjc = np.clip(jj, 0, E - 1)
            iic = np.clip(ii, 0, A - 1)
            nb = P[jjc + 0 * iic, iic + 0 * jjc]
            nidx = lin[jjc + 0 * iic, iic + 0 * jjc]
            cond = np.where(nidx < lin, P > nb, P >= nb)
            ok &= np.where(inside, cond, True)
            above_one |= inside & (P > nb)
    return np.flatnonzero((ok & above_one).ravel())


def select_peaks_2d(P: np.ndarray, peaks: np.ndarray, D: int) -> np.ndarray:
    """PeakSelection over a 2-D grid: the D largest by value, ties to the lower linear index."""
    flat = np.asarray(P, dtype=np.float64).ravel()
    return select_peaks(flat, peaks, D)


def estimate_2d(X: np.ndarray, pos: np.ndarray, D: int, az_grid, el_grid, alg: str, *,
                circular_az: bool = False) -> Estimate:
    """Table 2, Steps 1-6 for one frame over a 2-D grid (azimuth x polar angle of Eq. 2).

    ``az_grid`` and ``el_grid`` are (start, step, count) in degrees; Q and P have shape
    (n_el, n_az); peak indices are row-major (j * n_az + i); ``peak_angles`` holds
    (azimuth, polar angle) pairs."""
    R = covariance(X)
    lam, U = eig_desc(R)
    B = noise_subspace_matrix(alg, lam, U, D)
    az = grid_angles(*az_grid)
    el = grid_angles(*el_grid)
    Q, P = spectrum_factored_2d(B, pos, az, el)
    allp = find_peaks_2d(P, circular_az)
    sel = select_peaks_2d(P, allp, D)
    A = len(az)
    pairs = np.stack([az[sel % A], el[sel // A]], axis=1) if len(sel) else np.zeros((0, 2))
    return Estimate(R, lam, U, B, (az, el), Q, P, sel, pairs, allp)


def percent_error(y_meas: np.ndarray, y_true: np.ndarray) -> float:
    """Eq. 4: mean relative deviation in percent, 100/N * sum |y_meas - y_true| / |y_true|."""
    y_meas = np.asarray(y_meas, dtype=np.float64)
    y_true = np.asarray(y_true, dtype=np.float64)
    return float(100.0 / len(y_true) * np.sum(np.abs(y_meas - y_true) / np.abs(y_true)))
