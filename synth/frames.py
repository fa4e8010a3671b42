"""Seeded synthetic DOA frames (Section 3.1: signal model of Eq. 1, steering of Eq. 2).

Every frame is drawn from its own PCG64 stream seeded by
``SeedSequence(200714135, spawn_key=(config_index, frame_index))`` in a fixed order:
per-frame configuration draws -> source angles -> source waveforms S -> noise W.
Sources are unit-power circular complex Gaussian, i.e. (g1 + j g2)/sqrt(2); the noise is white
circular complex Gaussian with variance sigma^2 = 10^(-SNR/10), so the SNR is per source per
element.  Angles are sorted uniform draws redrawn until the minimum gap holds.  Data for the
complex64 workloads is rounded to complex64 once here; every consumer (oracle and GPU path)
reads the same bits.

Geometry: element positions are in wavelengths.  The uniform linear array (ULA) lies on the
x axis with its first element at the origin and half-wavelength spacing; the uniform circular
array (UCA) lies in the x-y plane.  Directions are azimuth theta measured from +y toward +x
in the horizontal plane (phi = 90 deg in Eq. 2).

The steering vector used here to synthesise the data is this module's own copy of Eq. 2 for
the source directions only; it is part of the data model, not of the estimator.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

ROOT_SEED = 200714135


def config_seed(config_index: int, frame_index: int) -> np.random.Generator:
    """Per-frame generator: PCG64 over SeedSequence(ROOT_SEED, spawn_key=(config, frame))."""
    ss = np.random.SeedSequence(ROOT_SEED, spawn_key=(int(config_index), int(frame_index)))
    return np.random.Generator(np.random.PCG64(ss))


def ula_positions(M: int, spacing: float = 0.5) -> np.ndarray:
    """Uniform linear array on the x axis, first element at the origin, (M, 3) in wavelengths."""
    pos = np.zeros((M, 3), dtype=np.float64)
    pos[:, 0] = spacing * np.arange(M, dtype=np.float64)
    return pos


def uca_positions(M: int, radius: float) -> np.ndarray:
    """Uniform circular array in the x-y plane, element m at angle 2*pi*m/M, (M, 3) in wavelengths."""
    ang = 2.0 * np.pi * np.arange(M, dtype=np.float64) / M
    pos = np.zeros((M, 3), dtype=np.float64)
    pos[:, 0] = radius * np.cos(ang)
    pos[:, 1] = radius * np.sin(ang)
    return pos


def _source_manifold(pos: np.ndarray, theta_deg: np.ndarray, phi_deg=None) -> np.ndarray:
    """Array manifold A (M x D) of Eq. 2: azimuth-plane sources (phi = 90 deg) unless polar
    angles phi_deg (one per source) are given."""
    th = np.deg2rad(np.asarray(theta_deg, dtype=np.float64))
    if phi_deg is None:
        cyc = np.outer(pos[:, 0], np.sin(th)) + np.outer(pos[:, 1], np.cos(th))
    else:
        ph = np.deg2rad(np.asarray(phi_deg, dtype=np.float64))
        cyc = (np.outer(pos[:, 0], np.sin(th) * np.sin(ph)) + np.outer(pos[:, 1], np.cos(th) * np.sin(ph))
               + np.outer(pos[:, 2], np.cos(ph)))
    return np.exp(2j * np.pi * cyc)


def draw_angles(rng: np.random.Generator, D: int, lo: float, hi: float, gap: float) -> np.ndarray:
    """D sorted angles uniform on {lo <= a_1 < ... < a_D <= hi, a_{k+1} - a_k >= gap}.

    Drawn exactly (no rejection loop): sort D uniforms on [lo, hi - (D-1) gap] and shift the
    k-th by k * gap.  The shift is a volume-preserving bijection onto the constrained set, so
    the result has the same law as redrawing plain sorted uniforms until the gaps hold.
    """
    span = hi - lo - (D - 1) * gap
    if span < 0:
        raise ValueError("cannot place %d sources %g deg apart in [%g, %g]" % (D, gap, lo, hi))
    y = np.sort(rng.uniform(lo, lo + span, size=D))
    return y + gap * np.arange(D, dtype=np.float64)


@dataclasses.dataclass
class Frame:
    """One frame of snapshots plus the parameters it was drawn with."""

    M: int
    N: int
    D: int
    pos: np.ndarray            # (M, 3) float64, wavelengths
    geometry: str              # "ula" | "uca"
    snr_db: float
    sigma2: float
    angles_deg: np.ndarray     # (D,) true source azimuths
    grid_start: float          # scan grid theta_l = start + l * step, l = 0..L-1
    grid_step: float
    grid_L: int
    X: np.ndarray              # (M, N) complex64 or complex128, element-major
    polar_deg: Optional[np.ndarray] = None  # (D,) true polar angles (phi of Eq. 2), None: all 90 deg

    @property
    def grid(self):
        return (self.grid_start, self.grid_step, self.grid_L)


@dataclasses.dataclass
class Config:
    name: str
    index: int
    n_frames: int
    dtype: type
    draw: callable             # rng -> dict of per-frame parameters
    description: str


def _grid_for_step(step: float):
    L = int(round(180.0 / step))
    return (-90.0, float(step), L)


def _c1(rng):
    M = 8
    return dict(M=M, geometry="ula", pos=ula_positions(M), D=2, N=1024, snr_db=10.0,
                angle_lo=-60.0, angle_hi=60.0, gap=10.0, grid=_grid_for_step(0.1))


def _c2(rng):
    M = 16
    snr = float(rng.uniform(0.0, 20.0))
    return dict(M=M, geometry="ula", pos=ula_positions(M), D=4, N=4096, snr_db=snr,
                angle_lo=-70.0, angle_hi=70.0, gap=5.0, grid=_grid_for_step(0.01))


def _c3(rng):
    M = int(rng.choice([8, 16, 32, 64]))
    geometry = "ula" if rng.uniform() < 0.5 else "uca"
    pos = ula_positions(M) if geometry == "ula" else uca_positions(M, 0.5 * M / np.pi)
    D = int(rng.integers(1, M // 4 + 1))
    N = int(round(math.exp(rng.uniform(math.log(256.0), math.log(8192.0)))))
    snr = float(rng.uniform(-5.0, 20.0))
    step = float(rng.choice([0.1, 0.01, 0.002]))
    return dict(M=M, geometry=geometry, pos=pos, D=D, N=N, snr_db=snr,
                angle_lo=-70.0, angle_hi=70.0, gap=5.0, grid=_grid_for_step(step))


def _c4(rng):
    M = 64
    return dict(M=M, geometry="ula", pos=ula_positions(M), D=8, N=16384, snr_db=5.0,
                angle_lo=-60.0, angle_hi=60.0, gap=1.0, grid=_grid_for_step(0.001))


def _c5(rng):
    M = 16
    D = int(rng.integers(1, 5))
    snr = float(rng.uniform(-5.0, 20.0))
    N = int(round(math.exp(rng.uniform(math.log(256.0), math.log(4096.0)))))
    return dict(M=M, geometry="ula", pos=ula_positions(M), D=D, N=N, snr_db=snr,
                angle_lo=-70.0, angle_hi=70.0, gap=5.0, grid=_grid_for_step(0.001))


def _c6(rng):
    # the paper's test scenario (Section 5): 8-element UCA of radius 10 m at 15 MHz (0.5 lambda),
    # two uncorrelated sources at 15 dB; snapshot count and directions are not given (readings:
    # N = 1024, azimuths uniform in [0, 330] deg at least 30 deg apart, so also 30 deg apart across
    # 0/360, polar angles uniform in [60, 90] deg); scanned over 0:1:359 deg of azimuth
    M = 8
    return dict(M=M, geometry="uca", pos=uca_positions(M, 0.5), D=2, N=1024, snr_db=15.0,
                angle_lo=0.0, angle_hi=330.0, gap=30.0, polar=(60.0, 90.0), grid=(0.0, 1.0, 360))


CONFIGS: Dict[str, Config] = {
    "c1": Config("c1", 0, 1, np.complex128, _c1,
                 "ULA M=8, D=2, N=1024, 10 dB, one frame, complex128, 0.1 deg grid"),
    "c2": Config("c2", 1, 256, np.complex64, _c2,
                 "ULA M=16, D=4, N=4096, SNR U[0,20] dB, 256 frames, complex64, 0.01 deg grid"),
    "c3": Config("c3", 2, 4096, np.complex64, _c3,
                 "uneven batch: M in {8,16,32,64}, ULA/UCA, D U{1..M/4}, N log-U[256,8192], "
                 "SNR U[-5,20] dB, step in {0.1,0.01,0.002} deg, 4096 frames, complex64"),
    "c4": Config("c4", 3, 64, np.complex64, _c4,
                 "ULA M=64, D=8 (gap 1 deg), N=16384, 5 dB, 64 frames, complex64, 0.001 deg grid"),
    "c5": Config("c5", 4, 8192, np.complex64, _c5,
                 "ULA M=16, D U{1..4}, SNR U[-5,20] dB, N log-U[256,4096], 0.001 deg grid"),
    "c6": Config("c6", 5, 1, np.complex64, _c6,
                 "UCA M=8 radius 0.5 lambda, D=2 at polar angles U[60,90] deg, N=1024, 15 dB, complex64, "
                 "azimuth 0:1:359 deg (2-D grids add polar angles)"),
}

# Polar-angle ranges of the 2-D scans of the paper's scenario (azimuth 0:1:359 x these), keyed by
# their point count: 360 x 1 is the horizontal plane; the larger ranges extend it away from the
# plane at 1 deg (reading: the paper names only the counts 1, 30, 60 and 90, and phi = 1..90 for
# the largest).
EL_GRIDS_2D = {1: (90.0, 1.0, 1), 30: (61.0, 1.0, 30), 60: (31.0, 1.0, 60), 90: (1.0, 1.0, 90)}


def make_frame(config: str, frame_index: int, *, N: Optional[int] = None,
               grid_step: Optional[float] = None, M: Optional[int] = None,
               D: Optional[int] = None) -> Frame:
    """Draw frame ``frame_index`` of ``config``; keyword overrides shrink the frame for tests.

    Overrides are applied after the configuration draws so that the random stream stays the
    same for every other quantity.
    """
    cfg = CONFIGS[config]
    rng = config_seed(cfg.index, frame_index)
    p = cfg.draw(rng)
    if M is not None and M != p["M"]:
        p["M"] = M
        p["pos"] = ula_positions(M) if p["geometry"] == "ula" else uca_positions(M, 0.5 * M / np.pi)
    if D is not None:
        p["D"] = D
    if N is not None:
        p["N"] = N
    if grid_step is not None:
        p["grid"] = _grid_for_step(grid_step)
    Mv, Dv, Nv = p["M"], p["D"], p["N"]
    angles = draw_angles(rng, Dv, p["angle_lo"], p["angle_hi"], p["gap"])
    polar = rng.uniform(p["polar"][0], p["polar"][1], size=Dv) if "polar" in p else None
    A = _source_manifold(p["pos"], angles, polar)
    # complex draws built part by part (the same values as re + 1j * im, without temporaries):
    # S = (g1 + j g2) / sqrt(2), W = sqrt(sigma2) (g3 + j g4) / sqrt(2), in this draw order
    S = np.empty((Dv, Nv), dtype=np.complex128)
    S.real = rng.standard_normal((Dv, Nv))
    S.imag = rng.standard_normal((Dv, Nv))
    S /= np.sqrt(2.0)
    sigma2 = 10.0 ** (-p["snr_db"] / 10.0)
    W = np.empty((Mv, Nv), dtype=np.complex128)
    W.real = rng.standard_normal((Mv, Nv))
    W.imag = rng.standard_normal((Mv, Nv))
    W.real *= np.sqrt(sigma2)
    W.imag *= np.sqrt(sigma2)
    W /= np.sqrt(2.0)
    W += A @ S
    X = W.astype(cfg.dtype)
    g = p["grid"]
    return Frame(M=Mv, N=Nv, D=Dv, pos=p["pos"], geometry=p["geometry"], snr_db=p["snr_db"],
                 sigma2=sigma2, angles_deg=angles, polar_deg=polar, grid_start=g[0], grid_step=g[1], grid_L=g[2],
                 X=X)


@dataclasses.dataclass
class FrameSet:
    """A batch of frames with their snapshots packed into one flat buffer.

    ``X_flat`` holds every frame's (M, ld) element-major block back to back; frame f starts at
    complex element ``x_off[f]`` and its rows are ``ld[f]`` complex elements apart.
    """

    frames: List[Frame]
    X_flat: np.ndarray
    x_off: np.ndarray
    ld: np.ndarray

    def __len__(self):
        return len(self.frames)


def pack_frames(frames: Sequence[Frame], dtype=None, align: int = 64) -> FrameSet:
    """Pack frames back to back; each block starts on a multiple of ``align`` complex elements."""
    if dtype is None:
        dtype = frames[0].X.dtype
    offs, lds = [], []
    cur = 0
    for fr in frames:
        cur = (cur + align - 1) // align * align
        offs.append(cur)
        lds.append(fr.N)
        cur += fr.M * fr.N
    flat = np.zeros(cur, dtype=dtype)
    for fr, o in zip(frames, offs):
        flat[o:o + fr.M * fr.N] = fr.X.astype(dtype).reshape(-1)
    return FrameSet(list(frames), flat, np.asarray(offs, dtype=np.int64), np.asarray(lds, dtype=np.int64))


def make_frames(config: str, n_frames: Optional[int] = None, start: int = 0, **overrides) -> FrameSet:
    """Frames ``start .. start+n_frames-1`` of ``config`` packed into one buffer."""
    cfg = CONFIGS[config]
    n = cfg.n_frames if n_frames is None else n_frames
    frames = [make_frame(config, start + i, **overrides) for i in range(n)]
    return pack_frames(frames, dtype=cfg.dtype)


def make_config(config: str) -> Config:
    return CONFIGS[config]


def integer_snapshots(rng: np.random.Generator, M: int, N: int, amp: int = 7,
                      dtype=np.complex64) -> np.ndarray:
    """Gaussian-integer snapshots with |re|, |im| <= amp (sums of their products are exact)."""
    re = rng.integers(-amp, amp + 1, size=(M, N))
    im = rng.integers(-amp, amp + 1, size=(M, N))
    return (re + 1j * im).astype(dtype)
