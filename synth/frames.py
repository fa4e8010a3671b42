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

import ast
import dataclasses
import json
import math
import operator
import os
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
    readings: List[str] = dataclasses.field(default_factory=list)
    recipe: Optional[dict] = None


def _grid_for_step(step: float):
    L = int(round(180.0 / step))
    return (-90.0, float(step), L)


# ---------------------------------------------------------------------------------------------
# Workload recipes: one JSON file per configuration under configs/.  "draws" lists the per-frame
# parameters in the order they are drawn from the frame's random stream; a value is
#   a literal (number, string, list)                      no draw
#   {"uniform": [lo, hi]}                                 float(rng.uniform(lo, hi))
#   {"choice": [v0, v1, ...]}                             rng.choice(values)
#   {"coin": [a, b]}                                      a if rng.uniform() < 0.5 else b
#   {"integers": [lo, hi]}                                int(rng.integers(lo, hi + 1)), inclusive
#   {"log_uniform_int": [lo, hi]}                         round(exp(rng.uniform(log lo, log hi)))
#   {"expr": "0.5 * M / pi"}                              arithmetic over earlier parameters
# and bounds may themselves be {"expr": ...}.  Derived: "pos" from "geometry", "M" and
# "uca_radius"; "grid" from "grid_step" unless given.
# ---------------------------------------------------------------------------------------------

CONFIG_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "configs")

_BINOPS = {ast.Add: operator.add, ast.Sub: operator.sub, ast.Mult: operator.mul,
           ast.Div: operator.truediv, ast.FloorDiv: operator.floordiv}


def _eval_expr(text: str, env: dict):
    """Evaluate +, -, *, /, // over numbers, ``pi`` and earlier parameters (nothing else)."""
    def ev(node):
        if isinstance(node, ast.Expression):
            return ev(node.body)
        if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)):
            return node.value
        if isinstance(node, ast.Name):
            if node.id == "pi":
                return math.pi
            if node.id in env and isinstance(env[node.id], (int, float)):
                return env[node.id]
            raise ValueError(f"unknown name {node.id!r} in {text!r}")
        if isinstance(node, ast.BinOp) and type(node.op) in _BINOPS:
            return _BINOPS[type(node.op)](ev(node.left), ev(node.right))
        if isinstance(node, ast.UnaryOp) and isinstance(node.op, ast.USub):
            return -ev(node.operand)
        raise ValueError(f"unsupported expression {text!r}")
    return ev(ast.parse(text, mode="eval"))


def _value(spec, env: dict, rng: np.random.Generator):
    if not isinstance(spec, dict):
        return spec
    if len(spec) != 1:
        raise ValueError(f"draw spec {spec!r} must have one key")
    (kind, arg), = spec.items()
    if kind == "expr":
        return _eval_expr(arg, env)
    bounds = [_value(b, env, rng) for b in arg] if kind != "choice" else arg
    if kind == "uniform":
        return float(rng.uniform(bounds[0], bounds[1]))
    if kind == "choice":
        v = rng.choice(arg)
        return int(v) if all(isinstance(x, int) for x in arg) else float(v)
    if kind == "coin":
        return bounds[0] if rng.uniform() < 0.5 else bounds[1]
    if kind == "integers":
        return int(rng.integers(int(bounds[0]), int(bounds[1]) + 1))
    if kind == "log_uniform_int":
        return int(round(math.exp(rng.uniform(math.log(bounds[0]), math.log(bounds[1])))))
    raise ValueError(f"unknown draw kind {kind!r}")


def _positions(p: dict) -> np.ndarray:
    if p["geometry"] == "ula":
        return ula_positions(p["M"])
    if p["geometry"] == "uca":
        return uca_positions(p["M"], p["uca_radius"])
    raise ValueError(f"unknown geometry {p['geometry']!r}")


def _recipe_draw(recipe: dict):
    def draw(rng: np.random.Generator) -> dict:
        p: dict = {}
        for name, spec in recipe["draws"]:
            p[name] = _value(spec, p, rng)
        p["pos"] = _positions(p)
        if "grid" in p:
            p["grid"] = (float(p["grid"][0]), float(p["grid"][1]), int(p["grid"][2]))
        else:
            p["grid"] = _grid_for_step(p["grid_step"])
        if "polar" in p:
            p["polar"] = tuple(p["polar"])
        return p
    return draw


def load_config(path: str) -> Config:
    """A workload configuration from its JSON recipe."""
    with open(path) as f:
        r = json.load(f)
    return Config(r["name"], int(r["index"]), int(r["frames"]), np.dtype(r["dtype"]).type,
                  _recipe_draw(r), r["description"], list(r.get("readings", [])), r)


CONFIGS: Dict[str, Config] = {
    c.name: c for c in (load_config(os.path.join(CONFIG_DIR, fn))
                        for fn in sorted(os.listdir(CONFIG_DIR)) if fn.endswith(".json"))
}

# Polar-angle ranges of the 2-D scans of the paper's scenario (azimuth 0:1:359 x these), keyed by
# their point count (the readings are stated in the scenario's recipe).
EL_GRIDS_2D = {int(k): (float(v[0]), float(v[1]), int(v[2]))
               for k, v in CONFIGS["c6"].recipe["polar_grids_2d"].items()}


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
        if p["geometry"] == "uca":
            # the radius follows M when the recipe gives it as an expression (never a new draw)
            spec = dict(cfg.recipe["draws"]).get("uca_radius")
            if isinstance(spec, dict) and "expr" in spec:
                p["uca_radius"] = _eval_expr(spec["expr"], p)
        p["pos"] = _positions(p)
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
