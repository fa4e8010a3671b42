"""Rounding-error model of the proposal network's bfloat16-operand kernels against exact FP64
arithmetic, evaluated from the FP64 oracle's own forward values (nothing from the GPU enters it).

Model (the standard probabilistic model of rounding errors): each rounding is an independent
relative error of variance ua^2 / 3 (ua: bfloat16 after FP32, 2^-8 + 2^-24 + 2^-32), FP32
accumulation adds K 2^-48 / 3 (sum |terms|)^2 per K-term sum, variances add through sums and
products to first order, a ReLU decision is uncertain where |z| <= 6 sigma_z, and an uncertain
decision contributes its whole term's square (the activation is either z or 0; backward, the
derivative is either t or 0).  The bound of a gradient entry is 6 sigma plus two FP32 roundings.
"""

import numpy as np

from oracle import mlp as omlp

UA = 2.0 ** -8 + 2.0 ** -24 + 2.0 ** -32    # bfloat16 rounding after FP32 rounding
UF = 2.0 ** -24
LAMBDA = 6.0                                 # standard deviations of the gate


def _prod_var(A, VA, B, VB):
    """Variance of the error of the FP32-accumulated product of the bfloat16-rounded operands of
    A @ B (A, B exact FP64 values; VA, VB the variances of the errors the GPU's copies already
    carry): each rounding is an independent relative error of variance ua^2 / 3."""
    vA = UA * UA / 3.0 * A * A + (1.0 + UA) ** 2 * VA
    vB = UA * UA / 3.0 * B * B + (1.0 + UA) ** 2 * VB
    acc = A.shape[1] * UF * UF / 3.0 * (np.abs(A) @ np.abs(B)) ** 2
    return (A * A) @ vB + vA @ (B * B) + vA @ vB + acc


def gradient_bounds(params, X, Y):
    """Per-entry bounds LAMBDA * sigma on the kernels' gradients minus the exact FP64 gradients
    (see the module docstring), from the oracle's FP64 forward pass, and the fraction of hidden
    pre-activations within LAMBDA * sigma of 0 (ReLU decision uncertain)."""
    z, acts = omlp.forward(params, X)
    n = z.size
    Vz, zs = [], []
    Vh = [np.zeros_like(acts[0])]
    h = acts[0]
    for li, (W, b) in enumerate(params):
        zl = h @ W.T + b
        V = _prod_var(h, Vh[-1], W.T, np.zeros_like(W.T)) + UF * UF / 3.0 * zl * zl
        Vz.append(V)
        zs.append(zl)
        if li < len(params) - 1:
            risky = np.abs(zl) <= LAMBDA * np.sqrt(V)
            # an uncertain decision: the activation is z or 0, an error of up to |z| + the noise
            Vh.append(np.where(risky, (np.abs(zl) + LAMBDA * np.sqrt(V)) ** 2, V))
            h = np.maximum(zl, 0.0)
    sig = 1.0 / (1.0 + np.exp(-zs[-1]))
    delta = (sig - Y) / n
    Vd = (Vz[-1] / 16.0 + (4.0 * UF) ** 2) / (n * n)
    bounds = [None] * len(params)
    at_risk = []
    for li in range(len(params) - 1, -1, -1):
        W, b = params[li]
        a = acts[li]
        VgW = _prod_var(delta.T, Vd.T, a, Vh[li])
        Vgb = Vd.sum(axis=0) + delta.shape[0] * UF * UF / 3.0 * np.abs(delta).sum(axis=0) ** 2
        gW = delta.T @ a
        gb = delta.sum(axis=0)
        bounds[li] = (LAMBDA * np.sqrt(VgW) + 2.0 * UF * np.abs(gW), LAMBDA * np.sqrt(Vgb) + 2.0 * UF * np.abs(gb))
        if li > 0:
            t = delta @ W
            Vt = _prod_var(delta, Vd, W, np.zeros_like(W))
            zp, Vzp = zs[li - 1], Vz[li - 1]
            risky = np.abs(zp) <= LAMBDA * np.sqrt(Vzp)
            at_risk.append(float(risky.mean()))
            delta = t * (zp > 0.0)
            Vd = np.where(risky, t * t + Vt, Vt)
    return bounds, at_risk[::-1]
