"""Initial weights of the proposal network: He-uniform weights, zero biases, from a seed."""

from __future__ import annotations

import numpy as np


def he_uniform(seed: int, sizes) -> np.ndarray:
    """Flat FP32 parameters in the C ABI order (W1, b1, W2, b2, W3, b3), W_l of shape
    (out_l, in_l) drawn uniformly from [-sqrt(6 / in_l), sqrt(6 / in_l)] by PCG64 seeded with
    SeedSequence(seed), layer after layer; biases zero."""
    gen = np.random.Generator(np.random.PCG64(np.random.SeedSequence(int(seed))))
    parts = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        bound = np.sqrt(6.0 / fan_in)
        parts.append(gen.uniform(-bound, bound, size=(fan_out, fan_in)).reshape(-1))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)
