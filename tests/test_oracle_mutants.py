"""Planted mistakes: each mutant below is a plausible error in an oracle function (a dropped
term, a swapped constant, a wrong index or operand), and each must fail at least one of the pins
written for that function.  The mutants are defined here, on the CPU; the oracle itself is
untouched."""

import numpy as np
import pytest

from oracle import mlp
from test_oracle_accuracy import check_percent_error_invariances, check_percent_error_worked_example
from test_oracle_mlp import (check_adam_alternating_gradient, check_adam_constant_gradient,
                             check_adam_scale_invariance)


def _adam(update):
    """An Adam step built from a per-array rule update(p, g, m, v, t, lr, b1, b2, eps)."""
    def step(params, grads, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
        newp, newm, newv = [], [], []
        for (W, b), (gW, gb), (mW, mb), (vW, vb) in zip(params, grads, m, v):
            rW = update(W, gW, mW, vW, t, lr, b1, b2, eps)
            rb = update(b, gb, mb, vb, t, lr, b1, b2, eps)
            newp.append((rW[0], rb[0]))
            newm.append((rW[1], rb[1]))
            newv.append((rW[2], rb[2]))
        return newp, newm, newv
    return step


def _no_bias_correction(p, g, m, v, t, lr, b1, b2, eps):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    return p - lr * m / (np.sqrt(v) + eps), m, v


def _bias_correction_at_t1(p, g, m, v, t, lr, b1, b2, eps):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    return p - lr * (m / (1 - b1)) / (np.sqrt(v / (1 - b2)) + eps), m, v


def _betas_swapped_in_moments(p, g, m, v, t, lr, b1, b2, eps):
    m = b2 * m + (1 - b2) * g
    v = b1 * v + (1 - b1) * g * g
    return p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps), m, v


def _eps_inside_sqrt(p, g, m, v, t, lr, b1, b2, eps):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    return p - lr * (m / (1 - b1 ** t)) / np.sqrt(v / (1 - b2 ** t) + eps), m, v


def _abs_gradient_in_v(p, g, m, v, t, lr, b1, b2, eps):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * np.abs(g)
    return p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps), m, v


def _bias_correction_off_by_one(p, g, m, v, t, lr, b1, b2, eps):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    return p - lr * (m / (1 - b1 ** (t + 1))) / (np.sqrt(v / (1 - b2 ** (t + 1))) + eps), m, v


ADAM_MUTANTS = [_no_bias_correction, _bias_correction_at_t1, _betas_swapped_in_moments, _eps_inside_sqrt,
                _abs_gradient_in_v, _bias_correction_off_by_one]


def _fails_some(checks, fn):
    for chk in checks:
        try:
            chk(fn)
        except AssertionError:
            return True
    return False


def test_adam_pins_pass_for_the_oracle():
    for chk in (check_adam_constant_gradient, check_adam_alternating_gradient, check_adam_scale_invariance):
        chk(mlp.adam_step)


@pytest.mark.parametrize("mutant", ADAM_MUTANTS, ids=lambda f: f.__name__.strip("_"))
def test_adam_mutant_fails_a_pin(mutant):
    checks = (check_adam_constant_gradient, check_adam_alternating_gradient, check_adam_scale_invariance)
    assert _fails_some(checks, _adam(mutant))


PERR_MUTANTS = {
    "relative_to_measurement": lambda m, t: 100.0 / len(t) * np.sum(np.abs(m - t) / np.abs(m)),
    "no_percent_factor": lambda m, t: 1.0 / len(t) * np.sum(np.abs(m - t) / np.abs(t)),
    "sum_not_mean": lambda m, t: 100.0 * np.sum(np.abs(m - t) / np.abs(t)),
    "signed_deviation": lambda m, t: 100.0 / len(t) * np.sum((m - t) / np.abs(t)),
    "signed_truth": lambda m, t: 100.0 / len(t) * np.sum(np.abs(m - t) / t),
    "ratio_of_sums": lambda m, t: 100.0 * np.sum(np.abs(m - t)) / np.sum(np.abs(t)),
}


@pytest.mark.parametrize("name", sorted(PERR_MUTANTS))
def test_percent_error_mutant_fails_a_pin(name):
    checks = (check_percent_error_worked_example, check_percent_error_invariances)
    assert _fails_some(checks, PERR_MUTANTS[name])
