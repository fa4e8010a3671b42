"""Pins for the oracle's accuracy statistic, Eq. 4: the mean relative deviation in percent,
100/N * sum_i |y_meas,i - y_true,i| / |y_true,i| (Section 5.1).  Written as checks of a callable
so that test_oracle_mutants.py can show that planted mistakes fail them."""

import numpy as np

from oracle import percent_error


def check_percent_error_worked_example(perr):
    # hand-worked: deviations 1 %, 10 %, 0 %, 10 % (|-4.4 - (-4)| / |-4| = 0.1), mean 5.25 %
    y_true = np.array([2.0, -4.0, 0.5, 10.0])
    y_meas = np.array([2.02, -4.4, 0.5, 9.0])
    assert abs(perr(y_meas, y_true) - 5.25) < 1e-12
    # one value 50 % high; one value 50 % low
    assert abs(perr(np.array([1.5]), np.array([1.0])) - 50.0) < 1e-12
    assert abs(perr(np.array([0.5]), np.array([1.0])) - 50.0) < 1e-12
    # a measurement equal to the truth has no error
    assert perr(y_true.copy(), y_true) == 0.0


def check_percent_error_invariances(perr):
    rng = np.random.default_rng(4)
    y_true = rng.uniform(0.5, 2.0, 37) * rng.choice([-1.0, 1.0], 37)
    y_meas = y_true * (1 + rng.normal(0, 1e-3, 37))
    e = perr(y_meas, y_true)
    # a common scale of both (either sign) leaves it unchanged; so does any reordering
    for c in (1e-6, -3.0, 1e5):
        assert abs(perr(c * y_meas, c * y_true) - e) <= 1e-12 * e
    perm = rng.permutation(37)
    assert abs(perr(y_meas[perm], y_true[perm]) - e) <= 1e-12 * e
    # a mean, not a sum: repeating the data leaves it unchanged
    assert abs(perr(np.tile(y_meas, 3), np.tile(y_true, 3)) - e) <= 1e-12 * e
    # every term is relative to the ground truth, not to the measurement
    assert abs(perr(np.array([2.0]), np.array([1.0])) - 100.0) < 1e-12


def test_percent_error_worked_example():
    check_percent_error_worked_example(percent_error)


def test_percent_error_invariances():
    check_percent_error_invariances(percent_error)
