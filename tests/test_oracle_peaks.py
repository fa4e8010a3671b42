"""Pins for the oracle's peak search and selection (Table 2, Step-6)."""

import json
import os

import numpy as np
import pytest

from oracle import find_peaks, select_peaks

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "peaks_cases.json")


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_peaks_golden(case):
    P = np.asarray(case["P"], dtype=np.float64)
    pk = find_peaks(P, circular=case["circular"])
    assert pk.tolist() == case["peaks"]
    assert select_peaks(P, pk, case["D"]).tolist() == case["selected"]


def _runs_bruteforce(P, circular):
    """Independent formulation: collapse equal neighbours into runs, a run is a peak when both
    neighbouring runs are lower (non-circular: the first and last runs have a missing side)."""
    L = len(P)
    runs = []          # (value, first index)
    for i in range(L):
        if runs and P[i] == runs[-1][0]:
            continue
        runs.append((P[i], i))
    if circular and len(runs) > 1 and runs[0][0] == runs[-1][0]:
        # the last run continues into the first: it starts at the last run's index
        runs = [(runs[-1][0], runs[-1][1])] + runs[1:-1]
    n = len(runs)
    out = []
    for k in range(n):
        if not circular and (k == 0 or k == n - 1):
            continue
        if circular and n < 2:
            continue
        lv = runs[(k - 1) % n][0]
        rv = runs[(k + 1) % n][0]
        if runs[k][0] > lv and runs[k][0] > rv:
            out.append(runs[k][1])
    return sorted(out)


@pytest.mark.parametrize("circular", [False, True])
def test_peaks_bruteforce_random_ties(circular):
    rng = np.random.default_rng(5 + circular)
    for trial in range(400):
        L = int(rng.integers(3, 40))
        P = rng.integers(0, 4, L).astype(np.float64)     # many plateaus and ties
        assert find_peaks(P, circular).tolist() == _runs_bruteforce(P, circular), (P, circular)


def test_select_is_sorted_topD():
    rng = np.random.default_rng(8)
    for trial in range(200):
        L = int(rng.integers(5, 60))
        P = rng.integers(0, 6, L).astype(np.float64)
        pk = find_peaks(P)
        D = int(rng.integers(1, 6))
        sel = select_peaks(P, pk, D)
        brute = sorted(pk.tolist(), key=lambda i: (-P[i], i))[:D]
        assert sel.tolist() == brute
