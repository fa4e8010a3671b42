"""Pins for the oracle of windowed estimation (the Step-5 scan and Step-6 search restricted to
proposal windows) and of the proposal windows themselves."""

import numpy as np

from oracle import estimate, estimate_windowed, grid_angles, steering
from oracle import mlp


def _ula(M):
    pos = np.zeros((M, 3))
    pos[:, 0] = 0.5 * np.arange(M)
    return pos


def _frame(seed=11, M=8, N=512, th=(-31.3, 12.7), s2=0.1):
    rng = np.random.default_rng(seed)
    pos = _ula(M)
    A = steering(pos, np.asarray(th)).T
    S = (rng.standard_normal((len(th), N)) + 1j * rng.standard_normal((len(th), N))) / np.sqrt(2)
    W = np.sqrt(s2) * (rng.standard_normal((M, N)) + 1j * rng.standard_normal((M, N))) / np.sqrt(2)
    return pos, A @ S + W


def test_whole_grid_window_is_the_plain_estimate():
    pos, X = _frame()
    grid = (-90.0, 0.1, 1800)
    for alg in ("music", "ev", "mn", "phd"):
        full = estimate(X, pos, 2, grid, alg)
        win = estimate_windowed(X, pos, 2, grid, alg, [(0, 1800)])
        assert np.array_equal(full.P, win.P)
        assert np.array_equal(full.peaks, win.peaks)
        assert np.array_equal(full.all_peaks, win.all_peaks)


def test_windows_around_the_peaks_find_them():
    # noise-free limit: exact R, true angles on grid points; windows around both
    M, ang = 8, grid_angles(-90.0, 0.01, 18000)
    idx = np.array([5870, 10270])
    pos = _ula(M)
    A = steering(pos, ang[idx]).T
    R = A @ A.conj().T + 0.2 * np.eye(M)
    # snapshots with exactly this covariance: X = R^(1/2) * sqrt(N) columns of an identity
    w, V = np.linalg.eigh(R)
    X = (V * np.sqrt(w)) @ V.conj().T * np.sqrt(M)
    X = np.concatenate([X, np.zeros((M, 0))], axis=1)
    full = estimate(X, pos, 2, (-90.0, 0.01, 18000), "music")
    assert sorted(full.peaks) == sorted(idx)
    win = estimate_windowed(X, pos, 2, (-90.0, 0.01, 18000), "music", [(5700, 6000), (10100, 10400)])
    assert sorted(win.peaks) == sorted(idx)
    assert np.isnan(win.P[:5700]).all() and np.isnan(win.P[6000:10100]).all() and np.isnan(win.P[10400:]).all()
    assert np.array_equal(win.P[5700:6000], full.P[5700:6000])


def test_window_end_is_never_a_peak():
    M, ang = 8, grid_angles(-90.0, 0.01, 18000)
    idx = np.array([5870, 10270])
    pos = _ula(M)
    A = steering(pos, ang[idx]).T
    R = A @ A.conj().T + 0.2 * np.eye(M)
    w, V = np.linalg.eigh(R)
    X = (V * np.sqrt(w)) @ V.conj().T * np.sqrt(M)
    # the first window ends exactly at the first peak, the second starts exactly at the second
    win = estimate_windowed(X, pos, 2, (-90.0, 0.01, 18000), "music", [(5700, 5871), (10270, 10400)])
    assert 5870 not in win.all_peaks and 10270 not in win.all_peaks
    # one point more on each side makes both interior again
    win = estimate_windowed(X, pos, 2, (-90.0, 0.01, 18000), "music", [(5700, 5872), (10269, 10400)])
    assert sorted(win.peaks) == [5870, 10270]


def test_peaks_of_windows_equal_brute_force():
    # random spectra: the windowed peaks are those l with both neighbours in the same window,
    # P[l] > P[l-1], and the run of values equal to P[l] ending inside the window in a smaller value
    from oracle.doa import find_peaks
    rng = np.random.default_rng(5)
    for trial in range(200):
        L = int(rng.integers(5, 60))
        P = rng.integers(0, 4, size=L).astype(float)
        cuts = sorted(set(int(c) for c in rng.integers(0, L + 1, size=4)))
        wins = [(a, b) for a, b in zip(cuts[:-1], cuts[1:]) if b > a][::2]
        got = []
        for a, b in wins:
            got.extend(int(i) + a for i in find_peaks(P[a:b]))
        brute = []
        for a, b in wins:
            for l in range(a + 1, b - 1):
                if not P[l] > P[l - 1]:
                    continue
                r = l
                while r < b and P[r] == P[l]:
                    r += 1
                if r < b and P[r] < P[l]:
                    brute.append(l)
        assert sorted(got) == sorted(brute), (P, wins)


def test_proposal_windows_threshold_nan_and_bin_width():
    s = np.full(180, -3.0)
    s[100] = 2.0                                   # centre 10.5 deg
    assert mlp.proposal_windows(s, 1, 1.0, -90.0, 0.01, 18000, threshold=0.0) == [(9950, 10151)]
    assert mlp.proposal_windows(s, 1, 1.0, -90.0, 0.01, 18000, threshold=2.5) == [(0, 18000)]
    s2 = np.full(180, np.nan)
    assert mlp.proposal_windows(s2, 3, 1.0, -90.0, 0.01, 18000, threshold=-1e30) == [(0, 18000)]
    assert mlp.proposal_windows(s2, 3, 1.0, -90.0, 0.01, 18000) == []
    s[7] = np.nan                                  # NaN never chosen, even among few bins
    got = mlp.proposal_windows(s, 2, 0.5, -90.0, 0.01, 18000)
    # bins 100 then 0 (lowest index among the -3.0 ties): centres 10.5 and -89.5
    assert got == [(0, 101), (10000, 10101)]
    # 90 bins of 2 degrees: bin 45 covers [0, 2), centre 1.0
    s3 = np.zeros(90)
    s3[45] = 1.0
    assert mlp.proposal_windows(s3, 1, 1.0, -90.0, 0.5, 360) == [(180, 185)]
    # a bin outside a partial grid gives an empty window, which is dropped
    assert mlp.proposal_windows(s, 1, 1.0, 20.0, 0.01, 1000) == []


def test_proposal_windows_floor_keeps_the_first_n_sure_bins():
    # scores 3 > 2 > 1 > 0.5 > 0.2 at bins 10, 50, 90, 130, 170 (centres -79.5, -39.5, 0.5, 40.5, 80.5)
    s = np.full(180, -5.0)
    for b, v in ((10, 3.0), (50, 2.0), (90, 1.0), (130, 0.5), (170, 0.2)):
        s[b] = v
    args = (5, 0.5, -90.0, 0.01, 18000)
    win = {10: (1000, 1101), 50: (5000, 5101), 90: (9000, 9101), 130: (13000, 13101), 170: (17000, 17101)}
    assert mlp.proposal_windows(s, *args) == [win[b] for b in (10, 50, 90, 130, 170)]
    # floor 0.75: the first two bins always, then only the one at score 1
    assert mlp.proposal_windows(s, *args, n_sure=2, floor=0.75) == [win[b] for b in (10, 50, 90)]
    # the first n_sure bins stay even below the floor
    assert mlp.proposal_windows(s, *args, n_sure=4, floor=10.0) == [win[b] for b in (10, 50, 90, 130)]
    assert mlp.proposal_windows(s, *args, n_sure=0, floor=10.0) == []
    # a floor at or below every chosen score changes nothing; topk still caps the count
    assert mlp.proposal_windows(s, 3, 0.5, -90.0, 0.01, 18000, n_sure=1, floor=-5.0) == [win[b] for b in (10, 50, 90)]
    # the threshold's whole-grid fallback is unaffected by the floor
    assert mlp.proposal_windows(s, *args, threshold=4.0, n_sure=1, floor=0.0) == [(0, 18000)]


def test_proposal_windows_with_fewer_finite_bins_than_topk():
    # -inf scores stay eligible (lowest first by bin), NaN never; no bin is chosen twice
    s = np.full(180, np.nan)
    s[40], s[100] = 1.0, -np.inf
    s[120] = -np.inf
    got = mlp.proposal_windows(s, 5, 0.5, -90.0, 0.01, 18000)
    assert got == [(4000, 4101), (10000, 10101), (12000, 12101)]   # centres -49.5, 10.5, 30.5


def test_proposed_estimate_rescues_a_missed_source():
    # scores that point at only one of two sources: the windows hold one peak, so the search runs
    # again over the whole grid and equals the plain estimate (non-circular grid: a whole-grid
    # window is the plain search)
    pos, X = _frame(seed=3, th=(-31.3, 12.7))
    grid = (-90.0, 0.01, 18000)
    full = estimate(X, pos, 2, grid, "music")
    s = np.full(180, -5.0)
    s[int(np.floor(-31.3 + 90))] = 3.0
    est, fb, rescued = mlp.estimate_proposed(X, pos, 2, grid, "music", s, 6, 1.0, 0.0)
    assert not fb and rescued
    assert np.array_equal(est.peaks, full.peaks) and np.array_equal(est.P, full.P)
    # both sources scored: no rescue, the windowed search alone finds both
    s[int(np.floor(12.7 + 90))] = 2.5
    est2, fb2, rescued2 = mlp.estimate_proposed(X, pos, 2, grid, "music", s, 6, 1.0, 0.0)
    assert not fb2 and not rescued2
    assert sorted(est2.peaks) == sorted(full.peaks)
    assert np.isnan(est2.P).sum() > 17000          # only the windows were scanned
    # a peak on a window's end: the window [l0, p + 1) ends at the first source's peak index
    p = int(full.peaks[np.argmin(full.angles[full.peaks])])
    wins = [(p - 150, p + 1)]
    w = estimate_windowed(X, pos, 2, grid, "music", wins)
    assert p not in w.all_peaks


def test_proposed_estimate_threshold_fallback_is_not_rescued():
    # every score below the threshold: one whole-grid window, flagged as fallback, never rescued
    pos, X = _frame(seed=4)
    grid = (-90.0, 0.1, 1800)
    s = np.full(180, -2.0)
    est, fb, rescued = mlp.estimate_proposed(X, pos, 2, grid, "ev", s, 6, 1.0, 0.0)
    assert fb and not rescued
    full = estimate(X, pos, 2, grid, "ev")
    assert np.array_equal(est.peaks, full.peaks)
    # a frame whose whole spectrum has fewer than D peaks stays with fewer after the rescue: a
    # 5-point grid 8..12 deg around one source at 10 deg; the window of bin 100 holds 10 and 11 deg
    # only (no interior point), the whole grid one peak, at 10 deg
    pos1, X1 = _frame(seed=5, th=(10.0,))
    g1 = (8.0, 1.0, 5)
    s1 = np.full(180, -5.0)
    s1[100] = 4.0
    assert mlp.proposal_windows(s1, 1, 1.0, *g1, threshold=0.0) == [(2, 4)]
    e1, fb1, r1 = mlp.estimate_proposed(X1, pos1, 2, g1, "music", s1, 1, 1.0, 0.0)
    f1 = estimate(X1, pos1, 2, g1, "music")
    assert r1 and not fb1
    assert list(e1.peaks) == list(f1.peaks) == [2]


def test_score_peaks_brute_force_and_cases():
    # hand cases: plateau at its first bin, a shoulder plateau that rises is no peak, ends count,
    # NaN is -inf and never a peak itself
    assert mlp.score_peaks(np.array([0.0, 2.0, 2.0, 1.0, 3.0])).tolist() == [1, 4]
    assert mlp.score_peaks(np.array([1.0, 2.0, 2.0, 3.0, 0.0])).tolist() == [3]
    assert mlp.score_peaks(np.array([5.0, 1.0, 1.0, 1.0])).tolist() == [0]
    assert mlp.score_peaks(np.array([1.0, 1.0, 1.0])).tolist() == [0]
    assert mlp.score_peaks(np.array([np.nan, 1.0, np.nan, 0.5])).tolist() == [1, 3]
    assert mlp.score_peaks(np.array([-np.inf, -np.inf, 0.0])).tolist() == [2]
    # brute force: a bin is a peak iff it is not NaN and no bin of its maximal equal run has a
    # larger neighbour, and the bin before the run (if any) is smaller
    rng = np.random.default_rng(3)
    for trial in range(300):
        s = rng.integers(0, 4, size=rng.integers(1, 12)).astype(np.float64)
        s[rng.uniform(size=len(s)) < 0.15] = np.nan
        v = np.where(np.isnan(s), -np.inf, s)
        ref = []
        for b in range(len(s)):
            if np.isnan(s[b]) or (b > 0 and v[b - 1] >= v[b]):
                continue
            e = b
            while e + 1 < len(s) and v[e + 1] == v[b]:
                e += 1
            if e + 1 < len(s) and v[e + 1] > v[b]:
                continue
            ref.append(b)
        assert mlp.score_peaks(s).tolist() == ref, (trial, s)


def test_proposal_windows_local_max_bins():
    # a source's bin and both its neighbours score high: only the best of the three gets a window;
    # the threshold test still uses the best score
    s = np.full(180, -4.0)
    s[99], s[100], s[101] = 2.5, 3.0, 2.8          # centres 9.5, 10.5, 11.5
    s[40] = 1.0
    args = (3, 1.0, -90.0, 0.01, 18000)
    # top 3 bins without the rule: the source's three, merged into one 3-degree window
    assert mlp.proposal_windows(s, *args) == [(9850, 10251)]
    # with it: the source's best bin and the next local maximum (bin 40)
    assert mlp.proposal_windows(s, *args, local_max=True) == [(3950, 4151), (9950, 10151)]
    got = mlp.proposal_windows(s, 2, 1.0, -90.0, 0.01, 18000, local_max=True)
    assert got == [(3950, 4151), (9950, 10151)]
    assert mlp.proposal_windows(s, 2, 1.0, -90.0, 0.01, 18000, threshold=3.0, local_max=True) == got
    assert mlp.proposal_windows(s, 2, 1.0, -90.0, 0.01, 18000, threshold=3.1, local_max=True) == [(0, 18000)]
