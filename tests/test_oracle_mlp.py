"""Pins for the learned-proposal oracle: gradients by central differences, closed forms of the
loss and of Adam (first step, every step of a constant gradient, every step of an alternating one,
gradient-scale invariance), feature invariances, bin labels and window arithmetic.  The Adam pins
are written as checks of a callable so that test_oracle_mutants.py can show that each of several
planted mistakes fails one of them."""

import numpy as np
import pytest

from oracle import mlp


def _small(seed=3):
    rng = np.random.default_rng(seed)
    params = mlp.init_params(seed, sizes=(7, 6, 5, 4))
    # nonzero biases so that every term of the gradient is exercised
    params = [(W, rng.normal(0, 0.1, size=b.shape)) for W, b in params]
    X = rng.normal(size=(5, 7))
    y = (rng.uniform(size=(5, 4)) < 0.3).astype(float)
    return params, X, y


def test_gradients_match_central_differences():
    params, X, y = _small()
    loss, grads = mlp.backward(params, X, y)
    h = 1e-6
    for li in range(3):
        for which in (0, 1):
            P = params[li][which]
            G = grads[li][which]
            it = np.nditer(P, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = P[idx]
                P[idx] = old + h
                lp = mlp.bce_with_logits(mlp.forward(params, X)[0], y)
                P[idx] = old - h
                lm = mlp.bce_with_logits(mlp.forward(params, X)[0], y)
                P[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - G[idx]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9, (li, which, idx, fd, G[idx])


def test_bce_closed_forms():
    assert abs(mlp.bce_with_logits(np.zeros((2, 3)), np.ones((2, 3))) - np.log(2.0)) < 1e-15
    assert mlp.bce_with_logits(np.array([[40.0]]), np.array([[1.0]])) < 1e-17
    assert abs(mlp.bce_with_logits(np.array([[40.0]]), np.array([[0.0]])) - 40.0) < 1e-12
    # symmetry: L(z, y) = L(-z, 1 - y)
    z = np.array([[0.3, -2.0, 5.0]])
    y = np.array([[1.0, 0.0, 1.0]])
    assert abs(mlp.bce_with_logits(z, y) - mlp.bce_with_logits(-z, 1 - y)) < 1e-15


def test_adam_first_step_closed_form():
    params, X, y = _small()
    _, grads = mlp.backward(params, X, y)
    m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    lr = 1e-3
    newp, _, _ = mlp.adam_step(params, grads, m, v, 1, lr)
    for (W, b), (W2, b2), (gW, gb) in zip(params, newp, grads):
        # bias-corrected first step: delta = -lr * g / (|g| + eps)
        assert np.allclose(W2 - W, -lr * gW / (np.abs(gW) + 1e-8), rtol=1e-12, atol=1e-18)
        assert np.allclose(b2 - b, -lr * gb / (np.abs(gb) + 1e-8), rtol=1e-12, atol=1e-18)


B1, B2, EPS = 0.9, 0.999, 1e-8


def _tree(rng):
    """A small parameter-shaped list [(W, b)] of random values."""
    return [(rng.normal(size=(3, 2)), rng.normal(size=3)), (rng.normal(size=(2, 3)), rng.normal(size=2))]


def _zeros(tree):
    return [(np.zeros_like(W), np.zeros_like(b)) for W, b in tree]


def check_adam_constant_gradient(adam, steps=7, lr=1e-3):
    """A constant gradient g gives m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2, so the bias-corrected
    moments are exactly g and g^2 and every step is -lr g / (|g| + eps): p_t = p_0 - t lr g / (|g| + eps)."""
    rng = np.random.default_rng(11)
    p0 = _tree(rng)
    g = [(rng.normal(size=W.shape) * 10.0 ** rng.uniform(-4, 1, size=W.shape),
          rng.normal(size=b.shape) * 10.0 ** rng.uniform(-4, 1, size=b.shape)) for W, b in p0]
    p, m, v = p0, _zeros(p0), _zeros(p0)
    for t in range(1, steps + 1):
        p, m, v = adam(p, g, m, v, t, lr)
        for (W, b), (W0, b0), (gW, gb) in zip(p, p0, g):
            assert np.allclose(W, W0 - t * lr * gW / (np.abs(gW) + EPS), rtol=1e-12, atol=1e-15), t
            assert np.allclose(b, b0 - t * lr * gb / (np.abs(gb) + EPS), rtol=1e-12, atol=1e-15), t


def check_adam_alternating_gradient(adam, steps=8, lr=1e-2):
    """g_t = (-1)^(t+1) g: v_t is as for a constant gradient, and the geometric series gives
    m_t = (1 - b1) (-1)^(t+1) g (1 - (-b1)^t) / (1 + b1), so step t moves p by
    -lr m_t / (1 - b1^t) / (|g| + eps)."""
    rng = np.random.default_rng(12)
    p0 = _tree(rng)
    g = [(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in p0]
    p, m, v = p0, _zeros(p0), _zeros(p0)
    for t in range(1, steps + 1):
        sgn = (-1.0) ** (t + 1)
        gt = [(sgn * gW, sgn * gb) for gW, gb in g]
        pn, m, v = adam(p, gt, m, v, t, lr)
        coef = (1 - B1) * sgn * (1 - (-B1) ** t) / (1 + B1) / (1 - B1 ** t)
        for (W, b), (Wn, bn), (gW, gb) in zip(p, pn, g):
            assert np.allclose(Wn - W, -lr * coef * gW / (np.abs(gW) + EPS), rtol=1e-10, atol=1e-17), t
            assert np.allclose(bn - b, -lr * coef * gb / (np.abs(gb) + EPS), rtol=1e-10, atol=1e-17), t
        p = pn


def check_adam_scale_invariance(adam, steps=5, lr=1e-3):
    """With eps = 0 the update depends on the gradients only through their ratios: scaling every
    gradient of a sequence by c > 0 leaves every step unchanged, and negating them negates it."""
    rng = np.random.default_rng(13)
    p0 = _tree(rng)
    seq = [[(rng.normal(size=W.shape), rng.normal(size=b.shape)) for W, b in p0] for _ in range(steps)]
    runs = {}
    for c in (1.0, 1e-5, 3e4, -1.0):
        p, m, v = p0, _zeros(p0), _zeros(p0)
        for t, g in enumerate(seq, start=1):
            p, m, v = adam(p, [(c * gW, c * gb) for gW, gb in g], m, v, t, lr, eps=0.0)
        runs[c] = [x - x0 for layer, layer0 in zip(p, p0) for x, x0 in zip(layer, layer0)]
    for c in (1e-5, 3e4, -1.0):
        for d, d1 in zip(runs[c], runs[1.0]):
            assert np.allclose(d, np.sign(c) * d1, rtol=1e-12, atol=1e-15), c


def test_adam_constant_gradient_every_step():
    check_adam_constant_gradient(mlp.adam_step)


def test_adam_alternating_gradient_closed_form():
    check_adam_alternating_gradient(mlp.adam_step)


def test_adam_gradient_scale_invariance():
    check_adam_scale_invariance(mlp.adam_step)


def test_features_layout_and_invariance():
    rng = np.random.default_rng(0)
    Z = rng.normal(size=(16, 40)) + 1j * rng.normal(size=(16, 40))
    R = Z @ Z.conj().T / 40
    f = mlp.features(R)
    assert f.shape == (272,)
    assert np.allclose(mlp.features(3.7 * R), f, rtol=1e-14, atol=1e-15)
    # diagonal entries sit at the start of each row of the upper triangle; their imaginary parts are 0
    pos, diag_re = 0, []
    for i in range(16):
        assert abs(f[2 * pos + 1]) < 1e-14
        diag_re.append(f[2 * pos])
        pos += 16 - i
    assert abs(sum(diag_re) - 16.0) < 1e-12          # trace of M R / trace(R)
    # first row: element (0, 1) follows (0, 0)
    Rn = R * 16 / np.trace(R).real
    assert np.isclose(f[2], Rn[0, 1].real) and np.isclose(f[3], Rn[0, 1].imag)


def test_bin_labels():
    y = mlp.bin_labels([-90.0, -0.5, 0.0, 89.999])
    assert y.sum() == 4 and y[0] == y[89] == y[90] == y[179] == 1
    assert mlp.bin_labels([90.0])[179] == 1          # clipped


def test_proposal_windows_arithmetic():
    s = np.zeros(180)
    s[90] = 0.9                                       # bin 90 = [0, 1) deg, centre 0.5
    w = mlp.proposal_windows(s, 1, 1.0, -90.0, 0.001, 180000)
    assert w == [(89500, 91501)]                      # -0.5 .. 1.5 deg inclusive: 2001 points
    s[91] = 0.8
    w = mlp.proposal_windows(s, 2, 1.0, -90.0, 0.001, 180000)
    assert w == [(89500, 92501)]                      # overlapping windows merge
    s[0] = 0.95                                       # centre -89.5: clipped at the grid start
    w = mlp.proposal_windows(s, 3, 1.0, -90.0, 0.001, 180000)
    assert w[0] == (0, 1501)


def test_bf16_round_matches_the_format():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(9)
    x = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 1e-3, 500), rng.normal(0, 1e4, 500)])
    # exact ties between two bfloat16 neighbours: 1 + 2^-8 (tie, rounds to even 1.0) and
    # 1 + 3 * 2^-8 (tie, rounds up to the even 1 + 2^-6), negative mirrors
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), -(1 + 3 * 2.0 ** -8)])
    x = np.concatenate([x, ties])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)
    assert mlp.bf16_round(ties).tolist() == [1.0, 1 + 2.0 ** -6, -1.0, -(1 + 2.0 ** -6)]


def test_bf16_mode_rounds_every_product_operand():
    params, X, y = _small()
    _, g = mlp.backward(params, X, y, precision="bf16")
    # rounding X or the weights beforehand changes nothing: they are rounded at every use
    _, gx = mlp.backward(params, mlp.bf16_round(X), y, precision="bf16")
    pr = [(mlp.bf16_round(W), b) for W, b in params]
    _, gw = mlp.backward(pr, X, y, precision="bf16")
    for a, b, c in zip(g, gx, gw):
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[0], c[0])
        assert np.array_equal(a[1], b[1]) and np.array_equal(a[1], c[1])
    # and the result is within bfloat16 rounding of the exact gradient, not equal to it
    _, g64 = mlp.backward(params, X, y)
    for (gw_, gb_), (ew, eb) in zip(g, g64):
        rel = np.linalg.norm(gw_ - ew) / np.linalg.norm(ew)
        assert 0 < rel < 0.05


def test_init_params_he_uniform():
    # He-uniform: W_l (out x in) uniform on [-sqrt(6/in), sqrt(6/in)] (variance 2/in), zero biases,
    # a function of the seed only
    p = mlp.init_params(21)
    assert [W.shape for W, _ in p] == [(512, 272), (512, 512), (180, 512)]
    for (W, b), fin in zip(p, (272, 512, 512)):
        lim = np.sqrt(6.0 / fin)
        n = W.size
        assert np.all(b == 0.0)
        assert np.all(np.abs(W) <= lim) and np.abs(W).max() > lim * (1 - 20.0 / n)
        assert abs(W.mean()) < 5 * lim / np.sqrt(3 * n)
        assert abs(W.var() / (2.0 / fin) - 1) < 5 * np.sqrt(0.8 / n)
        # uniform: each tenth of the interval holds a tenth of the values (5 sigma)
        h, _ = np.histogram(W, bins=10, range=(-lim, lim))
        assert np.all(np.abs(h - n / 10) < 5 * np.sqrt(n * 0.09))
    q = mlp.init_params(21)
    r = mlp.init_params(22)
    assert all(np.array_equal(a[0], c[0]) for a, c in zip(p, q))
    assert not np.array_equal(p[0][0], r[0][0])


def test_bf16_operand_gradients_within_the_rounding_bound():
    # The oracle's bfloat16-operand mode is one admissible rounding of every GEMM operand, so its
    # gradients must lie inside the probabilistic bound the GPU gradients are gated with; a bound
    # that wrongly drops a propagation term (here: the layer-2 decision uncertainty) fails.
    from mlp_bounds import gradient_bounds
    for seed, B in ((5, 257), (3, 64)):
        params = mlp.init_params(seed)
        rng = np.random.default_rng(seed)
        X = rng.normal(0, 1, size=(B, 272))
        Y = (rng.uniform(size=(B, 180)) < 0.02).astype(np.float64)
        bounds, risk = gradient_bounds(params, X, Y)
        _, g64 = mlp.backward(params, X, Y)
        _, g16 = mlp.backward(params, X, Y, precision="bf16")
        assert 0.0 < risk[0] < 0.1 and 0.0 < risk[1] < 0.1
        worst = 0.0
        for li in range(3):
            for w in range(2):
                worst = max(worst, float(np.max(np.abs(g16[li][w] - g64[li][w]) / bounds[li][w])))
        assert worst < 1.0, (seed, worst)
        # the bound is not vacuous for the output layer: well below the gradient itself
        assert np.median(bounds[2][0] / (np.abs(g64[2][0]) + 1e-300)) < 0.1
