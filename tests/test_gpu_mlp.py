"""GPU parity of the proposal network kernels against the FP64 MLP oracle.

The kernels round both operands of every matrix product to bfloat16 (unit roundoff 2^-9) and
accumulate in FP32.  Each product then carries a relative error of at most about 2^-8, and the
errors of the K <= 512 products of a sum are independent with random signs, so a gradient
component's relative error is of order 2^-8 only where its terms do not cancel; summed over a
layer (hundreds of thousands of components) the error vector's norm stays near 2^-8 of the
gradient's, i.e. a cosine of about 1 - 2^-17, plus the rare hidden units whose ReLU decision flips
under the rounding.  The binding gates are those of the learned-proposal oracle step: per layer the
gradient norm within 1e-2 relative and cosine >= 0.999 against the exact FP64 oracle, the logits
within 3e-2 of the largest.  Adam is checked step by step, at t = 1..5, against the oracle's update
applied to the kernels' own gradients and moments (FP32 arithmetic against FP64: a few ulps).  The
oracle's bfloat16-operand mode (the same operand roundings in FP64) is printed beside the FP64
figures as a diagnostic only: it shows how much of the difference is operand rounding.
"""

import numpy as np
import pytest

from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = (272, 512, 512, 180)


def _setup(batch, seed=5):
    import paper_2007_14135_amd as nd
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    params = omlp.init_params(seed)
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, size=(batch, 272))
    Y = (rng.uniform(size=(batch, 180)) < 0.02).astype(np.float64)
    net = nd.MLP(*SIZES[:2], SIZES[3], max_batch=max(batch, 64))
    net.load_params(nd.flatten_params(params))
    return nd, net, params, X, Y


def test_forward_matches_oracle():
    nd, net, params, X, Y = _setup(300)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    logits = torch.empty(300, 180, dtype=torch.float32, device="cuda")
    net.forward(Xd, logits)
    torch.cuda.synchronize()
    z16, _ = omlp.forward(params, X, precision="bf16")
    z, _ = omlp.forward(params, X)
    got = logits.cpu().numpy()
    scale = max(1.0, np.abs(z).max())
    row16 = np.abs(got - z16).max(axis=1)
    err = np.abs(got - z).max()
    off = int(np.sum(row16 > 1e-4 * scale))
    print("forward |dz| vs bf16-operand oracle: median row %.2e, max %.2e, %d of %d rows above 1e-4; "
          "vs FP64 oracle max %.3e (max |z| %.2f)" % (np.median(row16), row16.max(), off, len(row16), err, scale),
          flush=True)
    assert off <= max(3, len(row16) // 50)
    assert row16.max() <= 1e-2 * scale
    assert err <= 3e-2 * scale


def test_gradients_match_oracle():
    nd, net, params, X, Y = _setup(257)       # ragged batch (not a multiple of the 64-row tile)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Yd = torch.tensor(Y, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.train_step(Xd, Yd, 0.0, loss)          # lr = 0: parameters unchanged, gradients kept
    torch.cuda.synchronize()
    lo16, grads16 = omlp.backward(params, X, Y, precision="bf16")
    lo, grads = omlp.backward(params, X, Y)
    assert abs(float(loss.item()) - lo) <= 1e-3 * lo
    print("loss %.7f, FP64 oracle %.7f (bf16-operand oracle %.7f)" % (float(loss.item()), lo, lo16), flush=True)
    g = nd.unflatten_params(net.gradients().astype(np.float64), SIZES)
    _gate_gradients(g, grads, grads16)


def _gate_gradients(g, grads, grads16=None, tag=""):
    for li in range(3):
        for which, name in ((0, "W"), (1, "b")):
            a = g[li][which].ravel()
            b = grads[li][which].ravel()
            rel = abs(np.linalg.norm(a) - np.linalg.norm(b)) / np.linalg.norm(b)
            cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
            diag = ""
            if grads16 is not None:
                c = grads16[li][which].ravel()
                diag = "; bf16-operand oracle (diagnostic): norm rel %.2e cos %.7f" % (
                    abs(np.linalg.norm(a) - np.linalg.norm(c)) / np.linalg.norm(c),
                    a @ c / (np.linalg.norm(a) * np.linalg.norm(c)))
            print("%slayer %d %s vs FP64 oracle: norm rel %.2e cos %.7f%s" % (tag, li + 1, name, rel, cos, diag),
                  flush=True)
            assert rel <= 1e-2 and cos >= 0.999, (tag, li, name, rel, cos)


def test_adam_steps_match_oracle():
    # five training steps; at each one the gradients are gated against the FP64 oracle at the
    # network's current parameters, and the update against the oracle's Adam step t applied to
    # the kernels' gradients and moments (bias corrections 1 - beta^t change with t)
    nd, net, params, X, Y = _setup(192, seed=11)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Yd = torch.tensor(Y, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    lr = 2e-3
    for t in range(1, 6):
        p0, m0, v0, step0 = net.state()
        assert step0 == t - 1
        net.train_step(Xd, Yd, lr, loss)
        torch.cuda.synchronize()
        p1, m1, v1, step1 = net.state()
        assert step1 == t
        g = net.gradients().astype(np.float64)
        P0 = nd.unflatten_params(p0.astype(np.float64), SIZES)
        _, gref = omlp.backward(P0, X, Y)
        _gate_gradients(nd.unflatten_params(g, SIZES), gref, tag="step %d: " % t)
        G = nd.unflatten_params(g, SIZES)
        Mo = nd.unflatten_params(m0.astype(np.float64), SIZES)
        Vo = nd.unflatten_params(v0.astype(np.float64), SIZES)
        pn, mn, vn = omlp.adam_step(P0, G, Mo, Vo, t, lr)
        pe, me, ve = (nd.flatten_params(x) for x in (pn, mn, vn))
        # FP32 moment updates: a few roundings of the two terms' magnitudes (m may cancel)
        dm = np.abs(m1 - me) / (0.9 * np.abs(m0) + 0.1 * np.abs(g) + 1e-38)
        dv = np.abs(v1 - ve) / (0.999 * np.abs(v0) + 0.001 * g * g + 1e-45)
        # FP32 storage of p and the FP32 step (a value of magnitude <= lr / (1 - beta1^t) * ...)
        dp = np.abs(p1 - pe) / (np.spacing(np.abs(pe).astype(np.float32)).astype(np.float64) + lr * 2.0 ** -20)
        print("Adam step %d: max rel m %.2e, v %.2e; max |dp| %.2f ulp-units" % (t, dm.max(), dv.max(), dp.max()),
              flush=True)
        assert dm.max() <= 2.0 ** -20 and dv.max() <= 2.0 ** -20 and dp.max() <= 4.0, (t, dm.max(), dv.max(), dp.max())


def test_adam_step_and_checkpoint_roundtrip():
    nd, net, params, X, Y = _setup(128)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Yd = torch.tensor(Y, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.train_step(Xd, Yd, 1e-3, loss)
    torch.cuda.synchronize()
    g = net.gradients().astype(np.float64)
    p1, m1, v1, step = net.state()
    p0 = nd.flatten_params(params)
    assert step == 1
    # first Adam step from zero moments: m = 0.1 g, v = 0.001 g^2, delta = -lr g / (|g| + eps)
    assert np.allclose(m1, 0.1 * g, rtol=1e-5, atol=1e-12)
    expect = p0 - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(p1 - expect)) <= 1e-6
    # checkpoint -> new network -> one more step must equal continuing the original (bit for bit)
    blob = net.save()
    net2 = nd.MLP(272, 512, 180, max_batch=128)
    net2.load(blob)
    l1 = torch.zeros(1, dtype=torch.float32, device="cuda")
    l2 = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.train_step(Xd, Yd, 1e-3, l1)
    net2.train_step(Xd, Yd, 1e-3, l2)
    torch.cuda.synchronize()
    a, b = net.state(), net2.state()
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    assert a[3] == b[3] == 2 and float(l1.item()) == float(l2.item())


def test_training_reduces_loss_on_a_small_batch():
    nd, net, params, X, Y = _setup(64)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Yd = torch.tensor(Y, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    losses = []
    for _ in range(60):
        net.train_step(Xd, Yd, 3e-3, loss)
        losses.append(float(loss.item()))
    print("overfit: loss %.4f -> %.4f" % (losses[0], losses[-1]), flush=True)
    assert losses[-1] < 0.2 * losses[0]
