"""GPU parity of the proposal network kernels against the MLP oracle.

The kernels round both operands of every matrix product to bfloat16 and accumulate in FP32.  The
ReLU decisions of the network are taken on those values, so the parity comparison runs the
oracle in its bfloat16-operand mode (the same roundings, FP64 products and sums): the remaining
differences are FP32 accumulation and storage (K <= 512 terms: about 512 * 2^-24 relative), and
the gates are, per layer, gradient-norm relative error <= 1e-3 with cosine >= 0.9999, and logits
within 1e-4 (relative to the largest) in all but a few rows: a hidden value that lies within the
FP32-vs-FP64 accumulation difference of a bfloat16 rounding boundary rounds the other way on one
side (about 2^-24 / 2^-9 of the values), which moves that row's logits by up to one bfloat16
step of that value times its weights.  Against the exact FP64 oracle the differences are bfloat16-sized and
include ReLU decisions flipped by rounding; those are reported, with a cosine gate of 0.99.
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
    assert abs(float(loss.item()) - lo16) <= 1e-5 * lo16
    g = nd.unflatten_params(net.gradients().astype(np.float64), SIZES)
    for li in range(3):
        for which, name in ((0, "W"), (1, "b")):
            a = g[li][which].ravel()
            for ref, tag, rel_gate, cos_gate in ((grads16, "bf16-operand", 1e-3, 0.9999), (grads, "FP64", 5e-2, 0.99)):
                b = ref[li][which].ravel()
                rel = abs(np.linalg.norm(a) - np.linalg.norm(b)) / np.linalg.norm(b)
                cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
                print("layer %d %s vs %s oracle: norm rel %.2e cos %.7f" % (li + 1, name, tag, rel, cos), flush=True)
                assert rel <= rel_gate and cos >= cos_gate, (li, name, tag, rel, cos)


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
