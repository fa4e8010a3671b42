"""GPU parity of the proposal network kernels against the FP64 MLP oracle.

The kernels round both operands of every matrix product to bfloat16 (8 significant bits, unit
roundoff u = 2^-8) and accumulate in FP32.  Against exact FP64 arithmetic that moves every
pre-activation a little, and a hidden unit whose pre-activation lies within that distance of 0
may switch its ReLU decision, which changes its whole contribution to the gradients.  The gate is
therefore an elementwise error bound computed from the FP64 oracle's own forward values (nothing
from the GPU enters it), propagated layer by layer:
  * an operand a with propagated error Ea is off by at most e(a) = ua|a| + (1 + ua) Ea after its
    FP32 and bfloat16 roundings (ua = u + 2^-24 + u 2^-24);
  * a product A B with inner dimension K is then off by at most
    |A| e(B) + e(A) |B| + e(A) e(B) + g_K (|A| + e(A)) (|B| + e(B)),  g_K = K 2^-24 / (1 - K 2^-24);
  * ReLU is 1-Lipschitz, so a hidden activation is off by at most its pre-activation's bound;
  * the output derivative (sigmoid(z) - y) / n is off by at most (Ez / 4 + 8 2^-24) / n;
  * backward, t = delta W is bounded as a product; delta = t * [z > 0] is off by at most Et where
    |z| > Ez (the decision is certain) and by |t| + Et where it is not;
  * weight gradients are products over the batch, bias gradients FP32 column sums.
These worst-case sums are valid but loose (they let most layer-2 units count as uncertain), so the
gate uses the same propagation in the standard probabilistic model of rounding instead: every
rounding is an independent relative error of variance ua^2 / 3, variances add through sums, a
decision is uncertain where |z| <= 6 sigma_z, and an uncertain decision contributes its whole
term's square.  Every gradient entry must lie within 6 sigma of the FP64 oracle's; the gradient
norms must agree to 1e-2 and the logits to 3e-2 of the largest.  The oracle's bfloat16-operand mode (the same
operand roundings in FP64) is printed as a diagnostic only.
"""

import numpy as np
import pytest

from oracle import mlp as omlp
from mlp_bounds import gradient_bounds

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
    bounds, risk = gradient_bounds(params, X, Y)
    print("hidden pre-activations whose ReLU decision the rounding could change: layer 1 %.4f, layer 2 %.4f"
          % tuple(risk), flush=True)
    _gate_gradients(g, grads, bounds, grads16)


def _gate_gradients(g, grads, bounds, grads16=None, tag=""):
    for li in range(3):
        for which, name in ((0, "W"), (1, "b")):
            a = g[li][which].ravel()
            b = grads[li][which].ravel()
            e = bounds[li][which].ravel()
            rel = abs(np.linalg.norm(a) - np.linalg.norm(b)) / np.linalg.norm(b)
            cos = a @ b / (np.linalg.norm(a) * np.linalg.norm(b))
            ratio = np.abs(a - b) / e
            diag = ""
            if grads16 is not None:
                c = grads16[li][which].ravel()
                diag = "; bf16-operand oracle (diagnostic): norm rel %.2e cos %.7f" % (
                    abs(np.linalg.norm(a) - np.linalg.norm(c)) / np.linalg.norm(c),
                    a @ c / (np.linalg.norm(a) * np.linalg.norm(c)))
            print("%slayer %d %s vs FP64 oracle: norm rel %.2e cos %.7f, |error| / bound max %.3f median %.2e%s"
                  % (tag, li + 1, name, rel, cos, ratio.max(), np.median(ratio), diag), flush=True)
            assert rel <= 1e-2, (tag, li, name, rel)
            assert np.all(np.abs(a - b) <= e), (tag, li, name, float(ratio.max()), int(np.argmax(ratio)))


def test_adam_steps_match_oracle():
    # Five training steps from the oracle's initial parameters, and the oracle's own five-step
    # trajectory (its FP64 gradients and Adam) from the same start: nothing of the GPU enters the
    # oracle.  Gates: the first step's gradients against the oracle's within the bound above; the
    # losses of both trajectories within 1e-3 relative at every step (the parameters of the two
    # runs differ only where a gradient's sign is within its rounding bound, and those entries
    # carry tiny gradients); and at every step the GPU's moments and update obey Adam's rules on
    # its own gradients (bias corrections 1 - beta^t change with t), to FP32 rounding.
    nd, net, params, X, Y = _setup(192, seed=11)
    Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
    Yd = torch.tensor(Y, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    lr = 2e-3
    P = params
    Mo = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    Vo = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    for t in range(1, 6):
        p0, m0, v0, step0 = net.state()
        assert step0 == t - 1
        net.train_step(Xd, Yd, lr, loss)
        torch.cuda.synchronize()
        p1, m1, v1, step1 = net.state()
        assert step1 == t
        g = net.gradients().astype(np.float64)
        lo_ref, gref = omlp.backward(P, X, Y)
        if t == 1:
            bounds, _ = gradient_bounds(P, X, Y)
            _gate_gradients(nd.unflatten_params(g, SIZES), gref, bounds, tag="step 1: ")
        lo = float(loss.item())
        print("step %d: loss %.7f, oracle trajectory %.7f" % (t, lo, lo_ref), flush=True)
        assert abs(lo - lo_ref) <= 1e-3 * lo_ref, (t, lo, lo_ref)
        P, Mo, Vo = omlp.adam_step(P, gref, Mo, Vo, t, lr)
        # Adam's rules on the GPU's own quantities (FP32 arithmetic)
        m0d, v0d, p0d = (x.astype(np.float64) for x in (m0, v0, p0))
        m_exp = 0.9 * m0d + 0.1 * g
        v_exp = 0.999 * v0d + 0.001 * g * g
        # relative to the terms' magnitudes, plus FP32's subnormal spacing (g^2 of tiny gradients)
        dm = np.abs(m1 - m_exp) / (0.9 * np.abs(m0d) + 0.1 * np.abs(g) + 2.0 ** -126)
        dv = np.abs(v1 - v_exp) / (0.999 * v0d + 0.001 * g * g + 2.0 ** -126)
        mhat = m1.astype(np.float64) / (1.0 - 0.9 ** t)
        vhat = v1.astype(np.float64) / (1.0 - 0.999 ** t)
        p_exp = p0d - lr * mhat / (np.sqrt(vhat) + 1e-8)
        dp = np.abs(p1 - p_exp) / (np.spacing(np.abs(p_exp).astype(np.float32)).astype(np.float64) + lr * 2.0 ** -20)
        print("Adam step %d: max rel m %.2e, v %.2e; max |dp| %.2f ulp-units" % (t, dm.max(), dv.max(), dp.max()),
              flush=True)
        assert dm.max() <= 2.0 ** -20 and dv.max() <= 2.0 ** -20 and dp.max() <= 1.0, (t, dm.max(), dv.max(), dp.max())


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


def test_features_entry_point_against_the_oracle():
    # nssdoa_features after nssdoa_estimate: the proposal features of the covariances the estimate
    # computed, against the oracle's features of its own FP64 covariance (FP32 rounding of each
    # value, so within 2^-22 relative)
    from paper_2007_14135_amd.runner import prepare
    from synth import make_frames
    import oracle
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fs = make_frames("c5", n_frames=24, start=500)
    fr0 = fs.frames[0]
    frames = [(0, 0, fr.N, fr.D, int(fs.x_off[f]), int(fs.ld[f])) for f, fr in enumerate(fs.frames)]
    db = prepare([fr0.pos], [(-90.0, 0.1, 1800, 0)], frames, fs.X_flat, "music", "c64", 4)
    db.run()
    feats = torch.empty(len(fs), 272, dtype=torch.float32, device="cuda")
    db.batch.features(db.workspace, feats)
    got = feats.cpu().numpy().astype(np.float64)
    for f, fr in enumerate(fs.frames):
        ref = omlp.features(oracle.covariance(fr.X))
        assert np.all(np.abs(got[f] - ref) <= 2.0 ** -22 * np.abs(ref) + 1e-12), f
    from paper_2007_14135_amd import _abi
    with pytest.raises(_abi.NssdoaError):
        db.batch.features(db.workspace, torch.empty(len(fs), 270, dtype=torch.float32, device="cuda"))


def test_training_pipeline_runs_on_the_library(tmp_path):
    # the trainer end to end on 3072 frames: snapshots -> library estimate + features -> labels ->
    # one epoch of nssdoa_mlp_train_step; finite losses, weights and metadata written
    from paper_2007_14135_amd import train as tr
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = str(tmp_path / "w.npy")
    meta = tr.train(tr.argparse.Namespace(frames=3072, first_frame=tr.TRAIN_FIRST_FRAME + 7, epochs=1, batch=256,
                                          lr=1e-3, lr_min=1e-4, seed=3, workers=4, out=out, checkpoint="", resume=""))
    h = meta["history"][-1]
    assert np.isfinite(h["train_loss"]) and np.isfinite(h["val_loss"]) and 0.0 <= h["val_recall6"] <= 1.0
    w = np.load(out, allow_pickle=False)
    assert w.shape == (272 * 512 + 512 + 512 * 512 + 512 + 180 * 512 + 180,) and np.all(np.isfinite(w))
