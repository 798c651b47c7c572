"""The order-prediction network's GPU kernels (forward, loss gradient, Adam,
full-batch training) against the FP64 oracle of the same network.  FP32 on the
GPU: forward 1e-5, gradient 1e-4 relative (sums over samples in FP32 partials
combined in FP64), Adam 1e-6."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
F = pytest.importorskip("paper_2009_00767_amd")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def data(seed, m, scale=0.3):
    rng = np.random.default_rng(seed)
    w = rng.normal(0.0, scale, size=F.FMM_MLP_NPARAM)
    x = rng.normal(size=(m, 3))
    t = rng.normal(size=(m, 21))
    return w, x, t


def cuda32(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("m", [1, 37, 1000])
def test_forward_matches_oracle(m):
    w, x, _ = data(501, m)
    w32, x32 = np.float32(w), np.float32(x)
    y = torch.empty((m, 21), dtype=torch.float32, device="cuda")
    F.fmm_mlp_forward(cuda32(w32), cuda32(x32), y)
    torch.cuda.synchronize()
    want = oracle.mlp_forward(w32.astype(np.float64), x32.astype(np.float64))
    assert rel(y.cpu().numpy(), want) < 1e-5


@pytest.mark.parametrize("m", [1, 16, 17, 250, 3000])
def test_loss_gradient_matches_oracle(m):
    w, x, t = data(502 + m, m)
    w32, x32, t32 = np.float32(w), np.float32(x), np.float32(t)
    g = torch.empty(F.FMM_MLP_NPARAM, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    F.fmm_mlp_loss_grad(cuda32(w32), cuda32(x32), cuda32(t32), g, loss)
    wl, wg = oracle.mlp_loss_grad(w32.astype(np.float64), x32.astype(np.float64),
                                  t32.astype(np.float64))
    assert abs(float(loss.item()) - wl) < 1e-5 * wl
    gg = g.cpu().numpy()
    assert rel(gg, wg) < 1e-4
    # deterministic: a second call gives the same bits
    g2 = torch.empty_like(g)
    F.fmm_mlp_loss_grad(cuda32(w32), cuda32(x32), cuda32(t32), g2, loss)
    assert torch.equal(g, g2)


def test_adam_step_matches_oracle():
    rng = np.random.default_rng(510)
    n = F.FMM_MLP_NPARAM
    w0 = np.float32(rng.normal(size=n))
    g1, g2 = np.float32(rng.normal(size=n)), np.float32(rng.normal(size=n))
    w, m1, m2 = cuda32(w0), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    ow, om1, om2 = w0.astype(np.float64), np.zeros(n), np.zeros(n)
    for step, g in ((1, g1), (2, g2), (3, g1)):
        F.fmm_mlp_adam_step(w, cuda32(g), m1, m2, step, 2e-3)
        oracle.mlp_adam(ow, g.astype(np.float64), om1, om2, step, lr=2e-3)
    torch.cuda.synchronize()
    assert np.max(np.abs(w.cpu().numpy() - ow)) < 1e-6 * max(1.0, np.max(np.abs(ow)))
    assert rel(m2.cpu().numpy(), om2) < 1e-6


def test_training_fits_a_teacher_network():
    """Targets made by a random teacher network through the oracle: full-batch
    training on the GPU must drive the loss far below its start, and the first
    steps must follow the oracle's own Adam trajectory."""
    rng = np.random.default_rng(511)
    teacher = rng.normal(0.0, 0.3, size=F.FMM_MLP_NPARAM)
    x = rng.uniform(-1, 1, size=(2000, 3))
    t = oracle.mlp_forward(teacher, x)
    w0 = np.float32(rng.normal(0.0, 0.3, size=F.FMM_MLP_NPARAM))
    # three steps on the device against three oracle steps in FP64
    w = cuda32(w0)
    hist = F.fmm_mlp_train(w, cuda32(x), cuda32(t), 3, 1e-3)
    ow, om1, om2 = w0.astype(np.float64), np.zeros_like(teacher), np.zeros_like(teacher)
    x32, t32 = np.float32(x).astype(np.float64), np.float32(t).astype(np.float64)
    losses = []
    for step in (1, 2, 3):
        l, g = oracle.mlp_loss_grad(ow, x32, t32)
        losses.append(l)
        oracle.mlp_adam(ow, g, om1, om2, step, lr=1e-3)
    np.testing.assert_allclose(hist, losses, rtol=1e-5)
    # Adam's first steps move every weight by about lr; gradients near zero may
    # differ in sign between FP32 and FP64, so compare the typical weight
    wd = w.cpu().numpy() - ow
    assert np.median(np.abs(wd)) < 1e-6
    # longer training
    w = cuda32(w0)
    hist = np.concatenate([F.fmm_mlp_train(w, cuda32(x), cuda32(t), 1500, 3e-3),
                           F.fmm_mlp_train(w, cuda32(x), cuda32(t), 1500, 1e-3)])
    assert hist[-1] < 0.02 * hist[0]
    y = torch.empty((2000, 21), dtype=torch.float32, device="cuda")
    F.fmm_mlp_forward(w, cuda32(x), y)
    trained = w.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(y.cpu().numpy(), oracle.mlp_forward(trained, np.float32(x)),
                               rtol=1e-4, atol=1e-4)


def test_training_resumes_from_a_checkpoint(tmp_path):
    """Adam state checkpointed mid-schedule and resumed in a second call gives
    the same weights, bit for bit, as one uninterrupted fmm_mlp_train run."""
    from paper_2009_00767_amd import order_model
    rng = np.random.default_rng(41)
    X = rng.normal(size=(96, 3)).astype(np.float32)
    Y = rng.normal(size=(96, 21)).astype(np.float32)
    sched = ((40, 3e-3), (30, 1e-3))
    want, want_hist = order_model.train(X, Y, seed=3, schedule=sched)
    ck = str(tmp_path / "mlp.npz")
    w1, h1, done = order_model.train_resumable(X, Y, ck, seed=3, schedule=sched, every=16,
                                               max_steps=52)
    assert not done and len(h1) == 52
    st = order_model.load_checkpoint(ck)
    assert (st["stage"], st["step"]) == (1, 12) and np.any(st["m1"]) and np.any(st["m2"])
    w2, h2, done = order_model.train_resumable(X, Y, ck, seed=3, schedule=sched, every=16)
    assert done
    np.testing.assert_array_equal(w2, want)
    np.testing.assert_array_equal(h2, want_hist)
