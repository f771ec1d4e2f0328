"""Learned proposal on the GPU against the double-precision oracle.

Each matrix-core GEMM is checked on the GPU's own bf16 operands against the
double-precision sum of the same operands, within the fp32 accumulation bound
|err| <= 2 K 2^-24 sum_k |a_k b_k|; elementwise epilogues within one bf16 ulp
(the device erf/exp round differently from the oracle's); the whole gradient
against the oracle's independent backward pass; Adam against the oracle."""
import numpy as np
import pytest

from paper_2605_29663_amd import scenes

pytestmark = pytest.mark.gpu

T, NU, H = 40, 2, 256


@pytest.fixture(scope="module")
def pkg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2605_29663_amd as p
    p.load()
    return p


def _bound(A, B):
    K = A.shape[1]
    return 2.0 * K * 2.0 ** -24 * (np.abs(A) @ np.abs(B)) + 1e-7


def _setup(pkg, M=300, seed=0):
    import torch
    from oracle import mlp
    net = pkg.Proposal(T, NU, hidden=H, max_batch=512)
    rng = np.random.default_rng(seed)
    theta = net.init_params(seed).astype(np.float64)
    # non-zero biases
    W1, b1, W2, b2, W3, b3 = mlp.unpack(theta, net.in_dim, H, net.out_dim)
    theta = mlp.pack(W1, rng.normal(0, 0.1, H), W2, rng.normal(0, 0.1, H), W3,
                     rng.normal(0, 0.1, net.out_dim)).astype(np.float32)
    net.set_params(theta)
    X = rng.uniform(-1, 1, (M, net.in_dim)).astype(np.float32)
    Y = rng.uniform(-1, 1, (M, net.out_dim)).astype(np.float32)
    return net, theta.astype(np.float64), torch.tensor(X, device="cuda"), X, Y


def test_forward_layers_vs_oracle(pkg):
    from oracle import mlp
    net, theta, Xd, X, Y = _setup(pkg)
    M = X.shape[0]
    out = net.forward(Xd).cpu().numpy()
    W1, b1, W2, b2, W3, b3 = mlp.unpack(theta, net.in_dim, H, net.out_dim)
    g = lambda name, n: net.get_buffer(name, n).astype(np.float64).reshape(M, -1)
    x = g("x", M * net.in_dim)
    np.testing.assert_array_equal(x, mlp.bf16(X))
    pre1, a1, pre2, a2 = g("pre1", M * H), g("a1", M * H), g("pre2", M * H), g("a2", M * H)
    for A, Wt, b, pre in ((x, W1, b1, pre1), (a1, W2, b2, pre2), (a2, W3, b3, out)):
        ref = A @ mlp.bf16(Wt) + b
        assert np.all(np.abs(pre - ref) <= _bound(A, mlp.bf16(Wt)))
    # GELU on the fp32 pre-activation, rounded to bf16: one bf16 ulp (2^-7 relative)
    # plus the fp32 evaluation error of x (1 + erf(x / sqrt 2)) / 2, which cancels
    # for large negative x (about |x| 2^-23 absolute)
    for pre, act in ((pre1, a1), (pre2, a2)):
        ref = mlp.bf16(mlp.gelu(pre))
        assert np.all(np.abs(act - ref) <= 2.0 ** -7 * np.abs(ref) + np.abs(pre) * 2.0 ** -22)


def test_backward_layers_and_gradient_vs_oracle(pkg):
    import torch
    from oracle import mlp
    net, theta, Xd, X, Y = _setup(pkg, seed=1)
    M, O, In = X.shape[0], net.out_dim, net.in_dim
    net.train_step(Xd, torch.tensor(Y, device="cuda"), lr=0.0)
    g = lambda name, n: net.get_buffer(name, n).astype(np.float64).reshape(M, -1)
    x, a1, a2 = g("x", M * In), g("a1", M * H), g("a2", M * H)
    pre1, pre2, out = g("pre1", M * H), g("pre2", M * H), g("out", M * O)
    dout, dout_b = g("dout", M * O), g("dout_b", M * O)
    dh2, dh2_b, dh1, dh1_b = g("dh2", M * H), g("dh2_b", M * H), g("dh1", M * H), g("dh1_b", M * H)
    grad = net.get_buffer("grad", net.n_params).astype(np.float64)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(theta, In, H, O)
    gW1, gb1, gW2, gb2, gW3, gb3 = mlp.unpack(grad, In, H, O)
    np.testing.assert_allclose(dout, 2.0 * (out - Y) / (M * O), rtol=1e-6, atol=1e-12)
    np.testing.assert_array_equal(dout_b, mlp.bf16(dout))
    # weight gradients: A^T dY on the GPU's bf16 operands
    for A, dY, gW in ((a2, dout_b, gW3), (a1, dh2_b, gW2), (x, dh1_b, gW1)):
        ref = A.T @ dY
        assert np.all(np.abs(gW - ref) <= _bound(A.T, dY))
    np.testing.assert_allclose(gb3, dout.sum(0), rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(gb2, dh2.sum(0), rtol=1e-5, atol=1e-9)
    np.testing.assert_allclose(gb1, dh1.sum(0), rtol=1e-5, atol=1e-9)
    # activation gradients: (dY W^T) * gelu'(pre)
    for dY, Wt, pre, dh in ((dout_b, W3, pre2, dh2), (dh2_b, W2, pre1, dh1)):
        Wb = mlp.bf16(Wt).T
        lin = dY @ Wb
        ref = lin * mlp.gelu_grad(pre)
        tol = _bound(dY, Wb) * np.abs(mlp.gelu_grad(pre)) + 1e-6 * np.abs(ref) + 1e-12
        assert np.all(np.abs(dh - ref) <= tol)
    # whole gradient from the oracle's own forward and backward (bf16 at the same points)
    g_ref, _ = mlp.backward(theta, X.astype(np.float64), Y.astype(np.float64), In, H, O, bf=True)
    scale = np.abs(g_ref).max()
    assert np.max(np.abs(grad - g_ref)) <= 2e-2 * scale
    assert np.corrcoef(grad, g_ref)[0, 1] > 0.9999


def test_adam_step_vs_oracle(pkg):
    import torch
    from oracle import mlp
    net, theta, Xd, X, Y = _setup(pkg, seed=2)
    Yd = torch.tensor(Y, device="cuda")
    net.train_step(Xd, Yd, lr=0.0)                      # gradient at theta, moments updated
    g0 = net.get_buffer("grad", net.n_params).astype(np.float64)
    net.set_params(theta.astype(np.float32))            # reset moments and step count
    net.train_step(Xd, Yd, lr=1e-3)
    t1 = net.get_params().astype(np.float64)
    ref, _, _ = mlp.adam(theta, g0, np.zeros_like(theta), np.zeros_like(theta), 1, lr=1e-3)
    # the step lr m/(sqrt(v)+eps) is evaluated in fp32 (a few ulp of lr) and added to an
    # fp32 parameter (half an ulp of theta)
    np.testing.assert_allclose(t1, ref, rtol=1e-6, atol=1e-3 * 2.0 ** -20)


def test_training_reduces_loss_and_save_load(pkg, tmp_path):
    import torch
    net, theta, Xd, X, Y = _setup(pkg, M=512, seed=3)
    rng = np.random.default_rng(9)
    P = rng.normal(0, 1.0 / np.sqrt(net.in_dim), (net.in_dim, net.out_dim))
    Yd = torch.tensor(np.tanh(X @ P).astype(np.float32), device="cuda")
    losses = [net.train_step(Xd, Yd, lr=2e-3) for _ in range(150)]
    assert losses[-1] < 0.2 * losses[0]
    path = tmp_path / "net.bin"
    net.save(path)
    out1 = net.forward(Xd).cpu().numpy()
    net2 = pkg.Proposal(T, NU, hidden=H, max_batch=512)
    net2.load(path)
    np.testing.assert_array_equal(net2.forward(Xd).cpu().numpy(), out1)
    np.testing.assert_array_equal(net2.get_params(), net.get_params())


def test_features_bit_exact(pkg, orc):
    import torch
    prm, sc = scenes.config("c2")
    ctx = pkg.Context(0)
    ctx.set_footprint(pkg.POLYGON, sc["polygon"])
    valid = (np.arange(sc["ox"].size) % 7 != 0).astype(np.uint8)
    ctx.set_points(sc["ox"], sc["oy"], valid=valid)
    net = pkg.Proposal(prm["T"], prm["nu"], hidden=H, max_batch=64)
    net.set_scaling(prm)
    rng = np.random.default_rng(4)
    M = 9
    q0 = np.concatenate([rng.uniform(-1, 6, (M, 2)), rng.uniform(-3.5, 3.5, (M, 1))], 1).astype(np.float32)
    q0[0] = 0.0
    U = rng.uniform(-1.5, 1.5, (M, prm["T"], 2)).astype(np.float32)
    f = net.features(ctx, torch.tensor(q0, device="cuda"), torch.tensor(U, device="cuda")).cpu().numpy()
    for m in range(M):
        ref = orc.f32_features(sc["ox"], sc["oy"], valid, q0[m], prm["goal"], U[m], prm["u_min"],
                               prm["u_max"], 8.0)
        np.testing.assert_array_equal(f[m], ref)
    # sampling mean maps outputs back into the box; normalisation inverts it
    Xd = torch.tensor(f, device="cuda")
    y = net.forward(Xd)
    Um = net.mean(Xd).cpu().numpy()
    lo, hi = np.float32(prm["u_min"]), np.float32(prm["u_max"])
    ref = np.clip((hi + lo) / 2 + (hi - lo) / 2 * y.cpu().numpy().reshape(M, prm["T"], 2), lo, hi)
    np.testing.assert_allclose(Um, ref, rtol=1e-6, atol=1e-7)
    yn = net.normalize(torch.tensor(U, device="cuda")).cpu().numpy()
    np.testing.assert_allclose(yn.reshape(U.shape), (U - (hi + lo) / 2) / ((hi - lo) / 2), rtol=1e-6,
                               atol=1e-7)


def test_residual_mode_mean_and_targets(pkg):
    """Residual mode: the mean is the previous sequence (from the features)
    plus scale x output, in the control box; targets invert it."""
    import torch
    prm, sc = scenes.config("c2")
    ctx = pkg.Context(0)
    ctx.set_footprint(pkg.POLYGON, sc["polygon"])
    ctx.set_points(sc["ox"], sc["oy"])
    net = pkg.Proposal(prm["T"], prm["nu"], hidden=H, max_batch=64)
    net.init_params(3)
    net.set_scaling(prm)
    rng = np.random.default_rng(8)
    M = 7
    q0 = np.concatenate([rng.uniform(-1, 4, (M, 2)), rng.uniform(-3, 3, (M, 1))], 1).astype(np.float32)
    U = rng.uniform(-1.2, 1.2, (M, prm["T"], 2)).astype(np.float32)
    f = net.features(ctx, torch.tensor(q0, device="cuda"), torch.tensor(U, device="cuda"))
    y = net.forward(f).cpu().numpy().reshape(M, prm["T"], 2)
    s = 0.07
    net.set_residual(s)
    Um = net.mean(f).cpu().numpy()
    lo, hi = np.float32(prm["u_min"]), np.float32(prm["u_max"])
    mid, half = (hi + lo) / 2, (hi - lo) / 2
    prev = f.cpu().numpy()[:, 66:].reshape(M, prm["T"], 2)
    ref = np.clip(mid + half * (prev + s * y), lo, hi)
    np.testing.assert_allclose(Um, ref, rtol=1e-6, atol=1e-6)
    Ut = np.clip(U + 0.05 * rng.standard_normal(U.shape).astype(np.float32), lo, hi)
    t = net.normalize(torch.tensor(Ut, device="cuda"), f).cpu().numpy().reshape(M, prm["T"], 2)
    np.testing.assert_allclose(t, ((Ut - mid) / half - prev) / s, rtol=1e-5, atol=1e-4)
    with pytest.raises(pkg.MppiError):
        net.normalize(torch.tensor(Ut, device="cuda"))       # residual targets need features
    net.set_residual(0.0)
    np.testing.assert_allclose(net.mean(f).cpu().numpy(), np.clip(mid + half * y, lo, hi),
                               rtol=1e-6, atol=1e-6)


def test_training_resume_is_bitwise(pkg, tmp_path):
    """Checkpoint / resume: 6 Adam steps, save, load into a new proposal, 6
    more, equal bit for bit to 12 uninterrupted steps (weights and the Adam
    state travel in the file; every kernel is deterministic)."""
    import torch
    net, theta, Xd, X, Y = _setup(pkg, M=256, seed=11)
    Yd = torch.tensor(Y, device="cuda")
    ref = pkg.Proposal(T, NU, hidden=H, max_batch=512)
    ref.set_params(theta.astype(np.float32))
    for _ in range(12):
        ref.train_step(Xd, Yd, lr=1e-3, want_loss=False)
    for _ in range(6):
        net.train_step(Xd, Yd, lr=1e-3, want_loss=False)
    path = tmp_path / "ckpt.bin"
    net.save(path)
    res = pkg.Proposal(T, NU, hidden=H, max_batch=512)
    res.load(path)
    for _ in range(6):
        res.train_step(Xd, Yd, lr=1e-3, want_loss=False)
    np.testing.assert_array_equal(res.get_params(), ref.get_params())
