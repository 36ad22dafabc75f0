"""Pins of the FP64 surrogate oracle: its analytic gradient against central
finite differences of its own FP64 loss (brute force), its BF16 rounding
against torch's bfloat16 conversion (a library routine), and Adam against
the update written out for one scalar."""
import numpy as np
import torch

import rb_inputs as ri
from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(10000) * np.exp(rng.uniform(-20, 20, 10000)),
                        [0.0, -0.0, 1.0, -1.0, 1.00390625, 1.005859375, 3.0e38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)


def test_backward_matches_finite_differences():
    din, h, dout, B = 2, 8, 6, 5
    rng = np.random.default_rng(2)
    p = ri.mlp_init(3, din, h, dout).astype(np.float64)
    p += 0.05 * rng.standard_normal(p.size)  # nonzero biases too
    X = rng.uniform(-1, 1, (B, din))
    T = rng.standard_normal((B, dout))
    Y, Hs = mlp.forward(p, X, din, h, dout, bf16_round=False)
    _, dY = mlp.loss_and_grad_out(Y, T, bf16_round=False)
    g = mlp.backward(p, X, Hs, dY, din, h, dout, bf16_round=False)
    eps = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd[i] = (mlp.loss(pp, X, T, din, h, dout) - mlp.loss(pm, X, T, din, h, dout)) / (2 * eps)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)


def test_adam_scalar():
    w, m, v = np.array([1.0]), np.array([0.0]), np.array([0.0])
    g = np.array([0.5])
    w1, m1, v1 = mlp.adam(w, g, m, v, 1, 0.1)
    # first step: m_hat = g, v_hat = g^2, so the move is lr * g / (|g| + eps)
    np.testing.assert_allclose(w1, 1.0 - 0.1 * 0.5 / (0.5 + 1e-8))
    np.testing.assert_allclose(m1, 0.05)
    np.testing.assert_allclose(v1, 0.001 * 0.25)


def test_layout_and_init():
    lay = ri.mlp_layout(2, 256, 282)
    assert lay["total"] == 2 * 256 + 256 + 2 * (256 * 256 + 256) + 256 * 282 + 282
    p = ri.mlp_init(7, 2, 256, 282)
    o, n = lay["b2"]
    assert np.all(p[o:o + n] == 0)
    o, n = lay["W2"]
    assert 0 < np.abs(p[o:o + n]).max() <= np.sqrt(6 / 512)
    np.testing.assert_array_equal(ri.batch_indices(5, 1000, 100, 12)[:10].ravel().size, 1000)
    assert sorted(ri.batch_indices(5, 1000, 100, 10).ravel()) == list(range(1000))


def _torch_net(p, din, h, dout):
    """The same network as torch modules (nn.Linear holds W transposed)."""
    P = mlp.unpack(p, din, h, dout)
    layers = []
    for i, (a, b) in enumerate([(din, h), (h, h), (h, h), (h, dout)]):
        lin = torch.nn.Linear(a, b).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(P["W%d" % (i + 1)].T.copy()))
            lin.bias.copy_(torch.from_numpy(P["b%d" % (i + 1)].copy()))
        layers += [lin, torch.nn.Tanh()] if i < 3 else [lin]
    return torch.nn.Sequential(*layers)


def test_forward_and_backward_match_torch_autograd():
    """FP64 forward and gradients against torch.nn modules and autograd on
    the same weights (an independent implementation of the chain rule)."""
    din, h, dout, B = 2, 16, 10, 33
    rng = np.random.default_rng(4)
    p = ri.mlp_init(5, din, h, dout).astype(np.float64) + 0.05 * rng.standard_normal(
        ri.mlp_layout(din, h, dout)["total"])
    X = rng.uniform(-1, 1, (B, din))
    T = rng.standard_normal((B, dout))
    Y, Hs = mlp.forward(p, X, din, h, dout, bf16_round=False)
    _, dY = mlp.loss_and_grad_out(Y, T, bf16_round=False)
    g = mlp.unpack(mlp.backward(p, X, Hs, dY, din, h, dout, bf16_round=False), din, h, dout)
    net = _torch_net(p, din, h, dout)
    Yt = net(torch.from_numpy(X))
    np.testing.assert_allclose(Y, Yt.detach().numpy(), rtol=1e-13, atol=1e-15)
    torch.nn.functional.mse_loss(Yt, torch.from_numpy(T)).backward()
    lins = [m for m in net if isinstance(m, torch.nn.Linear)]
    for i, lin in enumerate(lins):
        np.testing.assert_allclose(g["W%d" % (i + 1)], lin.weight.grad.numpy().T, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(g["b%d" % (i + 1)], lin.bias.grad.numpy(), rtol=1e-12, atol=1e-15)


def test_adam_matches_torch_over_several_steps():
    """Ten Adam steps on a varying gradient sequence against torch.optim.Adam
    (bias-corrected, the same hyper-parameters)."""
    rng = np.random.default_rng(6)
    n = 50
    w0 = rng.standard_normal(n)
    grads = rng.standard_normal((10, n)) * np.exp(rng.uniform(-4, 2, (10, n)))
    w, m, v = w0.copy(), np.zeros(n), np.zeros(n)
    wt = torch.nn.Parameter(torch.from_numpy(w0.copy()))
    opt = torch.optim.Adam([wt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    for s in range(10):
        w, m, v = mlp.adam(w, grads[s], m, v, s + 1, 3e-3)
        wt.grad = torch.from_numpy(grads[s].copy())
        opt.step()
        np.testing.assert_allclose(w, wt.detach().numpy(), rtol=1e-13, atol=1e-15)
