"""Pins of the FP64 surrogate reference: finite differences, torch autograd
(CPU, float64) and torch's Adam (library routines)."""
import numpy as np
import torch

from oracle import mlp


def _setup(seed=0, dims=(5, 7, 2, 3), B=4):
    n_in, hidden, layers, n_out = dims
    shp = mlp.shapes(n_in, hidden, layers, n_out)
    rng = np.random.default_rng(seed)
    n = sum(r * c + r for r, c in shp)
    theta = rng.normal(0, 0.5, n)
    X = rng.normal(0, 1, (B, n_in))
    T = rng.normal(0, 1, (B, n_out))
    return shp, theta, X, T


def test_gradient_matches_central_differences():
    shp, theta, X, T = _setup()
    loss, g = mlp.loss_and_grad(theta, X, T, shp)
    h = 1e-6
    num = np.zeros_like(theta)
    for i in range(len(theta)):
        e = np.zeros_like(theta)
        e[i] = h
        num[i] = (mlp.loss_and_grad(theta + e, X, T, shp)[0] - mlp.loss_and_grad(theta - e, X, T, shp)[0]) / (2 * h)
    np.testing.assert_allclose(g, num, rtol=1e-6, atol=1e-9)


def test_forward_and_gradient_match_torch_autograd():
    shp, theta, X, T = _setup(seed=1, dims=(10, 16, 3, 4), B=6)
    layers = mlp.unpack(theta, shp)
    params = []
    a = torch.tensor(X, dtype=torch.float64)
    for li, (W, b) in enumerate(layers):
        Wt = torch.tensor(W, dtype=torch.float64, requires_grad=True)
        bt = torch.tensor(b, dtype=torch.float64, requires_grad=True)
        params += [Wt, bt]
        a = a @ Wt.T + bt
        if li < len(layers) - 1:
            a = torch.nn.functional.gelu(a)  # exact erf form
    loss = torch.mean((a - torch.tensor(T)) ** 2)
    loss.backward()
    ref = np.concatenate([p.grad.numpy().ravel() for p in params])
    l2, g = mlp.loss_and_grad(theta, X, T, shp)
    Y, _ = mlp.forward(theta, X, shp)
    np.testing.assert_allclose(Y, a.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert abs(l2 - loss.item()) < 1e-12
    np.testing.assert_allclose(g, ref, rtol=1e-10, atol=1e-12)


def test_adam_matches_torch():
    rng = np.random.default_rng(2)
    theta = rng.normal(0, 1, 50)
    p = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    for step in range(1, 6):
        g = rng.normal(0, 1, 50)
        p.grad = torch.tensor(g)
        opt.step()
        theta, m, v = mlp.adam(theta, m, v, g, step, 1e-2)
    np.testing.assert_allclose(theta, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_bf16_mode_rounds_only_product_operands():
    """With BF16 operand rounding the outputs move by a small relative amount
    (bfloat16 has 8 significand bits), never by a structural change."""
    shp, theta, X, T = _setup(seed=3, dims=(20, 32, 3, 5), B=8)
    Y64, _ = mlp.forward(theta, X, shp)
    Y16, _ = mlp.forward(theta, X, shp, bf16=True)
    rel = np.linalg.norm(Y16 - Y64) / np.linalg.norm(Y64)
    assert 1e-5 < rel < 3e-2
