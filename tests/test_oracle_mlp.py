"""Pins for oracle.mlp: central finite differences, and torch's CPU GELU
and Adam as independent implementations."""
import numpy as np
import pytest

import subap_inputs as si
from oracle import mlp


def small_net(seed=0):
    return si.mlp_init(widths=(4, 16, 12, 5), seed=seed)


def test_gradients_match_central_differences():
    params = small_net()
    rng = np.random.default_rng(1)
    P = rng.uniform(-1, 1, (7, 4))
    T = rng.standard_normal((7, 5))
    _, grads = mlp.loss_and_grads(params, P, T)
    eps = 1e-6
    for l, (W, b) in enumerate(params):
        for arr, g in ((W, grads[l][0]), (b, grads[l][1])):
            for idx in [tuple(rng.integers(s) for s in arr.shape) for _ in range(6)]:
                old = arr[idx]
                arr[idx] = old + eps
                lp, _ = mlp.loss_and_grads(params, P, T)
                arr[idx] = old - eps
                lm, _ = mlp.loss_and_grads(params, P, T)
                arr[idx] = old
                fd = (lp - lm) / (2 * eps)
                assert abs(fd - g[idx]) <= 1e-6 * max(1e-3, abs(fd)), (l, idx, fd, g[idx])


def test_gelu_matches_torch_exact():
    torch = pytest.importorskip("torch")
    x = np.linspace(-6, 6, 1001)
    ref = torch.nn.functional.gelu(torch.tensor(x, dtype=torch.float64)).numpy()
    assert np.abs(mlp.gelu(x) - ref).max() < 1e-15
    xt = torch.tensor(x, dtype=torch.float64, requires_grad=True)
    torch.nn.functional.gelu(xt).sum().backward()
    assert np.abs(mlp.gelu_grad(x) - xt.grad.numpy()).max() < 1e-14


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    params = small_net(3)
    rng = np.random.default_rng(4)
    opt = mlp.Adam(params, lr=1e-2)
    tparams = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for W, b in params for a in (W, b)]
    topt = torch.optim.Adam(tparams, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for _ in range(4):
        grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params]
        params = opt.step(params, grads)
        for t, g in zip(tparams, [a for pair in grads for a in pair]):
            t.grad = torch.tensor(g, dtype=torch.float64)
        topt.step()
    flat = [a for W, b in params for a in (W, b)]
    for a, t in zip(flat, tparams):
        assert np.abs(a - t.detach().numpy()).max() < 1e-14


def test_training_reduces_loss():
    params = small_net(5)
    rng = np.random.default_rng(6)
    P = rng.uniform(-1, 1, (256, 4))
    T = np.stack([np.sin(P @ rng.standard_normal(4)) for _ in range(5)], axis=1)
    opt = mlp.Adam(params, lr=1e-2)
    l0, _ = mlp.loss_and_grads(params, P, T)
    for _ in range(200):
        _, g = mlp.loss_and_grads(params, P, T)
        params = opt.step(params, g)
    l1, _ = mlp.loss_and_grads(params, P, T)
    assert l1 < 0.2 * l0
