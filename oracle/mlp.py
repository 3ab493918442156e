"""FP64 oracle for the learned p -> y surrogate (not part of the paper).

Test infrastructure only (see the package docstring).

The surrogate is a multilayer perceptron with GELU activations,
widths (d, 256, 256, r) by default:

    h_1 = gelu(W_1 p + b_1),  h_2 = gelu(W_2 h_1 + b_2),  out = W_3 h_2 + b_3,

trained on standardised SubApSnap coefficients t = (y - mu) / sd with the
mean-squared-error loss L = mean over batch and outputs of (out - t)^2 and
the Adam update (Kingma & Ba, 2015) with bias correction.  GELU is the
exact form x Phi(x) = x (1 + erf(x / sqrt 2)) / 2.

Parameters are a list of (W, b) pairs with W of shape (fan_out, fan_in);
activations are batch-major (batch x width).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / SQRT2))


def gelu_grad(x):
    """d/dx [x Phi(x)] = Phi(x) + x phi(x)."""
    return 0.5 * (1.0 + erf(x / SQRT2)) + x * INV_SQRT_2PI * np.exp(-0.5 * x * x)


def forward(params, P):
    """Returns (out, cache) for inputs P (batch x d)."""
    a = np.asarray(P, dtype=np.float64)
    cache = [a]
    L = len(params)
    for l, (W, b) in enumerate(params):
        z = a @ W.T + b
        if l < L - 1:
            cache.append(z)
            a = gelu(z)
            cache.append(a)
        else:
            a = z
    return a, cache


def mse_loss(out, T):
    return float(np.mean((out - T) ** 2))


def backward(params, cache, out, T):
    """Gradients of mse_loss w.r.t. every (W, b), in the same layout."""
    B = out.shape[0]
    g = 2.0 * (out - T) / out.size          # dL/d out
    grads = [None] * len(params)
    L = len(params)
    for l in range(L - 1, -1, -1):
        a_in = cache[0] if l == 0 else cache[2 * l]
        W, _ = params[l]
        grads[l] = (g.T @ a_in, g.sum(axis=0))
        if l > 0:
            z_prev = cache[2 * l - 1]
            g = (g @ W) * gelu_grad(z_prev)
    del B
    return grads


def loss_and_grads(params, P, T):
    out, cache = forward(params, P)
    return mse_loss(out, T), backward(params, cache, out, T)


class Adam:
    """Adam with bias correction; state is FP64 first/second moments."""

    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

    def step(self, params, grads, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for k, (w, g) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[l][k] + (1.0 - self.b1) * g
                v = self.b2 * self.v[l][k] + (1.0 - self.b2) * g * g
                self.m[l] = (m, self.m[l][1]) if k == 0 else (self.m[l][0], m)
                self.v[l] = (v, self.v[l][1]) if k == 0 else (self.v[l][0], v)
                new.append(w - lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
            out.append((new[0], new[1]))
        return out


def standardise(Y):
    """Per-component mean and standard deviation of the training targets."""
    mu = Y.mean(axis=0)
    sd = Y.std(axis=0)
    sd[sd == 0] = 1.0
    return mu, sd
