"""The learned surrogate's hand-written kernels against the FP64 oracle
(oracle.mlp): gradients of the mean-squared error, one Adam step, training
that reduces the loss, prediction, and the accept-or-fall-back solve.

Bars: gradients within 3e-2 relative per layer (BF16 products with FP32
accumulation, about 2^-8 per product); the first Adam step within 5e-2 lr
per entry where the gradient is not negligible (Adam's first step is close to
lr sign(g), so BF16 gradient error moves it little); fallback results equal
the plain batched solve bit for bit."""
import numpy as np
import pytest

import subap_inputs as si
from oracle import mlp
from oracle import offline as O
from oracle import online as On
from paper_2510_04825_amd import binding as B
from tests.gpu_util import device, header, to_dev

pytestmark = pytest.mark.gpu
WIDTHS = (4, 256, 256, 40)


def _layers(flat):
    return B.unflatten_mlp(flat, WIDTHS)


def test_gradient_matches_oracle():
    header("surrogate gradient")
    device()
    params = si.mlp_init(WIDTHS, seed=11)
    rng = np.random.default_rng(3)
    P = rng.uniform(-1, 1, (96, 4))
    T = rng.standard_normal((96, 40))
    s = B.subap_surrogate_create(4, 40, 256, B.flatten_mlp(params))
    try:
        g, loss = B.subap_surrogate_gradient(s, to_dev(P), to_dev(T))
        lo, go = mlp.loss_and_grads(params, P, T)
        assert abs(loss - lo) <= 2e-2 * lo
        for (gW, gb), (oW, ob) in zip(_layers(g), go):
            for a, b in ((gW, oW), (gb, ob)):
                assert np.linalg.norm(a - b) <= 3e-2 * np.linalg.norm(b), np.linalg.norm(a - b) / np.linalg.norm(b)
    finally:
        B.subap_surrogate_free(s)


def test_prediction_matches_oracle_forward():
    """subap_surrogate_predict element by element against the FP64 forward pass
    of oracle.mlp with the same weights (before training the standardisation
    is the identity, after it the prediction is destandardised with the
    training mean and deviation).  Bar per entry: 2^-6 (|y_oracle| + rms(y_oracle)):
    the hidden layers multiply bf16-rounded operands (2^-9 relative each) and
    the output layer's split product keeps its own error near FP32, so the
    error is that of two bf16 layers, a few times 2^-9 of the activations'
    scale."""
    import torch
    header("surrogate prediction vs oracle forward")
    device()
    params = si.mlp_init(WIDTHS, seed=14)
    rng = np.random.default_rng(6)
    P = rng.uniform(-1, 1, (777, 4))   # a ragged count of parameters
    s = B.subap_surrogate_create(4, 40, 256, B.flatten_mlp(params))
    try:
        y = torch.empty((777, 40), dtype=torch.float64, device="cuda")
        B.subap_surrogate_predict(s, to_dev(P), y)
        want, _ = mlp.forward(params, P)
        err = np.abs(y.cpu().numpy() - want)
        scale = np.abs(want) + np.sqrt(np.mean(want ** 2))
        print("max error / scale", (err / scale).max())
        assert (err <= 2.0 ** -6 * scale).all(), (err / scale).max()
        # after training: destandardised with the training statistics
        Ptr = rng.uniform(-1, 1, (512, 4))
        Ytr = rng.standard_normal((512, 40)) * 5.0 + 2.0
        B.subap_surrogate_train(s, to_dev(Ptr), to_dev(Ytr), epochs=1, batch=512, lr=1e-3, lr_min=1e-3)
        trained = _layers(B.subap_surrogate_weights(s))
        mu, sd = mlp.standardise(Ytr)
        B.subap_surrogate_predict(s, to_dev(P), y)
        out, _ = mlp.forward([(W.astype(np.float64), b.astype(np.float64)) for W, b in trained], P)
        want = out * sd + mu
        err = np.abs(y.cpu().numpy() - want)
        scale = np.abs(out) * sd + np.sqrt(np.mean(out ** 2)) * sd
        print("trained: max error / scale", (err / scale).max())
        assert (err <= 2.0 ** -6 * scale).all(), (err / scale).max()
    finally:
        B.subap_surrogate_free(s)


def test_first_adam_step_matches_oracle():
    header("surrogate adam step")
    device()
    params = si.mlp_init(WIDTHS, seed=12)
    rng = np.random.default_rng(4)
    P = rng.uniform(-1, 1, (128, 4))
    Y = rng.standard_normal((128, 40)) * 3.0 + 1.0
    mu, sd = mlp.standardise(Y)
    T = (Y - mu) / sd
    s = B.subap_surrogate_create(4, 40, 256, B.flatten_mlp(params))
    try:
        lr = 1e-3
        B.subap_surrogate_train(s, to_dev(P), to_dev(Y), epochs=1, batch=128, lr=lr, lr_min=lr)
        new = _layers(B.subap_surrogate_weights(s))
        _, go = mlp.loss_and_grads(params, P, T)
        ref = mlp.Adam(params, lr=lr).step(params, go)
        for (nW, nb), (rW, rb), (oW, ob), (gW, gb) in zip(new, ref, params, go):
            for n_, r_, o_, g_ in ((nW, rW, oW, gW), (nb, rb, ob, gb)):
                big = np.abs(g_) >= 1e-2 * np.sqrt(np.mean(g_ ** 2))
                d = np.abs((n_ - o_) - (r_ - o_))[big]
                assert d.max() <= 5e-2 * lr + 1e-7, d.max()
    finally:
        B.subap_surrogate_free(s)


@pytest.fixture(scope="module")
def small3d():
    w = si.diffusion3d(N=16, r=8, s=32, m=2048)
    off = O.offline(w)
    return w, off


def test_training_prediction_and_fallback(small3d):
    import torch
    w, off = small3d
    header("surrogate train / predict / fallback")
    M = B.Model(w, basis=off["Q"], rows=off["rows"])
    widths = (4, 256, 256, w["r"])
    s = B.subap_surrogate_create(4, w["r"], 256, B.flatten_mlp(si.mlp_init(widths, seed=13)))
    try:
        sg = si.surrogate(n_train=8192, n_infer=1024)
        Ptr = to_dev(sg["train_params"])
        ytr, _, st = M.solve(Ptr)
        assert np.all(st.cpu().numpy() == B.OK)
        losses = B.subap_surrogate_train(s, Ptr, ytr, epochs=40, batch=1024, lr=2e-3, lr_min=1e-5, seed=1)
        assert losses[-1] < 0.05 * losses[0], losses[[0, -1]]
        Pin = to_dev(sg["infer_params"])
        yhat = torch.empty((1024, w["r"]), dtype=torch.float64, device=Pin.device)
        B.subap_surrogate_predict(s, Pin, yhat)
        yref, _, _ = M.solve(Pin)
        rel = np.linalg.norm(yhat.cpu().numpy() - yref.cpu().numpy()) / np.linalg.norm(yref.cpu().numpy())
        assert rel < 0.05, rel
        # accept everything: y is the prediction
        y = torch.empty_like(yhat)
        acc = torch.zeros(1024, dtype=torch.uint8, device=Pin.device)
        n = B.subap_surrogate_solve_batch(M.handle, s, Pin, 1e30, y, acc)
        assert n == 1024 and torch.equal(y, yhat)
        # literal threshold: accepted predictions meet it, rejected ones equal the plain solve
        sts = torch.full((1024,), -1, dtype=torch.int32, device=Pin.device)
        _, rho_ref = M.sketched_residual(Pin, yref)
        tol = float(torch.quantile(rho_ref, 0.5)) * 1.5   # a threshold some predictions can meet
        n = B.subap_surrogate_solve_batch(M.handle, s, Pin, tol, y, acc, sts)
        a = acc.cpu().numpy().astype(bool)
        assert 0 <= n <= 1024 and a.sum() == n
        assert np.all(sts.cpu().numpy() == B.OK)
        yc, yrc = y.cpu().numpy(), yref.cpu().numpy()
        assert np.array_equal(yc[~a], yrc[~a])
        _, rho_acc = M.sketched_residual(Pin, y)
        assert np.all(rho_acc.cpu().numpy()[a] <= tol * (1 + 1e-12))
        print(f"accepted {n} of 1024 at tolerance {tol:.2e}; prediction error {rel:.2e}")
        # what the network gains over the method alone: at a threshold just above the
        # method's own sketched-residual floor most parameters skip the solve
        assert n >= 512, n
    finally:
        B.subap_surrogate_free(s)
        M.free()
