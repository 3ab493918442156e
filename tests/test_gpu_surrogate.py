"""The learned surrogate's hand-written kernels against the FP64 oracle
(oracle.mlp): gradients of the mean-squared error, one Adam step, training
that reduces the loss, prediction, and the accept-or-fall-back solve.

Bars: gradients within 1e-2 relative per layer (BF16 products with FP32
accumulation, about 2^-9 per rounded operand; measured at most 3.8e-3); the
first Adam step within 5e-2 lr
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
        rel = [np.linalg.norm(a - b) / np.linalg.norm(b)
               for (gW, gb), (oW, ob) in zip(_layers(g), go) for a, b in ((gW, oW), (gb, ob))]
        print("gradient relative errors per layer (W, b):", ["%.2e" % v for v in rel])
        assert max(rel) <= 1e-2, rel
    finally:
        B.subap_surrogate_free(s)


def test_prediction_matches_oracle_forward():
    """subap_surrogate_predict element by element against the FP64 forward pass
    of oracle.mlp with the same weights (before training the standardisation
    is the identity, after it the prediction is destandardised with the
    training mean and deviation).  Bar per entry: 2^-5 (|y_oracle| + rms(y_oracle)),
    sixteen bf16 rounding units: the inputs, the first two layers' weights and
    the hidden activations are rounded to bf16 (2^-9 relative each) before their
    MFMA products, and the output layer's split product keeps its own error
    near FP32, so the error is a sum of bf16 roundings through two layers of
    fan-in 4 and 256 (measured: 0.013 of the scale untrained, 0.017 after one
    training step)."""
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
        assert (err <= 2.0 ** -5 * scale).all(), (err / scale).max()
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
        assert (err <= 2.0 ** -5 * scale).all(), (err / scale).max()
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
        # acceptance by the normal-equation excess bound: with sigma at most
        # every sigma_min(G_p), an accepted prediction is within tau of the
        # SubApSnap solution in |G (y - y*)| / |S b|; rejected ones are the plain solve
        G = torch.empty((1024, w["s"], w["r"]), dtype=torch.float64, device=Pin.device)
        B.subap_reduced_matrix(M.handle, Pin, G)
        Gh = G.cpu().numpy()
        sig = float(np.linalg.svd(Gh, compute_uv=False)[:, -1].min())
        bound = torch.empty(1024, dtype=torch.float64, device=Pin.device)
        B.subap_excess_bound(M.handle, Pin, yhat, sig, bound)
        tau = float(torch.quantile(bound, 0.5))
        n = B.subap_surrogate_solve_batch_excess(M.handle, s, Pin, sig, tau, y, acc, sts)
        a = acc.cpu().numpy().astype(bool)
        assert a.sum() == n and 256 <= n <= 768, n
        assert np.all(sts.cpu().numpy() == B.OK)
        yc = y.cpu().numpy()
        assert np.array_equal(yc[~a], yrc[~a]) and np.array_equal(yc[a], yhat.cpu().numpy()[a])
        bS = np.asarray([off["family"].rhs_rows(p, off["rows"]) for p in sg["infer_params"]])
        dist = np.linalg.norm(np.einsum("psr,pr->ps", Gh, yc - yrc), axis=1) / np.linalg.norm(bS, axis=1)
        assert np.all(dist[a] <= tau * (1 + 1e-9)), dist[a].max() / tau
        print(f"excess bound: accepted {n} of 1024 at {tau:.2e} (sigma {sig:.2e}); "
              f"max distance of the accepted {dist[a].max():.2e}")
    finally:
        B.subap_surrogate_free(s)
        M.free()


@pytest.mark.parametrize("name", ["diff3d", "krr"])
def test_excess_bound_bounds_the_distance_to_subapsnap(name):
    """The acceptance measure beside the literal sketched-residual test: with
    G = S A(p) Q, r = G y - S b and sigma <= sigma_min(G),
    |G (y - y*)| / |S b| <= |G^T r| / (sigma |S b|), zero at y = y*.  The GPU's
    value (rows generated in FP64, no QR) against the oracle's G, y* and
    sigma_min on perturbed coefficients; and subap_reduced_matrix against the
    oracle's S A(p) Q."""
    import torch
    if name == "diff3d":
        w = si.diffusion3d(N=16, r=8, s=32, m=40)
    else:
        w = si.krr(n=1024, r=8, s=24, m=40)
    off = O.offline(w)
    fam, Q, rows = off["family"], off["Q"], off["rows"]
    header(f"excess bound {name}")
    device()
    M = B.Model(w, basis=Q, rows=rows)
    try:
        P = w["test_params"]
        Yo = On.solve(fam, Q, rows, P)
        rng = np.random.default_rng(8)
        Y = Yo + 10.0 ** rng.uniform(-8, -2, size=(len(P), 1)) * rng.standard_normal(Yo.shape)
        Y[0] = Yo[0]
        Gs = [On.reduced_matrix(fam, Q, rows, p) for p in P]
        sig = min(np.linalg.svd(G, compute_uv=False)[-1] for G in Gs)
        out = torch.empty(len(P), dtype=torch.float64, device="cuda")
        B.subap_excess_bound(M.handle, to_dev(P), to_dev(Y), sig, out)
        torch.cuda.synchronize()
        bound = out.cpu().numpy()
        for i, (p, G, y, yo) in enumerate(zip(P, Gs, Y, Yo)):
            bS = np.asarray(fam.rhs_rows(p, rows), dtype=np.float64)
            true = np.linalg.norm(G @ (y - yo)) / np.linalg.norm(bS)
            want = np.linalg.norm(G.T @ (G @ y - bS)) / (sig * np.linalg.norm(bS))
            # rounding of G^T r in FP64 (both sides): r is a difference of sums
            # of n products, with a rounding error near eps sqrt(n)
            # (|G| |y| + |S b|) in norm (random-walk accumulation), which G^T
            # carries with at most its norm |G|
            g2 = np.linalg.norm(G, 2)
            floor = 2.0 ** -52 * np.sqrt(w["n"]) * g2 * (g2 * np.linalg.norm(y) + np.linalg.norm(bS)) \
                / (sig * np.linalg.norm(bS))
            assert true <= bound[i] * (1 + 1e-9) + floor, (i, true, bound[i])
            assert abs(bound[i] - want) <= 1e-8 * want + floor, (i, bound[i], want, floor)
        assert bound[0] <= 1e-9
        Gg = torch.empty((5, w["s"], w["r"]), dtype=torch.float64, device="cuda")
        B.subap_reduced_matrix(M.handle, to_dev(P[:5]), Gg)
        torch.cuda.synchronize()
        for G, g in zip(Gs[:5], Gg.cpu().numpy()):
            assert np.abs(g - G).max() <= 1e-12 * np.abs(G).max()
    finally:
        M.free()
