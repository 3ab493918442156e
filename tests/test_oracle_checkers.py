"""Pins for the oracle's two checkers, delta_res and sketched_residual.

Every GPU parity test measures its result with these two functions, so they
are pinned against values that do not come from the oracle's own operator
code (family.matvec / family.rows):

* closed forms: on an eigenbasis of the operator, A(p) Q dy = Q diag(lam) dy,
  so |A(p) Q dy| = |lam * dy| exactly -- the shifted tridiagonal matrix of
  eq. (5.7) (eigenvalues 2 - 2 cos(k pi / (n + 1)) - p, sine eigenvectors)
  and the 5-point Laplacian the diffusion family reduces to at p = 0;
* dense operators assembled here entry by entry from the definitions
  (face-midpoint coefficients of -div(a grad u), Gaussian kernel plus ridge),
  with plain numpy norms.

A dropped A(p), a wrong norm, a transposed or missing factor, a wrong
denominator or a lost row weight each changes at least one of these values.
"""
import math

import numpy as np

from oracle import families as F
from oracle import online as On


def _sine_basis(n, ks):
    i = np.arange(1, n + 1)[:, None]
    return np.sqrt(2.0 / (n + 1)) * np.sin(i * np.asarray(ks)[None, :] * np.pi / (n + 1))


def test_delta_res_closed_form_on_the_tridiagonal_eigenbasis():
    n, p = 50, 0.3
    rng = np.random.default_rng(11)
    b0 = rng.standard_normal(n)
    fam = F.ShiftedTridiag(b0)
    ks = [1, 3, 7, 12, 40]
    Q = _sine_basis(n, ks)
    lam = np.array([2.0 - 2.0 * math.cos(k * math.pi / (n + 1)) for k in ks]) - p
    y1, y2 = rng.standard_normal(len(ks)), rng.standard_normal(len(ks))
    b = np.exp(b0 * math.sin(p / 10.0) * p)
    want = np.linalg.norm(lam * (y1 - y2)) / np.linalg.norm(b)
    got = On.delta_res(fam, Q, np.array([p]), y1, y2)
    assert abs(got - want) <= 1e-13 * want
    # swapping the two coefficient vectors leaves it unchanged; scaling dy scales it
    assert abs(On.delta_res(fam, Q, np.array([p]), y2, y1) - want) <= 1e-13 * want
    assert abs(On.delta_res(fam, Q, np.array([p]), 3.0 * y1, 3.0 * y2) - 3.0 * want) <= 1e-13 * want


def test_sketched_residual_closed_form_on_the_tridiagonal_eigenbasis():
    n, p = 40, -0.7
    rng = np.random.default_rng(12)
    b0 = rng.standard_normal(n)
    fam = F.ShiftedTridiag(b0)
    ks = [2, 5, 9]
    Q = _sine_basis(n, ks)
    lam = np.array([2.0 - 2.0 * math.cos(k * math.pi / (n + 1)) for k in ks]) - p
    rows = np.array([3, 17, 0, 39, 22, 8])
    y = rng.standard_normal(len(ks))
    b = np.exp(b0 * math.sin(p / 10.0) * p)
    # entry i of A Q y is sum_k lam_k y_k v_k(i), v_k the sine vectors, evaluated here by hand
    i = rows + 1
    AQy = sum(lam[c] * y[c] * math.sqrt(2.0 / (n + 1)) * np.sin(i * ks[c] * np.pi / (n + 1)) for c in range(len(ks)))
    res = AQy - b[rows]
    want = np.linalg.norm(res) / np.linalg.norm(b[rows])
    got = On.sketched_residual(fam, Q, rows, np.array([p]), y)
    assert abs(got - want) <= 1e-13 * want
    # with row weights the numerator is weighted and the denominator is the full |b|
    w = rng.uniform(0.5, 2.0, size=len(rows))
    want_w = np.linalg.norm(w * res) / np.linalg.norm(b)
    got_w = On.sketched_residual(fam, Q, rows, np.array([p]), y, weights=w)
    assert abs(got_w - want_w) <= 1e-13 * want_w


def test_delta_res_closed_form_on_the_laplacian_eigenbasis():
    # p = 0: a = 1, A is the 5-point Laplacian with eigenvectors
    # sin(a pi x) sin(b pi y) and eigenvalues (4/h^2)(sin^2(a pi h/2) + sin^2(b pi h/2))
    N = 9
    h = 1.0 / (N + 1)
    fam = F.Diffusion((N, N))
    modes = [(1, 1), (2, 1), (1, 3), (4, 4), (9, 2)]
    ix = np.arange(N * N) % N
    iy = np.arange(N * N) // N
    Q = np.stack([(2.0 / (N + 1)) * np.sin(a * np.pi * (ix + 1) * h) * np.sin(b * np.pi * (iy + 1) * h)
                  for a, b in modes], axis=1)
    assert np.allclose(Q.T @ Q, np.eye(len(modes)), atol=1e-14)
    lam = np.array([(4.0 / h ** 2) * (math.sin(a * math.pi * h / 2) ** 2 + math.sin(b * math.pi * h / 2) ** 2)
                    for a, b in modes])
    rng = np.random.default_rng(13)
    y1, y2 = rng.standard_normal(len(modes)), rng.standard_normal(len(modes))
    want = np.linalg.norm(lam * (y1 - y2)) / math.sqrt(N * N)  # b = 1
    got = On.delta_res(fam, Q, np.zeros(2), y1, y2)
    assert abs(got - want) <= 1e-12 * want


def _dense_diffusion(N, dim, p):
    """A(p) entry by entry: node i at ((ix+1)h, ...), face coefficient a at the
    midpoint between a node and each axis neighbour, diagonal sum a_f / h^2,
    off-diagonal -a_f / h^2 for neighbours inside the domain."""
    h = 1.0 / (N + 1)
    n = N ** dim
    A = np.zeros((n, n))

    def coef(x):
        if dim == 2:
            t = p[0] * math.sin(2 * math.pi * x[0]) + p[1] * math.cos(2 * math.pi * x[1])
        else:
            sx, cx = math.sin(2 * math.pi * x[0]), math.cos(2 * math.pi * x[0])
            sy, cy = math.sin(2 * math.pi * x[1]), math.cos(2 * math.pi * x[1])
            sz, cz = math.sin(2 * math.pi * x[2]), math.cos(2 * math.pi * x[2])
            t = p[0] * sx * cy + p[1] * sy * cz + p[2] * sz * cx + p[3] * cx * cy * cz
        return math.exp(t)

    for i in range(n):
        c = [(i // N ** a) % N for a in range(dim)]
        x = [(ci + 1) * h for ci in c]
        for axis in range(dim):
            for sgn in (-1, 1):
                face = list(x)
                face[axis] += sgn * h / 2
                af = coef(face) / h ** 2
                A[i, i] += af
                nb = list(c)
                nb[axis] += sgn
                if 0 <= nb[axis] < N:
                    A[i, sum(nb[a] * N ** a for a in range(dim))] -= af
    return A


def test_checkers_against_dense_diffusion_operators():
    rng = np.random.default_rng(14)
    for N, dim in ((6, 2), (4, 3)):
        d = 2 if dim == 2 else 4
        p = rng.uniform(-1, 1, size=d)
        A = _dense_diffusion(N, dim, p)
        n = N ** dim
        fam = F.Diffusion((N,) * dim)
        Q, _ = np.linalg.qr(rng.standard_normal((n, 5)))
        y1, y2 = rng.standard_normal(5), rng.standard_normal(5)
        b = np.ones(n)
        want = np.linalg.norm(A @ (Q @ (y1 - y2))) / np.linalg.norm(b)
        assert abs(On.delta_res(fam, Q, p, y1, y2) - want) <= 1e-12 * want
        rows = rng.choice(n, size=9, replace=False)
        res = (A @ (Q @ y1) - b)[rows]
        want_s = np.linalg.norm(res) / np.linalg.norm(b[rows])
        assert abs(On.sketched_residual(fam, Q, rows, p, y1) - want_s) <= 1e-12 * want_s


def test_checkers_against_a_dense_kernel_matrix():
    rng = np.random.default_rng(15)
    n, dim, lam, sig = 12, 3, 1e-2, 0.8
    pts = rng.standard_normal((n, dim))
    rhs = rng.standard_normal(n)
    K = np.empty((n, n))
    for i in range(n):
        for j in range(n):
            K[i, j] = math.exp(-sum((pts[i, q] - pts[j, q]) ** 2 for q in range(dim)) / (2 * sig * sig))
    A = K + lam * np.eye(n)
    fam = F.KernelRidge(pts, rhs, lam)
    Q, _ = np.linalg.qr(rng.standard_normal((n, 4)))
    y1, y2 = rng.standard_normal(4), rng.standard_normal(4)
    want = np.linalg.norm(A @ (Q @ (y1 - y2))) / np.linalg.norm(rhs)
    assert abs(On.delta_res(fam, Q, np.array([sig]), y1, y2) - want) <= 1e-13 * want
    rows = np.array([5, 0, 11, 7])
    res = (A @ (Q @ y1) - rhs)[rows]
    want_s = np.linalg.norm(res) / np.linalg.norm(rhs[rows])
    assert abs(On.sketched_residual(fam, Q, rows, np.array([sig]), y1) - want_s) <= 1e-13 * want_s


def test_delta_res_params_against_dense_kernel_matrices():
    """The many-parameter form (one pass over the kernel rows for all length
    scales, row blocks smaller than n) against dense matrices assembled entry
    by entry, and against the per-parameter delta_res."""
    rng = np.random.default_rng(16)
    n, dim, lam = 23, 2, 1e-2
    pts = rng.standard_normal((n, dim))
    rhs = rng.standard_normal(n)
    fam = F.KernelRidge(pts, rhs, lam)
    Q, _ = np.linalg.qr(rng.standard_normal((n, 5)))
    sigs = np.array([[0.3], [1.0], [2.5]])
    Y1, Y2 = rng.standard_normal((3, 5)), rng.standard_normal((3, 5))
    got = On.delta_res_params(fam, Q, sigs, Y1, Y2)
    for i, sig in enumerate(sigs[:, 0]):
        K = np.empty((n, n))
        for a in range(n):
            for b in range(n):
                K[a, b] = math.exp(-sum((pts[a, q] - pts[b, q]) ** 2 for q in range(dim)) / (2 * sig * sig))
        want = np.linalg.norm((K + lam * np.eye(n)) @ (Q @ (Y1[i] - Y2[i]))) / np.linalg.norm(rhs)
        assert abs(got[i] - want) <= 1e-13 * want
        assert abs(got[i] - On.delta_res(fam, Q, sigs[i], Y1[i], Y2[i])) <= 1e-13 * want
    V = fam.matvec_params(sigs, np.stack([Q @ Y1[i] for i in range(3)], axis=1), chunk=7)
    for i in range(3):
        assert np.allclose(V[:, i], fam.matvec(sigs[i], Q @ Y1[i]), rtol=1e-14, atol=1e-14)


def test_delta_res_params_without_a_batched_operator():
    """Families without matvec_params fall back to delta_res per parameter:
    closed form on the tridiagonal eigenbasis for two shifts."""
    n = 40
    fam = F.ShiftedTridiag(np.zeros(n))  # b = 1 for every p
    ks = [1, 4, 9]
    Q = _sine_basis(n, ks)
    lam0 = np.array([2.0 - 2.0 * math.cos(k * math.pi / (n + 1)) for k in ks])
    P = np.array([[0.5], [-1.5]])
    Y1 = np.array([[1.0, -2.0, 0.5], [0.3, 0.0, 1.0]])
    Y2 = np.zeros_like(Y1)
    got = On.delta_res_params(fam, Q, P, Y1, Y2)
    for i, p in enumerate(P[:, 0]):
        want = np.linalg.norm((lam0 - p) * Y1[i]) / math.sqrt(n)
        assert abs(got[i] - want) <= 1e-12 * want
