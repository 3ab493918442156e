"""Seeded synthetic inputs for SubApSnap workloads.

This module only draws random numbers and fixes sizes.  It holds none of the
method's arithmetic (no matrix rows, no solves, no contractions), so both the
FP64 CPU oracle and the GPU library's tests and benchmark can take their
inputs from it without sharing any computation.

Every generator returns a plain dict of numpy arrays and Python scalars.
Random streams come from ``numpy.random.SeedSequence(base).spawn(k)`` in a
fixed order (snapshot points, test points, data points, noise), so a given
base seed always yields the same workload on any machine.

Workloads (sizes follow the paper's problem classes: a parameter-dependent
diffusion PDE as in Section 6.1, and a Gaussian-kernel ridge regression as in
Section 6.3, eqs. (6.3)-(6.4)):

* ``diffusion2d``  -div(a grad u) = 1 on the unit square, 5-point stencil,
  a(x, y; p) = exp(p1 sin 2 pi x + p2 cos 2 pi y), p in [-1, 1]^2.
* ``diffusion3d``  7-point stencil on the unit cube with four sin/cos modes,
  p in [-1, 1]^4.
* ``krr``          (K_p + lambda I) x = b with a Gaussian kernel of length
  scale p, points from an 8-component Gaussian mixture in R^8,
  p log-uniform in [0.5, 2].
* ``uneven``       64 independent 2-D diffusion instances of varied size.
* ``tridiag``      the shifted tridiagonal family of eq. (5.7).
* ``affine``       a general affine family A(theta) = sum_q theta_q A_q
  (Section 3.1, "Computing S A(p*) X"): its terms are inputs of the family,
  given as sparse matrices, like the data points of ``krr``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "diffusion2d", "diffusion3d", "krr", "uneven", "tridiag", "identity",
    "surrogate", "sample_uniforms", "delay", "affine",
]


def _streams(base: int, k: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(base).spawn(k)]


def sample_uniforms(s: int, seed: int = 909) -> np.ndarray:
    """s seeded uniforms in [0, 1): the draws of a randomised row sampler."""
    return np.random.default_rng(seed).random(s)


def diffusion2d(N: int = 64, r: int = 16, s: int = 32, m: int = 64, seed: int = 101) -> dict:
    """2-D diffusion workload: N x N interior grid, n = N^2 (default 4096)."""
    g_snap, g_test = _streams(seed, 2)
    return dict(
        family="diff2d", grid=(N, N), n=N * N, d=2, r=r, s=s, m=m,
        snap_params=g_snap.uniform(-1.0, 1.0, size=(r, 2)),
        test_params=g_test.uniform(-1.0, 1.0, size=(m, 2)),
        select_param=np.zeros(2),
    )


def diffusion3d(N: int = 215, r: int = 40, s: int = 160, m: int = 65536,
                n_lift: int = 1024, seed: int = 303) -> dict:
    """3-D diffusion workload: N^3 interior grid (default n = 9,938,375)."""
    g_snap, g_test = _streams(seed, 2)
    return dict(
        family="diff3d", grid=(N, N, N), n=N ** 3, d=4, r=r, s=s, m=m,
        n_lift=min(n_lift, m),
        snap_params=g_snap.uniform(-1.0, 1.0, size=(r, 4)),
        test_params=g_test.uniform(-1.0, 1.0, size=(m, 4)),
        select_param=np.zeros(4),
    )


def krr(n: int = 16384, dim: int = 8, r: int = 32, s: int = 128, m: int = 4096,
        lam: float = 1e-2, components: int = 8, seed: int = 202) -> dict:
    """Kernel ridge regression workload.

    Points: equal-weight ``components``-component Gaussian mixture in R^dim,
    means uniform in [-3, 3]^dim, identity covariance.  Targets:
    sin(sum of coordinates) + 0.1 N(0, 1).  The parameter is the kernel
    length scale, drawn log-uniformly in [0.5, 2]; rows are selected at its
    geometric centre p = 1.
    """
    g_snap, g_test, g_pts, g_noise = _streams(seed, 4)
    snap = np.exp(g_snap.uniform(np.log(0.5), np.log(2.0), size=(r, 1)))
    test = np.exp(g_test.uniform(np.log(0.5), np.log(2.0), size=(m, 1)))
    means = g_pts.uniform(-3.0, 3.0, size=(components, dim))
    comp = g_pts.integers(components, size=n)
    points = means[comp] + g_pts.standard_normal(size=(n, dim))
    noise = g_noise.standard_normal(size=n)
    targets = np.sin(points.sum(axis=1)) + 0.1 * noise
    return dict(
        family="krr", n=n, dim=dim, d=1, r=r, s=s, m=m, lam=lam,
        points=points, rhs=targets,
        snap_params=snap, test_params=test, select_param=np.ones(1),
    )


def uneven(k: int = 64, seed: int = 404, max_m: int = 4096,
           grids=(32, 64, 128, 256, 512)) -> list:
    """List of ``k`` independent 2-D diffusion instances of uneven size.

    Instance i: grid side grids[i % len(grids)], r = (8, 16, 32, 64)[i % 4],
    s drawn uniformly in [2r, 4r], m = 2^j with j uniform in [4, 12] (capped at
    ``max_m``).  Each instance has its own snapshot and test points.
    """
    g_sizes, *g_inst = _streams(seed, 1 + 2 * k)
    out = []
    for i in range(k):
        N = grids[i % len(grids)]
        r = (8, 16, 32, 64)[i % 4]
        s = int(g_sizes.integers(2 * r, 4 * r + 1))
        m = min(int(2 ** g_sizes.integers(4, 13)), max_m)
        g_snap, g_test = g_inst[2 * i], g_inst[2 * i + 1]
        out.append(dict(
            family="diff2d", grid=(N, N), n=N * N, d=2, r=r, s=s, m=m,
            snap_params=g_snap.uniform(-1.0, 1.0, size=(r, 2)),
            test_params=g_test.uniform(-1.0, 1.0, size=(m, 2)),
            select_param=np.zeros(2),
        ))
    return out


def delay(n: int = 10 ** 7, r: int = 10, s: int = 40, m: int = 65536, seed: int = 606,
          p_range=(0.0, 10.0)) -> dict:
    """Delay system of Section 6.2.2 (tau = 0.1, kappa = 2.1, n = 10^7 by
    default) with a real parameter p uniform in p_range; b and the output
    vector c are seeded standard normal vectors (a constant b would be an
    eigenvector of T and make every solution a multiple of it)."""
    g_snap, g_test, g_vec = _streams(seed, 3)
    lo, hi = p_range
    return dict(
        family="delay", n=n, d=1, r=r, s=s, m=m, tau=0.1, kappa=2.1,
        rhs=g_vec.standard_normal(n), c_out=g_vec.standard_normal(n),
        snap_params=g_snap.uniform(lo, hi, size=(r, 1)),
        test_params=g_test.uniform(lo, hi, size=(m, 1)),
        select_param=np.array([0.5 * (lo + hi)]),
    )


def tridiag(n: int = 100, r: int = 7, m: int = 201, seed: int = 57) -> dict:
    """Shifted tridiagonal family of eq. (5.7): snapshots equispaced on [-10, -9]."""
    (g_b,) = _streams(seed, 1)
    return dict(
        family="tridiag", n=n, d=1, r=r, s=r, m=m,
        b0=g_b.standard_normal(size=n),
        snap_params=np.linspace(-10.0, -9.0, r).reshape(r, 1),
        test_params=np.linspace(-10.0, -9.0, m).reshape(m, 1),
        select_param=np.array([-9.5]),
    )


def identity(n: int = 200, r: int = 6, m: int = 32, seed: int = 58) -> dict:
    """Identity family (A = I): parameter points for the DEIM special case."""
    g_snap, g_test = _streams(seed, 2)
    return dict(
        family="identity", n=n, d=1, r=r, s=r, m=m,
        snap_params=g_snap.uniform(0.0, 1.0, size=(r, 1)),
        test_params=g_test.uniform(0.0, 1.0, size=(m, 1)),
        select_param=np.array([0.5]),
    )


def affine(N: int = 64, r: int = 12, s: int = 48, m: int = 4096, seed: int = 707) -> dict:
    """Three-term affine family on the N x N interior grid of the unit square,
    A(theta) = theta_0 L + theta_1 C + theta_2 R: L the 5-point negative
    Laplacian (h^-2 scaled), C the centred first difference in x (a
    convection term, skew-symmetric), R = diag(rho) with a seeded reaction
    field rho in [0.5, 1.5].  A(theta) is nonsymmetric, and its symmetric part
    theta_0 L + theta_2 R is positive definite, so it is nonsingular.  b is a
    seeded smooth source; theta_0 in [1, 2], theta_1 in [0, 500], theta_2 in
    [0, 5000], uniform."""
    import scipy.sparse as sps
    g_snap, g_test, g_field = _streams(seed, 3)
    n = N * N
    h = 1.0 / (N + 1)
    one = np.ones(N)
    d2 = sps.diags([-one[:-1], 2 * one, -one[:-1]], [-1, 0, 1])
    eye = sps.identity(N)
    lap = ((sps.kron(eye, d2) + sps.kron(d2, eye)) / (h * h)).tocsr()
    d1 = sps.diags([-0.5 * one[:-1], 0.5 * one[:-1]], [-1, 1])
    conv = (sps.kron(eye, d1) / h).tocsr()
    x = (np.arange(N) + 1) * h
    X, Y = np.meshgrid(x, x)
    amp = g_field.uniform(-0.5, 0.5, size=3)
    rho = 1.0 + amp[0] * np.sin(2 * np.pi * X) * np.cos(np.pi * Y) + amp[1] * X * Y
    rho = np.clip(rho, 0.5, 1.5).reshape(-1)
    react = sps.diags(rho).tocsr()
    rhs = (np.sin(np.pi * X) * np.sin(2 * np.pi * Y) + 1.0 + 0.1 * amp[2]).reshape(-1)
    lo = np.array([1.0, 0.0, 0.0])
    hi = np.array([2.0, 500.0, 5000.0])
    return dict(
        family="affine", n=n, d=3, r=r, s=s, m=m, grid=(N, N),
        terms=[lap, conv, react], rhs=rhs,
        snap_params=lo + (hi - lo) * g_snap.random((r, 3)),
        test_params=lo + (hi - lo) * g_test.random((m, 3)),
        select_param=0.5 * (lo + hi),
    )


def surrogate(n_train: int = 1 << 18, n_infer: int = 1 << 20, d: int = 4,
              seed: int = 505) -> dict:
    """Parameter sets for the learned surrogate on the 3-D family."""
    g_train, g_infer, g_init = _streams(seed, 3)
    return dict(
        train_params=g_train.uniform(-1.0, 1.0, size=(n_train, d)),
        infer_params=g_infer.uniform(-1.0, 1.0, size=(n_infer, d)),
        init_seed=int(g_init.integers(1 << 31)),
    )


def mlp_init(widths=(4, 256, 256, 40), seed: int = 506) -> list:
    """He-style uniform initial weights for an MLP, as (W, b) pairs, FP64.

    W_l has shape (fan_out, fan_in) and is uniform in +-sqrt(6/fan_in); b_l = 0.
    """
    (g,) = _streams(seed, 1)
    params = []
    for fi, fo in zip(widths[:-1], widths[1:]):
        lim = np.sqrt(6.0 / fi)
        params.append((g.uniform(-lim, lim, size=(fo, fi)), np.zeros(fo)))
    return params
