"""Pins of the oracle's general affine family A(theta) = sum_q theta_q A_q
(Section 3.1, "Computing S A(p*) X") against facts that do not go through
its own arithmetic:

* the delay system of Section 6.2.2 is the two-term family A_q = (I, A_1),
  theta = (p, -(3 + e^{tau p})): the oracle's Delay rows, built from their
  own definition, must agree;
* brute force on tiny dense terms: the assembled matrix is the plain sum;
* at a snapshot parameter the solution lies in span(Q), so SubApSnap
  reproduces the snapshot (zero least-squares residual, Section 3).
"""
import numpy as np
import scipy.sparse as sp

import subap_inputs as si
from oracle import families as F
from oracle import offline as O
from oracle import online as On


def test_delay_is_a_two_term_affine_family():
    w = si.delay(n=300, r=6, s=12, m=8)
    dl = F.from_workload(w)
    A1 = dl.A1()
    af = F.Affine([sp.identity(w["n"], format="csr"), A1], w["rhs"])
    idx = np.array([0, 1, 57, 150, 298, 299])
    for p in (0.0, 0.37, 4.2, 9.9):
        theta = np.array([p, -(3.0 + np.exp(w["tau"] * p))])
        a = af.rows(theta, idx).toarray()
        b = dl.rows(np.array([p]), idx).toarray()
        assert np.abs(a - b).max() <= 1e-14 * np.abs(b).max()
        x = np.random.default_rng(1).standard_normal(w["n"])
        np.testing.assert_allclose(af.matvec(theta, x), dl.matvec(np.array([p]), x), rtol=0, atol=1e-12)


def test_affine_matrix_is_the_plain_sum():
    rng = np.random.default_rng(7)
    T = [rng.standard_normal((6, 6)) for _ in range(3)]
    af = F.Affine([sp.csr_matrix(t) for t in T], np.ones(6))
    theta = np.array([0.5, -2.0, 3.25])
    dense = np.zeros((6, 6))
    for t, c in zip(T, theta):
        for i in range(6):
            for j in range(6):
                dense[i, j] += c * t[i, j]
    assert np.abs(af.matrix(theta).toarray() - dense).max() <= 1e-14
    assert np.abs(af.rows(theta, [4, 1]).toarray() - dense[[4, 1]]).max() <= 1e-14
    x = rng.standard_normal(6)
    assert np.abs(af.matvec(theta, x) - dense @ x).max() <= 1e-13


def test_affine_reproduces_snapshots():
    w = si.affine(N=20, r=8, s=24, m=4)
    off = O.offline(w)
    fam, Q, rows = off["family"], off["Q"], off["rows"]
    Y = On.solve(fam, Q, rows, w["snap_params"])
    for i, y in enumerate(Y):
        x = off["X"][:, i]
        assert np.linalg.norm(Q @ y - x) <= 1e-9 * np.linalg.norm(x), i
