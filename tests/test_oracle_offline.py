"""Pins for oracle.offline (Algorithm 3.1 steps 1-3)."""
import numpy as np
import pytest
import scipy.linalg as sla

import subap_inputs as si
from oracle import families as F
from oracle import offline as O


def test_snapshots_solve_the_systems():
    w = si.diffusion2d(N=16, r=5, s=10)
    fam = F.from_workload(w)
    X = O.snapshots(fam, w["snap_params"])
    for i, p in enumerate(w["snap_params"]):
        r = fam.matvec(p, X[:, i]) - fam.rhs(p)
        assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(fam.rhs(p))


def test_krr_snapshots_solve_the_systems():
    w = si.krr(n=400, r=4, s=8)
    fam = F.from_workload(w)
    X = O.snapshots(fam, w["snap_params"])
    for i, p in enumerate(w["snap_params"]):
        r = fam.matvec(p, X[:, i]) - fam.rhs(p)
        assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(fam.rhs(p))


def test_orthonormalise_is_a_qr_with_positive_diagonal():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((200, 12))
    Q, R = O.orthonormalise(X)
    assert np.abs(Q.T @ Q - np.eye(12)).max() < 1e-14
    assert np.abs(Q @ R - X).max() < 1e-13 * np.abs(X).max()
    assert np.all(np.diag(R) > 0)
    assert np.abs(np.tril(R, -1)).max() == 0.0
    # unique: equals LAPACK's QR after fixing the signs
    Q2, R2 = sla.qr(X, mode="economic")
    sg = np.sign(np.diag(R2))
    assert np.abs(Q2 * sg - Q).max() < 1e-13


@pytest.mark.parametrize("shape", [(6, 40), (10, 300), (16, 64)])
def test_cpqr_pivots_equal_lapack_on_tie_free_input(shape):
    rng = np.random.default_rng(shape[1])
    M = rng.standard_normal(shape)
    k = shape[0]
    _, _, piv = sla.qr(M, pivoting=True, mode="economic")
    assert np.array_equal(O.cpqr_pivots(M, k), piv[:k])


def test_cpqr_tie_rule_takes_smallest_index():
    rng = np.random.default_rng(1)
    base = rng.standard_normal((4, 6))
    # columns 7 and 2 are exact copies of the largest column; 7 + 1e-9 noise
    big = 10 * rng.standard_normal(4)
    M = np.concatenate([base[:, :2], big[:, None], base[:, 2:], big[:, None] * (1 + 1e-9)], axis=1)
    assert M.shape[1] == 8
    piv = O.cpqr_pivots(M, 1)
    assert piv[0] == 2
    # with the rule switched off (tolerance 0) the larger copy wins
    assert O.cpqr_pivots(M, 1, tie_rtol=0.0)[0] == 7


def test_select_rows_rounds():
    rng = np.random.default_rng(5)
    M = rng.standard_normal((5, 60))
    rows = O.select_rows(M, 5)
    assert np.array_equal(rows, O.cpqr_pivots(M, 5))
    rows = O.select_rows(M, 13)
    assert len(rows) == 13 and len(set(rows.tolist())) == 13
    assert np.array_equal(rows[:5], O.cpqr_pivots(M, 5))
    rest = np.setdiff1d(np.arange(60), rows[:5])
    assert np.array_equal(rows[5:10], rest[O.cpqr_pivots(M[:, rest], 5)])
    with pytest.raises(ValueError):
        O.select_rows(M, 4)


def test_offline_pipeline_c1_shape():
    w = si.diffusion2d()
    off = O.offline(w)
    assert off["Q"].shape == (4096, 16)
    assert len(off["rows"]) == 32 and len(set(off["rows"].tolist())) == 32
    sv = np.linalg.svd(off["X"], compute_uv=False)
    assert sv[-1] / sv[0] > 1e-8  # full-rank snapshots: index parity is meaningful
