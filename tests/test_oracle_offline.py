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


# --- leverage-score sampling with weights (Section 5.3) and the residual
# estimate (Section 5.3.1)

def test_leverage_scores_equal_the_projector_diagonal():
    # diag(B (B^T B)^{-1} B^T), by normal equations instead of QR; sum = rank
    rng = np.random.default_rng(11)
    B = rng.standard_normal((60, 5)) * rng.uniform(0.1, 10.0, size=(60, 1))
    sc = O.leverage_scores(B)
    direct = np.einsum("ij,ji->i", B, np.linalg.solve(B.T @ B, B.T))
    np.testing.assert_allclose(sc, direct, rtol=1e-12, atol=1e-15)
    assert abs(sc.sum() - 5.0) < 1e-12
    assert np.all(sc >= 0.0) and np.all(sc <= 1.0 + 1e-12)


def test_leverage_sample_with_equal_scores_is_floor_u_n():
    n, s = 37, 200
    u = np.random.default_rng(12).random(s)
    rows, w = O.leverage_sample(np.ones(n), u)
    np.testing.assert_array_equal(rows, np.floor(u * n).astype(np.int64))
    np.testing.assert_allclose(w, np.sqrt(n / s), rtol=1e-15)


def test_leverage_sample_matches_a_linear_scan():
    sc = np.array([0.5, 0.0, 2.0, 1e-3, 0.0, 1.25, 0.25])
    u = np.concatenate([np.linspace(0.0, 0.999999, 97), [0.1249, 0.1251, 0.6253, 0.9999999]])
    rows, w = O.leverage_sample(sc, u)
    total = 0.0
    for v in sc:
        total += v
    for k, uk in enumerate(u):
        acc, pick = 0.0, None
        for i, v in enumerate(sc):
            acc += v
            if acc > uk * total:
                pick = i
                break
        assert rows[k] == pick
        assert sc[pick] > 0.0
        assert abs(w[k] - 1.0 / np.sqrt(u.size * sc[pick] / total)) <= 1e-14 * w[k]


def test_weighted_sketch_is_unbiased():
    # E |W S v|^2 = |v|^2; stratified draws u_k = (k + 1/2) / K make the sample
    # frequencies equal to pi_i up to one count, so the sum converges
    rng = np.random.default_rng(13)
    sc = rng.uniform(0.2, 3.0, size=40)
    v = rng.standard_normal(40)
    K = 40000
    rows, w = O.leverage_sample(sc, (np.arange(K) + 0.5) / K)
    est = np.sum((w * v[rows]) ** 2)
    assert abs(est / (v @ v) - 1.0) < 2e-3


def test_all_rows_once_with_unit_weights_is_apsnap():
    # equal scores and one draw per row: W S is a permutation, so the weighted
    # SubApSnap problem is ApSnap's (eq. (3.1))
    from oracle import online as On
    w = si.diffusion2d(N=10, r=4, s=100)
    off = O.offline(w)
    rows, wt = O.leverage_sample(np.ones(w["n"]), (np.arange(w["n"]) + 0.5) / w["n"])
    np.testing.assert_array_equal(np.sort(rows), np.arange(w["n"]))
    np.testing.assert_allclose(wt, 1.0, rtol=1e-15)
    for p in w["test_params"][:4]:
        y = On.solve_one(off["family"], off["Q"], rows, p, wt)
        ya = On.apsnap_solve(off["family"], off["Q"], p)
        np.testing.assert_allclose(y, ya, rtol=1e-10, atol=1e-12 * np.abs(ya).max())


def test_a_repeated_row_equals_one_row_of_summed_squared_weight():
    from oracle import online as On
    w = si.diffusion2d(N=10, r=4, s=12)
    off = O.offline(w)
    rows = np.array([3, 3, 17, 40, 41, 55, 60, 71, 88, 90, 97, 5])
    wt = np.linspace(0.5, 2.0, rows.size)
    wt[1] = wt[0]
    rows2 = rows[1:]
    wt2 = wt[1:].copy()
    wt2[0] = np.sqrt(2.0) * wt[0]
    p = w["test_params"][0]
    y1 = On.solve_one(off["family"], off["Q"], rows, p, wt)
    y2 = On.solve_one(off["family"], off["Q"], rows2, p, wt2)
    np.testing.assert_allclose(y1, y2, rtol=1e-11, atol=1e-13 * np.abs(y1).max())


def test_leverage_selection_estimates_the_full_residual():
    # At p_sel, the weighted sketch of span([A X, b]) keeps every residual in
    # that span within (1 +- eps) of its full norm for nearly every draw
    # (Section 5.3.1); eps = k log k / s with k = r + 1
    from oracle import online as On
    w = si.diffusion2d(N=16, r=5, s=96)
    off = O.offline(w)
    fam, Q, p = off["family"], off["Q"], w["select_param"]
    B = O.leverage_matrix(fam, Q, p)
    sc = O.span_scores(B)
    lo_hi_ok, ratios = 0, []
    for seed in range(20):
        rows, wt = O.leverage_sample(sc, si.sample_uniforms(w["s"], seed=seed))
        y = On.solve_one(fam, Q, rows, p, wt)
        full = On.residual(fam, Q @ y, p)
        est = On.sketched_residual(fam, Q, rows, p, y, wt)
        lo, hi = O.residual_bounds(est, w["r"], w["s"])
        ratios.append(est / full)
        lo_hi_ok += lo <= full <= hi
    assert lo_hi_ok >= 18, ratios
    assert 0.7 < np.median(ratios) < 1.3


def test_residual_bounds_default_eps():
    lo, hi = O.residual_bounds(1e-3, 15, 64)
    eps = 16 * np.log(16) / 64
    assert abs(lo - 1e-3 / (1 + eps)) < 1e-18 and abs(hi - 1e-3 / (1 - eps)) < 1e-18
    assert O.residual_bounds(1.0, 40, 41)[1] == np.inf


def test_offline_with_sample_u_returns_weighted_rows():
    w = si.diffusion2d(N=12, r=4, s=20)
    u = si.sample_uniforms(20, seed=3)
    off = O.offline(w, sample_u=u)
    B = O.leverage_matrix(off["family"], off["Q"], w["select_param"])
    rows, wt = O.leverage_sample(O.span_scores(B), u)
    np.testing.assert_array_equal(off["rows"], rows)
    np.testing.assert_array_equal(off["weights"], wt)
    assert O.offline(w)["weights"] is None


def test_span_scores_drop_a_right_hand_side_inside_the_span():
    # b in span(A Q): span([A Q, b]) is r-dimensional, the scores are those of
    # A Q and sum to r; a generic b adds its direction and the sum is r + 1
    rng = np.random.default_rng(14)
    AQ = rng.standard_normal((80, 6))
    inside = np.column_stack([AQ, AQ @ rng.standard_normal(6)])
    np.testing.assert_allclose(O.span_scores(inside), O.leverage_scores(AQ), rtol=1e-10, atol=1e-14)
    assert abs(O.span_scores(inside).sum() - 6.0) < 1e-12
    generic = np.column_stack([AQ, rng.standard_normal(80)])
    np.testing.assert_allclose(O.span_scores(generic), O.leverage_scores(generic), rtol=1e-12)
    assert abs(O.span_scores(generic).sum() - 7.0) < 1e-12


# --- LU with partial pivoting (Section 5.3) and the union of pivots (Section 5.3.2)

def test_lupp_pivots_equal_lapack_partial_pivoting():
    rng = np.random.default_rng(15)
    W = rng.standard_normal((40, 7))
    _, ipiv = sla.lu_factor(W)
    perm = np.arange(40)
    for j, pj in enumerate(ipiv):
        perm[[j, pj]] = perm[[pj, j]]
    np.testing.assert_array_equal(O.lupp_pivots(W, 7), perm[:7])


def test_lupp_on_a_basis_is_the_deim_greedy_selection():
    # DEIM's indices (eq. (3.5)): first argmax |u_1|, then argmax of the
    # residual of interpolating u_l at the indices so far
    rng = np.random.default_rng(16)
    U, _ = np.linalg.qr(rng.standard_normal((60, 6)))
    idx = [int(np.argmax(np.abs(U[:, 0])))]
    for l in range(1, 6):
        c = np.linalg.solve(U[idx, :l], U[idx, l])
        res = U[:, l] - U[:, :l] @ c
        idx.append(int(np.argmax(np.abs(res))))
    np.testing.assert_array_equal(O.lupp_pivots(U, 6), idx)


def test_lu_rounds_and_union():
    rng = np.random.default_rng(17)
    W = rng.standard_normal((50, 5))
    rows = O.select_rows_lu(W, 12)
    assert rows.size == 12 and np.unique(rows).size == 12
    np.testing.assert_array_equal(rows[:5], O.lupp_pivots(W, 5))
    rest = np.setdiff1d(np.arange(50), rows[:5])
    np.testing.assert_array_equal(rows[5:10], rest[O.lupp_pivots(W[rest], 5)])
    np.testing.assert_array_equal(O.union_rows([[3, 1, 4], [1, 5, 9], [2, 6, 5]]), [3, 1, 4, 5, 9, 2, 6])


def test_offline_union_of_pivots_at_several_points():
    w = si.diffusion2d(N=12, r=4, s=4)
    pts = np.array([[-0.5, 0.5], [0.0, 0.0], [0.7, -0.2]])
    off = O.offline(w, selection="lu", select_params=pts)
    fam, Q = off["family"], off["Q"]
    sets = [O.select_rows_lu(O.selection_matrix(fam, Q, p).T, 4) for p in pts]
    np.testing.assert_array_equal(off["rows"], O.union_rows(sets))
    assert 4 <= off["rows"].size <= 12
