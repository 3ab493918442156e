"""Pins for oracle.online against facts the paper states (Sections 3-5)."""
import numpy as np
import pytest
import scipy.linalg as sla

import subap_inputs as si
from oracle import families as F
from oracle import offline as O
from oracle import online as On


@pytest.fixture(scope="module")
def c1_small():
    w = si.diffusion2d(N=24, r=8, s=16, m=12)
    return w, O.offline(w)


def test_householder_lsq_matches_svd_lstsq():
    rng = np.random.default_rng(11)
    G = rng.standard_normal((40, 9))
    b = rng.standard_normal(40)
    y, R, rho = On.householder_lsq(G, b)
    ref, res, *_ = np.linalg.lstsq(G, b, rcond=None)
    assert np.abs(y - ref).max() < 1e-13 * np.abs(ref).max()
    assert rho == pytest.approx(np.sqrt(res[0]), rel=1e-12)


def test_snapshot_point_reproduces_snapshot(c1_small):
    # Section 5.2 / Fig. 1: at p* = p_i the snapshot x(p_i) lies in span(X)
    w, off = c1_small
    fam, Q, X, rows = off["family"], off["Q"], off["X"], off["rows"]
    for i, p in enumerate(w["snap_params"]):
        y = On.solve_one(fam, Q, rows, p)
        assert np.linalg.norm(Q @ y - X[:, i]) <= 1e-12 * np.linalg.norm(X[:, i])


def test_manufactured_solution_in_span_is_recovered(c1_small):
    # Lemma 5.1: if b = B c exactly then the subsampled problem returns c
    w, off = c1_small
    Q, rows = off["Q"], off["rows"]
    rng = np.random.default_rng(2)
    p = rng.uniform(-1, 1, 2)
    c = rng.standard_normal(Q.shape[1])
    base = F.Diffusion(w["grid"])
    fam = F.Diffusion(w["grid"], rhs=base.matvec(p, Q @ c))
    y = On.solve_one(fam, Q, rows, p)
    assert np.linalg.norm(y - c) <= 1e-11 * np.linalg.norm(c)


def test_s_equal_r_interpolates_selected_rows():
    # Section 3: with s = r, A(p*) x_hat equals b on the r selected rows
    w = si.diffusion2d(N=24, r=8, s=8)
    off = O.offline(w)
    fam, Q, rows = off["family"], off["Q"], off["rows"]
    for p in w["test_params"][:5]:
        x = Q @ On.solve_one(fam, Q, rows, p)
        r_S = fam.rows(p, rows) @ x - fam.rhs_rows(p, rows)
        assert np.abs(r_S).max() <= 1e-10 * np.abs(fam.rhs_rows(p, rows)).max()


def test_identity_family_reduces_to_deim():
    # Section 3.4, eq. (3.5): with A = I SubApSnap is DEIM; for s = r
    # x_hat = Q (S Q)^{-1} S y(p*), exact on the selected rows.
    w = si.identity()
    off = O.offline(w)
    fam, Q, rows = off["family"], off["Q"], off["rows"]
    for p in w["test_params"][:6]:
        x = Q @ On.solve_one(fam, Q, rows, p)
        yS = fam.rhs_rows(p, rows)
        deim = Q @ sla.lu_solve(sla.lu_factor(Q[rows]), yS)
        assert np.abs(x - deim).max() <= 1e-10 * np.abs(deim).max()
        assert np.abs(x[rows] - yS).max() <= 1e-12
    # Q-DEIM: rows are the pivoted-QR pivots of Q^T
    assert np.array_equal(rows, O.cpqr_pivots(Q.T, Q.shape[1]))


def test_orthonormalisation_does_not_change_the_solution(c1_small):
    # Section 3.1: replacing X by Q_X leaves X c unchanged (same S)
    w, off = c1_small
    fam, Q, X, rows = off["family"], off["Q"], off["X"], off["rows"]
    for p in w["test_params"][:4]:
        xq = Q @ On.solve_one(fam, Q, rows, p)
        xx = X @ On.solve_one(fam, X, rows, p)
        assert np.linalg.norm(xq - xx) <= 1e-9 * np.linalg.norm(xq)


def test_all_rows_is_apsnap_and_apsnap_is_never_worse(c1_small):
    # S = I_n turns SubApSnap into ApSnap (eq. (3.1)); Lemma 5.1: ApSnap <= SubApSnap
    w, off = c1_small
    fam, Q, rows = off["family"], off["Q"], off["rows"]
    allrows = np.arange(fam.n)
    for p in w["test_params"][:4]:
        c_full = On.apsnap_solve(fam, Q, p)
        c_all = On.solve_one(fam, Q, allrows, p)
        assert np.linalg.norm(c_full - c_all) <= 1e-10 * np.linalg.norm(c_full)
        sub = On.residual(fam, Q @ On.solve_one(fam, Q, rows, p), p)
        full = On.residual(fam, Q @ c_full, p)
        assert full <= sub * (1 + 1e-12)


def _polar_u(B):
    W, _, Vt = np.linalg.svd(B, full_matrices=False)
    return W @ Vt


def test_lemma_5_1_bounds(c1_small):
    # eq. (5.2): ratio <= |S| / sigma_min(S U); eq. (5.3): ratio <= kappa_2(S U~)
    w, off = c1_small
    fam, Q, rows = off["family"], off["Q"], off["rows"]
    for p in w["test_params"]:
        B = np.asarray(fam.matvec(p, Q))
        b = fam.rhs(p)
        c = On.apsnap_solve(fam, Q, p)
        ch = On.solve_one(fam, Q, rows, p)
        ratio = np.linalg.norm(B @ ch - b) / np.linalg.norm(B @ c - b)
        U = _polar_u(B)
        Ut = _polar_u(np.column_stack([B, b]))
        b52 = 1.0 / np.linalg.svd(U[rows], compute_uv=False)[-1]
        sv = np.linalg.svd(Ut[rows], compute_uv=False)
        b53 = sv[0] / sv[-1]
        assert 1.0 - 1e-12 <= ratio <= b52 * (1 + 1e-10)
        assert ratio <= b53 * (1 + 1e-10)


def test_corollary_5_3_on_tridiagonal_example():
    # eq. (5.7) with 7 equispaced snapshots on [-10, -9]; L = 1 since
    # |A(p) - A(p')|_2 = |p - p'|.  Bound (5.5) with the nearest snapshot,
    # bound (5.6) with the grid spacing; residuals vanish at snapshots.
    w = si.tridiag()
    off = O.offline(w)
    fam, Q, rows, X = off["family"], off["Q"], off["rows"], off["X"]
    snaps = w["snap_params"][:, 0]
    smin = lambda M: np.linalg.svd(M, compute_uv=False)[-1]
    sU = {i: smin(_polar_u(fam.matrix([pi]) @ Q)[rows]) for i, pi in enumerate(snaps)}
    sA = {i: smin(fam.matrix([pi]) @ Q) for i, pi in enumerate(snaps)}
    hgrid = (snaps[1] - snaps[0]) / 2
    C_hat = 3.0 / min(sA.values())
    den2 = min(sU.values()) - C_hat * hgrid
    checked = 0
    for p in w["test_params"][:, 0]:
        i = int(np.argmin(np.abs(snaps - p)))
        dist = abs(p - snaps[i])
        B = fam.matrix([p]) @ Q
        b = fam.rhs([p])
        ch = On.solve_one(fam, Q, rows, [p])
        if dist < 1e-12:
            assert np.linalg.norm(B @ ch - b) <= 1e-10 * np.linalg.norm(b)
            continue
        c = np.linalg.lstsq(B, b, rcond=None)[0]
        ratio = np.linalg.norm(B @ ch - b) / np.linalg.norm(B @ c - b)
        den1 = sU[i] - 3.0 / sA[i] * dist
        if den1 > 0:
            assert ratio <= 1.0 / den1 * (1 + 1e-8)
            checked += 1
        if den2 > 0:
            assert ratio <= 1.0 / den2 * (1 + 1e-8)
    assert checked > 100  # the bound is not vacuous on this example


def test_sketched_residual_is_zero_for_interpolation():
    w = si.diffusion2d(N=16, r=6, s=6)
    off = O.offline(w)
    fam, Q, rows = off["family"], off["Q"], off["rows"]
    p = w["test_params"][0]
    y = On.solve_one(fam, Q, rows, p)
    assert On.sketched_residual(fam, Q, rows, p, y) < 1e-10
    # and delta_res of a vector with itself is zero
    assert On.delta_res(fam, Q, p, y, y) == 0.0


# --- polishing by conjugate gradients (Section 3.1)

def test_cg_polish_terminates_in_n_steps():
    # CG on an SPD n x n system reaches the solution within n iterations
    from oracle import families as Fm
    w = si.diffusion2d(N=5, r=3, s=6)
    fam = Fm.from_workload(w)
    p = w["test_params"][0]
    xs = np.linalg.solve(fam.matrix(p).toarray(), fam.rhs(p))
    for jac in (True, False):
        x, rr = On.cg_polish(fam, p, np.zeros(fam.n), fam.n, jacobi=jac)
        np.testing.assert_allclose(x, xs, rtol=1e-9, atol=1e-12 * np.abs(xs).max())
        assert rr < 1e-9


def test_cg_polish_keeps_the_solution_and_lowers_the_energy_error():
    from oracle import families as Fm
    w = si.diffusion2d(N=12, r=3, s=6)
    fam = Fm.from_workload(w)
    p = w["test_params"][1]
    A = fam.matrix(p)
    xs = np.linalg.solve(A.toarray(), fam.rhs(p))
    x, rr = On.cg_polish(fam, p, xs, 3)
    assert rr < 1e-12 and np.abs(x - xs).max() <= 1e-12 * np.abs(xs).max()
    x0 = np.zeros(fam.n)
    errs = []
    for k in range(0, 12, 2):
        xk, _ = On.cg_polish(fam, p, x0, k)
        e = xk - xs
        errs.append(float(e @ (A @ e)))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs, errs[1:])), errs
