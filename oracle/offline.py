"""Offline phase of SubApSnap (Algorithm 3.1, steps 1-3), FP64 CPU oracle.

Test infrastructure only (see the package docstring).

* ``snapshots``      step 1: solve A(p_i) x_i = b(p_i) directly for every
                     snapshot point and stack X = [x_1 ... x_r].
* ``orthonormalise`` step 2 / Section 3.1 ("Postprocessing the snapshot
                     matrix"): thin Householder QR X = Q R, X <- Q.  The sign
                     of each column is fixed so that diag(R) > 0, which makes
                     Q unique for full-rank X.
* ``cpqr_pivots``    column-pivoted QR (Businger-Golub), one of the row
                     selectors of Section 5.3 applied to (A(p_i) X)^T.
* ``select_rows``    s >= r rows by rounds of pivoted QR: each round runs a
                     fresh pivoted QR on the columns not chosen yet and takes
                     min(r, s - chosen) pivots.  With s = r this is exactly
                     one pivoted QR (interpolation, Section 3).
* ``leverage_scores`` / ``span_scores`` / ``leverage_sample``  the randomised selector of
                     Section 5.3 the paper recommends when s > r: rows drawn
                     with probability proportional to the squared row norms of
                     the orthonormal factor of [A(p_sel) X, b(p_sel)] (the span
                     Section 5.3.1 samples so that the sketched residual
                     estimates the full one), each sampled row weighted by
                     1/sqrt(s pi_i) as the Section 5.3 footnote prescribes.
* ``lupp_pivots`` / ``select_rows_lu``  LU with partial pivoting on
                     A(p_sel) X, the other deterministic selector of Section
                     5.3 (rounds for s > r, as for pivoted QR).
* ``union_rows``     the union of the pivots found at several points
                     (Section 5.3.2).
* ``offline``        all of the above for a workload.

Readings where the paper is silent (kept identical in the GPU library):
the tie rule of the pivot search takes the smallest column index among the
candidates whose residual norm is >= (1 - 1e-6) of the maximum, with the
residual norms recomputed exactly at every step; rows are selected at the
centre of the parameter domain.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import families as fam

TIE_RTOL = 1e-6


def snapshots(family, snap_params) -> np.ndarray:
    """Step 1 of Algorithm 3.1: X[:, i] = A(p_i)^{-1} b(p_i), direct solves."""
    P = np.atleast_2d(np.asarray(snap_params, dtype=np.float64))
    X = np.empty((family.n, P.shape[0]))
    for i, p in enumerate(P):
        A = family.matrix(p)
        b = family.rhs(p)
        if sp.issparse(A):
            X[:, i] = spla.spsolve(A.tocsc(), b)
        else:
            c, low = sla.cho_factor(A)
            X[:, i] = sla.cho_solve((c, low), b)
    return X


def orthonormalise(X):
    """Thin Householder QR X = Q R with diag(R) > 0; returns (Q, R)."""
    Q, R = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return Q * sgn, R * sgn[:, None]


def cpqr_pivots(M, k, tie_rtol=TIE_RTOL):
    """First k pivot columns of a column-pivoted Householder QR of M (m x N).

    At step j the residual norms |R[j:, c]| of the columns not pivoted yet
    are recomputed from scratch; the pivot is the smallest column index
    whose norm is >= (1 - tie_rtol) * max.  The Householder reflector that
    zeros the pivot column below row j is then applied to every column.
    """
    R = np.array(M, dtype=np.float64, copy=True)
    m, N = R.shape
    k = min(k, m, N)
    free = np.ones(N, dtype=bool)
    piv = []
    for j in range(k):
        norms = np.sqrt(np.sum(R[j:, :] ** 2, axis=0))
        norms[~free] = -1.0
        top = norms.max()
        c = int(np.flatnonzero(norms >= (1.0 - tie_rtol) * top)[0])
        piv.append(c)
        free[c] = False
        # Householder reflector H = I - 2 v v^T / (v^T v) mapping R[j:, c] to -sign * |.| e_1
        x = R[j:, c].copy()
        alpha = -np.copysign(np.linalg.norm(x), x[0])
        v = x
        v[0] -= alpha
        vv = v @ v
        if vv > 0.0:
            R[j:, :] -= np.outer(v, (2.0 / vv) * (v @ R[j:, :]))
    return np.array(piv, dtype=np.int64)


def select_rows(M, s, tie_rtol=TIE_RTOL):
    """s row indices of A(p_sel) X by rounds of pivoted QR on M = (A(p_sel) X)^T.

    Returns the indices in selection order (round 1 first).
    """
    M = np.asarray(M, dtype=np.float64)
    r, n = M.shape
    if not (r <= s <= n):
        raise ValueError("need r <= s <= n")
    chosen = []
    remaining = np.arange(n)
    while len(chosen) < s:
        take = min(r, s - len(chosen))
        piv = cpqr_pivots(M[:, remaining], take, tie_rtol)
        new = remaining[piv]
        chosen.extend(int(v) for v in new)
        keep = np.ones(remaining.size, dtype=bool)
        keep[piv] = False
        remaining = remaining[keep]
    return np.array(chosen, dtype=np.int64)


def leverage_scores(B):
    """Squared row norms of the orthonormal factor of B (n x k): thin QR of B
    (Section 5.3, leverage scores of span(B)).  They sum to rank(B)."""
    Qb, _ = np.linalg.qr(np.asarray(B, dtype=np.float64), mode="reduced")
    return np.sum(Qb * Qb, axis=1)


def leverage_sample(scores, u):
    """Leverage-score sampling with weights (Section 5.3 and its footnote).

    One row per uniform draw u_k in [0, 1), with replacement: row i is drawn
    with probability pi_i = scores_i / sum(scores), by taking the first i whose
    running sum scores_0 + ... + scores_i exceeds u_k * sum(scores) (a draw at
    or beyond the total, possible only through rounding, takes the last row
    with a positive score).  Weight w_k = 1 / sqrt(s pi_i), so that
    E |W S v|^2 = |v|^2 for every v.  Returns (rows int64, weights).
    """
    sc = np.asarray(scores, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    s = u.size
    run = np.cumsum(sc)
    total = run[-1]
    rows = np.searchsorted(run, u * total, side="right")
    last = int(np.flatnonzero(sc > 0.0)[-1])
    rows = np.where(rows >= sc.size, last, rows)
    pi = sc[rows] / total
    return rows.astype(np.int64), 1.0 / np.sqrt(s * pi)


SPAN_RTOL = 1e-8


def leverage_matrix(family, Q, select_param):
    """B = [A(p_sel) Q, b(p_sel)] (n x (r+1)), whose span is sampled."""
    AQ = np.asarray(family.matvec(select_param, Q))
    return np.column_stack([AQ, family.rhs(select_param)])


def span_scores(B, rtol=SPAN_RTOL):
    """Leverage scores of span([A(p_sel) Q, b]) for B = that n x (r+1) matrix.

    When b lies in span(A(p_sel) Q) up to |R[r, r]| <= rtol |b| (R of the
    Householder QR of B), the last direction is rounding noise and the span
    is r-dimensional: the scores come from the first r columns only."""
    B = np.asarray(B, dtype=np.float64)
    r = B.shape[1] - 1
    Qb, Rb = np.linalg.qr(B, mode="reduced")
    k = r if abs(Rb[r, r]) <= rtol * np.linalg.norm(B[:, r]) else r + 1
    return np.sum(Qb[:, :k] * Qb[:, :k], axis=1)


def residual_bounds(rho, r, s, eps=None):
    """Bounds on the full relative residual from the weighted sketched one
    (Section 5.3.1): with probability close to 1 at p_sel,
    (1 - eps) |Bc - b| <= |W S (Bc - b)| <= (1 + eps) |Bc - b|, so the full
    value lies in [rho / (1 + eps), rho / (1 - eps)].  eps defaults to the
    paper's k log k / s with k = r + 1, the dimension of span([B, b])."""
    if eps is None:
        k = r + 1
        eps = k * np.log(k) / s
    hi = rho / (1.0 - eps) if eps < 1.0 else np.inf
    return rho / (1.0 + eps), hi


def lupp_pivots(W, k, tie_rtol=TIE_RTOL):
    """First k pivot rows of Gaussian elimination with partial pivoting on the
    n x r matrix W (Section 5.3, LUPP on A(p_i) X).

    At step j the pivot is the smallest row index, among rows not pivoted yet,
    whose |W[i, j]| is >= (1 - tie_rtol) * max; every other row not pivoted
    yet then loses the multiple W[i, j] / W[piv, j] of the pivot row."""
    W = np.array(W, dtype=np.float64, copy=True)
    n, r = W.shape
    k = min(k, n, r)
    free = np.ones(n, dtype=bool)
    piv = []
    for j in range(k):
        mag = np.abs(W[:, j])
        mag[~free] = -1.0
        top = mag.max()
        i = int(np.flatnonzero(mag >= (1.0 - tie_rtol) * top)[0])
        piv.append(i)
        free[i] = False
        if W[i, j] != 0.0:
            f = W[free, j] / W[i, j]
            W[np.ix_(free, np.arange(j + 1, r))] -= np.outer(f, W[i, j + 1:])
    return np.array(piv, dtype=np.int64)


def select_rows_lu(W, s, tie_rtol=TIE_RTOL):
    """s row indices of W = A(p_sel) X by rounds of LUPP: each round runs a
    fresh elimination on the rows not chosen yet and takes min(r, s - chosen)
    pivots (s = r is one LUPP)."""
    W = np.asarray(W, dtype=np.float64)
    n, r = W.shape
    if not (r <= s <= n):
        raise ValueError("need r <= s <= n")
    chosen = []
    remaining = np.arange(n)
    while len(chosen) < s:
        take = min(r, s - len(chosen))
        piv = lupp_pivots(W[remaining], take, tie_rtol)
        new = remaining[piv]
        chosen.extend(int(v) for v in new)
        keep = np.ones(remaining.size, dtype=bool)
        keep[piv] = False
        remaining = remaining[keep]
    return np.array(chosen, dtype=np.int64)


def union_rows(row_sets):
    """Union of several row selections in order of first appearance
    (Section 5.3.2: r pivots at each of t points, collected)."""
    out, seen = [], set()
    for rows in row_sets:
        for v in rows:
            if int(v) not in seen:
                seen.add(int(v))
                out.append(int(v))
    return np.array(out, dtype=np.int64)


def selection_matrix(family, Q, select_param):
    """M = (A(p_sel) Q)^T, the r x n matrix whose columns are pivoted."""
    return np.asarray(family.matvec(select_param, Q)).T


def offline(workload: dict, basis=None, rows=None, sample_u=None, selection="cpqr", select_params=None):
    """Algorithm 3.1 steps 1-3 for a ``subap_inputs`` workload.

    ``basis``: optional n x r matrix used instead of the snapshot solves (it
    is still orthonormalised).  ``rows``: optional row indices used instead of
    the pivoted-QR selection.  ``sample_u``: s uniforms in [0, 1); when given,
    rows come from leverage-score sampling of [A(p_sel) Q, b(p_sel)] and carry
    weights.  ``selection``: "cpqr" (pivoted QR on (A(p_sel) Q)^T) or "lu"
    (LUPP on A(p_sel) Q).  ``select_params``: several points (t x d); the rows
    are then the union of r pivots at each (Section 5.3.2), and s is their
    count.  Returns dict(family, X (raw snapshots or None), Q, R, rows,
    weights (None for unweighted rows)).
    """
    family = fam.from_workload(workload)
    if basis is None:
        X = snapshots(family, workload["snap_params"])
    else:
        X = np.asarray(basis, dtype=np.float64)
    Q, R = orthonormalise(X)
    weights = None
    if sample_u is not None:
        B = leverage_matrix(family, Q, workload["select_param"])
        rows, weights = leverage_sample(span_scores(B), sample_u)
    elif rows is None:
        def pick(p, k):
            M = selection_matrix(family, Q, p)
            return select_rows_lu(M.T, k) if selection == "lu" else select_rows(M, k)
        if select_params is not None:
            rows = union_rows([pick(p, Q.shape[1]) for p in np.atleast_2d(select_params)])
        else:
            rows = pick(workload["select_param"], workload["s"])
    return dict(family=family, X=X, Q=Q, R=R, rows=np.asarray(rows, dtype=np.int64), weights=weights)
