"""Online phase of SubApSnap (Algorithm 3.1, step 4), FP64 CPU oracle.

Test infrastructure only (see the package docstring).

For each new parameter p*:

1. generate the selected rows S A(p*) and entries S b(p*) (Section 3.1:
   only s rows of A and s entries of b are needed);
2. form the s x r matrix S A(p*) X (eq. (3.4));
3. solve min_c |S A(p*) X c - S b(p*)| (eq. (3.3)) by Householder QR
   (numpy.linalg.qr, LAPACK dgeqrf) and back substitution;
4. lift x = X c.

Also: ApSnap, the full-sampling problem of eq. (3.1); the paper's relative
residual |A(p) x - b(p)| / |b(p)|; the sketched residual
|S(A(p) X y - b)| / |S b|; and delta_res(p) = |A(p) X (y1 - y2)| / |b(p)|,
the residual-norm distance between two coefficient vectors that the GPU
parity tests use.

With leverage-score rows (Section 5.3) every function takes the row weights:
row k of S A(p) X and entry k of S b are multiplied by weights[k], and the
sketched residual is |W S(A(p) X y - b)| / |b| (the weighted sketch estimates
the full residual norm, Section 5.3.1; b is the same for every p here, so its
full norm is known).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def _w(weights, v):
    return v if weights is None else np.asarray(weights, dtype=np.float64).reshape((-1,) + (1,) * (v.ndim - 1)) * v


def reduced_matrix(family, Q, rows, p, weights=None):
    """S A(p) Q (s x r): the selected rows of A(p), times Q (eq. (3.4));
    row k scaled by weights[k] when given."""
    A_S = family.rows(p, rows)
    return _w(weights, np.asarray(A_S @ Q))


def householder_lsq(G, b):
    """argmin_y |G y - b| by thin Householder QR; returns (y, R, rho).

    rho = |G y - b| is the least-squares residual norm.
    """
    Qg, Rg = np.linalg.qr(G, mode="reduced")
    y = sla.solve_triangular(Rg, Qg.T @ b, lower=False)
    rho = float(np.linalg.norm(G @ y - b))
    return y, Rg, rho


def solve_one(family, Q, rows, p, weights=None):
    """SubApSnap coefficients y(p) for one parameter (eq. (3.3))."""
    G = reduced_matrix(family, Q, rows, p, weights)
    bS = _w(weights, np.asarray(family.rhs_rows(p, rows), dtype=np.float64))
    y, _, _ = householder_lsq(G, bS)
    return y


def solve(family, Q, rows, params, weights=None):
    """y for every parameter row of ``params`` (m x d) -> (m x r)."""
    P = np.atleast_2d(np.asarray(params, dtype=np.float64))
    return np.stack([solve_one(family, Q, rows, p, weights) for p in P])


def lift(Q, y):
    """x = Q y (n,) or Q Y^T for a batch y (m x r) -> (n x m)."""
    y = np.asarray(y, dtype=np.float64)
    return Q @ (y if y.ndim == 1 else y.T)


def apsnap_solve(family, Q, p):
    """ApSnap (eq. (3.1)): argmin_c |A(p) Q c - b(p)| over all n rows."""
    B = np.asarray(family.matvec(p, Q))
    c, *_ = np.linalg.lstsq(B, family.rhs(p), rcond=None)
    return c


def output(c, Q, y):
    """c^T x for x = Q y (Section 6.2.2: H(p*) ~ (c^T X) c_hat); y (r,) or (m, r)."""
    return (np.asarray(c, dtype=np.float64) @ np.asarray(Q)) @ np.asarray(y, dtype=np.float64).T


def cg_polish(family, p, x0, iters, jacobi=True):
    """Polishing from x0 by conjugate gradients on A(p) x = b (Section 3.1
    mentions polishing the SubApSnap solution; every family here is
    symmetric positive definite, so CG is the Krylov method).  ``jacobi``:
    precondition with 1 / diag(A(p)).  Exactly ``iters`` iterations (a step
    with p^T A p = 0 or r^T z = 0 leaves the iterate unchanged).  Returns
    (x, |r| / |b|) with r the recursively updated residual."""
    A = family.matrix(p)
    b = np.asarray(family.rhs(p), dtype=np.float64)
    dinv = 1.0 / np.asarray(A.diagonal()) if jacobi else np.ones(b.size)
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x
    z = dinv * r
    d = z.copy()
    rz = r @ z
    for _ in range(iters):
        q = A @ d
        dq = d @ q
        alpha = 0.0 if dq == 0.0 else rz / dq
        x = x + alpha * d
        r = r - alpha * q
        z = dinv * r
        rz_new = r @ z
        beta = 0.0 if rz == 0.0 else rz_new / rz
        rz = rz_new
        d = z + beta * d
    return x, float(np.linalg.norm(r) / np.linalg.norm(b))


def residual(family, x, p):
    """|A(p) x - b(p)|_2 / |b(p)|_2 (the measure of Tables 3-4)."""
    b = family.rhs(p)
    return float(np.linalg.norm(family.matvec(p, x) - b) / np.linalg.norm(b))


def delta_res(family, Q, p, y1, y2):
    """|A(p) Q (y1 - y2)|_2 / |b(p)|_2."""
    dy = np.asarray(y1, dtype=np.float64) - np.asarray(y2, dtype=np.float64)
    b = family.rhs(p)
    return float(np.linalg.norm(family.matvec(p, Q @ dy)) / np.linalg.norm(b))


def delta_res_params(family, Q, params, Y1, Y2):
    """delta_res for every row of params (m x d) against coefficient rows of
    Y1, Y2 (m x r).  Families with ``matvec_params`` evaluate all parameters
    in one pass over A's rows; the others call ``delta_res`` per parameter."""
    P = np.atleast_2d(np.asarray(params, dtype=np.float64))
    dY = np.asarray(Y1, dtype=np.float64) - np.asarray(Y2, dtype=np.float64)
    if not hasattr(family, "matvec_params"):
        return np.array([delta_res(family, Q, p, a, b) for p, a, b in zip(P, Y1, Y2)])
    V = family.matvec_params(P, Q @ dY.T)
    return np.array([np.linalg.norm(V[:, i]) / np.linalg.norm(family.rhs(p)) for i, p in enumerate(P)])


def sketched_residual(family, Q, rows, p, y, weights=None):
    """|S(A(p) Q y - b(p))|_2 / |S b(p)|_2, from the s selected rows only.
    With weights: |W S(A(p) Q y - b(p))|_2 / |b(p)|_2."""
    A_S = family.rows(p, rows)
    bS = np.asarray(family.rhs_rows(p, rows), dtype=np.float64)
    res = _w(weights, A_S @ (Q @ np.asarray(y)) - bS)
    den = np.linalg.norm(bS) if weights is None else np.linalg.norm(family.rhs(p))
    return float(np.linalg.norm(res) / den)
