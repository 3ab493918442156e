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


def selection_matrix(family, Q, select_param):
    """M = (A(p_sel) Q)^T, the r x n matrix whose columns are pivoted."""
    return np.asarray(family.matvec(select_param, Q)).T


def offline(workload: dict, basis=None, rows=None):
    """Algorithm 3.1 steps 1-3 for a ``subap_inputs`` workload.

    ``basis``: optional n x r matrix used instead of the snapshot solves (it
    is still orthonormalised).  ``rows``: optional row indices used instead of
    the pivoted-QR selection.  Returns dict(family, X (raw snapshots or None),
    Q, R, rows).
    """
    family = fam.from_workload(workload)
    if basis is None:
        X = snapshots(family, workload["snap_params"])
    else:
        X = np.asarray(basis, dtype=np.float64)
    Q, R = orthonormalise(X)
    if rows is None:
        M = selection_matrix(family, Q, workload["select_param"])
        rows = select_rows(M, workload["s"])
    return dict(family=family, X=X, Q=Q, R=R, rows=np.asarray(rows, dtype=np.int64))
