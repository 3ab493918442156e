"""Parameter-dependent linear systems A(p) x(p) = b(p) (eq. (1.1)), FP64.

Each family exposes:

* ``n``, ``d``                 size and parameter dimension;
* ``matrix(p)``                the full A(p) (scipy.sparse CSR or dense) --
                               only for sizes where that is cheap;
* ``matvec(p, x)``             A(p) @ x without assembling A (any size);
* ``rows(p, idx)``             the rows idx of A(p) as a sparse CSR (len(idx) x n)
                               or dense array, generated directly from the
                               definition: SubApSnap only needs these rows
                               (Section 3.1, "Computing S A(p*) X");
* ``rhs(p)`` / ``rhs_rows(p, idx)``  b(p) and its entries idx.

Finite-difference diffusion (reading of the PDE examples of Section 6.1)
------------------------------------------------------------------------
-div(a grad u) = f on (0,1)^D, u = 0 on the boundary.  Interior nodes at
x = (i + 1) h, i = 0..N-1, h = 1/(N+1); lexicographic index
idx = ix + N iy (+ N^2 iz), x fastest.  Row idx of A(p): for each of the 2D
faces between the node and its axis neighbours, the coefficient a evaluated
at the face midpoint, a_f; diagonal sum_f a_f / h^2, off-diagonal -a_f / h^2
for neighbours inside the domain (boundary neighbours carry u = 0 and drop
out).  a(x; p) = exp(sum_k p_k phi_k(x)).

Kernel ridge regression (Section 6.3, eqs. (6.3)-(6.4))
-------------------------------------------------------
A(p) = K_p + lambda I, K_p[i, j] = exp(-|t_i - t_j|^2 / (2 p^2)); the
parameter p is the kernel length scale; b is the target vector.

Shifted tridiagonal (eq. (5.7))
-------------------------------
A(p) = A0 - p I with A0 = tridiag(-1, 2, -1); b(p) = exp(b0 sin(p/10) p)
componentwise.

Delay system (Section 6.2.2), real parameter
--------------------------------------------
A(p) = p I - A_0 - e^{tau p} A_1 with A_1 = (T - kappa I) / tau, A_0 = 3 A_1,
T the n x n matrix with ones on the first off-diagonals and at the two ends
of the diagonal (T[0,0] = T[n-1,n-1] = 1); b is fixed and the output of
interest is H(p) = c^T x(p).  The paper evaluates the transfer function; here
p is real, which keeps A(p) symmetric positive definite for p > -3 (kappa - 2)
/ tau.

Affine (Section 3.1, "Computing S A(p*) X")
-------------------------------------------
A(theta) = sum_q theta_q A_q with given sparse terms A_q and a fixed b; the
parameter is the coefficient vector theta itself (any theta_q(p) of a
physical parameter p is evaluated by the caller).  The delay system is the
two-term case A_q = (I, A_1), theta = (p, -(3 + e^{tau p})).

Identity (DEIM special case, eq. (3.5))
---------------------------------------
A(p) = I; b(p) = y(p) with y_i(p) = 1 / (1 + 25 (t_i - p)^2) on t_i = i/(n-1),
a smooth family whose snapshots have rapidly decaying singular values.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

TWO_PI = 2.0 * np.pi


# --------------------------------------------------------------------------
# coefficient modes phi_k for the diffusion families
# --------------------------------------------------------------------------
def modes_2d(x, y):
    """phi_1 = sin(2 pi x), phi_2 = cos(2 pi y)."""
    return np.stack([np.sin(TWO_PI * x), np.cos(TWO_PI * y)], axis=-1)


def modes_3d(x, y, z):
    """Four sin/cos product modes on the unit cube.

    phi_1 = sin(2 pi x) cos(2 pi y), phi_2 = sin(2 pi y) cos(2 pi z),
    phi_3 = sin(2 pi z) cos(2 pi x), phi_4 = cos(2 pi x) cos(2 pi y) cos(2 pi z).
    """
    sx, cx = np.sin(TWO_PI * x), np.cos(TWO_PI * x)
    sy, cy = np.sin(TWO_PI * y), np.cos(TWO_PI * y)
    sz, cz = np.sin(TWO_PI * z), np.cos(TWO_PI * z)
    return np.stack([sx * cy, sy * cz, sz * cx, cx * cy * cz], axis=-1)


class Diffusion:
    """Finite-difference -div(a grad u) = f with a = exp(sum_k p_k phi_k)."""

    def __init__(self, grid, rhs=None):
        self.grid = tuple(int(g) for g in grid)
        self.dim = len(self.grid)
        if self.dim not in (2, 3) or len(set(self.grid)) != 1:
            raise ValueError("grid must be N x N or N x N x N")
        self.N = self.grid[0]
        self.n = self.N ** self.dim
        self.h = 1.0 / (self.N + 1)
        self.d = 2 if self.dim == 2 else 4
        self._rhs = None if rhs is None else np.asarray(rhs, dtype=np.float64)

    # geometry ------------------------------------------------------------
    def coords(self, idx):
        """Integer grid coordinates (ix, iy[, iz]) of lexicographic indices."""
        idx = np.asarray(idx, dtype=np.int64)
        N = self.N
        out = [idx % N, (idx // N) % N]
        if self.dim == 3:
            out.append(idx // (N * N))
        return out

    def coefficient(self, pts, p):
        """a(x; p) at points pts[..., dim] (physical coordinates)."""
        p = np.asarray(p, dtype=np.float64)
        if self.dim == 2:
            phi = modes_2d(pts[..., 0], pts[..., 1])
        else:
            phi = modes_3d(pts[..., 0], pts[..., 1], pts[..., 2])
        return np.exp(phi @ p)

    # rows ------------------------------------------------------------------
    def rows(self, p, idx):
        """Rows idx of A(p), built node by node from the definition (CSR)."""
        idx = np.asarray(idx, dtype=np.int64)
        h, N, D = self.h, self.N, self.dim
        data, cols, indptr = [], [], [0]
        for i in idx:
            c = [int(v[0]) for v in self.coords([i])]
            x = np.array([(ci + 1) * h for ci in c])
            diag = 0.0
            entries = {}
            for axis in range(D):
                for sgn in (-1, +1):
                    face = x.copy()
                    face[axis] += sgn * 0.5 * h
                    a_f = float(self.coefficient(face, p))
                    diag += a_f / h ** 2
                    nb = list(c)
                    nb[axis] += sgn
                    if 0 <= nb[axis] < N:
                        j = nb[0] + N * nb[1] + (N * N * nb[2] if D == 3 else 0)
                        entries[j] = entries.get(j, 0.0) - a_f / h ** 2
            entries[int(i)] = entries.get(int(i), 0.0) + diag
            for j in sorted(entries):
                cols.append(j)
                data.append(entries[j])
            indptr.append(len(cols))
        return sp.csr_matrix((data, cols, indptr), shape=(len(idx), self.n))

    # full operator ------------------------------------------------------------
    def _face_coeffs(self, p):
        """For each axis, a at the faces between node i and its +axis
        neighbour: array of shape grid with an extra leading face at the low
        boundary, i.e. (N+1) faces along that axis."""
        h, N, D = self.h, self.N, self.dim
        centres = (np.arange(N) + 1) * h
        faces = (np.arange(N + 1) + 0.5) * h
        out = []
        for axis in range(D):
            axes = [centres] * D
            axes[axis] = faces
            mesh = np.meshgrid(*axes, indexing="ij")  # mesh[k][i0, i1, ...] coordinate k
            pts = np.stack(mesh, axis=-1)
            out.append(self.coefficient(pts, p))      # indexed [ix, iy(, iz)]
        return out

    def matrix(self, p):
        """Full sparse A(p) (CSR), assembled from face coefficients."""
        h, N, D = self.h, self.N, self.dim
        fc = self._face_coeffs(p)
        shape = (N,) * D
        diag = np.zeros(shape)
        rows, cols, vals = [], [], []
        lin = np.arange(self.n).reshape(shape[::-1]).transpose()  # lin[ix, iy, iz]
        for axis in range(D):
            a = fc[axis] / h ** 2
            lo = np.take(a, np.arange(N), axis=axis)       # face below node
            hi = np.take(a, np.arange(1, N + 1), axis=axis)  # face above node
            diag += lo + hi
            # coupling between node k and k+1 along axis uses face k+1 (interior faces)
            src = np.take(lin, np.arange(N - 1), axis=axis).ravel()
            dst = np.take(lin, np.arange(1, N), axis=axis).ravel()
            w = np.take(a, np.arange(1, N), axis=axis).ravel()
            rows += [src, dst]
            cols += [dst, src]
            vals += [-w, -w]
        rows.append(lin.ravel())
        cols.append(lin.ravel())
        vals.append(diag.ravel())
        A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(self.n, self.n))
        return A.tocsr()

    def matvec(self, p, x):
        """A(p) @ x for x of shape (n,) or (n, k), without assembling A."""
        h, N, D = self.h, self.N, self.dim
        x = np.asarray(x, dtype=np.float64)
        vec = x.ndim == 1
        k = 1 if vec else x.shape[1]
        # grid view u[ix, iy, (iz,) col]: index = ix + N iy + N^2 iz (x fastest)
        u = x.reshape((-1, k)).reshape(((N,) * D)[::-1] + (k,))
        u = np.moveaxis(u, list(range(D)), list(range(D))[::-1])  # -> [ix, iy, iz, col]
        y = np.zeros_like(u)
        fc = self._face_coeffs(p)
        for axis in range(D):
            a = (fc[axis] / h ** 2)[..., None]
            pad = [(0, 0)] * (D + 1)
            pad[axis] = (1, 1)
            up = np.pad(u, pad)  # Dirichlet zeros
            lo_nb = np.take(up, np.arange(0, N), axis=axis)
            hi_nb = np.take(up, np.arange(2, N + 2), axis=axis)
            a_lo = np.take(a, np.arange(N), axis=axis)
            a_hi = np.take(a, np.arange(1, N + 1), axis=axis)
            y += a_lo * (u - lo_nb) + a_hi * (u - hi_nb)
        y = np.moveaxis(y, list(range(D))[::-1], list(range(D)))
        y = y.reshape((-1, k))
        return y[:, 0] if vec else y

    # right-hand side ------------------------------------------------------------
    def rhs(self, p=None):
        return np.ones(self.n) if self._rhs is None else self._rhs.copy()

    def rhs_rows(self, p, idx):
        return self.rhs(p)[np.asarray(idx, dtype=np.int64)]


class KernelRidge:
    """A(p) = K_p + lambda I with the Gaussian kernel of eq. (6.4)."""

    def __init__(self, points, rhs, lam):
        self.points = np.asarray(points, dtype=np.float64)
        self.n, self.dim = self.points.shape
        self.d = 1
        self.lam = float(lam)
        self._rhs = np.asarray(rhs, dtype=np.float64)

    def sqdist_rows(self, idx):
        """|t_i - t_j|^2 for i in idx, all j, by explicit differences."""
        idx = np.asarray(idx, dtype=np.int64)
        out = np.empty((len(idx), self.n))
        for k, i in enumerate(idx):
            diff = self.points - self.points[i]
            out[k] = np.sum(diff * diff, axis=1)
        return out

    def rows(self, p, idx):
        idx = np.asarray(idx, dtype=np.int64)
        sigma = float(np.asarray(p).reshape(-1)[0])
        K = np.exp(-self.sqdist_rows(idx) / (2.0 * sigma * sigma))
        K[np.arange(len(idx)), idx] += self.lam
        return K

    def matrix(self, p):
        return self.rows(p, np.arange(self.n))

    def matvec(self, p, x, chunk=1024):
        x = np.asarray(x, dtype=np.float64)
        out = np.empty((self.n,) + x.shape[1:])
        for a in range(0, self.n, chunk):
            idx = np.arange(a, min(a + chunk, self.n))
            out[idx] = self.rows(p, idx) @ x
        return out

    def matvec_params(self, params, X, chunk=1024):
        """Column i of the result is A(params[i]) @ X[:, i]: the same sums as
        ``matvec`` one parameter at a time, with each block of squared
        distances computed once for all parameters."""
        P = np.atleast_2d(np.asarray(params, dtype=np.float64))
        X = np.asarray(X, dtype=np.float64)
        out = np.empty((self.n, P.shape[0]))
        for a in range(0, self.n, chunk):
            idx = np.arange(a, min(a + chunk, self.n))
            D = self.sqdist_rows(idx)
            for i, p in enumerate(P):
                sigma = float(p[0])
                K = np.exp(-D / (2.0 * sigma * sigma))
                K[np.arange(len(idx)), idx] += self.lam
                out[idx, i] = K @ X[:, i]
        return out

    def rhs(self, p=None):
        return self._rhs.copy()

    def rhs_rows(self, p, idx):
        return self._rhs[np.asarray(idx, dtype=np.int64)]


class ShiftedTridiag:
    """A(p) = A0 - p I, b(p) = exp(b0 sin(p/10) p) (eq. (5.7))."""

    def __init__(self, b0):
        self.b0 = np.asarray(b0, dtype=np.float64)
        self.n = self.b0.size
        self.d = 1

    def matrix(self, p):
        pv = float(np.asarray(p).reshape(-1)[0])
        n = self.n
        return sp.diags([-np.ones(n - 1), (2.0 - pv) * np.ones(n), -np.ones(n - 1)],
                        [-1, 0, 1], format="csr")

    def rows(self, p, idx):
        return self.matrix(p)[np.asarray(idx, dtype=np.int64)]

    def matvec(self, p, x):
        return self.matrix(p) @ x

    def rhs(self, p):
        pv = float(np.asarray(p).reshape(-1)[0])
        return np.exp(self.b0 * np.sin(pv / 10.0) * pv)

    def rhs_rows(self, p, idx):
        return self.rhs(p)[np.asarray(idx, dtype=np.int64)]


class Identity:
    """A(p) = I, b(p) = y(p) (DEIM as SubApSnap without A, eq. (3.5))."""

    def __init__(self, n):
        self.n = int(n)
        self.d = 1
        self.t = np.linspace(0.0, 1.0, self.n)

    def matrix(self, p):
        return sp.identity(self.n, format="csr")

    def rows(self, p, idx):
        return self.matrix(p)[np.asarray(idx, dtype=np.int64)]

    def matvec(self, p, x):
        return np.array(x, dtype=np.float64, copy=True)

    def rhs(self, p):
        pv = float(np.asarray(p).reshape(-1)[0])
        return 1.0 / (1.0 + 25.0 * (self.t - pv) ** 2)

    def rhs_rows(self, p, idx):
        return self.rhs(p)[np.asarray(idx, dtype=np.int64)]


class Delay:
    """A(p) = p I - A_0 - e^{tau p} A_1, A_1 = (T - kappa I)/tau, A_0 = 3 A_1 (Section 6.2.2)."""

    def __init__(self, n, tau, kappa, rhs, c_out=None):
        self.n = int(n)
        self.d = 1
        self.tau = float(tau)
        self.kappa = float(kappa)
        self._rhs = np.asarray(rhs, dtype=np.float64)
        self.c_out = None if c_out is None else np.asarray(c_out, dtype=np.float64)

    def T(self):
        n = self.n
        off = np.ones(n - 1)
        main = np.zeros(n)
        main[0] = main[-1] = 1.0
        return sp.diags([off, main, off], [-1, 0, 1], format="csr")

    def A1(self):
        return (self.T() - self.kappa * sp.identity(self.n, format="csr")) / self.tau

    def matrix(self, p):
        pv = float(np.asarray(p).reshape(-1)[0])
        A1 = self.A1()
        A0 = 3.0 * A1
        return (pv * sp.identity(self.n, format="csr") - A0 - np.exp(self.tau * pv) * A1).tocsr()

    def rows(self, p, idx):
        return self.matrix(p)[np.asarray(idx, dtype=np.int64)]

    def matvec(self, p, x):
        return self.matrix(p) @ x

    def rhs(self, p=None):
        return self._rhs.copy()

    def rhs_rows(self, p, idx):
        return self._rhs[np.asarray(idx, dtype=np.int64)]


class Affine:
    """A(theta) = sum_q theta_q A_q, terms given as sparse matrices, b fixed."""

    def __init__(self, terms, rhs):
        self.terms = [sp.csr_matrix(T, dtype=np.float64) for T in terms]
        self.n = self.terms[0].shape[0]
        self.d = len(self.terms)
        self._rhs = np.asarray(rhs, dtype=np.float64)

    def matrix(self, theta):
        th = np.asarray(theta, dtype=np.float64).reshape(-1)
        A = th[0] * self.terms[0]
        for t, T in zip(th[1:], self.terms[1:]):
            A = A + t * T
        return sp.csr_matrix(A)

    def rows(self, theta, idx):
        return self.matrix(theta)[np.asarray(idx, dtype=np.int64)]

    def matvec(self, theta, x):
        th = np.asarray(theta, dtype=np.float64).reshape(-1)
        y = th[0] * (self.terms[0] @ x)
        for t, T in zip(th[1:], self.terms[1:]):
            y = y + t * (T @ x)
        return y

    def rhs(self, theta=None):
        return self._rhs.copy()

    def rhs_rows(self, theta, idx):
        return self._rhs[np.asarray(idx, dtype=np.int64)]


def from_workload(w: dict):
    """Build the family object described by a ``subap_inputs`` workload dict."""
    fam = w["family"]
    if fam in ("diff2d", "diff3d"):
        return Diffusion(w["grid"], rhs=w.get("rhs"))
    if fam == "krr":
        return KernelRidge(w["points"], w["rhs"], w["lam"])
    if fam == "tridiag":
        return ShiftedTridiag(w["b0"])
    if fam == "identity":
        return Identity(w["n"])
    if fam == "delay":
        return Delay(w["n"], w["tau"], w["kappa"], w["rhs"], w.get("c_out"))
    if fam == "affine":
        return Affine(w["terms"], w["rhs"])
    raise ValueError(f"unknown family {fam!r}")
