"""Pins for oracle.families: each row generator is checked against an
independent construction (Kronecker sums, a manufactured solution with the
analytic operator, scikit-learn's RBF kernel), not against itself."""
import numpy as np
import pytest
import scipy.sparse as sp

import subap_inputs as si
from oracle import families as F


def lap1d(N, h):
    return sp.diags([-np.ones(N - 1), 2 * np.ones(N), -np.ones(N - 1)], [-1, 0, 1]) / h ** 2


def op1d(face_vals, h):
    """1-D -(a u')' with face coefficients a_{i-1/2}, i = 0..N (N+1 values)."""
    lo, hi = face_vals[:-1], face_vals[1:]
    return sp.diags([-face_vals[1:-1], lo + hi, -face_vals[1:-1]], [-1, 0, 1]) / h ** 2


@pytest.mark.parametrize("N", [5, 8])
def test_diffusion2d_at_zero_is_five_point_laplacian(N):
    fam = F.Diffusion((N, N))
    L = lap1d(N, fam.h)
    I = sp.identity(N)
    ref = sp.kron(I, L) + sp.kron(L, I)
    assert abs(fam.matrix(np.zeros(2)) - ref).max() < 1e-9 * abs(ref).max()


def test_diffusion3d_at_zero_is_seven_point_laplacian():
    N = 5
    fam = F.Diffusion((N, N, N))
    L = lap1d(N, fam.h)
    I = sp.identity(N)
    ref = sp.kron(I, sp.kron(I, L)) + sp.kron(I, sp.kron(L, I)) + sp.kron(L, sp.kron(I, I))
    assert abs(fam.matrix(np.zeros(4)) - ref).max() < 1e-9 * abs(ref).max()


def test_diffusion2d_separable_coefficient_kron_form():
    # a = exp(p1 sin 2 pi x) exp(p2 cos 2 pi y) = f(x) g(y), so
    # A = diag(g(y_nodes)) (x) Lx[f] + Ly[g] (x) diag(f(x_nodes)) with x fastest.
    N, p = 7, np.array([0.7, -0.4])
    fam = F.Diffusion((N, N))
    h = fam.h
    nodes = (np.arange(N) + 1) * h
    faces = (np.arange(N + 1) + 0.5) * h
    f = lambda x: np.exp(p[0] * np.sin(2 * np.pi * x))
    g = lambda y: np.exp(p[1] * np.cos(2 * np.pi * y))
    ref = sp.kron(sp.diags(g(nodes)), op1d(f(faces), h)) + sp.kron(op1d(g(faces), h), sp.diags(f(nodes)))
    A = fam.matrix(p)
    assert abs(A - ref).max() < 1e-10 * abs(ref).max()


def _analytic_operator_3d(p, x, y, z):
    """-div(a grad u) for u = sin(pi x) sin(pi y) sin(pi z), a = exp(sum p_k phi_k)."""
    tp = 2 * np.pi
    sx, cx, sy, cy, sz, cz = (np.sin(tp * x), np.cos(tp * x), np.sin(tp * y), np.cos(tp * y),
                              np.sin(tp * z), np.cos(tp * z))
    phi = p[0] * sx * cy + p[1] * sy * cz + p[2] * sz * cx + p[3] * cx * cy * cz
    a = np.exp(phi)
    gx = tp * (p[0] * cx * cy - p[2] * sz * sx - p[3] * sx * cy * cz)
    gy = tp * (-p[0] * sx * sy + p[1] * cy * cz - p[3] * cx * sy * cz)
    gz = tp * (-p[1] * sy * sz + p[2] * cz * cx - p[3] * cx * cy * sz)
    pi = np.pi
    u = np.sin(pi * x) * np.sin(pi * y) * np.sin(pi * z)
    ux = pi * np.cos(pi * x) * np.sin(pi * y) * np.sin(pi * z)
    uy = pi * np.sin(pi * x) * np.cos(pi * y) * np.sin(pi * z)
    uz = pi * np.sin(pi * x) * np.sin(pi * y) * np.cos(pi * z)
    lap = -3 * pi ** 2 * u
    return -a * (lap + gx * ux + gy * uy + gz * uz), u


def test_diffusion3d_second_order_consistency():
    p = np.array([0.6, -0.8, 0.5, 0.9])
    errs = []
    for N in (16, 32, 64):
        fam = F.Diffusion((N, N, N))
        c = (np.arange(N) + 1) * fam.h
        X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
        Lu, u = _analytic_operator_3d(p, X, Y, Z)
        # lexicographic ordering with x fastest == Fortran order of [ix, iy, iz]
        Au = fam.matvec(p, u.ravel(order="F"))
        errs.append(np.abs(Au - Lu.ravel(order="F")).max() / np.abs(Lu).max())
    assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0, errs


def test_diffusion2d_second_order_consistency():
    p = np.array([0.9, -0.7])
    errs = []
    for N in (16, 32, 64):
        fam = F.Diffusion((N, N))
        c = (np.arange(N) + 1) * fam.h
        X, Y = np.meshgrid(c, c, indexing="ij")
        tp, pi = 2 * np.pi, np.pi
        a = np.exp(p[0] * np.sin(tp * X) + p[1] * np.cos(tp * Y))
        ax = a * p[0] * tp * np.cos(tp * X)
        ay = -a * p[1] * tp * np.sin(tp * Y)
        u = np.sin(pi * X) * np.sin(pi * Y)
        ux = pi * np.cos(pi * X) * np.sin(pi * Y)
        uy = pi * np.sin(pi * X) * np.cos(pi * Y)
        Lu = -(a * (-2 * pi ** 2 * u) + ax * ux + ay * uy)
        Au = fam.matvec(p, u.ravel(order="F"))
        errs.append(np.abs(Au - Lu.ravel(order="F")).max() / np.abs(Lu).max())
    assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0, errs


@pytest.mark.parametrize("grid", [(6, 6), (4, 4, 4)])
def test_diffusion_rows_matvec_and_matrix_agree(grid):
    fam = F.Diffusion(grid)
    rng = np.random.default_rng(0)
    p = rng.uniform(-1, 1, fam.d)
    A = fam.matrix(p)
    idx = rng.choice(fam.n, size=10, replace=False)
    assert abs(fam.rows(p, idx) - A[idx]).max() < 1e-12 * abs(A).max()
    x = rng.standard_normal((fam.n, 3))
    assert np.abs(fam.matvec(p, x) - A @ x).max() < 1e-12 * np.abs(A @ x).max()


def test_diffusion_symmetric_positive_definite():
    fam = F.Diffusion((6, 6))
    A = fam.matrix(np.array([1.0, -1.0])).toarray()
    assert np.abs(A - A.T).max() == 0.0
    assert np.linalg.eigvalsh(A).min() > 0.0


def test_krr_rows_match_sklearn_rbf():
    from sklearn.metrics.pairwise import rbf_kernel
    w = si.krr(n=300, m=4)
    fam = F.from_workload(w)
    sigma = 0.8
    ref = rbf_kernel(w["points"], gamma=1.0 / (2 * sigma ** 2)) + w["lam"] * np.eye(300)
    idx = np.array([0, 17, 299, 5])
    assert np.abs(fam.rows(np.array([sigma]), idx) - ref[idx]).max() < 1e-13
    assert np.allclose(np.diag(fam.matrix(np.array([sigma]))), 1.0 + w["lam"], rtol=0, atol=1e-15)


def test_krr_kernel_closed_form_two_points():
    pts = np.array([[0.0, 0.0], [3.0, 4.0]])  # distance 5
    fam = F.KernelRidge(pts, np.ones(2), lam=0.5)
    K = fam.matrix(np.array([2.0]))
    assert K[0, 1] == pytest.approx(np.exp(-25.0 / 8.0), rel=1e-15)
    assert K[0, 0] == pytest.approx(1.5, rel=1e-15)


def test_tridiag_family_definition():
    b0 = np.array([0.5, -1.0, 2.0])
    fam = F.ShiftedTridiag(b0)
    A = fam.matrix(np.array([-9.5])).toarray()
    assert np.allclose(A, [[11.5, -1, 0], [-1, 11.5, -1], [0, -1, 11.5]], rtol=0, atol=0)
    p = -9.5
    assert np.allclose(fam.rhs(np.array([p])), [np.exp(v * np.sin(p / 10) * p) for v in b0], rtol=1e-15)


# --- delay system (Section 6.2.2), real parameter

def _delay(n=12):
    return F.Delay(n, 0.1, 2.1, np.random.default_rng(5).standard_normal(n),
                   np.random.default_rng(6).standard_normal(n))


def test_delay_ones_vector_is_an_eigenvector():
    # T 1 = 2 * 1 needs the two corner ones, so A(p) 1 = (p - (3 + e^{tau p}) (2 - kappa) / tau) 1
    fam = _delay(15)
    for p in (0.0, 2.5, 9.0):
        lam = p - (3.0 + np.exp(0.1 * p)) * (2.0 - 2.1) / 0.1
        np.testing.assert_allclose(fam.matvec(p, np.ones(15)), lam * np.ones(15), rtol=1e-13)


def test_delay_spectrum_closed_form():
    # eigenvalues of T are 2 cos(pi k / n), k = 0..n-1, so those of A(p) are
    # p + (3 + e^{tau p}) (kappa - 2 cos(pi k / n)) / tau: all positive for p >= 0
    n = 12
    fam = _delay(n)
    for p in (0.0, 4.0):
        ev = np.linalg.eigvalsh(fam.matrix(p).toarray())
        th = 3.0 + np.exp(0.1 * p)
        want = np.sort(p + th * (2.1 - 2.0 * np.cos(np.pi * np.arange(n) / n)) / 0.1)
        np.testing.assert_allclose(ev, want, rtol=1e-12)
        assert ev.min() > 0.0


def test_delay_rows_are_the_affine_combination():
    # Section 6.2.2: S A(p) X = p S X - S A_0 X - e^{tau p} S A_1 X with A_0 = 3 A_1
    fam = _delay(20)
    X = np.random.default_rng(7).standard_normal((20, 4))
    idx = np.array([0, 3, 19, 7])
    T = np.zeros((20, 20))
    for i in range(19):
        T[i, i + 1] = T[i + 1, i] = 1.0
    T[0, 0] = T[19, 19] = 1.0
    A1X = (T @ X - 2.1 * X) / 0.1
    for p in (0.5, 7.0):
        want = p * X[idx] - (3.0 + np.exp(0.1 * p)) * A1X[idx]
        np.testing.assert_allclose(fam.rows(p, idx) @ X, want, rtol=1e-12, atol=1e-12)


def test_delay_output_with_a_full_basis_is_the_transfer_function():
    # r = n snapshots span R^n, and with S = I SubApSnap is the exact solve,
    # so (c^T Q) y = c^T A(p)^{-1} b
    from oracle import offline as O
    from oracle import online as On
    n = 10
    fam = _delay(n)
    Q, _ = O.orthonormalise(np.random.default_rng(8).standard_normal((n, n)))
    for p in (1.0, 6.0):
        y = On.solve_one(fam, Q, np.arange(n), p)
        H = fam.c_out @ np.linalg.solve(fam.matrix(p).toarray(), fam.rhs(p))
        assert abs(On.output(fam.c_out, Q, y) - H) <= 1e-12 * abs(H)
