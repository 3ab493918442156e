"""GPU parity for the finite-difference families against the FP64 oracle.

Bars: row indices bit-exact; FP64 solves within delta_res <= 1e-12 of the
oracle (delta_res(p) = |A(p) Q (y_gpu - y_oracle)| / |b|), the residual-norm
distance the oracle defines; full-chain runs (GPU snapshots by CG) within
1e-8 because the snapshots themselves differ by the CG tolerance.
"""
import numpy as np
import pytest

import subap_inputs as si
from oracle import offline as O
from oracle import online as On
from paper_2510_04825_amd import binding as B
from tests.gpu_util import device, header, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    w = si.diffusion2d()
    return w, O.offline(w)


def _dres(fam, Q, P, Yg, Yo):
    return np.array([On.delta_res(fam, Q, p, a, b) for p, a, b in zip(P, Yg, Yo)])


def test_c1_rows_from_oracle_basis_are_bit_exact(c1):
    w, off = c1
    header("c1 given-basis rows")
    device()
    M = B.Model(w, basis=off["Q"])
    try:
        assert np.array_equal(M.rows(), off["rows"])
        assert np.abs(M.basis() - off["Q"]).max() < 1e-13
    finally:
        M.free()


def test_c1_fp64_solve_matches_oracle(c1):
    w, off = c1
    fam, Q, rows = off["family"], off["Q"], off["rows"]
    header("c1 fp64 solve given basis and rows")
    M = B.Model(w, basis=Q, rows=rows)
    try:
        P = w["test_params"]
        y, rho, st = M.solve(to_dev(P))
        y = y.cpu().numpy()
        assert np.all(st.cpu().numpy() == B.OK)
        Yo = On.solve(fam, Q, rows, P)
        dres = _dres(fam, Q, P, y, Yo)
        assert dres.max() <= 1e-12, dres.max()
        # rows come in mirror pairs here, so the sketched residual is rounding noise (~1e-12)
        rho_o = [On.sketched_residual(fam, Q, rows, p, yo) for p, yo in zip(P, Yo)]
        assert np.allclose(rho.cpu().numpy(), rho_o, rtol=1e-6, atol=1e-10)
    finally:
        M.free()


def test_c1_full_chain(c1):
    w, off = c1
    fam = off["family"]
    header("c1 full offline on GPU")
    M = B.Model(w)
    try:
        sv = np.linalg.svd(off["X"], compute_uv=False)
        assert sv[-1] / sv[0] > 1e-8
        assert np.array_equal(M.rows(), off["rows"])
        Qg = M.basis()
        assert np.abs(Qg.T @ Qg - np.eye(w["r"])).max() < 1e-13
        # same subspace as the oracle's snapshots
        assert np.linalg.norm(Qg - off["Q"] @ (off["Q"].T @ Qg)) < 1e-8
        P = w["test_params"]
        y, _, st = M.solve(to_dev(P))
        xg = Qg @ y.cpu().numpy().T
        xo = off["Q"] @ On.solve(fam, off["Q"], off["rows"], P).T
        b = fam.rhs()
        for i, p in enumerate(P):
            assert np.linalg.norm(fam.matvec(p, xg[:, i] - xo[:, i])) <= 1e-8 * np.linalg.norm(b)
    finally:
        M.free()


def test_c1_refinement_and_fp32_forms(c1):
    w, off = c1
    fam, Q, rows = off["family"], off["Q"], off["rows"]
    header("c1 fp32 contraction + refinement")
    M = B.Model(w, basis=Q, rows=rows)
    try:
        P = w["test_params"]
        Yo = On.solve(fam, Q, rows, P)
        y1, _, _ = M.solve(to_dev(P), contraction=B.FP64, refine_steps=1)
        assert _dres(fam, Q, P, y1.cpu().numpy(), Yo).max() <= 1e-12
        y32, _, _ = M.solve(to_dev(P), contraction=B.FP32, refine_steps=0)
        d32 = _dres(fam, Q, P, y32.cpu().numpy(), Yo)
        y32r, _, _ = M.solve(to_dev(P), contraction=B.FP32, refine_steps=2)
        d32r = _dres(fam, Q, P, y32r.cpu().numpy(), Yo)
        assert d32r.max() <= 1e-6, (d32.max(), d32r.max())
        assert d32r.max() <= d32.max()
        # corrected semi-normal equations (the column-per-lane solver takes these
        # rows although s < 96): G^T r_S from the FP64 table
        for steps in (1, 2):
            yc, _, stc = M.solve(to_dev(P), contraction=B.FP32, refine_steps=steps, csne=True)
            assert np.all(stc.cpu().numpy() == B.OK)
            dc = _dres(fam, Q, P, yc.cpu().numpy(), Yo)
            print(f"c1 fp32 + {steps} csne steps: delta_res {dc.max():.2e}")
            assert dc.max() <= 1e-6
        yc, _, _ = M.solve(to_dev(P), contraction=B.FP64, refine_steps=1, csne=True)
        assert _dres(fam, Q, P, yc.cpu().numpy(), Yo).max() <= 1e-12
    finally:
        M.free()


def test_c1_edge_cases(c1):
    import torch
    w, off = c1
    header("c1 edge cases")
    M = B.Model(w, basis=off["Q"], rows=off["rows"])
    try:
        dev = device()
        # m = 0 is a no-op
        y, rho, st = M.solve(torch.empty((0, 2), dtype=torch.float64, device=dev))
        assert y.shape == (0, 16)
        # ragged batch, non-finite parameter
        P = np.array(w["test_params"][:13])
        P[5, 1] = np.nan
        y, rho, st = M.solve(to_dev(P))
        st = st.cpu().numpy()
        y = y.cpu().numpy()
        assert st[5] == B.E_NONFINITE and np.all(np.isnan(y[5]))
        ok = np.arange(13) != 5
        assert np.all(st[ok] == B.OK)
        Yo = On.solve(off["family"], off["Q"], off["rows"], P[ok])
        assert _dres(off["family"], off["Q"], P[ok], y[ok], Yo).max() <= 1e-12
        # single parameter equals its batched value
        y1, _, _ = M.solve(to_dev(P[:1]))
        assert np.array_equal(y1.cpu().numpy()[0], y[0])
        # option values outside their range are rejected before any device work
        import ctypes as C
        lib = B.load()
        Pd = to_dev(P[:4])
        yb = torch.empty((4, 16), dtype=torch.float64, device=dev)
        for opts in (B.SolveOpts(0, 1, 2), B.SolveOpts(0, 5, 0), B.SolveOpts(9, 0, 0), B.SolveOpts(0, -1, 1)):
            rc = lib.subap_solve_batch(C.c_void_p(M.handle), C.c_void_p(Pd.data_ptr()), 4,
                                       C.c_void_p(yb.data_ptr()), None, None, C.byref(opts), None)
            assert rc == B.E_INVALID, (opts.contraction, opts.refine_steps, opts.refine_csne)
    finally:
        M.free()


def test_rank_deficient_rows_report_rank_status():
    # basis = unit vectors at nodes two or more cells away from the selected
    # rows, so S A(p) Q = 0 and the least-squares problem has no unique solution
    w = si.diffusion2d(N=16, r=4, s=8, m=6)
    Q = np.zeros((256, 4))
    for c, node in enumerate((150, 170, 200, 230)):
        Q[node, c] = 1.0
    rows = np.arange(8)
    header("rank-deficient S A Q")
    M = B.Model(w, basis=Q, rows=rows)
    try:
        y, _, st = M.solve(to_dev(w["test_params"]))
        assert np.all(st.cpu().numpy() == B.E_RANK)
        assert np.all(np.isnan(y.cpu().numpy()))
    finally:
        M.free()


@pytest.mark.parametrize("dim,N,r,s,m", [(2, 32, 16, 100, 37), (2, 40, 32, 131, 21), (3, 16, 40, 96, 9),
                                         (3, 20, 40, 191, 15), (2, 32, 31, 97, 6), (3, 20, 47, 256, 13),
                                         (3, 16, 24, 120, 11)])
def test_fd_tall_fp64_shapes(dim, N, r, s, m):
    """FP64 solves of tall problems (s >= 96: the matrix-core semi-normal
    solve for 16 <= r <= 47) with ragged row groups, an odd batch and a
    non-finite parameter; y within delta_res 1e-12 of the oracle and rho equal
    to the oracle's sketched residual.  r = 31 puts S b in the last column of
    the second 16-column tile; r = 47, s = 256 in 3-D takes the largest
    factors (three 16-column tiles full) and four full 64-row chunks; r = 24
    in 3-D is the two-tile build with six faces."""
    w = si.diffusion2d(N=N, r=r, s=s, m=m) if dim == 2 else si.diffusion3d(N=N, r=r, s=s, m=m)
    off = O.offline(w)
    fam, Q, rows = off["family"], off["Q"], off["rows"]
    header(f"tall fp64 dim={dim} N={N} r={r} s={s} m={m}")
    M = B.Model(w, basis=Q, rows=rows)
    try:
        P = np.array(w["test_params"])
        P[3, 0] = np.nan
        y, rho, st = M.solve(to_dev(P))
        st, y, rho = st.cpu().numpy(), y.cpu().numpy(), rho.cpu().numpy()
        assert st[3] == B.E_NONFINITE and np.all(np.isnan(y[3]))
        ok = np.arange(m) != 3
        assert np.all(st[ok] == B.OK)
        Yo = On.solve(fam, Q, rows, P[ok])
        assert _dres(fam, Q, P[ok], y[ok], Yo).max() <= 1e-12
        ro = np.array([On.sketched_residual(fam, Q, rows, p, yo) for p, yo in zip(P[ok], Yo)])
        assert np.allclose(rho[ok], ro, rtol=1e-6, atol=1e-10), np.abs(rho[ok] - ro).max()
    finally:
        M.free()


@pytest.mark.parametrize("dim,N,r,s,m", [(2, 40, 64, 128, 9), (2, 32, 32, 100, 11), (3, 16, 40, 160, 7),
                                         (2, 40, 64, 70, 5)])
def test_fd_column_kernel_forms(dim, N, r, s, m):
    """Column-per-lane kernel in every form: r = 64 (S b carried by every
    lane), FP32 contraction with one and two FP64 refinement steps
    (corrections from R^T R dy = G^T r_S), and a shape the register team
    kernel has no instantiation for (r = 64, s = 70)."""
    w = si.diffusion2d(N=N, r=r, s=s, m=m) if dim == 2 else si.diffusion3d(N=N, r=r, s=s, m=m)
    off = O.offline(w)
    fam, Q, rows = off["family"], off["Q"], off["rows"]
    header(f"column kernel forms dim={dim} N={N} r={r} s={s} m={m}")
    M = B.Model(w, basis=Q, rows=rows)
    try:
        P = w["test_params"]
        Yo = On.solve(fam, Q, rows, P)
        y64, rho64, st = M.solve(to_dev(P))
        assert np.all(st.cpu().numpy() == B.OK)
        assert _dres(fam, Q, P, y64.cpu().numpy(), Yo).max() <= 1e-12
        ro = np.array([On.sketched_residual(fam, Q, rows, p, yo) for p, yo in zip(P, Yo)])
        assert np.allclose(rho64.cpu().numpy(), ro, rtol=1e-6, atol=1e-10)
        y0, _, _ = M.solve(to_dev(P), contraction=B.FP32, refine_steps=0)
        y1, rho1, st1 = M.solve(to_dev(P), contraction=B.FP32, refine_steps=1)
        y2, _, st2 = M.solve(to_dev(P), contraction=B.FP32, refine_steps=2)
        assert np.all(st1.cpu().numpy() == B.OK) and np.all(st2.cpu().numpy() == B.OK)
        d0 = _dres(fam, Q, P, y0.cpu().numpy(), Yo)
        d1 = _dres(fam, Q, P, y1.cpu().numpy(), Yo)
        d2 = _dres(fam, Q, P, y2.cpu().numpy(), Yo)
        print(f"fp32: before {d0.max():.2e}, 1 step {d1.max():.2e}, 2 steps {d2.max():.2e}")
        assert d1.max() <= 1e-6 and d1.max() < d0.max()
        assert d2.max() <= max(d1.max(), 1e-12)
        # rho after refinement is the FP64 sketched residual of the refined y
        rg = np.array([On.sketched_residual(fam, Q, rows, p, yg) for p, yg in zip(P, y1.cpu().numpy())])
        assert np.allclose(rho1.cpu().numpy(), rg, rtol=1e-9, atol=1e-13)
        # corrected semi-normal equations: fixed point at the oracle's solution
        yc, rhoc, stc = M.solve(to_dev(P), contraction=B.FP32, refine_steps=1, csne=True)
        assert np.all(stc.cpu().numpy() == B.OK)
        dc = _dres(fam, Q, P, yc.cpu().numpy(), Yo)
        print(f"fp32 + 1 csne step: {dc.max():.2e}")
        assert dc.max() <= 1e-6
        rg = np.array([On.sketched_residual(fam, Q, rows, p, yg) for p, yg in zip(P, yc.cpu().numpy())])
        assert np.allclose(rhoc.cpu().numpy(), rg, rtol=1e-9, atol=1e-13)
    finally:
        M.free()


def test_rank_deficient_tall_problem():
    # unit-vector basis at nodes 13 or more grid lines away from the 96 selected
    # rows (the first three lines): S A(p) Q = 0
    w = si.diffusion2d(N=32, r=16, s=96, m=5)
    Q = np.zeros((1024, 16))
    for c in range(16):
        Q[512 + 32 * c, c] = 1.0
    header("rank-deficient tall S A Q")
    M = B.Model(w, basis=Q, rows=np.arange(96))
    try:
        y, _, st = M.solve(to_dev(w["test_params"]))
        assert np.all(st.cpu().numpy() == B.E_RANK)
        assert np.all(np.isnan(y.cpu().numpy()))
    finally:
        M.free()


@pytest.mark.parametrize("eps", [1e-8, 1e-4])
def test_fd_tall_ill_conditioned_rows(eps):
    """An orthonormal basis of unit vectors at grid nodes, one column mixing a
    node far from every selected row (weight sqrt(1 - eps^2)) with a selected
    one (weight eps): kappa(S A(p) Q) grows like 1/eps.  At eps = 1e-8 the
    semi-normal equations cannot resolve it and the parameters go to the
    Householder solver; at 1e-4 the corrected semi-normal steps settle it.
    The weak direction of S A Q is strong in A Q, so y itself is fixed only to
    kappa^2 eps and the full-row delta_res of any two stable solvers differs
    at that level; the bars are on what a backward-stable solver fixes to
    about kappa eps: the fitted values |S A Q (y - y_oracle)| / |S b| and the
    sketched residual, each within 10 eps kappa (plus 1e-13)."""
    w = si.diffusion3d(N=20, r=40, s=160, m=13)
    N, n, r, s = 20, w["n"], w["r"], w["s"]
    from oracle import families as Fm
    fam = Fm.from_workload(w)
    far = N // 2 + N * (N // 2) + N * N * (N // 2)
    ijk = np.stack([np.arange(n) % N, (np.arange(n) // N) % N, np.arange(n) // (N * N)], axis=1)
    dist = np.abs(ijk - ijk[far]).sum(axis=1)
    rng = np.random.default_rng(31)
    cand = np.flatnonzero(dist > 2)
    nodes = rng.choice(cand, size=r, replace=False)
    extra = rng.choice(np.setdiff1d(cand, nodes), size=s - r, replace=False)
    rows = np.sort(np.concatenate([nodes, extra]))
    Q = np.zeros((n, r))
    Q[nodes, np.arange(r)] = 1.0
    Q[nodes[7], 7] = eps
    Q[far, 7] = np.sqrt(1.0 - eps * eps)
    header(f"tall ill-conditioned rows eps={eps}")
    M = B.Model(w, basis=Q, rows=rows)
    try:
        P = w["test_params"]
        y, rho, st = M.solve(to_dev(P))
        st, y, rho = st.cpu().numpy(), y.cpu().numpy(), rho.cpu().numpy()
        assert np.all(st == B.OK)
        Yo = On.solve(fam, Q, rows, P)
        worst = 0.0
        for p, yg, yo, rg in zip(P, y, Yo, rho):
            G = On.reduced_matrix(fam, Q, rows, p)
            sv = np.linalg.svd(G, compute_uv=False)
            kappa = sv[0] / sv[-1]
            bS = np.asarray(fam.rhs_rows(p, rows))
            fit = np.linalg.norm(G @ (yg - yo)) / np.linalg.norm(bS)
            ro = np.linalg.norm(G @ yo - bS) / np.linalg.norm(bS)
            bar = 10 * 2.0 ** -52 * kappa + 1e-13
            worst = max(worst, fit / bar)
            assert fit <= bar, (kappa, fit, bar)
            assert abs(rg - ro) <= bar * max(ro, 1.0), (kappa, rg, ro)
        print(f"kappa {kappa:.1e}: worst fitted-value error / bar {worst:.2e}")
    finally:
        M.free()


@pytest.mark.parametrize("N,r,s", [(16, 8, 32), (24, 40, 160)])
def test_diffusion3d_given_basis(N, r, s):
    w = si.diffusion3d(N=N, r=r, s=s, m=50)
    off = O.offline(w)
    fam, Q, rows = off["family"], off["Q"], off["rows"]
    header(f"3-D N={N} r={r} s={s}")
    M = B.Model(w, basis=Q)
    try:
        assert np.array_equal(M.rows(), rows)
        P = w["test_params"]
        y, _, st = M.solve(to_dev(P))
        assert np.all(st.cpu().numpy() == B.OK)
        Yo = On.solve(fam, Q, rows, P)
        assert _dres(fam, Q, P, y.cpu().numpy(), Yo).max() <= 1e-12
    finally:
        M.free()


def _check_lift32(x32, ref, Q, Y):
    """FP32 lift bar.  Q and y are rounded to FP32 and split exactly into three
    bf16 parts; the kernel accumulates 6 r part products in FP32 and drops
    terms below 2^-24 |q||y|.  The worst case is therefore
    |x - Q y| <= (6 r + 3) u32 (|Q| |y|) elementwise (u32 = 2^-24); the typical
    error is a few u32."""
    u = 2.0 ** -24
    r = Q.shape[1]
    mag = (np.abs(Q) @ np.abs(Y.T)).T
    err = np.abs(x32 - ref)
    assert np.all(err <= (6 * r + 3) * u * mag + 1e-300)
    rel = err / np.maximum(mag, 1e-300)
    print(f"lift fp32: median {np.median(rel) / u:.2f} u32, max {rel.max() / u:.2f} u32")
    assert np.median(rel) <= 2 * u


def test_lift_matches_q_times_y(c1):
    import torch
    w, off = c1
    header("lift")
    M = B.Model(w, basis=off["Q"], rows=off["rows"])
    try:
        rng = np.random.default_rng(0)
        Y = rng.standard_normal((70, 16))
        x64 = M.lift(to_dev(Y), precision=B.FP64).cpu().numpy()
        Qg = M.basis()
        ref = (Qg @ Y.T).T
        assert np.abs(x64 - ref).max() <= 1e-14 * np.abs(ref).max()
        x32 = M.lift(to_dev(Y), precision=B.FP32).cpu().numpy()
        _check_lift32(x32, ref, Qg, Y)
    finally:
        M.free()


@pytest.mark.parametrize("k,pad", [(1, 0), (33, 0), (130, 0), (70, 32), (70, 5), (45, 4), (1, 32)])
def test_lift_3d_many_vectors(k, pad):
    """FP32 lift on a 3-D basis (N = 41, n = 68921, odd, r = 40) with a vector
    count that leaves a ragged tile, with ld = n and with padded leading
    dimensions (aligned to 32 and not); checked against FP64 Q y on the host,
    padding rows must keep their contents."""
    import torch
    header(f"lift 3-D k={k} pad={pad}")
    dev = device()
    w = si.diffusion3d(N=41, r=40, s=160, m=8)
    n = w["n"]
    rng = np.random.default_rng(11)
    Q0, _ = np.linalg.qr(rng.standard_normal((n, w["r"])))
    M = B.Model(w, basis=Q0)
    try:
        Y = rng.standard_normal((k, w["r"])) * np.logspace(0, -6, w["r"])
        ld = n if pad == 0 else (n + 31) // 32 * 32 + (0 if pad == 32 else pad)
        x = torch.full((k, ld), 7.5, dtype=torch.float32, device=dev)
        B.subap_lift(M.handle, to_dev(Y), x, B.FP32)
        xh = x.cpu().numpy()
        assert np.all(xh[:, n:] == 7.5)
        Qg = M.basis()
        ref = (Qg @ Y.T).T
        _check_lift32(xh[:, :n], ref, Qg, Y)
        # FP64 lift with the same leading dimension
        x64 = torch.full((k, ld), -2.5, dtype=torch.float64, device=dev)
        B.subap_lift(M.handle, to_dev(Y), x64, B.FP64)
        x64h = x64.cpu().numpy()
        assert np.all(x64h[:, n:] == -2.5)
        assert np.abs(x64h[:, :n] - ref).max() <= 1e-14 * np.abs(ref).max()
    finally:
        M.free()


@pytest.fixture(scope="module")
def d3_full():
    """Full 3-D configuration size (215^3 nodes, r = 40, s = 160) with an
    oracle-made orthonormal basis and seeded rows: the online solve does not
    depend on where they came from, and every oracle input stays independent
    of the GPU path."""
    from oracle import families as F
    w = si.diffusion3d()
    fam = F.from_workload(w)
    rng = np.random.default_rng(2025)
    Q, _ = O.orthonormalise(rng.standard_normal((w["n"], w["r"])))
    rows = np.sort(rng.choice(w["n"], size=w["s"], replace=False))
    return w, fam, Q, rows


@pytest.mark.slow
@pytest.mark.parametrize("prec,refine,csne", [(B.FP64, 0, False), (B.FP32, 1, True)])
def test_diffusion3d_full_size_sampled(d3_full, prec, refine, csne):
    """All 65,536 parameters in one launch (the benchmark's configuration);
    the oracle recomputes 12 sampled parameters one by one and measures
    delta_res = |A(p) Q (y_gpu - y_oracle)| / |b| over all n rows: <= 1e-11
    for FP64, <= 1e-6 for the FP32 contraction with one step of the corrected
    semi-normal equations (a random basis makes the sketched residual of
    order one, where simple refinement stops at a biased fixed point)."""
    w, fam, Q, rows = d3_full
    header(f"3-D full size prec={prec} refine={refine} csne={csne}")
    M = B.Model(w, basis=Q, rows=rows)
    try:
        P = w["test_params"]
        y, _, st = M.solve(to_dev(P), contraction=prec, refine_steps=refine, csne=csne)
        st = st.cpu().numpy()
        y = y.cpu().numpy()
        assert np.all(st == B.OK)
        idx = np.concatenate([np.random.default_rng(9).choice(len(P), size=10, replace=False), [0, len(P) - 1]])
        bar = 1e-11 if prec == B.FP64 else 1e-6
        for i in idx:
            yo = On.solve_one(fam, Q, rows, P[i])
            d = On.delta_res(fam, Q, P[i], y[i], yo)
            print(f"p[{i}] delta_res {d:.2e} (bar {bar:.0e})", flush=True)
            assert d <= bar, (i, d, bar)
    finally:
        M.free()
