"""GPU parity of leverage-score row sampling with weights (Section 5.3) and of
the weighted online solve and residual estimate (Section 5.3.1) against the
FP64 oracle.

Bars:
* rows bit-exact for the same uniforms.  A draw may differ only where
  u_k * sum(l) lies within 1e-12 * sum(l) of a running-sum boundary.  There
  the GPU's chunked summation order may round to the other side, and both
  rows are valid draws.
* weights within 1e-12 relative.
* the weighted solve within delta_res <= 1e-12 (FP64 contraction) and
  <= 1e-6 (FP32 / FP16X3 contraction + one FP64 refinement step).
* rho within 1e-9 relative of the oracle's |W S (A Q y - b)| / |b|.
* residual bounds within 1e-12 relative of the oracle's.
"""
import numpy as np
import pytest

import subap_inputs as si
from oracle import offline as O
from oracle import online as On
from paper_2510_04825_amd import binding as B
from tests.gpu_util import device, header, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    "diff2d": lambda: si.diffusion2d(N=24, r=6, s=28, m=24),
    "diff3d": lambda: si.diffusion3d(N=9, r=8, s=40, m=24),
    "krr": lambda: si.krr(n=1024, r=8, s=48, m=24),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def lev(request):
    w = CASES[request.param]()
    u = si.sample_uniforms(w["s"], seed=31)
    off = O.offline(w, sample_u=u)
    B_ = O.leverage_matrix(off["family"], off["Q"], w["select_param"])
    sc = O.span_scores(B_)
    device()
    M = B.Model(w, basis=off["Q"], sample_u=u)
    yield request.param, w, off, u, sc, M
    M.free()


def test_leverage_rows_and_weights(lev):
    name, w, off, u, sc, M = lev
    header(f"leverage rows {name}")
    rows, wt = M.rows(), M.weights()
    diff = np.flatnonzero(rows != off["rows"])
    for k in diff:
        run = np.cumsum(sc)
        t = u[k] * run[-1]
        lo = min(rows[k], off["rows"][k])
        assert abs(run[lo] - t) <= 1e-12 * run[-1], (name, k, rows[k], off["rows"][k])
    assert diff.size <= 1
    same = rows == off["rows"]
    np.testing.assert_allclose(wt[same], off["weights"][same], rtol=1e-12)
    # every weight is 1 / sqrt(s pi) of its own row
    np.testing.assert_allclose(wt, 1.0 / np.sqrt(w["s"] * sc[rows] / sc.sum()), rtol=1e-12)


@pytest.mark.parametrize("form", ["fp64", "reduced+1"])
def test_weighted_solve_matches_oracle(lev, form):
    import torch
    name, w, off, u, sc, M = lev
    header(f"leverage solve {name} {form}")
    rows, wt = M.rows(), M.weights()  # the GPU's draw, so a boundary draw cannot differ
    fam, Q = off["family"], off["Q"]
    P = w["test_params"]
    yo = On.solve(fam, Q, rows, P, wt)
    if form == "fp64":
        prec, ref, tol = B.FP64, 0, 1e-12
    else:
        prec, ref, tol = (B.FP16X3 if name == "krr" else B.FP32), 1, 1e-6
    y, rho, st = M.solve(to_dev(P), prec, ref)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == B.OK)
    yg = y.cpu().numpy()
    d = max(On.delta_res(fam, Q, p, a, b) for p, a, b in zip(P, yg, yo))
    assert d <= tol, (name, form, d)
    rho_o = np.array([On.sketched_residual(fam, Q, rows, p, a, wt) for p, a in zip(P, yg)])
    rtol = 1e-9 if form == "fp64" else 1e-6
    np.testing.assert_allclose(rho.cpu().numpy(), rho_o, rtol=rtol)


def test_residual_bounds_match_oracle_and_hold_at_select_param(lev):
    import torch
    name, w, off, u, sc, M = lev
    header(f"leverage bounds {name}")
    fam, Q = off["family"], off["Q"]
    P = np.vstack([np.atleast_2d(w["select_param"]), w["test_params"][:7]])
    y, rho, st = M.solve(to_dev(P))
    lo, hi = M.residual_bounds(rho)
    torch.cuda.synchronize()
    rh = rho.cpu().numpy()
    for i, p in enumerate(P):
        lo_o, hi_o = O.residual_bounds(rh[i], w["r"], w["s"])
        np.testing.assert_allclose([lo.cpu().numpy()[i], hi.cpu().numpy()[i]], [lo_o, hi_o], rtol=1e-12)
    # at p_sel the estimate brackets the full relative residual
    full = On.residual(fam, Q @ y.cpu().numpy()[0], P[0])
    assert lo.cpu().numpy()[0] <= full <= hi.cpu().numpy()[0], (name, full, rh[0])
    # an explicit eps
    lo2, hi2 = M.residual_bounds(rho, eps=0.25)
    torch.cuda.synchronize()
    np.testing.assert_allclose(lo2.cpu().numpy(), rh / 1.25, rtol=1e-15)
    np.testing.assert_allclose(hi2.cpu().numpy(), rh / 0.75, rtol=1e-15)


def test_weighted_model_in_a_plan(lev):
    import torch
    name, w, off, u, sc, M = lev
    header(f"leverage plan {name}")
    P = to_dev(w["test_params"])
    y1, _, _ = M.solve(P)
    y2 = torch.empty_like(y1)
    B.subap_solve_multi([M.handle], [P], [y2])
    torch.cuda.synchronize()
    a, b = y1.cpu().numpy(), y2.cpu().numpy()
    assert np.abs(a - b).max() <= 1e-10 * np.abs(a).max()


def test_leverage_rejects_bad_uniforms():
    w = si.diffusion2d(N=8, r=3, s=6)
    device()
    for bad in (np.full(6, 1.0), np.array([0.1, 0.2, np.nan, 0.3, 0.4, 0.5]), np.full(6, -0.1)):
        with pytest.raises(B.SubapError):
            B.Model(w, sample_u=bad)


@pytest.mark.slow
def test_leverage_full_size_3d():
    """The 3-D benchmark size (215^3 nodes, r = 40, s = 160) with an oracle-made
    orthonormal basis: the GPU's leverage rows and weights against the
    oracle's sampling of the same uniforms (a draw may differ only on a
    running-sum boundary), then the weighted batch of 65,536 parameters,
    sampled parameters recomputed by the oracle (sketched distance <= 1e-11)."""
    import torch
    from oracle import families as Fm
    w = si.diffusion3d()
    header("leverage full size 3-D")
    fam = Fm.from_workload(w)
    rng = np.random.default_rng(2028)
    Q, _ = O.orthonormalise(rng.standard_normal((w["n"], w["r"])))
    u = si.sample_uniforms(w["s"], seed=909)
    sc = O.span_scores(O.leverage_matrix(fam, Q, w["select_param"]))
    rows_o, wt_o = O.leverage_sample(sc, u)
    device()
    M = B.Model(w, basis=Q, sample_u=u)
    try:
        rows, wt = M.rows(), M.weights()
        run = np.cumsum(sc)
        for k in np.flatnonzero(rows != rows_o):
            lo = min(rows[k], rows_o[k])
            # two QR codes on a 9.9M-row matrix agree to about eps kappa(A) in the
            # scores, so the running sums may differ by ~1e-11 of the total
            assert abs(run[lo] - u[k] * run[-1]) <= 1e-9 * run[-1], (k, rows[k], rows_o[k])
        same = rows == rows_o
        np.testing.assert_allclose(wt[same], wt_o[same], rtol=1e-9)
        P = w["test_params"]
        y, _, st = M.solve(to_dev(P))
        torch.cuda.synchronize()
        assert np.all(st.cpu().numpy() == B.OK)
        y = y.cpu().numpy()
        for i in np.concatenate([rng.choice(len(P), size=8, replace=False), [0, len(P) - 1]]):
            G = On.reduced_matrix(fam, Q, rows, P[i], wt)
            bS = wt * fam.rhs_rows(P[i], rows)
            yo, _, _ = On.householder_lsq(G, bS)
            d = np.linalg.norm(G @ (y[i] - yo)) / np.linalg.norm(bS)
            assert d <= 1e-11, (i, d)
    finally:
        M.free()
