"""GPU parity for kernel ridge regression against the FP64 oracle.

Bars: row indices bit-exact (given basis); FP64 contraction within
delta_res <= 1e-11 of the oracle (the GPU's polynomial exp2 is accurate to
FP64 rounding there, to 5.5e-11 per kernel entry in a first refinement step and
to FP64 rounding in later steps); FP32 and split-bf16 contractions followed by one
FP64 refinement step within delta_res <= 1e-6, the tolerance the method's
reduced-precision forms are held to.  At the full configuration size the
oracle checks sampled parameters through the sketched distance
|S A(p) Q (y_gpu - y_oracle)| / |S b| (same bars), computed from the s rows.
"""
import numpy as np
import pytest

import subap_inputs as si
from oracle import families as F
from oracle import offline as O
from oracle import online as On
from paper_2510_04825_amd import binding as B
from tests.gpu_util import device, header, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def krr_small():
    w = si.krr(n=2048, m=96)
    return w, O.offline(w)


def _dres(fam, Q, P, Yg, Yo):
    return np.array([On.delta_res(fam, Q, p, a, b) for p, a, b in zip(P, Yg, Yo)])


def test_krr_rows_bit_exact_given_basis(krr_small):
    w, off = krr_small
    header("krr given-basis rows")
    device()
    M = B.Model(w, basis=off["Q"])
    try:
        assert np.array_equal(M.rows(), off["rows"])
    finally:
        M.free()


@pytest.fixture(scope="module")
def krr_model(krr_small):
    w, off = krr_small
    device()
    M = B.Model(w, basis=off["Q"], rows=off["rows"])
    yield M
    M.free()


@pytest.fixture(scope="module")
def krr_oracle_y(krr_small):
    w, off = krr_small
    return On.solve(off["family"], off["Q"], off["rows"], w["test_params"])


def test_krr_fp64_matches_oracle(krr_small, krr_model, krr_oracle_y):
    w, off = krr_small
    header("krr fp64 batched")
    P = w["test_params"]
    y, rho, st = krr_model.solve(to_dev(P))
    assert np.all(st.cpu().numpy() == B.OK)
    d = _dres(off["family"], off["Q"], P, y.cpu().numpy(), krr_oracle_y)
    assert d.max() <= 1e-11, d.max()


@pytest.mark.parametrize("prec", [B.FP32, B.BF16X3, B.FP16X3])
def test_krr_reduced_precision_with_refinement(krr_small, krr_model, krr_oracle_y, prec):
    w, off = krr_small
    header(f"krr precision {prec}")
    P = w["test_params"]
    y0, _, _ = krr_model.solve(to_dev(P), contraction=prec, refine_steps=0)
    y1, rho, st = krr_model.solve(to_dev(P), contraction=prec, refine_steps=1)
    assert np.all(st.cpu().numpy() == B.OK)
    d0 = _dres(off["family"], off["Q"], P, y0.cpu().numpy(), krr_oracle_y)
    d1 = _dres(off["family"], off["Q"], P, y1.cpu().numpy(), krr_oracle_y)
    print(f"precision {prec}: delta_res before {d0.max():.2e} after one step {d1.max():.2e}")
    assert d1.max() <= 1e-6
    assert d1.max() < d0.max()
    # the reported sketched residual is the oracle's (after refinement)
    rho_o = np.array([On.sketched_residual(off["family"], off["Q"], off["rows"], p, yo)
                      for p, yo in zip(P, krr_oracle_y)])
    # After a refinement step rho is the part of the FP64 residual outside the
    # range of the computed S A Q; it carries an absolute error of about
    # (contraction error ~1e-5) x (residual change of the step <= 3e-4 |S b|).
    rg = rho.cpu().numpy()
    print("rho gpu", rg[:6], "oracle", rho_o[:6], "max abs diff", np.abs(rg - rho_o).max())
    assert np.allclose(rg, rho_o, rtol=1e-2, atol=5e-8)


@pytest.mark.parametrize("prec", [B.FP32, B.FP16X3])
def test_krr_two_refinement_steps(krr_small, krr_model, krr_oracle_y, prec):
    """The second step runs with FP64-rounding kernel entries: it must not
    lose what the first step gained."""
    w, off = krr_small
    header(f"krr two refinement steps precision {prec}")
    P = w["test_params"]
    y1, _, _ = krr_model.solve(to_dev(P), contraction=prec, refine_steps=1)
    y2, _, st = krr_model.solve(to_dev(P), contraction=prec, refine_steps=2)
    assert np.all(st.cpu().numpy() == B.OK)
    d1 = _dres(off["family"], off["Q"], P, y1.cpu().numpy(), krr_oracle_y)
    d2 = _dres(off["family"], off["Q"], P, y2.cpu().numpy(), krr_oracle_y)
    print(f"precision {prec}: delta_res after 1 step {d1.max():.2e}, after 2 steps {d2.max():.2e}")
    assert d2.max() <= 1e-9
    assert d2.max() <= 2.0 * d1.max() + 1e-13


def test_krr_per_parameter_calls_match_batched(krr_small, krr_model, krr_oracle_y):
    w, off = krr_small
    header("krr per-p plain")
    P = w["test_params"][:6]
    ys = []
    for i in range(len(P)):
        y, _, st = krr_model.solve(to_dev(P[i:i + 1]))
        assert st.cpu().numpy()[0] == B.OK
        ys.append(y.cpu().numpy()[0])
    d = _dres(off["family"], off["Q"], P, np.array(ys), krr_oracle_y[:6])
    assert d.max() <= 1e-11


def test_krr_nonpositive_length_scale(krr_model):
    header("krr invalid parameter")
    P = np.array([[1.0], [0.0], [-1.0], [np.inf], [0.7]])
    y, _, st = krr_model.solve(to_dev(P), contraction=B.BF16X3, refine_steps=1)
    st = st.cpu().numpy()
    assert list(st) == [B.OK, B.E_NONFINITE, B.E_NONFINITE, B.E_NONFINITE, B.OK]
    y = y.cpu().numpy()
    assert np.all(np.isnan(y[1:4])) and np.all(np.isfinite(y[[0, 4]]))


@pytest.mark.parametrize("prec,refine", [(B.FP64, 0), (B.FP16X3, 1)])
def test_krr_extreme_length_scales(krr_small, krr_model, prec, refine):
    """Length scales far outside the snapshot range: tiny p makes every
    off-point entry underflow (the refinement takes its clamped reduction for
    those parameter blocks), huge p makes K_p nearly the all-ones matrix.
    The first 16 parameters are ordinary, so one block of the refinement
    takes the unclamped reduction in the same launch.  p = 1e4 is checked in
    FP64 only: S A(p) Q then has a condition number near n / lambda, and one
    refinement step from a contraction accurate to 2^-18 cannot reach 1e-6."""
    w, off = krr_small
    header(f"krr extreme length scales prec {prec} refine {refine}")
    extra = [[1e-5], [1.0], [3e-6], [1e-3], [0.05]] + ([[1e4]] if prec == B.FP64 else [])
    P = np.concatenate([w["test_params"][:16], extra])
    y, _, st = krr_model.solve(to_dev(P), contraction=prec, refine_steps=refine)
    assert np.all(st.cpu().numpy() == B.OK)
    yo = On.solve(off["family"], off["Q"], off["rows"], P)
    d = _dres(off["family"], off["Q"], P, y.cpu().numpy(), yo)
    print("delta_res", d)
    assert d.max() <= (1e-11 if prec == B.FP64 else 1e-6), d.max()


def test_krr_full_chain_on_gpu(krr_small):
    w, off = krr_small
    fam = off["family"]
    header("krr full offline on GPU")
    M = B.Model(w, snap_tol=1e-12)
    try:
        Qg = M.basis()
        assert np.abs(Qg.T @ Qg - np.eye(w["r"])).max() < 1e-12
        P = w["test_params"][:8]
        y, _, st = M.solve(to_dev(P), contraction=B.BF16X3, refine_steps=1)
        assert np.all(st.cpu().numpy() == B.OK)
        yo = On.solve(fam, off["Q"], off["rows"], P)
        for i, p in enumerate(P):
            rg = On.residual(fam, Qg @ y.cpu().numpy()[i], p)
            ro = On.residual(fam, off["Q"] @ yo[i], p)
            assert rg <= max(10 * ro, 1e-8), (rg, ro)
    finally:
        M.free()


@pytest.fixture(scope="module")
def krr_full():
    """Full configuration size with an oracle-made orthonormal basis: the
    online solve does not depend on where the basis came from, and this
    keeps every oracle input independent of the GPU path."""
    w = si.krr()
    fam = F.from_workload(w)
    rng = np.random.default_rng(2024)
    Q, _ = O.orthonormalise(rng.standard_normal((w["n"], w["r"])))
    rows = O.select_rows(O.selection_matrix(fam, Q, w["select_param"]), w["s"])
    return w, fam, Q, rows


# First-order size of the contraction error relative to |S A Q|, per form:
# generous upper bounds (2x or more over CPU emulation of each form).
U_EFF = {B.BF16X3: 2.0 ** -15, B.FP16X3: 2.0 ** -18, B.FP32: 2.0 ** -18, B.FP64: 0.0}


@pytest.mark.parametrize("prec,refine", [(B.FP64, 0), (B.BF16X3, 1), (B.FP16X3, 1), (B.FP32, 1)])
def test_krr_full_size_sampled(krr_full, prec, refine):
    """Full sizes, bench launch configuration (s = 128, m = 4096).

    With s > r, simple refinement converges to the solution whose FP64
    residual is orthogonal to the range of the computed S A Q, not of the
    exact one: a bias of about u_eff kappa(S A Q) rho*, with rho* the sketched
    relative residual.  The synthetic random basis used at full size makes
    rho* of order one, so the bar is 1e-6 plus that bias (FP64: 1e-11).
    """
    w, fam, Q, rows = krr_full
    header(f"krr full size prec={prec} refine={refine}")
    M = B.Model(w, basis=Q, rows=rows)
    try:
        assert np.array_equal(M.rows(), rows)
        P = w["test_params"]
        y, _, st = M.solve(to_dev(P), contraction=prec, refine_steps=refine)
        st = st.cpu().numpy()
        y = y.cpu().numpy()
        assert np.all(st == B.OK)
        idx = np.random.default_rng(7).choice(len(P), size=12, replace=False)
        idx = np.concatenate([idx, [0, len(P) - 1]])
        for i in idx:
            G = On.reduced_matrix(fam, Q, rows, P[i])
            bS = fam.rhs_rows(P[i], rows)
            yo, _, rho = On.householder_lsq(G, bS)
            sv = np.linalg.svd(G, compute_uv=False)
            tol = 1e-11 if prec == B.FP64 else 1e-6 + U_EFF[prec] * sv[0] / sv[-1] * rho / np.linalg.norm(bS)
            d = np.linalg.norm(G @ (y[i] - yo)) / np.linalg.norm(bS)
            print(f"p[{i}]={P[i, 0]:.3f} sketched distance {d:.2e} (bar {tol:.1e})")
            assert d <= tol, (i, d, tol)
    finally:
        M.free()


@pytest.mark.parametrize("prec", [B.BF16X3, B.FP16X3, B.FP32])
def test_krr_full_size_interpolation(krr_full, prec):
    """s = r (interpolation, zero sketched residual): no refinement bias, so
    reduced-precision forms plus one FP64 step are held to 1e-6 at full size."""
    w, fam, Q, rows = krr_full
    r = w["r"]
    wi = dict(w, s=r)
    rows_i = rows[:r]
    header(f"krr full size interpolation prec={prec}")
    M = B.Model(wi, basis=Q, rows=rows_i)
    try:
        P = w["test_params"]
        y, _, st = M.solve(to_dev(P), contraction=prec, refine_steps=1)
        assert np.all(st.cpu().numpy() == B.OK)
        y = y.cpu().numpy()
        for i in np.random.default_rng(8).choice(len(P), size=12, replace=False):
            G = On.reduced_matrix(fam, Q, rows_i, P[i])
            bS = fam.rhs_rows(P[i], rows_i)
            yo, _, _ = On.householder_lsq(G, bS)
            d = np.linalg.norm(G @ (y[i] - yo)) / np.linalg.norm(bS)
            print(f"p[{i}]={P[i, 0]:.3f} interpolation distance {d:.2e}")
            assert d <= 1e-6, (i, d)
    finally:
        M.free()
