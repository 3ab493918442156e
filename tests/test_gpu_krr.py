"""GPU parity for kernel ridge regression against the FP64 oracle.

Bars: row indices bit-exact (given basis); FP64 contraction within
delta_res <= 1e-11 of the oracle (the GPU's polynomial exp2 is accurate to
FP64 rounding there, to 5.5e-11 per kernel entry in a first refinement step and
to FP64 rounding in later steps); FP32 and split 16-bit contractions followed
by FP64 refinement within delta_res <= 1e-6, the tolerance the method's
reduced-precision forms are held to.  delta_res = |A(p) Q (y_gpu - y_oracle)|
/ |b| over all n rows (oracle.online.delta_res).  At the full configuration
size the refinement solves the corrected semi-normal equations, and the
oracle recomputes sampled parameters one by one on its own snapshot basis and
on a random one.
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


@pytest.mark.parametrize("prec", [B.FP64, B.FP32, B.BF16X3, B.FP16X3])
def test_krr_csne_refinement(krr_small, krr_model, krr_oracle_y, prec):
    """Corrected semi-normal equations: each step solves R^T R dy = G^T r_S
    with an FP64 G^T r_S, so the fixed point is the exact solution of eq.
    (3.3).  One step from FP32 or a split contraction lands within 1e-6 of
    the oracle (FP64: 1e-11), and a second step does not lose it."""
    w, off = krr_small
    header(f"krr csne precision {prec}")
    P = w["test_params"]
    y1, rho1, st1 = krr_model.solve(to_dev(P), contraction=prec, refine_steps=1, csne=True)
    y2, _, st2 = krr_model.solve(to_dev(P), contraction=prec, refine_steps=2, csne=True)
    assert np.all(st1.cpu().numpy() == B.OK) and np.all(st2.cpu().numpy() == B.OK)
    d1 = _dres(off["family"], off["Q"], P, y1.cpu().numpy(), krr_oracle_y)
    d2 = _dres(off["family"], off["Q"], P, y2.cpu().numpy(), krr_oracle_y)
    print(f"precision {prec}: csne delta_res after 1 step {d1.max():.2e}, after 2 steps {d2.max():.2e}")
    assert d1.max() <= (1e-11 if prec == B.FP64 else 1e-6)
    assert d2.max() <= max(1e-9, 2.0 * d1.max()) if prec != B.FP64 else d2.max() <= 1e-11
    # rho: the FP64 residual before the step, outside the computed Q factor's range
    rho_o = np.array([On.sketched_residual(off["family"], off["Q"], off["rows"], p, yo)
                      for p, yo in zip(P, krr_oracle_y)])
    assert np.allclose(rho1.cpu().numpy(), rho_o, rtol=1e-2, atol=5e-8)


def test_krr_csne_weighted_rows():
    """CSNE with leverage-score rows: the weights enter G^T r_S through the
    kernel part (w o r_S) and through Q_S, which carries them."""
    w = si.krr(n=1536, r=12, s=40, m=40)
    u = si.sample_uniforms(w["s"])
    off = O.offline(w, sample_u=u)
    header("krr csne weighted rows")
    M = B.Model(w, basis=off["Q"], sample_u=u, selection=B.SELECT_LEVERAGE)
    try:
        assert np.array_equal(M.rows(), off["rows"])
        P = w["test_params"]
        Yo = On.solve(off["family"], off["Q"], off["rows"], P, off["weights"])
        y, _, st = M.solve(to_dev(P), contraction=B.FP16X3, refine_steps=1, csne=True)
        assert np.all(st.cpu().numpy() == B.OK)
        d = _dres(off["family"], off["Q"], P, y.cpu().numpy(), Yo)
        print("weighted csne delta_res", d.max())
        assert d.max() <= 1e-6
    finally:
        M.free()


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


@pytest.mark.parametrize("prec,refine,csne", [(B.FP64, 0, False), (B.FP16X3, 1, False), (B.FP16X3, 1, True)])
def test_krr_extreme_length_scales(krr_small, krr_model, prec, refine, csne):
    """Length scales far outside the snapshot range: tiny p makes every
    off-point entry underflow (the refinement takes its clamped reduction for
    those parameter blocks), huge p makes K_p nearly the all-ones matrix.
    The first 16 parameters are ordinary, so one block of the refinement
    takes the unclamped reduction in the same launch.  p = 1e4 is checked in
    FP64 only: S A(p) Q then has a condition number near n / lambda, and one
    refinement step from a contraction accurate to 2^-18 cannot reach 1e-6."""
    w, off = krr_small
    header(f"krr extreme length scales prec {prec} refine {refine} csne {csne}")
    extra = [[1e-5], [1.0], [3e-6], [1e-3], [0.05]] + ([[1e4]] if prec == B.FP64 else [])
    P = np.concatenate([w["test_params"][:16], extra])
    y, _, st = krr_model.solve(to_dev(P), contraction=prec, refine_steps=refine, csne=csne)
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


def _golden_krr_basis(w):
    """The oracle's own offline result for this configuration (snapshot solves,
    QR, pivoted-QR rows), stored by tests/golden/make_krr_basis.py."""
    import os
    import sys
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, here)
    try:
        import make_krr_basis as mk
    finally:
        sys.path.remove(here)
    z = np.load(mk.PATH, allow_pickle=False)
    assert str(z["fingerprint"]) == mk.fingerprint(w), "krr_c2_basis.npz does not match the workload generator"
    return z["Q"], z["rows"]


# Forms of the full-size runs: (contraction, refinement steps, CSNE).  The
# split bf16 contraction (relative error ~2^-15) needs a second CSNE step: one
# step multiplies the error by about kappa x 2^-15.
FULL_FORMS = [(B.FP64, 0, False), (B.FP16X3, 1, True), (B.FP32, 1, True), (B.BF16X3, 2, True)]


@pytest.fixture(scope="module", params=["snapshot", "random"])
def krr_full_results(request, krr_full):
    """Every form of FULL_FORMS at full size in the benchmark's launch
    (s = 128, m = 4096), on the oracle's snapshot basis (the configuration
    itself) and on a random orthonormal basis (sketched residual of order one,
    the hardest case for the refinement).  The oracle then recomputes 16
    parameters one by one, 14 sampled plus the smallest and largest length
    scale of the batch, and gives delta_res over all n rows for each form."""
    w, fam, Qr, rows_r = krr_full
    if request.param == "snapshot":
        Q, rows = _golden_krr_basis(w)
    else:
        Q, rows = Qr, rows_r
    P = w["test_params"]
    idx = np.random.default_rng(7).choice(len(P), size=14, replace=False)
    idx = np.concatenate([idx, [int(np.argmin(P[:, 0])), int(np.argmax(P[:, 0]))]])
    header(f"krr full size, {request.param} basis")
    M = B.Model(w, basis=Q, rows=rows)
    try:
        assert np.array_equal(M.rows(), rows)
        Ys = {}
        for prec, refine, csne in FULL_FORMS:
            header(f"krr full size {request.param} prec={prec} refine={refine} csne={csne}")
            y, _, st = M.solve(to_dev(P), contraction=prec, refine_steps=refine, csne=csne)
            assert np.all(st.cpu().numpy() == B.OK), (prec, refine, csne)
            Ys[(prec, refine, csne)] = y.cpu().numpy()[idx]
    finally:
        M.free()
    Yo = On.solve(fam, Q, rows, P[idx])
    forms = list(Ys)
    Pall = np.concatenate([P[idx]] * len(forms))
    Yall = np.concatenate([Ys[f] for f in forms])
    d = On.delta_res_params(fam, Q, Pall, Yall, np.concatenate([Yo] * len(forms)))
    dres = {f: d[i * len(idx):(i + 1) * len(idx)] for i, f in enumerate(forms)}
    return request.param, P[idx], dres


@pytest.mark.parametrize("form", FULL_FORMS)
def test_krr_full_size_sampled(krr_full_results, form):
    """delta_res = |A(p) Q (y_gpu - y_oracle)| / |b| over all n rows <= 1e-6
    for the reduced-precision forms with CSNE refinement, <= 1e-11 for FP64."""
    basis, P, dres = krr_full_results
    d = dres[form]
    for p, v in zip(P[:, 0], d):
        print(f"{basis} basis form {form}: p={p:.4f} delta_res {v:.2e}")
    bar = 1e-11 if form[0] == B.FP64 else 1e-6
    assert d.max() <= bar, (basis, form, d.max())


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


def test_exp2_rate_microbenchmark():
    """subap_exp2_rate: positive, finite rates; the degree-11 polynomial costs
    more than degree 7 (four more FMAs per evaluation); bad forms and counts
    are rejected before any device work."""
    import ctypes as C
    header("exp2 rate")
    device()
    r7, r11, r0 = (B.subap_exp2_rate(f, 1 << 30) for f in (7, 11, 0))
    print(f"2^(c d) per second: degree 7 {r7:.3e}, degree 11 {r11:.3e}, v_exp_f32 {r0:.3e}")
    assert all(np.isfinite(v) and v > 0 for v in (r7, r11, r0))
    assert r11 < r7
    lib = B.load()
    out = C.c_double()
    assert lib.subap_exp2_rate(5, 1 << 20, C.byref(out), None) == B.E_INVALID
    assert lib.subap_exp2_rate(7, 0, C.byref(out), None) == B.E_INVALID
    assert lib.subap_exp2_rate(7, 1 << 20, None, None) == B.E_INVALID
