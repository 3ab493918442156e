"""The oracle against its stored outputs (tests/golden/, written by
tests/golden/make_golden.py from the oracle alone).  A change of the oracle's
row selection or least-squares arithmetic shows up here first; a deliberate
change regenerates the fixtures in the same commit."""
import os

import numpy as np

import subap_inputs as si
from oracle import offline as O
from oracle import online as On

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#", ndmin=2)


def test_c1_rows_and_coefficients_match_golden():
    w = si.diffusion2d()
    off = O.offline(w)
    rows = _load("c1_rows.txt").astype(np.int64).ravel()
    assert np.array_equal(off["rows"], rows)
    Y = On.solve(off["family"], off["Q"], off["rows"], w["test_params"][:8])
    Yg = _load("c1_y.txt")
    # BLAS builds may differ in rounding order: agreement to a few hundred ulps
    assert np.abs(Y - Yg).max() <= 1e-10 * np.abs(Yg).max()


def test_krr_golden_basis_is_the_oracles():
    """krr_c2_basis.npz (written by make_krr_basis.py from the oracle only)
    belongs to the current workload generator, holds an orthonormal basis, and
    its rows are the oracle's pivoted-QR rounds on (A(p_sel) Q)^T for that
    basis (Algorithm 3.1 step 3, readings R3/R4)."""
    import os
    import sys
    import subap_inputs as si
    from oracle import families as F
    from oracle import offline as O
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, here)
    try:
        import make_krr_basis as mk
    finally:
        sys.path.remove(here)
    w = si.krr()
    z = np.load(mk.PATH, allow_pickle=False)
    assert str(z["fingerprint"]) == mk.fingerprint(w)
    Q, rows = z["Q"], z["rows"]
    assert Q.shape == (w["n"], w["r"]) and rows.shape == (w["s"],)
    assert np.abs(Q.T @ Q - np.eye(w["r"])).max() <= 1e-14
    fam = F.from_workload(w)
    assert np.array_equal(O.select_rows(O.selection_matrix(fam, Q, w["select_param"]), w["s"]), rows)
