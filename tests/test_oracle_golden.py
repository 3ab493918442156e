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
