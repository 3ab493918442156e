"""Saving and loading a model: the loaded model has the same rows, weights
and output vector and solves bit-identically (its tables are rebuilt from
the saved basis, rows and weights by the same kernels)."""
import numpy as np
import pytest

import subap_inputs as si
from paper_2510_04825_amd import binding as B
from tests.gpu_util import device, header, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    "diff2d_cpqr": (lambda: si.diffusion2d(N=20, r=6, s=20, m=16), {}),
    "diff3d_leverage": (lambda: si.diffusion3d(N=8, r=6, s=24, m=16), {"sample_u": si.sample_uniforms(24, 4)}),
    "krr_lu": (lambda: si.krr(n=600, r=6, s=18, m=16), {"selection": B.SELECT_LU}),
    "delay_output": (lambda: si.delay(n=1500, r=5, s=15, m=16), {}),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_save_load_roundtrip(name, tmp_path):
    import torch
    make, kw = CASES[name]
    w = make()
    header(f"model file {name}")
    device()
    M = B.Model(w, snap_tol=1e-12, **kw)
    L = None
    try:
        P = to_dev(w["test_params"])
        prec = B.FP16X3 if w["family"] == "krr" else B.FP32
        y1, rho1, st1 = M.solve(P)
        y1r, rho1r, _ = M.solve(P, prec, 1)
        path = tmp_path / f"{name}.subap"
        M.save(str(path))
        rows, wts = M.rows(), M.weights()
        H1 = M.output(y1) if w["family"] == "delay" else None
        M.free()
        L = B.Model.load(str(path))
        assert (L.n, L.r, L.s, L.d) == (w["n"], w["r"], rows.size, w["d"])
        np.testing.assert_array_equal(L.rows(), rows)
        np.testing.assert_array_equal(L.weights(), wts)
        y2, rho2, st2 = L.solve(P)
        y2r, rho2r, _ = L.solve(P, prec, 1)
        torch.cuda.synchronize()
        assert torch.equal(y1, y2) and torch.equal(rho1, rho2) and torch.equal(st1, st2)
        assert torch.equal(y1r, y2r) and torch.equal(rho1r, rho2r)
        if H1 is not None:
            assert torch.equal(H1, L.output(y2))
    finally:
        M.free()
        if L is not None:
            L.free()
