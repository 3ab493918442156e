"""subap_solve_batch_noalloc against subap_solve_batch, through the C ABI.

The entry point keeps its workspace in the library's fixed device array
instead of allocating; its results must equal subap_solve_batch's bit for
bit (the same kernels on the same parameter blocks).  Two calls in a row, the
second with a smaller batch, so that the second reuses the array the first
left behind; the kernel ridge batch is larger than one scratch-full, so the
first call also runs in several chunks.
"""
import ctypes as C

import numpy as np
import pytest

import subap_inputs as si
from oracle import offline as O
from oracle import online as On
from paper_2510_04825_amd import binding as B
from tests.gpu_util import device, header, to_dev

pytestmark = pytest.mark.gpu


def _call(fn, M, P, r, opts):
    import torch
    m = P.shape[0]
    y = torch.full((m, r), -3.0, dtype=torch.float64, device="cuda")
    rho = torch.full((m,), -3.0, dtype=torch.float64, device="cuda")
    st = torch.full((m,), -3, dtype=torch.int32, device="cuda")
    rc = fn(C.c_void_p(M.handle), C.c_void_p(P.data_ptr()), m, C.c_void_p(y.data_ptr()),
            C.c_void_p(rho.data_ptr()), C.c_void_p(st.data_ptr()), C.byref(opts), None)
    assert rc == B.OK, B.load().subap_last_error()
    torch.cuda.synchronize()
    return y.cpu().numpy(), rho.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("form", [(B.FP16X3, 1, 1), (B.FP64, 0, 0), (B.FP32, 2, 0)])
def test_noalloc_matches_solve_batch_krr(form):
    w = si.krr(n=2048, r=32, s=128, m=1500)
    off = O.offline(w, basis=np.random.default_rng(31).standard_normal((w["n"], w["r"])))
    header(f"noalloc krr form {form}")
    device()
    M = B.Model(w, basis=off["Q"], rows=off["rows"])
    lib = B.load()
    try:
        opts = B.SolveOpts(*form)
        for m in (1500, 37):  # two calls in a row, the second smaller
            P = to_dev(w["test_params"][:m])
            ya, ra, sa = _call(lib.subap_solve_batch, M, P, w["r"], opts)
            yb, rb, sb = _call(lib.subap_solve_batch_noalloc, M, P, w["r"], opts)
            assert np.array_equal(sa, sb) and np.all(sb == B.OK)
            assert np.array_equal(ya, yb), np.abs(ya - yb).max()
            assert np.array_equal(ra, rb)
        # and both are the oracle's solution (the bar of the form)
        Yo = On.solve(off["family"], off["Q"], off["rows"], w["test_params"][:37])
        d = max(On.delta_res(off["family"], off["Q"], p, a, b) for p, a, b in zip(w["test_params"][:37], yb, Yo))
        assert d <= (1e-11 if form[0] == B.FP64 else 1e-6), d
    finally:
        M.free()


def test_noalloc_matches_solve_batch_diffusion():
    w = si.diffusion2d(N=32, r=8, s=16, m=300)
    off = O.offline(w)
    header("noalloc diffusion")
    device()
    M = B.Model(w, basis=off["Q"], rows=off["rows"])
    lib = B.load()
    try:
        opts = B.SolveOpts(B.FP64, 0, 0)
        for m in (300, 11):
            P = to_dev(w["test_params"][:m])
            ya, ra, sa = _call(lib.subap_solve_batch, M, P, w["r"], opts)
            yb, rb, sb = _call(lib.subap_solve_batch_noalloc, M, P, w["r"], opts)
            assert np.array_equal(ya, yb) and np.array_equal(ra, rb) and np.array_equal(sa, sb)
    finally:
        M.free()
