"""The C-ABI library loads, exports every symbol include/subap.h declares,
and rejects bad arguments with status codes before touching a device
(these tests run without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2510_04825_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "subap.h")).read()
    return sorted(set(re.findall(r"SUBAP_API\s+[\w\s\*]*?\b(subap_\w+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libsubap.so not built (run __graft_entry__.build())")
    return B.load()


def test_header_declares_the_binding_exports():
    assert header_functions() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in header_functions():
        assert hasattr(lib, name), name


def test_status_strings(lib):
    assert lib.subap_status_string(0) == b"ok"
    assert lib.subap_status_string(4) == b"rank deficient"


def _pd(**kw):
    base = dict(family=B.FAMILY_DIFF2D, grid=16, n=0, dim=0, points=None, rhs=None, lam=0.0)
    base.update(kw)
    return B.ProblemDesc(**base)


def _opts(**kw):
    snap = np.zeros((4, 2))
    sel = np.zeros(2)
    base = dict(r=4, s=8, snap_params=snap.ctypes.data, select_param=sel.ctypes.data, snap_tol=0.0,
                snap_maxiter=0, basis_in=None, rows_in=None)
    base.update(kw)
    return B.OfflineOpts(**base), (snap, sel)


@pytest.mark.parametrize("pd_kw,opt_kw", [
    (dict(family=9), {}),
    (dict(grid=1), {}),
    (dict(), dict(r=0)),
    (dict(), dict(r=65)),
    (dict(), dict(s=3)),
    (dict(), dict(s=300)),
    (dict(), dict(snap_params=None)),
    (dict(), dict(select_param=None)),
    (dict(), dict(snap_tol=-1.0)),
    (dict(family=B.FAMILY_KRR, n=100, dim=8), {}),          # points/rhs missing
])
def test_offline_rejects_bad_arguments(lib, pd_kw, opt_kw):
    pd = _pd(**pd_kw)
    op, keep = _opts(**opt_kw)
    h = C.c_void_p()
    rc = lib.subap_offline(C.byref(pd), C.byref(op), None, C.byref(h))
    assert rc == B.E_INVALID
    assert h.value is None
    assert len(lib.subap_last_error()) > 0


def test_offline_rejects_bad_rows(lib):
    pd = _pd()
    rows = np.array([0, 1, 2, 3, 4, 5, 6, 6], dtype=np.int64)  # duplicate
    op, keep = _opts(rows_in=rows.ctypes.data)
    h = C.c_void_p()
    assert lib.subap_offline(C.byref(pd), C.byref(op), None, C.byref(h)) == B.E_INVALID
    rows[-1] = 16 * 16  # out of range
    assert lib.subap_offline(C.byref(pd), C.byref(op), None, C.byref(h)) == B.E_INVALID


def test_offline_rejects_nonfinite_inputs(lib):
    pd = _pd()
    op, keep = _opts()
    keep[0][0, 0] = np.nan
    h = C.c_void_p()
    assert lib.subap_offline(C.byref(pd), C.byref(op), None, C.byref(h)) == B.E_INVALID


def test_null_model_calls(lib):
    assert lib.subap_offline(None, None, None, None) == B.E_INVALID
    opts = B.SolveOpts(0, 0)
    assert lib.subap_solve_batch(None, None, 4, None, None, None, C.byref(opts), None) == B.E_INVALID
    assert lib.subap_lift(None, None, 1, None, 0, 0, None) == B.E_INVALID
    assert lib.subap_model_rows(None, None) == B.E_INVALID
    assert lib.subap_model_free(None) == B.OK


@pytest.mark.parametrize("opt_kw", [
    dict(selection=7),
    dict(selection=B.SELECT_LEVERAGE),                     # sample_u missing
    dict(selection=B.SELECT_LU, n_select=3),               # select_params missing
    dict(n_select=-1),
])
def test_offline_rejects_bad_selection(lib, opt_kw):
    pd = _pd()
    op, keep = _opts(**opt_kw)
    h = C.c_void_p()
    assert lib.subap_offline(C.byref(pd), C.byref(op), None, C.byref(h)) == B.E_INVALID
    assert h.value is None


def test_offline_rejects_uniforms_outside_the_unit_interval(lib):
    pd = _pd()
    for bad in (1.0, -0.25, np.nan):
        u = np.full(8, 0.5)
        u[3] = bad
        op, keep = _opts(selection=B.SELECT_LEVERAGE, sample_u=u.ctypes.data)
        h = C.c_void_p()
        assert lib.subap_offline(C.byref(pd), C.byref(op), None, C.byref(h)) == B.E_INVALID


@pytest.mark.parametrize("pd_kw", [
    dict(tau=0.0, kappa=2.1),
    dict(tau=0.1, kappa=2.0),
    dict(tau=0.1, kappa=2.1, rhs=None),
    dict(tau=0.1, kappa=2.1, n=1),
])
def test_offline_rejects_bad_delay_problems(lib, pd_kw):
    b = np.ones(50)
    base = dict(family=B.FAMILY_DELAY, n=50, rhs=b.ctypes.data)
    base.update(pd_kw)
    pd = _pd(**base)
    snap = np.zeros((4, 1))
    sel = np.zeros(1)
    op, keep = _opts(snap_params=snap.ctypes.data, select_param=sel.ctypes.data)
    h = C.c_void_p()
    assert lib.subap_offline(C.byref(pd), C.byref(op), None, C.byref(h)) == B.E_INVALID


def test_null_model_calls_of_the_other_entry_points(lib):
    assert lib.subap_model_weights(None, None) == B.E_INVALID
    assert lib.subap_output(None, None, 1, None, None) == B.E_INVALID
    assert lib.subap_full_residual(None, None, 1, None, None, None) == B.E_INVALID
    assert lib.subap_apsnap_solve(None, None, 1, None, None, None) == B.E_INVALID
    assert lib.subap_polish(None, None, 1, None, 5, 0.0, None, None) == B.E_INVALID
    assert lib.subap_residual_bounds(None, None, 1, 0.0, None, None, None) == B.E_INVALID


def test_model_load_rejects_bad_files(lib, tmp_path):
    h = C.c_void_p()
    assert lib.subap_model_load(os.fsencode(str(tmp_path / "missing.bin")), None, C.byref(h)) == B.E_INVALID
    bad = tmp_path / "garbage.bin"
    bad.write_bytes(b"not a model file at all")
    assert lib.subap_model_load(os.fsencode(str(bad)), None, C.byref(h)) == B.E_INVALID
    # right magic, inconsistent header (r = 0)
    hdr = np.zeros(12, dtype=np.int64)
    hdr[:9] = [1, 8, 2, 64, 0, 4, 2, 4, 0]
    cut = tmp_path / "header.bin"
    cut.write_bytes(b"SUBAPMD1" + hdr.tobytes() + np.zeros(8).tobytes())
    assert lib.subap_model_load(os.fsencode(str(cut)), None, C.byref(h)) == B.E_INVALID
    # consistent header, arrays missing
    hdr[4] = 2
    cut.write_bytes(b"SUBAPMD1" + hdr.tobytes() + np.zeros(8).tobytes() + np.zeros(10).tobytes())
    assert lib.subap_model_load(os.fsencode(str(cut)), None, C.byref(h)) == B.E_INVALID
    assert h.value is None
    assert lib.subap_model_save(None, b"x") == B.E_INVALID


def test_model_load_rejects_a_grid_that_does_not_match_n(lib, tmp_path):
    # a 2-D model whose N disagrees with n would index neighbours outside the
    # basis; the header check refuses it before any device work
    n, r, s = 64, 2, 4
    hdr = np.array([B.FAMILY_DIFF2D, 7, 2, n, r, s, 2, 4, 0, 0, 0, 0], dtype=np.int64)
    body = np.zeros(n * r + n).tobytes() + np.arange(s, dtype=np.int64).tobytes() + np.ones(s).tobytes()
    f = tmp_path / "grid.bin"
    f.write_bytes(b"SUBAPMD1" + hdr.tobytes() + np.zeros(8).tobytes() + body)
    h = C.c_void_p()
    assert lib.subap_model_load(os.fsencode(str(f)), None, C.byref(h)) == B.E_INVALID
    assert b"inconsistent" in lib.subap_last_error()


def test_model_load_checks_the_payload_size_before_allocating(lib, tmp_path):
    # a self-consistent header that describes a 3-D model of 1290^3 nodes and
    # 64 columns (about 1.1 TB of basis) over a file of a few bytes: refused
    # from the file size, with no host or device allocation attempted
    N, r, s = 1290, 64, 128
    hdr = np.array([B.FAMILY_DIFF3D, N, 3, N ** 3, r, s, 4, 6, 0, 0, 0, 0], dtype=np.int64)
    f = tmp_path / "huge.bin"
    f.write_bytes(b"SUBAPMD1" + hdr.tobytes() + np.zeros(8).tobytes() + np.zeros(16).tobytes())
    h = C.c_void_p()
    assert lib.subap_model_load(os.fsencode(str(f)), None, C.byref(h)) == B.E_INVALID
    assert b"payload" in lib.subap_last_error()
    assert h.value is None
    # one byte too many is refused as well
    n, r, s = 64, 2, 4
    hdr = np.array([B.FAMILY_DIFF2D, 8, 2, n, r, s, 2, 4, 0, 0, 0, 0], dtype=np.int64)
    body = np.zeros(n * r + n).tobytes() + np.arange(s, dtype=np.int64).tobytes() + np.ones(s).tobytes()
    f.write_bytes(b"SUBAPMD1" + hdr.tobytes() + np.zeros(8).tobytes() + body + b"x")
    assert lib.subap_model_load(os.fsencode(str(f)), None, C.byref(h)) == B.E_INVALID
    assert b"payload" in lib.subap_last_error()
