"""GPU parity of the other row selectors of Section 5.3: LU with partial
pivoting on A(p_sel) X (in rounds for s > r) and the union of the pivots
found at several points (Section 5.3.2), against the FP64 oracle with the
oracle's basis passed in.  Row indices must match bit-exactly; the solve on
the selected rows within delta_res <= 1e-12 (FP64)."""
import numpy as np
import pytest

import subap_inputs as si
from oracle import families as F
from oracle import offline as O
from oracle import online as On
from paper_2510_04825_amd import binding as B
from tests.gpu_util import device, header, to_dev

pytestmark = pytest.mark.gpu

CASES = {
    "diff2d_s_eq_r": lambda: si.diffusion2d(N=20, r=6, s=6, m=16),
    "diff2d_rounds": lambda: si.diffusion2d(N=20, r=6, s=22, m=16),
    "diff3d": lambda: si.diffusion3d(N=8, r=7, s=21, m=16),
    "krr": lambda: si.krr(n=800, r=6, s=18, m=16),
    "delay": lambda: si.delay(n=1500, r=6, s=18, m=16),
}


def _basis(w):
    X = O.snapshots(F.from_workload(w), w["snap_params"])
    return O.orthonormalise(X)[0]


@pytest.mark.parametrize("name", sorted(CASES))
def test_lu_rows_bit_exact_and_solve(name):
    import torch
    w = CASES[name]()
    header(f"LU rows {name}")
    Q = _basis(w)
    off = O.offline(w, basis=Q, selection="lu")
    device()
    M = B.Model(w, basis=Q, selection=B.SELECT_LU)
    try:
        assert np.array_equal(M.rows(), off["rows"]), (M.rows(), off["rows"])
        P = w["test_params"]
        y, _, st = M.solve(to_dev(P))
        torch.cuda.synchronize()
        assert np.all(st.cpu().numpy() == B.OK)
        yo = On.solve(off["family"], off["Q"], off["rows"], P)
        d = max(On.delta_res(off["family"], off["Q"], p, a, b) for p, a, b in zip(P, y.cpu().numpy(), yo))
        assert d <= 1e-12, d
    finally:
        M.free()


@pytest.mark.parametrize("name,selection", [("diff2d_s_eq_r", "cpqr"), ("diff2d_s_eq_r", "lu"), ("krr", "lu"),
                                            ("delay", "cpqr")])
def test_union_of_pivots(name, selection):
    import torch
    w = CASES[name]()
    header(f"union {name} {selection}")
    Q = _basis(w)
    d = w["d"]
    if w["family"] == "krr":
        pts = np.array([[0.6], [1.0], [1.7]])
    elif w["family"] == "delay":
        pts = np.array([[1.0], [5.0], [9.0]])
    else:
        pts = np.random.default_rng(9).uniform(-1.0, 1.0, size=(4, d))
    off = O.offline(w, basis=Q, selection=selection, select_params=pts)
    device()
    sel = B.SELECT_LU if selection == "lu" else B.SELECT_CPQR
    M = B.Model(w, basis=Q, selection=sel, select_params=pts)
    try:
        assert M.s == off["rows"].size
        assert np.array_equal(M.rows(), off["rows"])
        P = w["test_params"]
        y, _, st = M.solve(to_dev(P))
        torch.cuda.synchronize()
        assert np.all(st.cpu().numpy() == B.OK)
        yo = On.solve(off["family"], off["Q"], off["rows"], P)
        dd = max(On.delta_res(off["family"], off["Q"], p, a, b) for p, a, b in zip(P, y.cpu().numpy(), yo))
        assert dd <= 1e-12, dd
    finally:
        M.free()


@pytest.mark.parametrize("name", ["diff2d_rounds", "diff3d"])
def test_rows_per_nearest_snapshot(name):
    """The other variant of Section 5.3.2: each parameter takes the rows
    selected at its nearest snapshot point.  It is built from existing parts:
    one model per snapshot on the shared basis, each selecting at its own
    point, and one plan that solves every parameter with its snapshot's
    model.  Rows bit-exact per snapshot; FP64 delta_res <= 1e-12 for every
    parameter against the oracle on the same rows."""
    import torch
    w = CASES[name]()
    w = dict(w, test_params=np.random.default_rng(31).uniform(-1.0, 1.0, size=(48, w["d"])), m=48)
    header(f"nearest-snapshot rows {name}")
    Q = _basis(w)
    snaps = w["snap_params"]
    P = w["test_params"]
    near = np.argmin(((P[:, None, :] - snaps[None, :, :]) ** 2).sum(axis=2), axis=1)
    used = [i for i in range(len(snaps)) if np.any(near == i)]
    assert len(used) >= 2
    offs = {i: O.offline(dict(w, select_param=snaps[i]), basis=Q) for i in used}
    device()
    models = {}
    try:
        for i in used:
            models[i] = B.Model(dict(w, select_param=snaps[i]), basis=Q)
            assert np.array_equal(models[i].rows(), offs[i]["rows"]), i
        params = [to_dev(P[near == i]) for i in used]
        ys = [torch.full((int(np.sum(near == i)), w["r"]), -7.0, dtype=torch.float64, device=params[0].device)
              for i in used]
        sts = [torch.full((int(np.sum(near == i)),), -1, dtype=torch.int32, device=params[0].device) for i in used]
        plan = B.subap_plan_create([models[i].handle for i in used], params, ys, None, sts, B.FP64, 0, 0)
        try:
            B.subap_plan_execute(plan)
            torch.cuda.synchronize()
        finally:
            B.subap_plan_free(plan)
        for i, y, st in zip(used, ys, sts):
            assert np.all(st.cpu().numpy() == B.OK)
            Pi = P[near == i]
            off = offs[i]
            yo = On.solve(off["family"], off["Q"], off["rows"], Pi)
            dd = max(On.delta_res(off["family"], off["Q"], p, a, b) for p, a, b in zip(Pi, y.cpu().numpy(), yo))
            assert dd <= 1e-12, (i, dd)
    finally:
        for M in models.values():
            M.free()
