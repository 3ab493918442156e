"""GPU parity of the batched persistent solve (many uneven finite-difference
instances in one launch) against the FP64 oracle, with and without hipGraph
replay and autotuning.  Bars as for the single-model solve: delta_res
<= 1e-12 (FP64), <= 1e-6 (FP32 contraction + one FP64 refinement)."""
import numpy as np
import pytest

import subap_inputs as si
from oracle import offline as O
from oracle import online as On
from paper_2510_04825_amd import binding as B
from tests.gpu_util import device, header, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def uneven_small():
    # every r of the uneven workload (8..64) and s in [2r, 4r], on grids the
    # oracle solves in seconds; m capped to keep the oracle loop short
    insts = si.uneven(k=8, grids=(16, 24, 20), max_m=64)
    out = []
    for w in insts:
        off = O.offline(w)
        yo = On.solve(off["family"], off["Q"], off["rows"], w["test_params"])
        out.append((w, off, yo))
    return out


def _models(uneven_small):
    device()
    return [B.Model(w, basis=off["Q"], rows=off["rows"]) for w, off, _ in uneven_small]


@pytest.mark.parametrize("prec,refine,tol,flags", [
    (B.FP64, 0, 1e-12, 0),
    (B.FP64, 0, 1e-12, B.PLAN_GRAPH | B.PLAN_AUTOTUNE),
    (B.FP32, 1, 1e-6, B.PLAN_GRAPH),
    (B.FP32, -1, 1e-6, B.PLAN_GRAPH),  # one step of the corrected semi-normal equations
])
def test_plan_matches_oracle(uneven_small, prec, refine, tol, flags, tmp_path, monkeypatch):
    import torch
    monkeypatch.setenv("SUBAP_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    csne = refine < 0
    refine = abs(refine)
    header(f"plan prec={prec} refine={refine} csne={csne} flags={flags}")
    models = _models(uneven_small)
    try:
        params = [to_dev(w["test_params"]) for w, _, _ in uneven_small]
        ys = [torch.full((w["m"], w["r"]), -7.0, dtype=torch.float64, device=params[0].device)
              for w, _, _ in uneven_small]
        sts = [torch.full((w["m"],), -1, dtype=torch.int32, device=params[0].device) for w, _, _ in uneven_small]
        plan = B.subap_plan_create([M.handle for M in models], params, ys, None, sts, prec, refine, flags,
                                   csne=csne)
        try:
            for rep in range(3):  # replays with eager work between them
                for y in ys:
                    y.fill_(-7.0)
                B.subap_plan_execute(plan)
                torch.cuda.synchronize()
                for (w, off, yo), y, st in zip(uneven_small, ys, sts):
                    assert np.all(st.cpu().numpy() == B.OK)
                    yg = y.cpu().numpy()
                    d = max(On.delta_res(off["family"], off["Q"], p, a, b)
                            for p, a, b in zip(w["test_params"], yg, yo))
                    assert d <= tol, (rep, w["r"], w["s"], d)
            t, b = B.subap_plan_shape(plan)
            assert t in (64, 128, 256) and b > 0
        finally:
            B.subap_plan_free(plan)
    finally:
        for M in models:
            M.free()


def test_plan_equals_single_model_solves(uneven_small):
    import torch
    header("plan vs per-model batch solves")
    models = _models(uneven_small)
    try:
        params = [to_dev(w["test_params"]) for w, _, _ in uneven_small]
        ys = [torch.empty((w["m"], w["r"]), dtype=torch.float64, device=params[0].device)
              for w, _, _ in uneven_small]
        B.subap_solve_multi([M.handle for M in models], params, ys)
        for (w, off, _), M, P, y in zip(uneven_small, models, params, ys):
            y1, _, _ = M.solve(P)
            assert np.abs(y1.cpu().numpy() - y.cpu().numpy()).max() <= 1e-9 * np.abs(y1.cpu().numpy()).max()
    finally:
        for M in models:
            M.free()


def test_autotune_cache_is_reused(uneven_small, tmp_path, monkeypatch):
    import torch
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SUBAP_AUTOTUNE_CACHE", str(cache))
    header("autotune cache")
    models = _models(uneven_small)
    try:
        params = [to_dev(w["test_params"]) for w, _, _ in uneven_small]
        ys = [torch.empty((w["m"], w["r"]), dtype=torch.float64, device=params[0].device)
              for w, _, _ in uneven_small]
        p1 = B.subap_plan_create([M.handle for M in models], params, ys, flags=B.PLAN_AUTOTUNE)
        shape1 = B.subap_plan_shape(p1)
        B.subap_plan_free(p1)
        lines = cache.read_text().strip().splitlines()
        assert len(lines) == 1 and lines[0].startswith("fd_multi/")
        p2 = B.subap_plan_create([M.handle for M in models], params, ys, flags=B.PLAN_AUTOTUNE)
        assert B.subap_plan_shape(p2) == shape1
        B.subap_plan_free(p2)
        assert len(cache.read_text().strip().splitlines()) == 1  # looked up, not re-tuned
    finally:
        for M in models:
            M.free()


@pytest.mark.parametrize("prec,refine", [(B.FP64, 0), (B.FP32, 1)])
def test_plan_with_fewer_blocks_than_xcd_groups(uneven_small, prec, refine, tmp_path, monkeypatch):
    """The instances are split into eight groups, one per XCD (block id mod
    8), and a wavefront takes items from its own group first, then from the
    others.  With three blocks, five groups have no block of their own and are
    solved only by taking items from them: every output must still equal the
    default launch's, bit for bit (the same kernel and per-item arithmetic).
    The shape is forced through the autotune cache."""
    import torch
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("SUBAP_AUTOTUNE_CACHE", str(cache))
    header(f"plan on 3 blocks prec={prec} refine={refine}")
    models = _models(uneven_small)
    try:
        params = [to_dev(w["test_params"]) for w, _, _ in uneven_small]
        dev = params[0].device
        ref = [torch.full((w["m"], w["r"]), -7.0, dtype=torch.float64, device=dev) for w, _, _ in uneven_small]
        p1 = B.subap_plan_create([M.handle for M in models], params, ref, contraction=prec, refine_steps=refine,
                                 flags=B.PLAN_AUTOTUNE)
        B.subap_plan_execute(p1)
        torch.cuda.synchronize()
        B.subap_plan_free(p1)
        key = cache.read_text().split()[0]
        cache.write_text(f"{key} 64 3\n")
        ys = [torch.full((w["m"], w["r"]), -7.0, dtype=torch.float64, device=dev) for w, _, _ in uneven_small]
        p2 = B.subap_plan_create([M.handle for M in models], params, ys, contraction=prec, refine_steps=refine,
                                 flags=B.PLAN_AUTOTUNE)
        try:
            assert B.subap_plan_shape(p2) == (64, 3)
            B.subap_plan_execute(p2)
            torch.cuda.synchronize()
        finally:
            B.subap_plan_free(p2)
        for a, b in zip(ys, ref):
            assert torch.equal(a, b)
    finally:
        for M in models:
            M.free()


@pytest.mark.parametrize("prec,refine,csne", [(B.FP64, 0, False), (B.FP32, 1, True)])
def test_plan_with_every_family(uneven_small, prec, refine, csne):
    """A plan holding two diffusion models with a kernel-family model, the
    delay system, eq. (5.7), the identity family and an affine family,
    captured in one hipGraph
    and replayed three times with eager work between the replays.  Every other
    member equals subap_solve_batch with the same options bit for bit (its
    family's solver, the plan's workspace); the diffusion members stay within
    delta_res 1e-12 (FP64) or 1e-6 (FP32 + one CSNE step) of the oracle."""
    import torch
    header(f"plan with every family prec={prec} refine={refine} csne={csne}")
    dev = device()
    ws = [si.krr(n=1024, r=8, s=24, m=40), si.delay(n=3000, r=10, s=40, m=33), si.tridiag(m=50),
          si.identity(m=20), si.affine(N=16, r=6, s=18, m=24)]
    others = [B.Model(w, basis=O.offline(w)["Q"]) for w in ws]
    diff = uneven_small[:2]
    dmodels = [B.Model(w, basis=off["Q"], rows=off["rows"]) for w, off, _ in diff]
    try:
        models = dmodels + others
        allw = [w for w, _, _ in diff] + ws
        params = [to_dev(w["test_params"]) for w in allw]
        ys = [torch.full((w["m"], w["r"]), -7.0, dtype=torch.float64, device=dev) for w in allw]
        sts = [torch.full((w["m"],), -1, dtype=torch.int32, device=dev) for w in allw]
        plan = B.subap_plan_create([M.handle for M in models], params, ys, None, sts, prec, refine,
                                   B.PLAN_GRAPH, csne=csne)
        try:
            refs = []
            for M, P in zip(others, params[2:]):
                y1, _, st1 = M.solve(P, contraction=prec, refine_steps=refine, csne=csne)
                refs.append((y1, st1))
            for rep in range(3):
                for y in ys:
                    y.fill_(-7.0)
                B.subap_plan_execute(plan)
                torch.cuda.synchronize()
                for (y1, st1), y, st in zip(refs, ys[2:], sts[2:]):
                    assert torch.equal(y, y1) and torch.equal(st, st1)
                tol = 1e-12 if prec == B.FP64 else 1e-6
                for (w, off, yo), y, st in zip(diff, ys[:2], sts[:2]):
                    assert np.all(st.cpu().numpy() == B.OK)
                    d = max(On.delta_res(off["family"], off["Q"], p, a, b)
                            for p, a, b in zip(w["test_params"], y.cpu().numpy(), yo))
                    assert d <= tol, d
                torch.zeros(1 << 20, device=dev).sum()  # eager work between replays
        finally:
            B.subap_plan_free(plan)
    finally:
        for M in dmodels + others:
            M.free()


@pytest.fixture(scope="module")
def cubes_small():
    # 3-D models for plans that hold 3-D instances only or mix them with 2-D ones
    out = []
    for N, r, s, m in ((8, 8, 24, 32), (10, 64, 160, 16)):
        w = si.diffusion3d(N=N, r=r, s=s, m=m, seed=500 + N)
        off = O.offline(w)
        out.append((w, off, On.solve(off["family"], off["Q"], off["rows"], w["test_params"])))
    return out


@pytest.mark.parametrize("mix", ["3d_only", "2d_and_3d"])
@pytest.mark.parametrize("prec,refine,tol", [(B.FP64, 0, 1e-12), (B.FP32, 1, 1e-6)])
def test_plan_with_3d_models(uneven_small, cubes_small, mix, prec, refine, tol, tmp_path, monkeypatch):
    import torch
    monkeypatch.setenv("SUBAP_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    header(f"plan {mix} prec={prec} refine={refine}")
    cases = list(cubes_small) + (list(uneven_small[:3]) if mix == "2d_and_3d" else [])
    device()
    models = [B.Model(w, basis=off["Q"], rows=off["rows"]) for w, off, _ in cases]
    try:
        params = [to_dev(w["test_params"]) for w, _, _ in cases]
        ys = [torch.full((w["m"], w["r"]), -7.0, dtype=torch.float64, device=params[0].device) for w, _, _ in cases]
        sts = [torch.full((w["m"],), -1, dtype=torch.int32, device=params[0].device) for w, _, _ in cases]
        plan = B.subap_plan_create([M.handle for M in models], params, ys, None, sts, prec, refine,
                                   B.PLAN_GRAPH | B.PLAN_AUTOTUNE)
        try:
            B.subap_plan_execute(plan)
            torch.cuda.synchronize()
            for (w, off, yo), y, st in zip(cases, ys, sts):
                assert np.all(st.cpu().numpy() == B.OK)
                d = max(On.delta_res(off["family"], off["Q"], p, a, b)
                        for p, a, b in zip(w["test_params"], y.cpu().numpy(), yo))
                assert d <= tol, (mix, w["family"], w["r"], w["s"], d)
        finally:
            B.subap_plan_free(plan)
    finally:
        for M in models:
            M.free()


@pytest.mark.slow
def test_uneven_full_size_sampled(tmp_path, monkeypatch):
    """The benchmark's uneven batch: all 64 instances (grids 32^2..512^2,
    r in {8, 16, 32, 64}) in one persistent, autotuned, graph-replayed launch,
    in both forms the benchmark times (FP64 without refinement, and FP32
    contraction + one FP64 refinement), with oracle-made orthonormal bases and
    seeded rows.  Two sampled parameters per instance are recomputed by the
    oracle.  Bars on the sketched distance: FP64 1e-12 plus the backward-error
    term 2^-46 kappa(S A Q) rho*; FP32 + refinement 1e-6 plus the
    simple-refinement bias bound 2^-20 kappa(S A Q) rho* (rho* is of order one
    for a random basis)."""
    import torch
    from oracle import families as Fm
    monkeypatch.setenv("SUBAP_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    insts = si.uneven()
    header("uneven full size")
    rng = np.random.default_rng(2027)
    device()
    models, bases, rowsets = [], [], []
    try:
        for w in insts:
            Q, _ = O.orthonormalise(rng.standard_normal((w["n"], w["r"])))
            rows = np.sort(rng.choice(w["n"], size=w["s"], replace=False))
            bases.append(Q)
            rowsets.append(rows)
            models.append(B.Model(w, basis=Q, rows=rows))
        params = [to_dev(w["test_params"]) for w in insts]
        ys = [torch.empty((w["m"], w["r"]), dtype=torch.float64, device=params[0].device) for w in insts]
        sts = [torch.empty(w["m"], dtype=torch.int32, device=params[0].device) for w in insts]
        picks = [rng.choice(w["m"], size=min(2, w["m"]), replace=False) for w in insts]
        forms = ((B.FP64, 0, False, 1e-12, 2.0 ** -46), (B.FP32, 1, False, 1e-6, 2.0 ** -20),
                 (B.FP32, 1, True, 1e-6, None))
        for prec, refine, csne, base, scale in forms:
            header(f"uneven full size prec={prec} refine={refine} csne={csne}")
            plan = B.subap_plan_create([M.handle for M in models], params, ys, None, sts, prec, refine,
                                       B.PLAN_GRAPH | B.PLAN_AUTOTUNE, csne=csne)
            try:
                B.subap_plan_execute(plan)
                torch.cuda.synchronize()
            finally:
                B.subap_plan_free(plan)
            for w, Q, rows, y, st, pick in zip(insts, bases, rowsets, ys, sts, picks):
                assert np.all(st.cpu().numpy() == B.OK)
                fam = Fm.from_workload(w)
                yg = y.cpu().numpy()
                for i in pick:
                    p = w["test_params"][i]
                    G = On.reduced_matrix(fam, Q, rows, p)
                    bS = fam.rhs_rows(p, rows)
                    yo, _, rho = On.householder_lsq(G, bS)
                    if scale is None:
                        # corrected semi-normal equations: flat bar on delta_res over all n rows
                        d = On.delta_res(fam, Q, p, yg[i], yo)
                        assert d <= base, (prec, w["n"], w["r"], w["s"], i, d)
                        continue
                    sv = np.linalg.svd(G, compute_uv=False)
                    tol = base + scale * sv[0] / sv[-1] * rho / np.linalg.norm(bS)
                    d = np.linalg.norm(G @ (yg[i] - yo)) / np.linalg.norm(bS)
                    assert d <= tol, (prec, w["n"], w["r"], w["s"], i, d, tol)
    finally:
        for M in models:
            M.free()


@pytest.fixture(scope="module")
def tall_small():
    # diffusion models whose FP64 form without refinement the matrix-core
    # semi-normal solve takes (s >= 96, 16 <= r <= 47): a 3-D one with 16
    # parameters per CU (a plan routes it to that solve; the oracle checks
    # every 16th parameter) and a 2-D one with 21 (it stays in the
    # persistent launch)
    import torch
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = []
    for w, step in ((si.diffusion3d(N=12, r=20, s=100, m=16 * cus, seed=710), 16),
                    (si.diffusion2d(N=24, r=24, s=104, m=21, seed=711), 1)):
        off = O.offline(w)
        sample = np.arange(0, w["m"], step)
        out.append((w, off, sample, On.solve(off["family"], off["Q"], off["rows"], w["test_params"][sample])))
    return out


def _check_oracle(w, off, sample, yo, y, tol):
    yg = y.cpu().numpy()
    d = max(On.delta_res(off["family"], off["Q"], w["test_params"][j], yg[j], b) for j, b in zip(sample, yo))
    assert d <= tol, (w["r"], w["s"], d)


@pytest.mark.parametrize("prec,refine,tol", [(B.FP64, 0, 1e-12), (B.FP32, 1, 1e-6)])
def test_plan_gives_tall_members_to_the_matrix_core_solve(uneven_small, tall_small, prec, refine, tol):
    """A graph-captured plan of a large tall model, a small tall model and one
    other diffusion member.  In FP64 without refinement the large tall model
    leaves the persistent launch for the matrix-core semi-normal solve: it
    equals subap_solve_batch bit for bit, on three replays with eager work
    between them.  Every member is held to the oracle (the large one on every
    16th parameter); in the refined form all stay in the persistent launch."""
    import torch
    header(f"plan with tall members prec={prec} refine={refine}")
    dev = device()
    w0, off0, yo0 = uneven_small[0]
    cases = list(tall_small) + [(w0, off0, np.arange(w0["m"]), yo0)]
    models = [B.Model(w, basis=off["Q"], rows=off["rows"]) for w, off, _, _ in cases]
    try:
        params = [to_dev(w["test_params"]) for w, _, _, _ in cases]
        ys = [torch.full((w["m"], w["r"]), -7.0, dtype=torch.float64, device=dev) for w, _, _, _ in cases]
        sts = [torch.full((w["m"],), -1, dtype=torch.int32, device=dev) for w, _, _, _ in cases]
        plan = B.subap_plan_create([M.handle for M in models], params, ys, None, sts, prec, refine, B.PLAN_GRAPH)
        try:
            y1, _, st1 = models[0].solve(params[0], contraction=prec, refine_steps=refine)
            for rep in range(3):
                for y in ys:
                    y.fill_(-7.0)
                B.subap_plan_execute(plan)
                torch.cuda.synchronize()
                for (w, off, sample, yo), y, st in zip(cases, ys, sts):
                    assert np.all(st.cpu().numpy() == B.OK)
                    _check_oracle(w, off, sample, yo, y, tol)
                if prec == B.FP64:
                    assert torch.equal(ys[0], y1) and torch.equal(sts[0], st1)
                torch.zeros(1 << 20, device=dev).sum()  # eager work between replays
        finally:
            B.subap_plan_free(plan)
        if prec == B.FP64:
            # a plan of the large tall model alone has no persistent launch
            plan = B.subap_plan_create([models[0].handle], params[:1], ys[:1], None, sts[:1], prec, refine,
                                       B.PLAN_GRAPH)
            try:
                ys[0].fill_(-7.0)
                B.subap_plan_execute(plan)
                torch.cuda.synchronize()
                assert B.subap_plan_shape(plan)[1] == 0
                assert torch.equal(ys[0], y1)
            finally:
                B.subap_plan_free(plan)
    finally:
        for M in models:
            M.free()
