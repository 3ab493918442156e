"""ctypes binding of libsubap.so (include/subap.h).

Argument marshalling only: every step of SubApSnap runs inside the HIP
library.  Device buffers are torch tensors on the GPU (their data pointers
are passed through); the HIP stream is torch's current stream unless one is
given.  Functions keep the C names; ``Model`` is a small owner of a
``subap_model`` handle built from a ``subap_inputs`` workload dict.

Loading fails loudly if the library has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsubap.so")

# subap_status
OK, E_INVALID, E_NOMEM, E_HIP, E_RANK, E_NOCONV, E_NONFINITE, E_UNSUPPORTED = range(8)
# subap_family
FAMILY_DIFF2D, FAMILY_DIFF3D, FAMILY_KRR, FAMILY_DELAY, FAMILY_TRIDIAG_SHIFT, FAMILY_IDENTITY = 1, 2, 3, 4, 5, 6
FAMILY_AFFINE = 7
# subap_precision
FP64, FP32, BF16X3, FP16X3 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3, "fp16x3": FP16X3}
FAMILIES = {"diff2d": FAMILY_DIFF2D, "diff3d": FAMILY_DIFF3D, "krr": FAMILY_KRR, "delay": FAMILY_DELAY,
            "tridiag": FAMILY_TRIDIAG_SHIFT, "identity": FAMILY_IDENTITY, "affine": FAMILY_AFFINE}

EXPORTS = ("subap_offline", "subap_solve_batch", "subap_lift", "subap_sketched_residual", "subap_model_dims",
           "subap_model_rows", "subap_model_basis", "subap_model_free", "subap_profile_enable",
           "subap_profile_reset", "subap_profile_entry", "subap_plan_create", "subap_plan_execute",
           "subap_plan_shape", "subap_plan_free", "subap_solve_multi", "subap_surrogate_create",
           "subap_surrogate_weights", "subap_surrogate_gradient", "subap_surrogate_train",
           "subap_surrogate_predict", "subap_surrogate_solve_batch", "subap_surrogate_free",
           "subap_surrogate_nparams", "subap_profile_count", "subap_status_string", "subap_last_error",
           "subap_model_weights", "subap_residual_bounds", "subap_output", "subap_full_residual",
           "subap_apsnap_solve", "subap_polish", "subap_model_save", "subap_model_load",
           "subap_delta_residual", "subap_solve_batch_noalloc", "subap_excess_bound", "subap_reduced_matrix",
           "subap_surrogate_solve_batch_excess", "subap_exp2_rate")
PLAN_GRAPH, PLAN_AUTOTUNE = 1, 2
# subap_selection
SELECT_CPQR, SELECT_LEVERAGE, SELECT_LU = 0, 1, 2


class ProblemDesc(C.Structure):
    _fields_ = [("family", C.c_int32), ("grid", C.c_int32), ("n", C.c_int64), ("dim", C.c_int32),
                ("points", C.c_void_p), ("rhs", C.c_void_p), ("lam", C.c_double), ("tau", C.c_double),
                ("kappa", C.c_double), ("c_out", C.c_void_p), ("nterms", C.c_int32),
                ("term_rowptr", C.c_void_p), ("term_cols", C.c_void_p), ("term_vals", C.c_void_p)]


class OfflineOpts(C.Structure):
    _fields_ = [("r", C.c_int32), ("s", C.c_int32), ("snap_params", C.c_void_p),
                ("select_param", C.c_void_p), ("snap_tol", C.c_double), ("snap_maxiter", C.c_int32),
                ("basis_in", C.c_void_p), ("rows_in", C.c_void_p), ("selection", C.c_int32),
                ("sample_u", C.c_void_p), ("n_select", C.c_int32), ("select_params", C.c_void_p)]


class SolveOpts(C.Structure):
    _fields_ = [("contraction", C.c_int32), ("refine_steps", C.c_int32), ("refine_csne", C.c_int32)]


class TrainOpts(C.Structure):
    _fields_ = [("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_double), ("lr_min", C.c_double),
                ("seed", C.c_uint64)]


class SubapError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"subap error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load libsubap.so once and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(python -m paper_2510_04825_amd.build); there is no CPU fallback")
    # torch's HIP context first: device memory and streams come from torch,
    # and the library's first runtime call must not precede its initialisation
    import torch
    if torch.cuda.is_available():
        torch.cuda.init()
    lib = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    lib.subap_offline.argtypes = [C.POINTER(ProblemDesc), C.POINTER(OfflineOpts), vp, C.POINTER(vp)]
    lib.subap_solve_batch.argtypes = [vp, vp, i64, vp, vp, vp, C.POINTER(SolveOpts), vp]
    lib.subap_solve_batch_noalloc.argtypes = [vp, vp, i64, vp, vp, vp, C.POINTER(SolveOpts), vp]
    lib.subap_lift.argtypes = [vp, vp, i64, vp, i64, i32, vp]
    lib.subap_sketched_residual.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    lib.subap_profile_enable.argtypes = [i32]
    lib.subap_profile_reset.argtypes = []
    lib.subap_profile_count.argtypes = []
    lib.subap_profile_count.restype = i32
    lib.subap_profile_entry.argtypes = [i32, C.POINTER(C.c_char_p), C.POINTER(i64), C.POINTER(C.c_double)]
    lib.subap_model_dims.argtypes = [vp, C.POINTER(i64), C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)]
    lib.subap_model_rows.argtypes = [vp, vp]
    lib.subap_model_weights.argtypes = [vp, vp]
    lib.subap_model_save.argtypes = [vp, C.c_char_p]
    lib.subap_model_load.argtypes = [C.c_char_p, vp, C.POINTER(vp)]
    lib.subap_output.argtypes = [vp, vp, i64, vp, vp]
    lib.subap_full_residual.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.subap_delta_residual.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    lib.subap_excess_bound.argtypes = [vp, vp, i64, vp, C.c_double, vp, vp]
    lib.subap_reduced_matrix.argtypes = [vp, vp, i64, vp, vp]
    lib.subap_apsnap_solve.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.subap_polish.argtypes = [vp, vp, i64, vp, i32, C.c_double, vp, vp]
    lib.subap_residual_bounds.argtypes = [vp, vp, i64, C.c_double, vp, vp, vp]
    lib.subap_model_basis.argtypes = [vp, vp]
    lib.subap_model_free.argtypes = [vp]
    pp = C.POINTER(vp)
    lib.subap_plan_create.argtypes = [pp, i32, pp, C.POINTER(i64), pp, pp, pp, C.POINTER(SolveOpts), i32, vp,
                                      C.POINTER(vp)]
    lib.subap_plan_execute.argtypes = [vp, vp]
    lib.subap_plan_shape.argtypes = [vp, C.POINTER(i32), C.POINTER(i32)]
    lib.subap_plan_free.argtypes = [vp]
    lib.subap_solve_multi.argtypes = [pp, i32, pp, C.POINTER(i64), pp, pp, pp, C.POINTER(SolveOpts), vp]
    dp = C.POINTER(C.c_double)
    lib.subap_surrogate_create.argtypes = [i32, i32, i32, vp, C.POINTER(vp)]
    lib.subap_surrogate_nparams.argtypes = [vp]
    lib.subap_surrogate_nparams.restype = i64
    lib.subap_surrogate_weights.argtypes = [vp, vp]
    lib.subap_surrogate_gradient.argtypes = [vp, vp, vp, i64, vp, dp, vp]
    lib.subap_surrogate_train.argtypes = [vp, vp, vp, i64, C.POINTER(TrainOpts), vp, vp]
    lib.subap_surrogate_predict.argtypes = [vp, vp, i64, vp, vp]
    lib.subap_surrogate_solve_batch.argtypes = [vp, vp, vp, i64, C.c_double, vp, vp, vp, C.POINTER(SolveOpts),
                                                C.POINTER(i64), vp]
    lib.subap_surrogate_solve_batch_excess.argtypes = [vp, vp, vp, i64, C.c_double, C.c_double, vp, vp, vp,
                                                       C.POINTER(SolveOpts), C.POINTER(i64), vp]
    lib.subap_exp2_rate.argtypes = [i32, i64, C.POINTER(C.c_double), vp]
    lib.subap_surrogate_free.argtypes = [vp]
    for name in EXPORTS[:23]:
        getattr(lib, name).restype = C.c_int
    lib.subap_status_string.argtypes = [C.c_int]
    lib.subap_status_string.restype = C.c_char_p
    lib.subap_last_error.argtypes = []
    lib.subap_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _check(rc: int):
    if rc != OK:
        lib = load()
        raise SubapError(rc, f"{lib.subap_status_string(rc).decode()}: {lib.subap_last_error().decode()}")


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _expect(t, shape, dtype, name):
    """Host-side check that a device tensor has the layout the kernels assume."""
    if tuple(t.shape) != tuple(shape) or str(t.dtype) != f"torch.{dtype}" or not t.is_contiguous() \
            or not t.is_cuda:
        raise ValueError(f"{name}: expected a contiguous cuda {dtype} tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


def _host(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
# C entry points
# ---------------------------------------------------------------------------
def subap_offline(family, grid=0, n=0, dim=0, points=None, rhs=None, lam=0.0, r=1, s=1,
                  snap_params=None, select_param=None, snap_tol=0.0, snap_maxiter=0,
                  basis_in=None, rows_in=None, sample_u=None, tau=0.0, kappa=0.0, c_out=None, selection=None,
                  select_params=None, stream=None, terms=None):
    """Run the offline phase; returns the opaque model handle (int).  With
    sample_u (s uniforms in [0, 1)) the rows come from leverage-score sampling;
    selection SELECT_LU picks rows by LU with partial pivoting; select_params
    (t x d, t > 1) takes the union of the r pivots at each point.  terms
    (affine family): the sparse matrices A_q (anything with indptr, indices
    and data in CSR form)."""
    lib = load()
    keep = [_host(points, np.float64), _host(rhs, np.float64), _host(snap_params, np.float64),
            _host(select_param, np.float64), _host(basis_in, np.float64), _host(rows_in, np.int64),
            _host(sample_u, np.float64), _host(c_out, np.float64), _host(select_params, np.float64)]
    addr = [None if a is None else a.ctypes.data for a in keep]
    pd = ProblemDesc(family, grid, n, dim, addr[0], addr[1], lam, tau, kappa, addr[7])
    if terms is not None:
        csr = [(np.ascontiguousarray(T.indptr, dtype=np.int64), np.ascontiguousarray(T.indices, dtype=np.int32),
                np.ascontiguousarray(T.data, dtype=np.float64)) for T in terms]
        keep.append(csr)
        ptrs = [(C.c_void_p * len(csr))(*[c[i].ctypes.data for c in csr]) for i in range(3)]
        keep.append(ptrs)
        pd.nterms = len(csr)
        pd.term_rowptr, pd.term_cols, pd.term_vals = (C.cast(a, C.c_void_p).value for a in ptrs)
    if selection is None:
        selection = SELECT_LEVERAGE if sample_u is not None else SELECT_CPQR
    nsel = 0 if select_params is None else int(np.atleast_2d(select_params).shape[0])
    op = OfflineOpts(r, s, addr[2], addr[3], snap_tol, snap_maxiter, addr[4], addr[5], selection, addr[6], nsel,
                     addr[8])
    h = C.c_void_p()
    _check(lib.subap_offline(C.byref(pd), C.byref(op), _stream(stream), C.byref(h)))
    return h.value


def subap_solve_batch(model, params, y, rho=None, status=None, contraction=FP64, refine_steps=0,
                      stream=None, csne=False):
    """params: (m, d) float64 cuda tensor; y: (m, r) float64; rho: (m,) float64; status: (m,) int32."""
    lib = load()
    m = params.shape[0]
    _, r, _, d = subap_model_dims(model)
    _expect(params, (m, d), "float64", "params")
    _expect(y, (m, r), "float64", "y")
    if rho is not None:
        _expect(rho, (m,), "float64", "rho")
    if status is not None:
        _expect(status, (m,), "int32", "status")
    opts = SolveOpts(int(contraction), int(refine_steps), int(bool(csne)))
    _check(lib.subap_solve_batch(C.c_void_p(model), _ptr(params), m, _ptr(y), _ptr(rho), _ptr(status),
                                 C.byref(opts), _stream(stream)))


def subap_solve_batch_noalloc(model, params, y, rho=None, status=None, contraction=FP64, refine_steps=0,
                              stream=None, csne=False):
    """subap_solve_batch with the library's fixed device scratch instead of allocations."""
    lib = load()
    m = params.shape[0]
    _, r, _, d = subap_model_dims(model)
    _expect(params, (m, d), "float64", "params")
    _expect(y, (m, r), "float64", "y")
    if rho is not None:
        _expect(rho, (m,), "float64", "rho")
    if status is not None:
        _expect(status, (m,), "int32", "status")
    opts = SolveOpts(int(contraction), int(refine_steps), int(bool(csne)))
    _check(lib.subap_solve_batch_noalloc(C.c_void_p(model), _ptr(params), m, _ptr(y), _ptr(rho), _ptr(status),
                                         C.byref(opts), _stream(stream)))


def subap_lift(model, y, x, precision=FP64, stream=None):
    """y: (k, r) float64 cuda tensor; x: (k, ldx) tensor with ldx >= n, float64 or
    float32 (row i of x holds column i of the lift in its first n entries)."""
    lib = load()
    n, r, _, _ = subap_model_dims(model)
    k = y.shape[0]
    _expect(y, (k, r), "float64", "y")
    dt = "float64" if precision == FP64 else "float32"
    if x.dim() != 2 or x.shape[0] != k or x.shape[1] < n or not x.is_contiguous() or str(x.dtype) != "torch." + dt \
            or not x.is_cuda:
        raise ValueError(f"x must be a contiguous {dt} cuda tensor of shape ({k}, >= {n}), got "
                         f"{tuple(x.shape)} {x.dtype}")
    _check(lib.subap_lift(C.c_void_p(model), _ptr(y), k, _ptr(x), int(x.shape[1]), int(precision), _stream(stream)))


def subap_sketched_residual(model, params, y, res=None, norm=None, stream=None):
    """FP64 sketched residual of coefficients y: res (m, s) and/or norm (m,) float64 cuda tensors."""
    lib = load()
    m = params.shape[0]
    _, r, s, d = subap_model_dims(model)
    _expect(params, (m, d), "float64", "params")
    _expect(y, (m, r), "float64", "y")
    if res is not None:
        _expect(res, (m, s), "float64", "res")
    if norm is not None:
        _expect(norm, (m,), "float64", "norm")
    _check(lib.subap_sketched_residual(C.c_void_p(model), _ptr(params), m, _ptr(y), _ptr(res), _ptr(norm),
                                       _stream(stream)))


def subap_profile_enable(on=True):
    _check(load().subap_profile_enable(1 if on else 0))


def subap_profile_reset():
    _check(load().subap_profile_reset())


def subap_profile_read():
    """{kernel name: (launches, total ms)} recorded since the last reset."""
    lib = load()
    out = {}
    for i in range(lib.subap_profile_count()):
        name, calls, ms = C.c_char_p(), C.c_int64(), C.c_double()
        _check(lib.subap_profile_entry(i, C.byref(name), C.byref(calls), C.byref(ms)))
        out[name.value.decode()] = (calls.value, ms.value)
    return out


def _ptr_array(items):
    arr = (C.c_void_p * len(items))()
    for i, t in enumerate(items):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def _multi_args(models, params, ys, rhos, statuses):
    k = len(models)
    for mdl, p, y in zip(models, params, ys):
        _, r, _, d = subap_model_dims(mdl)
        m = p.shape[0]
        _expect(p, (m, d), "float64", "params")
        _expect(y, (m, r), "float64", "y")
    for lst, dt in ((rhos, "float64"), (statuses, "int32")):
        if lst is not None:
            for t, p in zip(lst, params):
                if t is not None:
                    _expect(t, (p.shape[0],), dt, "rho/status")
    hm = (C.c_void_p * k)(*models)
    mm = (C.c_int64 * k)(*[p.shape[0] for p in params])
    return (hm, k, _ptr_array(params), mm, _ptr_array(ys),
            _ptr_array(rhos) if rhos is not None else None,
            _ptr_array(statuses) if statuses is not None else None)


def subap_plan_create(models, params, ys, rhos=None, statuses=None, contraction=FP64, refine_steps=0,
                      flags=0, stream=None, csne=False):
    """Plan over model handles with per-model (m, d) params and (m, r) outputs; returns the handle."""
    lib = load()
    a = _multi_args(models, params, ys, rhos, statuses)
    opts = SolveOpts(int(contraction), int(refine_steps), int(bool(csne)))
    h = C.c_void_p()
    _check(lib.subap_plan_create(*a, C.byref(opts), int(flags), _stream(stream), C.byref(h)))
    return h.value


def subap_plan_execute(plan, stream=None):
    _check(load().subap_plan_execute(C.c_void_p(plan), _stream(stream)))


def subap_plan_shape(plan):
    t, b = C.c_int32(), C.c_int32()
    _check(load().subap_plan_shape(C.c_void_p(plan), C.byref(t), C.byref(b)))
    return t.value, b.value


def subap_plan_free(plan):
    _check(load().subap_plan_free(C.c_void_p(plan)))


def subap_solve_multi(models, params, ys, rhos=None, statuses=None, contraction=FP64, refine_steps=0,
                      stream=None, csne=False):
    lib = load()
    a = _multi_args(models, params, ys, rhos, statuses)
    opts = SolveOpts(int(contraction), int(refine_steps), int(bool(csne)))
    _check(lib.subap_solve_multi(*a, C.byref(opts), _stream(stream)))


def flatten_mlp(params):
    """[(W1, b1), (W2, b2), (W3, b3)] -> the library's flat FP64 weight vector."""
    return np.concatenate([a.ravel() for W, b in params for a in (W, b)]).astype(np.float64)


def unflatten_mlp(flat, widths):
    out, o = [], 0
    for fi, fo in zip(widths[:-1], widths[1:]):
        W = flat[o:o + fo * fi].reshape(fo, fi)
        o += fo * fi
        b = flat[o:o + fo]
        o += fo
        out.append((W, b))
    return out


def subap_surrogate_create(d, r, hidden, weights):
    w = np.ascontiguousarray(weights, dtype=np.float64)
    if w.size != hidden * d + hidden + hidden * hidden + hidden + r * hidden + r:
        raise ValueError("weights length does not match (d, hidden, r)")
    h = C.c_void_p()
    _check(load().subap_surrogate_create(d, r, hidden, w.ctypes.data, C.byref(h)))
    return h.value


def subap_surrogate_nparams(s):
    return int(load().subap_surrogate_nparams(C.c_void_p(s)))


def subap_surrogate_weights(s):
    out = np.empty(subap_surrogate_nparams(s), dtype=np.float64)
    _check(load().subap_surrogate_weights(C.c_void_p(s), out.ctypes.data))
    return out


def subap_surrogate_gradient(s, params, targets, stream=None):
    """(grad (nparams,), loss) for standardised targets (m, r) on device."""
    g = np.empty(subap_surrogate_nparams(s), dtype=np.float64)
    loss = C.c_double()
    _check(load().subap_surrogate_gradient(C.c_void_p(s), _ptr(params), _ptr(targets), params.shape[0],
                                           g.ctypes.data, C.byref(loss), _stream(stream)))
    return g, loss.value


def subap_surrogate_train(s, params, y, epochs, batch=0, lr=0.0, lr_min=0.0, seed=0, stream=None):
    losses = np.zeros(epochs)
    o = TrainOpts(int(epochs), int(batch), float(lr), float(lr_min), int(seed))
    _check(load().subap_surrogate_train(C.c_void_p(s), _ptr(params), _ptr(y), params.shape[0], C.byref(o),
                                        losses.ctypes.data, _stream(stream)))
    return losses


def subap_surrogate_predict(s, params, y, stream=None):
    _check(load().subap_surrogate_predict(C.c_void_p(s), _ptr(params), params.shape[0], _ptr(y), _stream(stream)))


def subap_surrogate_solve_batch(model, s, params, accept_tol, y, accepted=None, status=None, contraction=FP64,
                                refine_steps=0, stream=None, csne=False):
    """Returns the number of accepted predictions."""
    _, r, _, d = subap_model_dims(model)
    m = params.shape[0]
    _expect(params, (m, d), "float64", "params")
    _expect(y, (m, r), "float64", "y")
    if accepted is not None:
        _expect(accepted, (m,), "uint8", "accepted")
    if status is not None:
        _expect(status, (m,), "int32", "status")
    opts = SolveOpts(int(contraction), int(refine_steps), int(bool(csne)))
    n = C.c_int64()
    _check(load().subap_surrogate_solve_batch(C.c_void_p(model), C.c_void_p(s), _ptr(params), m, float(accept_tol),
                                              _ptr(y), _ptr(accepted), _ptr(status), C.byref(opts), C.byref(n),
                                              _stream(stream)))
    return n.value


def subap_surrogate_solve_batch_excess(model, s, params, sigma_min, accept_tol, y, accepted=None, status=None,
                                       contraction=FP64, refine_steps=0, stream=None, csne=False):
    """Acceptance by the normal-equation excess bound; returns the number of accepted predictions."""
    _, r, _, d = subap_model_dims(model)
    m = params.shape[0]
    _expect(params, (m, d), "float64", "params")
    _expect(y, (m, r), "float64", "y")
    if accepted is not None:
        _expect(accepted, (m,), "uint8", "accepted")
    if status is not None:
        _expect(status, (m,), "int32", "status")
    opts = SolveOpts(int(contraction), int(refine_steps), int(bool(csne)))
    n = C.c_int64()
    _check(load().subap_surrogate_solve_batch_excess(C.c_void_p(model), C.c_void_p(s), _ptr(params), m,
                                                     float(sigma_min), float(accept_tol), _ptr(y), _ptr(accepted),
                                                     _ptr(status), C.byref(opts), C.byref(n), _stream(stream)))
    return n.value


def subap_exp2_rate(form, evals=1 << 34, stream=None):
    """2^(c d) evaluations per second on the device (form 7/9/11: FP64 polynomial degree; 0: v_exp_f32)."""
    rate = C.c_double()
    _check(load().subap_exp2_rate(int(form), int(evals), C.byref(rate), _stream(stream)))
    return rate.value


def subap_surrogate_free(s):
    _check(load().subap_surrogate_free(C.c_void_p(s)))


def subap_model_dims(model):
    lib = load()
    n, r, s, d = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
    _check(lib.subap_model_dims(C.c_void_p(model), C.byref(n), C.byref(r), C.byref(s), C.byref(d)))
    return n.value, r.value, s.value, d.value


def subap_model_rows(model):
    lib = load()
    _, _, s, _ = subap_model_dims(model)
    out = np.empty(s, dtype=np.int64)
    _check(lib.subap_model_rows(C.c_void_p(model), out.ctypes.data))
    return out


def subap_full_residual(model, params, x, res, stream=None):
    """params (m, d); x (m, n) float64 cuda tensor, row k = x_k (column-major n x m); res (m,)."""
    n, _, _, d = subap_model_dims(model)
    m = params.shape[0]
    _expect(params, (m, d), "float64", "params")
    _expect(x, (m, n), "float64", "x")
    _expect(res, (m,), "float64", "res")
    _check(load().subap_full_residual(C.c_void_p(model), _ptr(params), m, _ptr(x), _ptr(res), _stream(stream)))


def subap_delta_residual(model, params, y1, y2, res, stream=None):
    """|A(p_k) Q (y1_k - y2_k)| / |b| over all n rows: params (m, d), y1 and y2 (m, r), res (m,)."""
    _, r, _, d = subap_model_dims(model)
    m = params.shape[0]
    _expect(params, (m, d), "float64", "params")
    _expect(y1, (m, r), "float64", "y1")
    _expect(y2, (m, r), "float64", "y2")
    _expect(res, (m,), "float64", "res")
    _check(load().subap_delta_residual(C.c_void_p(model), _ptr(params), m, _ptr(y1), _ptr(y2), _ptr(res),
                                       _stream(stream)))


def subap_excess_bound(model, params, y, sigma_min, out, stream=None):
    """|G^T (G y - S b)| / (sigma_min |S b|) per parameter: params (m, d), y (m, r), out (m,)."""
    _, r, _, d = subap_model_dims(model)
    m = params.shape[0]
    _expect(params, (m, d), "float64", "params")
    _expect(y, (m, r), "float64", "y")
    _expect(out, (m,), "float64", "out")
    _check(load().subap_excess_bound(C.c_void_p(model), _ptr(params), m, _ptr(y), float(sigma_min), _ptr(out),
                                     _stream(stream)))


def subap_reduced_matrix(model, params, G, stream=None):
    """G_k = S A(p_k) Q in FP64: params (m, d), G (m, s, r)."""
    _, r, s, d = subap_model_dims(model)
    m = params.shape[0]
    _expect(params, (m, d), "float64", "params")
    _expect(G, (m, s, r), "float64", "G")
    _check(load().subap_reduced_matrix(C.c_void_p(model), _ptr(params), m, _ptr(G), _stream(stream)))


def subap_apsnap_solve(model, params, y, rho=None, stream=None):
    _, r, _, d = subap_model_dims(model)
    m = params.shape[0]
    _expect(params, (m, d), "float64", "params")
    _expect(y, (m, r), "float64", "y")
    if rho is not None:
        _expect(rho, (m,), "float64", "rho")
    _check(load().subap_apsnap_solve(C.c_void_p(model), _ptr(params), m, _ptr(y), _ptr(rho), _stream(stream)))


def subap_polish(model, params, x, max_iter, tol=0.0, res=None, stream=None):
    """x (m, n) float64 cuda tensor (row k = x_k), overwritten by the CG iterate."""
    n, _, _, d = subap_model_dims(model)
    m = params.shape[0]
    _expect(params, (m, d), "float64", "params")
    _expect(x, (m, n), "float64", "x")
    if res is not None:
        _expect(res, (m,), "float64", "res")
    _check(load().subap_polish(C.c_void_p(model), _ptr(params), m, _ptr(x), int(max_iter), float(tol), _ptr(res),
                               _stream(stream)))


def subap_output(model, y, out, stream=None):
    """y: (m, r) float64 cuda tensor; out: (m,) float64 -> c^T Q y per row."""
    m = y.shape[0]
    _, r, _, _ = subap_model_dims(model)
    _expect(y, (m, r), "float64", "y")
    _expect(out, (m,), "float64", "out")
    _check(load().subap_output(C.c_void_p(model), _ptr(y), m, _ptr(out), _stream(stream)))


def subap_model_weights(model):
    lib = load()
    _, _, s, _ = subap_model_dims(model)
    out = np.empty(s, dtype=np.float64)
    _check(lib.subap_model_weights(C.c_void_p(model), out.ctypes.data))
    return out


def subap_residual_bounds(model, rho, lo, hi, eps=0.0, stream=None):
    """rho, lo, hi: (m,) float64 cuda tensors; eps <= 0 takes k ln k / s, k = r + 1."""
    m = rho.shape[0]
    for t, name in ((rho, "rho"), (lo, "lo"), (hi, "hi")):
        _expect(t, (m,), "float64", name)
    _check(load().subap_residual_bounds(C.c_void_p(model), _ptr(rho), m, float(eps), _ptr(lo), _ptr(hi),
                                        _stream(stream)))


def subap_model_basis(model):
    lib = load()
    n, r, _, _ = subap_model_dims(model)
    out = np.empty((r, n), dtype=np.float64)  # column-major n x r == row-major r x n
    _check(lib.subap_model_basis(C.c_void_p(model), out.ctypes.data))
    return out.T


def subap_model_save(model, path):
    _check(load().subap_model_save(C.c_void_p(model), os.fsencode(path)))


def subap_model_load(path, stream=None):
    h = C.c_void_p()
    _check(load().subap_model_load(os.fsencode(path), _stream(stream), C.byref(h)))
    return h.value


def subap_model_free(model):
    _check(load().subap_model_free(C.c_void_p(model)))


# ---------------------------------------------------------------------------
# convenience owner
# ---------------------------------------------------------------------------
class Model:
    """Owns a subap_model built from a ``subap_inputs`` workload dict."""

    def __init__(self, workload: dict, basis=None, rows=None, snap_tol=0.0, snap_maxiter=0, stream=None,
                 sample_u=None, selection=None, select_params=None):
        w = workload
        fam = FAMILIES[w["family"]]
        kw = dict(r=w["r"], s=w["s"], snap_params=w.get("snap_params"), select_param=w.get("select_param"),
                  snap_tol=snap_tol, snap_maxiter=snap_maxiter, basis_in=None, rows_in=rows, sample_u=sample_u,
                  selection=selection, select_params=select_params, stream=stream)
        if basis is not None:
            kw["basis_in"] = np.asfortranarray(basis, dtype=np.float64).T  # column-major n x r
        if fam == FAMILY_KRR:
            self.handle = subap_offline(fam, n=w["n"], dim=w["dim"], points=w["points"], rhs=w["rhs"],
                                        lam=w["lam"], **kw)
        elif fam == FAMILY_TRIDIAG_SHIFT:
            self.handle = subap_offline(fam, n=w["n"], rhs=w["b0"], **kw)
        elif fam == FAMILY_IDENTITY:
            self.handle = subap_offline(fam, n=w["n"], **kw)
        elif fam == FAMILY_AFFINE:
            self.handle = subap_offline(fam, n=w["n"], rhs=w["rhs"], terms=[T.tocsr() for T in w["terms"]], **kw)
        elif fam == FAMILY_DELAY:
            self.handle = subap_offline(fam, n=w["n"], rhs=w["rhs"], tau=w["tau"], kappa=w["kappa"],
                                        c_out=w.get("c_out"), **kw)
        else:
            self.handle = subap_offline(fam, grid=w["grid"][0], rhs=w.get("rhs"), **kw)
        self.n, self.r, self.s, self.d = subap_model_dims(self.handle)

    def rows(self):
        return subap_model_rows(self.handle)

    def basis(self):
        return subap_model_basis(self.handle)

    def weights(self):
        return subap_model_weights(self.handle)

    def save(self, path):
        subap_model_save(self.handle, path)

    @classmethod
    def load(cls, path, stream=None):
        """A model rebuilt from a file written by save()."""
        self = cls.__new__(cls)
        self.handle = subap_model_load(path, stream)
        self.n, self.r, self.s, self.d = subap_model_dims(self.handle)
        return self

    def output(self, y, stream=None):
        """c^T Q y for each row of y (m, r) -> (m,) cuda tensor."""
        import torch
        out = torch.empty(y.shape[0], dtype=torch.float64, device=y.device)
        subap_output(self.handle, y, out, stream)
        return out

    def residual_bounds(self, rho, eps=0.0, stream=None):
        """(lo, hi) cuda tensors bracketing the full relative residual (leverage rows)."""
        import torch
        lo, hi = torch.empty_like(rho), torch.empty_like(rho)
        subap_residual_bounds(self.handle, rho, lo, hi, eps, stream)
        return lo, hi

    def solve(self, params, contraction=FP64, refine_steps=0, stream=None, with_status=True, csne=False):
        """params: (m, d) float64 cuda tensor -> (y, rho, status) cuda tensors.
        csne: refinement steps solve the corrected semi-normal equations."""
        import torch
        m = params.shape[0]
        y = torch.empty((m, self.r), dtype=torch.float64, device=params.device)
        rho = torch.empty(m, dtype=torch.float64, device=params.device)
        st = torch.empty(m, dtype=torch.int32, device=params.device) if with_status else None
        subap_solve_batch(self.handle, params, y, rho, st, contraction, refine_steps, stream, csne)
        return y, rho, st

    def sketched_residual(self, params, y, vector=False, stream=None):
        """(res (m, s) or None, norm (m,)) cuda tensors."""
        import torch
        m = params.shape[0]
        norm = torch.empty(m, dtype=torch.float64, device=params.device)
        res = torch.empty((m, self.s), dtype=torch.float64, device=params.device) if vector else None
        subap_sketched_residual(self.handle, params, y, res, norm, stream)
        return res, norm

    def lift(self, y, precision=FP64, stream=None, ldx=None):
        """x = Q y for the rows of y; returns a (k, n) view of a (k, ldx) tensor."""
        import torch
        dt = torch.float64 if precision == FP64 else torch.float32
        x = torch.empty((y.shape[0], ldx or self.n), dtype=dt, device=y.device)
        subap_lift(self.handle, y, x, precision, stream)
        return x[:, :self.n]

    def free(self):
        if getattr(self, "handle", None):
            subap_model_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
