// C ABI entry points (include/subap.h): argument validation, model
// lifetime, and dispatch to the offline and online kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <unordered_set>
#include <vector>

#include "common.h"
#include "profile.h"

namespace subap {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }

subap_status dmalloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    set_error("hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? SUBAP_E_NOMEM : SUBAP_E_HIP;
  }
  return SUBAP_OK;
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

// ---- per-kernel timing registry ----
namespace {
struct ProfPending {
  const char* name;
  hipEvent_t a, b;
};
struct ProfTotal {
  int64_t calls = 0;
  double ms = 0.0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfPending> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
std::map<std::string, ProfTotal> g_prof_totals;
std::vector<std::string> g_prof_names;

// Fold finished event pairs into the totals (caller holds the lock).
void prof_drain() {
  for (const ProfPending& e : g_prof_pending) {
    float ms = 0.0f;
    if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      ProfTotal& t = g_prof_totals[e.name];
      t.calls += 1;
      t.ms += ms;
    }
    g_prof_pool.push_back(e.a);
    g_prof_pool.push_back(e.b);
  }
  g_prof_pending.clear();
  g_prof_names.clear();
  for (const auto& kv : g_prof_totals) g_prof_names.push_back(kv.first);
}
}  // namespace

bool profiling_enabled() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  return g_prof_on;
}

hipEvent_t profile_event() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void profile_push(const char* name, hipEvent_t a, hipEvent_t b) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_pending.push_back({name, a, b});
  if (g_prof_pending.size() > 4096) prof_drain();
}

subap_status ensure_work(subap_model_s* M, size_t bytes) {
  if (M->work_bytes >= bytes) return SUBAP_OK;
  dfree(M->work);
  M->work = nullptr;
  M->work_bytes = 0;
  SUBAP_TRY(dmalloc(&M->work, bytes));
  M->work_bytes = bytes;
  return SUBAP_OK;
}

namespace {

void free_model(subap_model_s* M) {
  if (!M) return;
  void* bufs[] = {M->Q, M->rows_d, M->wS, M->cQ, M->bS, M->QS, M->rhs, M->phi, M->delta64, M->delta32, M->delta64T, M->delta32T, M->points,
                  M->Dt64, M->D32, M->Qrm, M->Q32, M->Qhi, M->Qlo, M->Qh16, M->Ql16, M->colscale_inv,
                  M->rowdat, M->work, M->aff_rp, M->aff_ci, M->aff_v};
  for (void* b : bufs) dfree(b);
  delete M;
}

subap_status invalid(const std::string& msg) {
  set_error(msg);
  return SUBAP_E_INVALID;
}

bool all_finite(const double* v, int64_t len) {
  for (int64_t i = 0; i < len; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

// Maps a host-side C++ exception escaping an entry point to a status code:
// no exception crosses the C ABI.
subap_status host_exception() {
  try {
    throw;
  } catch (const std::bad_alloc&) {
    set_error("host memory allocation failed");
    return SUBAP_E_NOMEM;
  } catch (const std::length_error&) {
    set_error("host buffer size out of range");
    return SUBAP_E_NOMEM;
  } catch (const std::exception& e) {
    set_error(std::string("host exception: ") + e.what());
    return SUBAP_E_INVALID;
  } catch (...) {
    set_error("unknown host exception");
    return SUBAP_E_INVALID;
  }
}

}  // namespace
}  // namespace subap

using namespace subap;

extern "C" {

const char* subap_status_string(subap_status s) {
  switch (s) {
    case SUBAP_OK: return "ok";
    case SUBAP_E_INVALID: return "invalid argument";
    case SUBAP_E_NOMEM: return "out of memory";
    case SUBAP_E_HIP: return "HIP runtime error";
    case SUBAP_E_RANK: return "rank deficient";
    case SUBAP_E_NOCONV: return "no convergence";
    case SUBAP_E_NONFINITE: return "non-finite value";
    case SUBAP_E_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* subap_last_error(void) { return g_last_error.c_str(); }

subap_status subap_offline(const subap_problem_desc* pd, const subap_offline_opts* o, void* hip_stream,
                           subap_model* out) {
  try {
    clear_error();
    if (!pd || !o || !out) return invalid("problem, opts and out must not be NULL");
    *out = nullptr;
    subap_model_s tmp;
    tmp.family = pd->family;
    if (pd->family == SUBAP_FAMILY_DIFF2D || pd->family == SUBAP_FAMILY_DIFF3D) {
      const int dimx = pd->family == SUBAP_FAMILY_DIFF2D ? 2 : 3;
      if (pd->grid < 2 || pd->grid > 46340) return invalid("grid must be in [2, 46340]");
      double nn = std::pow(static_cast<double>(pd->grid), dimx);
      if (nn > 2147483647.0) return invalid("grid^dim exceeds 2^31 - 1 unknowns");
      tmp.N = pd->grid;
      tmp.dimx = dimx;
      tmp.n = static_cast<int64_t>(nn);
      tmp.d = dimx == 2 ? 2 : 4;
      tmp.F = 2 * dimx;
      tmp.h = 1.0 / (pd->grid + 1);
      tmp.inv_h2 = 1.0 / (tmp.h * tmp.h);
      if (pd->rhs && !all_finite(pd->rhs, tmp.n)) return invalid("rhs has non-finite entries");
    } else if (pd->family == SUBAP_FAMILY_KRR) {
      if (pd->n < 1 || pd->n > 2147483647LL) return invalid("KRR n must be in [1, 2^31 - 1]");
      if (pd->dim < 1 || pd->dim > 16) return invalid("KRR point dimension must be in [1, 16]");
      if (!pd->points || !pd->rhs) return invalid("KRR needs points and rhs");
      if (!(pd->lambda > 0.0) || !std::isfinite(pd->lambda)) return invalid("KRR lambda must be finite and > 0");
      tmp.n = pd->n;
      tmp.dimx = pd->dim;
      tmp.d = 1;
      tmp.lambda = pd->lambda;
      if (!all_finite(pd->points, pd->n * pd->dim) || !all_finite(pd->rhs, pd->n))
        return invalid("points or rhs have non-finite entries");
    } else if (pd->family == SUBAP_FAMILY_DELAY) {
      if (pd->n < 2 || pd->n > 2147483647LL) return invalid("delay n must be in [2, 2^31 - 1]");
      if (!(pd->tau > 0.0) || !std::isfinite(pd->tau)) return invalid("delay tau must be finite and > 0");
      if (!(pd->kappa > 2.0) || !std::isfinite(pd->kappa)) return invalid("delay kappa must be finite and > 2");
      if (!pd->rhs || !all_finite(pd->rhs, pd->n)) return invalid("delay needs a finite rhs");
      tmp.n = pd->n;
      tmp.dimx = 1;
      tmp.d = 1;
      tmp.F = 2;
      tmp.h = 1.0;
      tmp.inv_h2 = 1.0;
      tmp.tau = pd->tau;
      tmp.kappa = pd->kappa;
      tmp.aff_c0 = 3.0;  // A_0 = 3 A_1
    } else if (pd->family == SUBAP_FAMILY_TRIDIAG_SHIFT || pd->family == SUBAP_FAMILY_IDENTITY) {
      if (pd->n < 2 || pd->n > 2147483647LL) return invalid("n must be in [2, 2^31 - 1]");
      if (pd->family == SUBAP_FAMILY_TRIDIAG_SHIFT && (!pd->rhs || !all_finite(pd->rhs, pd->n)))
        return invalid("the shifted tridiagonal family needs finite b0 in rhs");
      tmp.n = pd->n;
      tmp.dimx = 1;
      tmp.d = 1;
      tmp.F = pd->family == SUBAP_FAMILY_TRIDIAG_SHIFT ? 2 : 1;
      tmp.h = 1.0;
      tmp.inv_h2 = 1.0;
    } else if (pd->family == SUBAP_FAMILY_AFFINE) {
      if (pd->n < 1 || pd->n > 2147483647LL) return invalid("affine n must be in [1, 2^31 - 1]");
      if (pd->nterms < 1 || pd->nterms > kMaxAffineTerms) return invalid("affine nterms must be in [1, 4]");
      if (!pd->term_rowptr || !pd->term_cols || !pd->term_vals || !pd->rhs)
        return invalid("the affine family needs its terms and rhs");
      for (int q = 0; q < pd->nterms; ++q) {
        const int64_t* rp = pd->term_rowptr[q];
        if (!rp || rp[0] != 0) return invalid("affine term row offsets must start at 0");
        for (int64_t i = 0; i < pd->n; ++i)
          if (rp[i + 1] < rp[i]) return invalid("affine term row offsets must not decrease");
        const int64_t nnz = rp[pd->n];
        if (nnz > 0 && (!pd->term_cols[q] || !pd->term_vals[q])) return invalid("affine term arrays missing");
        for (int64_t e = 0; e < nnz; ++e)
          if (pd->term_cols[q][e] < 0 || pd->term_cols[q][e] >= pd->n) return invalid("affine column out of range");
        if (!all_finite(pd->term_vals[q], nnz)) return invalid("affine term values not finite");
      }
      if (!all_finite(pd->rhs, pd->n)) return invalid("rhs has non-finite entries");
      if (!o->basis_in) {
        set_error("the affine family takes its basis from basis_in (no snapshot solver for general terms)");
        return SUBAP_E_UNSUPPORTED;
      }
      tmp.n = pd->n;
      tmp.dimx = 1;
      tmp.d = pd->nterms;
      tmp.F = pd->nterms;
      tmp.h = 1.0;
      tmp.inv_h2 = 1.0;
    } else {
      return invalid("unknown family");
    }
    if (pd->c_out && !all_finite(pd->c_out, tmp.n)) return invalid("c_out has non-finite entries");
    if (o->r < 1 || o->r > kMaxR) return invalid("r must be in [1, 64]");
    const bool uni = !o->rows_in && o->n_select > 1 && o->selection != SUBAP_SELECT_LEVERAGE;
    if (o->n_select < 0) return invalid("n_select must be >= 0");
    if (uni) {
      if (!o->select_params) return invalid("n_select > 1 needs select_params");
      if (o->r > tmp.n) return invalid("r must not exceed n");
    } else if (o->s < o->r || o->s > kMaxS || o->s > tmp.n) {
      return invalid("s must satisfy r <= s <= min(n, 256)");
    }
    if (o->snap_tol < 0.0 || !std::isfinite(o->snap_tol)) return invalid("snap_tol must be finite and >= 0");
    if (o->snap_maxiter < 0) return invalid("snap_maxiter must be >= 0");
    tmp.r = o->r;
    tmp.s = uni ? o->r : o->s;  // a union of pivots sets s after the selection
    if (!o->basis_in) {
      if (!o->snap_params) return invalid("snap_params needed without basis_in");
      if (!all_finite(o->snap_params, static_cast<int64_t>(o->r) * tmp.d)) return invalid("snap_params not finite");
      if (pd->family == SUBAP_FAMILY_KRR)
        for (int i = 0; i < o->r; ++i)
          if (!(o->snap_params[i] > 0.0)) return invalid("KRR length scales must be > 0");
    } else if (!all_finite(o->basis_in, tmp.n * o->r)) {
      return invalid("basis_in has non-finite entries");
    }
    if (!o->rows_in) {
      if (o->selection != SUBAP_SELECT_CPQR && o->selection != SUBAP_SELECT_LEVERAGE &&
          o->selection != SUBAP_SELECT_LU)
        return invalid("selection must be SUBAP_SELECT_CPQR, SUBAP_SELECT_LEVERAGE or SUBAP_SELECT_LU");
      if (o->selection == SUBAP_SELECT_LEVERAGE) {
        if (rhs_varies(pd->family)) {
          set_error("leverage-score selection needs a right-hand side independent of p");
          return SUBAP_E_UNSUPPORTED;
        }
        if (!o->sample_u) return invalid("leverage-score selection needs sample_u");
        for (int k = 0; k < o->s; ++k)
          if (!(o->sample_u[k] >= 0.0 && o->sample_u[k] < 1.0)) return invalid("sample_u must lie in [0, 1)");
      }
      if (uni) {
        if (!all_finite(o->select_params, static_cast<int64_t>(o->n_select) * tmp.d))
          return invalid("select_params not finite");
        if (pd->family == SUBAP_FAMILY_KRR)
          for (int t = 0; t < o->n_select; ++t)
            if (!(o->select_params[t] > 0.0)) return invalid("KRR select_params must be > 0");
      } else {
        if (!o->select_param) return invalid("select_param needed without rows_in");
        if (!all_finite(o->select_param, tmp.d)) return invalid("select_param not finite");
        if (pd->family == SUBAP_FAMILY_KRR && !(o->select_param[0] > 0.0))
          return invalid("KRR select_param must be > 0");
      }
    } else {
      std::unordered_set<int64_t> seen;
      for (int k = 0; k < o->s; ++k) {
        const int64_t v = o->rows_in[k];
        if (v < 0 || v >= tmp.n) return invalid("rows_in index out of range");
        if (!seen.insert(v).second) return invalid("rows_in has duplicates");
      }
    }
    subap_model_s* M = new (std::nothrow) subap_model_s(tmp);
    if (!M) return SUBAP_E_NOMEM;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    subap_status rc = offline_build(pd, o, st, M);
    if (rc != SUBAP_OK) {
      (void)hipStreamSynchronize(st);
      free_model(M);
      return rc;
    }
    *out = M;
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_solve_batch(subap_model M, const double* params, int64_t m, double* y, double* rho,
                               int32_t* status, const subap_solve_opts* opts, void* hip_stream) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (m < 0) return invalid("m must be >= 0");
    if (m == 0) return SUBAP_OK;
    if (!params || !y) return invalid("params and y must not be NULL");
    const int prec = opts ? opts->contraction : SUBAP_FP64;
    const int refine = opts ? opts->refine_steps : 0;
    const int csne = opts ? opts->refine_csne : 0;
    if (prec < SUBAP_FP64 || prec > SUBAP_FP16X3) return invalid("unknown contraction precision");
    if (refine < 0 || refine > 4) return invalid("refine_steps must be in [0, 4]");
    if (csne != 0 && csne != 1) return invalid("refine_csne must be 0 or 1");
    if (m > (int64_t(1) << 31) / 64) return invalid("m too large for one call");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (M->family == SUBAP_FAMILY_KRR) return krr_solve(M, params, m, y, rho, status, prec, refine, csne, st);
    if (prec == SUBAP_BF16X3 || prec == SUBAP_FP16X3) {
      set_error("the split 16-bit contractions are implemented for the kernel family only");
      return SUBAP_E_UNSUPPORTED;
    }
    return fd_solve(M, params, m, y, rho, status, prec, refine, csne, st);
  } catch (...) {
    return host_exception();
  }
}

// ---------------------------------------------------------------------------
// subap_solve_batch_noalloc: the same solve with its device workspace in a
// file-scope array instead of a library allocation.  The array exists once
// per GPU the library runs on (the loader places it with the code object);
// host code reaches it only through the address hipGetSymbolAddress returns
// for the current device, taken on the first call there and kept.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

subap_status scratch_on_current_device(void** out) {
  int dev = 0;
  SUBAP_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index out of the scratch table's range");
    return SUBAP_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    SUBAP_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return SUBAP_OK;
}

}  // namespace

subap_status subap_solve_batch_noalloc(subap_model M, const double* params, int64_t m, double* y, double* rho,
                                       int32_t* status, const subap_solve_opts* opts, void* hip_stream) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (m < 0) return invalid("m must be >= 0");
    if (m == 0) return SUBAP_OK;
    if (!params || !y) return invalid("params and y must not be NULL");
    const int prec = opts ? opts->contraction : SUBAP_FP64;
    const int refine = opts ? opts->refine_steps : 0;
    const int csne = opts ? opts->refine_csne : 0;
    if (prec < SUBAP_FP64 || prec > SUBAP_FP16X3) return invalid("unknown contraction precision");
    if (refine < 0 || refine > 4) return invalid("refine_steps must be in [0, 4]");
    if (csne != 0 && csne != 1) return invalid("refine_csne must be 0 or 1");
    if (m > (int64_t(1) << 31) / 64) return invalid("m too large for one call");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (M->family != SUBAP_FAMILY_KRR) {
      // the finite-difference and delay solves keep everything in registers
      // and LDS: no device workspace
      if (prec == SUBAP_BF16X3 || prec == SUBAP_FP16X3) {
        set_error("the split 16-bit contractions are implemented for the kernel family only");
        return SUBAP_E_UNSUPPORTED;
      }
      return fd_solve(M, params, m, y, rho, status, prec, refine, csne, st);
    }
    const int64_t chunk = krr_chunk(M, prec, refine, csne != 0, kScratchBytes);
    if (chunk < 1) {
      set_error("one block of parameters needs more workspace than the 64 MiB scratch");
      return SUBAP_E_UNSUPPORTED;
    }
    void* ws = nullptr;
    SUBAP_TRY(scratch_on_current_device(&ws));
    for (int64_t c0 = 0; c0 < m; c0 += chunk) {
      const int64_t cnt = std::min(chunk, m - c0);
      SUBAP_TRY(krr_solve_ws(M, params + c0 * M->d, cnt, y + c0 * M->r, rho ? rho + c0 : nullptr,
                             status ? status + c0 : nullptr, prec, refine, csne != 0, ws, st));
    }
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_lift(subap_model M, const double* y, int64_t k, void* x, int64_t ldx, int32_t precision,
                        void* hip_stream) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (k < 0) return invalid("k must be >= 0");
    if (ldx != 0 && ldx < M->n) return invalid("ldx must be 0 or >= n");
    if (k == 0) return SUBAP_OK;
    if (!y || !x) return invalid("y and x must not be NULL");
    if (precision != SUBAP_FP64 && precision != SUBAP_FP32) return invalid("lift precision must be FP64 or FP32");
    return lift(M, y, k, x, ldx == 0 ? M->n : ldx, precision, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_model_dims(subap_model M, int64_t* n, int32_t* r, int32_t* s, int32_t* d) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (n) *n = M->n;
    if (r) *r = M->r;
    if (s) *s = M->s;
    if (d) *d = M->d;
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_model_rows(subap_model M, int64_t* rows_host) {
  try {
    clear_error();
    if (!M || !rows_host) return invalid("model and rows_host must not be NULL");
    std::memcpy(rows_host, M->rows.data(), sizeof(int64_t) * M->rows.size());
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_full_residual(subap_model M, const double* params, int64_t m, const double* x, double* res,
                                 void* hip_stream) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (m < 0) return invalid("m must be >= 0");
    if (m == 0) return SUBAP_OK;
    if (!params || !x || !res) return invalid("params_dev, x_dev and res_dev must not be NULL");
    return subap::full_residual(M, params, m, x, res, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_delta_residual(subap_model M, const double* params, int64_t m, const double* y1,
                                  const double* y2, double* res, void* hip_stream) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (m < 0) return invalid("m must be >= 0");
    if (m == 0) return SUBAP_OK;
    if (!params || !y1 || !y2 || !res) return invalid("params_dev, y1_dev, y2_dev and res_dev must not be NULL");
    return subap::delta_residual(M, params, m, y1, y2, res, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_apsnap_solve(subap_model M, const double* params, int64_t m, double* y, double* rho,
                                void* hip_stream) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (m < 0) return invalid("m must be >= 0");
    if (m == 0) return SUBAP_OK;
    if (!params || !y) return invalid("params_dev and y_dev must not be NULL");
    if (rhs_varies(M->family)) {
      set_error("ApSnap is implemented for right-hand sides independent of p");
      return SUBAP_E_UNSUPPORTED;
    }
    return subap::apsnap_solve(M, params, m, y, rho, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_polish(subap_model M, const double* params, int64_t m, double* x, int32_t max_iter, double tol,
                          double* res, void* hip_stream) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (m < 0) return invalid("m must be >= 0");
    if (max_iter < 0) return invalid("max_iter must be >= 0");
    if (!(tol >= 0.0) || !std::isfinite(tol)) return invalid("tol must be finite and >= 0");
    if (m == 0) return SUBAP_OK;
    if (!params || !x) return invalid("params_dev and x_dev must not be NULL");
    if (M->family == SUBAP_FAMILY_AFFINE) {
      set_error("polishing runs conjugate gradients, which the affine family's general terms do not allow");
      return SUBAP_E_UNSUPPORTED;
    }
    if (rhs_varies(M->family)) {
      set_error("polishing is implemented for right-hand sides independent of p");
      return SUBAP_E_UNSUPPORTED;
    }
    return subap::polish(M, params, m, x, max_iter, tol, res, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_output(subap_model M, const double* y, int64_t m, double* out, void* hip_stream) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (!M->cQ) return invalid("the model was built without an output vector (c_out)");
    if (m < 0) return invalid("m must be >= 0");
    if (m == 0) return SUBAP_OK;
    if (!y || !out) return invalid("y_dev and out_dev must not be NULL");
    return subap::output_apply(M, y, m, out, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return host_exception();
  }
}

// ---- model files ----
// Layout (native byte order): 8-byte magic, a header of 12 int64 and 8 double
// fields, then the arrays Q (n r), rhs (n), rows (s int64), weights (s),
// points (n dimx, KRR only) and c^T Q (r, when present).
namespace {
constexpr char kMagic[8] = {'S', 'U', 'B', 'A', 'P', 'M', 'D', '1'};
constexpr int kHdrInts = 12, kHdrDoubles = 8;

struct FileCloser {
  std::FILE* f;
  ~FileCloser() {
    if (f) std::fclose(f);
  }
};

bool put(std::FILE* f, const void* p, size_t bytes) { return bytes == 0 || std::fwrite(p, 1, bytes, f) == bytes; }
bool get(std::FILE* f, void* p, size_t bytes) { return bytes == 0 || std::fread(p, 1, bytes, f) == bytes; }
}  // namespace

subap_status subap_model_save(subap_model M, const char* path) {
  try {
    clear_error();
    if (!M || !path) return invalid("model and path must not be NULL");
    if (M->family == SUBAP_FAMILY_AFFINE) {
      set_error("model files do not hold the affine family's terms");
      return SUBAP_E_UNSUPPORTED;
    }
    const int64_t n = M->n;
    const int r = M->r, s = M->s;
    std::vector<double> Q(static_cast<size_t>(n) * r), rhs(static_cast<size_t>(n)), pts, cq;
    SUBAP_HIP_TRY(hipDeviceSynchronize());
    SUBAP_HIP_TRY(hipMemcpy(Q.data(), M->Q, sizeof(double) * Q.size(), hipMemcpyDeviceToHost));
    SUBAP_HIP_TRY(hipMemcpy(rhs.data(), M->rhs, sizeof(double) * n, hipMemcpyDeviceToHost));
    if (M->family == SUBAP_FAMILY_KRR) {
      pts.resize(static_cast<size_t>(n) * M->dimx);
      SUBAP_HIP_TRY(hipMemcpy(pts.data(), M->points, sizeof(double) * pts.size(), hipMemcpyDeviceToHost));
    }
    if (M->cQ) {
      cq.resize(r);
      SUBAP_HIP_TRY(hipMemcpy(cq.data(), M->cQ, sizeof(double) * r, hipMemcpyDeviceToHost));
    }
    const int64_t hi[kHdrInts] = {M->family, M->N, M->dimx, n, r, s, M->d, M->F, M->selection,
                                   M->cQ ? 1 : 0, static_cast<int64_t>(pts.size()), 0};
    const double hd[kHdrDoubles] = {M->h, M->inv_h2, M->lambda, M->tau, M->kappa, M->aff_c0, M->dmax, 0.0};
    FileCloser fc{std::fopen(path, "wb")};
    if (!fc.f) return invalid(std::string("cannot open ") + path + " for writing");
    const bool ok = put(fc.f, kMagic, sizeof(kMagic)) && put(fc.f, hi, sizeof(hi)) && put(fc.f, hd, sizeof(hd)) &&
                    put(fc.f, Q.data(), sizeof(double) * Q.size()) && put(fc.f, rhs.data(), sizeof(double) * n) &&
                    put(fc.f, M->rows.data(), sizeof(int64_t) * s) &&
                    put(fc.f, M->weights.data(), sizeof(double) * s) &&
                    put(fc.f, pts.data(), sizeof(double) * pts.size()) && put(fc.f, cq.data(), sizeof(double) * cq.size());
    if (!ok || std::fflush(fc.f) != 0) return invalid(std::string("writing ") + path + " failed");
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_model_load(const char* path, void* hip_stream, subap_model* out) {
  try {
    clear_error();
    if (!path || !out) return invalid("path and out must not be NULL");
    *out = nullptr;
    FileCloser fc{std::fopen(path, "rb")};
    if (!fc.f) return invalid(std::string("cannot open ") + path);
    char magic[8];
    int64_t hi[kHdrInts];
    double hd[kHdrDoubles];
    if (!get(fc.f, magic, sizeof(magic)) || std::memcmp(magic, kMagic, sizeof(kMagic)) != 0)
      return invalid(std::string(path) + " is not a SubApSnap model file");
    if (!get(fc.f, hi, sizeof(hi)) || !get(fc.f, hd, sizeof(hd))) return invalid(std::string(path) + " is truncated");
    subap_model_s tmp;
    tmp.family = static_cast<int>(hi[0]);
    tmp.N = static_cast<int>(hi[1]);
    tmp.dimx = static_cast<int>(hi[2]);
    tmp.n = hi[3];
    tmp.r = static_cast<int>(hi[4]);
    tmp.s = static_cast<int>(hi[5]);
    tmp.d = static_cast<int>(hi[6]);
    tmp.F = static_cast<int>(hi[7]);
    tmp.selection = static_cast<int>(hi[8]);
    const bool has_cq = hi[9] != 0;
    const int64_t npts = hi[10];
    tmp.h = hd[0];
    tmp.inv_h2 = hd[1];
    tmp.lambda = hd[2];
    tmp.tau = hd[3];
    tmp.kappa = hd[4];
    tmp.aff_c0 = hd[5];
    tmp.dmax = hd[6];
    // the family's geometry must agree with n (the table builders index
    // neighbours from it); derived constants are recomputed, not trusted
    bool geo = false;
    if (tmp.family == SUBAP_FAMILY_DIFF2D || tmp.family == SUBAP_FAMILY_DIFF3D) {
      const int dx = tmp.family == SUBAP_FAMILY_DIFF2D ? 2 : 3;
      geo = tmp.N >= 2 && tmp.N <= 46340 && tmp.dimx == dx && tmp.d == (dx == 2 ? 2 : 4) && tmp.F == 2 * dx &&
            std::pow(static_cast<double>(tmp.N), dx) == static_cast<double>(tmp.n);
      tmp.h = 1.0 / (tmp.N + 1);
      tmp.inv_h2 = 1.0 / (tmp.h * tmp.h);
    } else if (tmp.family == SUBAP_FAMILY_KRR) {
      geo = tmp.dimx >= 1 && tmp.dimx <= 16 && tmp.d == 1 && npts == tmp.n * tmp.dimx && tmp.lambda > 0.0 &&
            std::isfinite(tmp.lambda);
    } else if (tmp.family == SUBAP_FAMILY_DELAY) {
      geo = tmp.n >= 2 && tmp.dimx == 1 && tmp.d == 1 && tmp.F == 2 && tmp.tau > 0.0 && std::isfinite(tmp.tau) &&
            tmp.kappa > 2.0 && std::isfinite(tmp.kappa);
      tmp.h = 1.0;
      tmp.inv_h2 = 1.0;
      tmp.aff_c0 = 3.0;
    } else if (tmp.family == SUBAP_FAMILY_TRIDIAG_SHIFT || tmp.family == SUBAP_FAMILY_IDENTITY) {
      geo = tmp.n >= 2 && tmp.dimx == 1 && tmp.d == 1 &&
            tmp.F == (tmp.family == SUBAP_FAMILY_TRIDIAG_SHIFT ? 2 : 1) && tmp.selection != SUBAP_SELECT_LEVERAGE;
      tmp.h = 1.0;
      tmp.inv_h2 = 1.0;
    }
    if (!geo || tmp.n < 1 || tmp.n > 2147483647LL || tmp.r < 1 || tmp.r > kMaxR || tmp.s < tmp.r ||
        tmp.s > kMaxS || tmp.s > tmp.n || (tmp.family != SUBAP_FAMILY_KRR && npts != 0) ||
        (tmp.selection != SUBAP_SELECT_CPQR && tmp.selection != SUBAP_SELECT_LEVERAGE &&
         tmp.selection != SUBAP_SELECT_LU))
      return invalid(std::string(path) + " has an inconsistent header");
    {  // the payload the header implies must be exactly what the file holds, before anything is allocated
      const int64_t payload = 8 * (tmp.n * tmp.r + tmp.n + 2 * int64_t(tmp.s) + npts + (has_cq ? tmp.r : 0));
      const long here = std::ftell(fc.f);
      if (here < 0 || std::fseek(fc.f, 0, SEEK_END) != 0) return invalid(std::string("cannot seek in ") + path);
      const long end = std::ftell(fc.f);
      if (end < 0 || std::fseek(fc.f, here, SEEK_SET) != 0) return invalid(std::string("cannot seek in ") + path);
      if (static_cast<int64_t>(end - here) != payload)
        return invalid(std::string(path) + " does not hold the payload its header describes");
    }
    std::vector<double> Q(static_cast<size_t>(tmp.n) * tmp.r), rhs(static_cast<size_t>(tmp.n)),
        w(static_cast<size_t>(tmp.s)), pts(static_cast<size_t>(npts)), cq(has_cq ? tmp.r : 0);
    std::vector<int64_t> rows(static_cast<size_t>(tmp.s));
    if (!get(fc.f, Q.data(), sizeof(double) * Q.size()) || !get(fc.f, rhs.data(), sizeof(double) * rhs.size()) ||
        !get(fc.f, rows.data(), sizeof(int64_t) * rows.size()) || !get(fc.f, w.data(), sizeof(double) * w.size()) ||
        !get(fc.f, pts.data(), sizeof(double) * pts.size()) || !get(fc.f, cq.data(), sizeof(double) * cq.size()))
      return invalid(std::string(path) + " is truncated");
    for (int64_t v : rows)
      if (v < 0 || v >= tmp.n) return invalid(std::string(path) + " has a row index out of range");
    if (!all_finite(Q.data(), static_cast<int64_t>(Q.size())) || !all_finite(rhs.data(), tmp.n) ||
        !all_finite(w.data(), tmp.s) || !all_finite(pts.data(), npts) || !all_finite(cq.data(), static_cast<int64_t>(cq.size())))
      return invalid(std::string(path) + " has non-finite entries");
    if (tmp.family == SUBAP_FAMILY_KRR) {  // bound on every squared distance, as the offline phase computes it
      double rmax = 0.0;
      for (int64_t i = 0; i < tmp.n; ++i) {
        double t2 = 0.0;
        for (int q = 0; q < tmp.dimx; ++q) t2 += pts[i * tmp.dimx + q] * pts[i * tmp.dimx + q];
        rmax = std::max(rmax, t2);
      }
      tmp.dmax = 4.0 * rmax;
    }
    subap_model_s* M = new (std::nothrow) subap_model_s(tmp);
    if (!M) return SUBAP_E_NOMEM;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    subap_status rc = subap::restore_model(M, Q.data(), rows.data(), w.data(), rhs.data(),
                                           npts ? pts.data() : nullptr, has_cq ? cq.data() : nullptr, st);
    if (rc != SUBAP_OK) {
      (void)hipStreamSynchronize(st);
      free_model(M);
      return rc;
    }
    *out = M;
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_model_weights(subap_model M, double* weights_host) {
  try {
    clear_error();
    if (!M || !weights_host) return invalid("model and weights_host must not be NULL");
    std::memcpy(weights_host, M->weights.data(), sizeof(double) * M->weights.size());
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_residual_bounds(subap_model M, const double* rho, int64_t m, double eps, double* lo, double* hi,
                                   void* hip_stream) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (M->selection != SUBAP_SELECT_LEVERAGE) return invalid("residual bounds need leverage-score rows");
    if (m < 0) return invalid("m must be >= 0");
    if (!std::isfinite(eps)) return invalid("eps must be finite");
    if (m == 0) return SUBAP_OK;
    if (!rho || !lo || !hi) return invalid("rho_dev, lo_dev and hi_dev must not be NULL");
    if (!(eps > 0.0)) {
      const double k = M->r + 1.0;
      eps = k * std::log(k) / M->s;
    }
    return subap::residual_bounds(rho, m, eps, lo, hi, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_model_basis(subap_model M, double* Q_host) {
  try {
    clear_error();
    if (!M || !Q_host) return invalid("model and Q_host must not be NULL");
    SUBAP_HIP_TRY(hipDeviceSynchronize());
    SUBAP_HIP_TRY(hipMemcpy(Q_host, M->Q, sizeof(double) * M->n * M->r, hipMemcpyDeviceToHost));
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_sketched_residual(subap_model M, const double* params, int64_t m, const double* y, double* res,
                                     double* norm, void* hip_stream) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (m < 0) return invalid("m must be >= 0");
    if (m == 0) return SUBAP_OK;
    if (!params || !y) return invalid("params and y must not be NULL");
    if (!res && !norm) return invalid("at least one of res and norm must be given");
    if (m > (int64_t(1) << 31) / 64) return invalid("m too large for one call");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (M->family == SUBAP_FAMILY_KRR) return krr_residual(M, params, m, y, res, norm, st);
    return fd_residual(M, params, m, y, res, norm, st);
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_excess_bound(subap_model M, const double* params, int64_t m, const double* y, double sigma_min,
                                double* out, void* hip_stream) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (m < 0) return invalid("m must be >= 0");
    if (!(sigma_min > 0.0) || !std::isfinite(sigma_min)) return invalid("sigma_min must be finite and > 0");
    if (m == 0) return SUBAP_OK;
    if (!params || !y || !out) return invalid("params, y and out must not be NULL");
    if (m > (int64_t(1) << 31) / 64) return invalid("m too large for one call");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (M->family == SUBAP_FAMILY_KRR) return krr_excess(M, params, m, y, sigma_min, out, st);
    return fd_excess(M, params, m, y, sigma_min, out, st);
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_reduced_matrix(subap_model M, const double* params, int64_t m, double* G, void* hip_stream) {
  try {
    clear_error();
    if (!M) return invalid("model must not be NULL");
    if (m < 0) return invalid("m must be >= 0");
    if (m == 0) return SUBAP_OK;
    if (!params || !G) return invalid("params and G must not be NULL");
    if (m > (int64_t(1) << 40) / (static_cast<int64_t>(M->s) * M->r)) return invalid("m too large for one call");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    if (M->family == SUBAP_FAMILY_KRR) return krr_reduced_matrix(M, params, m, G, st);
    return fd_reduced_matrix(M, params, m, G, st);
  } catch (...) {
    return host_exception();
  }
}

static subap_status plan_args(const subap_model* models, int32_t k, const double* const* params, const int64_t* m,
                              double* const* y, const subap_solve_opts* opts, int* prec, int* refine,
                              bool* csne) {
  if (!models || !params || !m || !y || k < 1) return invalid("models, params, m and y must be given and k >= 1");
  *prec = opts ? opts->contraction : SUBAP_FP64;
  *refine = opts ? opts->refine_steps : 0;
  const int cs = opts ? opts->refine_csne : 0;
  if (*prec != SUBAP_FP64 && *prec != SUBAP_FP32) return invalid("batched plans take FP64 or FP32 contractions");
  if (*refine < 0 || *refine > 4) return invalid("refine_steps must be in [0, 4]");
  if (cs != 0 && cs != 1) return invalid("refine_csne must be 0 or 1");
  *csne = cs != 0;
  int64_t total = 0;
  for (int i = 0; i < k; ++i) {
    if (!models[i]) return invalid("model must not be NULL");
    if (m[i] < 0) return invalid("m must be >= 0");
    if (m[i] > 0 && (!params[i] || !y[i])) return invalid("params and y must not be NULL when m > 0");
    total += m[i];
  }
  if (total > (int64_t(1) << 40)) return invalid("too many parameters in one plan");
  return SUBAP_OK;
}

subap_status subap_plan_create(const subap_model* models, int32_t k, const double* const* params, const int64_t* m,
                               double* const* y, double* const* rho, int32_t* const* status,
                               const subap_solve_opts* opts, int32_t flags, void* hip_stream, subap_plan* out) {
  try {
    clear_error();
    if (!out) return invalid("out must not be NULL");
    *out = nullptr;
    int prec = 0, refine = 0;
    bool csne = false;
    SUBAP_TRY(plan_args(models, k, params, m, y, opts, &prec, &refine, &csne));
    subap_plan_s* h = new (std::nothrow) subap_plan_s{nullptr};
    if (!h) return SUBAP_E_NOMEM;
    subap_status rc = plan_build(models, k, params, m, y, rho, status, prec, refine, csne, flags,
                                 static_cast<hipStream_t>(hip_stream), &h->impl);
    if (rc != SUBAP_OK) {
      delete h;
      return rc;
    }
    *out = h;
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_plan_execute(subap_plan plan, void* hip_stream) {
  try {
    clear_error();
    if (!plan || !plan->impl) return invalid("plan must not be NULL");
    return plan_execute(plan->impl, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_plan_shape(subap_plan plan, int32_t* threads, int32_t* blocks) {
  try {
    clear_error();
    if (!plan || !plan->impl) return invalid("plan must not be NULL");
    int t = 0, b = 0;
    plan_shape(plan->impl, &t, &b);
    if (threads) *threads = t;
    if (blocks) *blocks = b;
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_plan_free(subap_plan plan) {
  try {
    clear_error();
    if (!plan) return SUBAP_OK;
    (void)hipDeviceSynchronize();
    plan_free(plan->impl);
    delete plan;
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_solve_multi(const subap_model* models, int32_t k, const double* const* params, const int64_t* m,
                               double* const* y, double* const* rho, int32_t* const* status,
                               const subap_solve_opts* opts, void* hip_stream) {
  try {
    subap_plan plan = nullptr;
    SUBAP_TRY(subap_plan_create(models, k, params, m, y, rho, status, opts, 0, hip_stream, &plan));
    subap_status rc = subap_plan_execute(plan, hip_stream);
    if (rc == SUBAP_OK) rc = hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)) == hipSuccess
                                 ? SUBAP_OK : SUBAP_E_HIP;
    subap_plan_free(plan);
    return rc;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_surrogate_create(int32_t d, int32_t r, int32_t hidden, const double* w, subap_surrogate* out) {
  try {
    clear_error();
    if (!out || !w) return invalid("weights and out must not be NULL");
    *out = nullptr;
    if (d < 1 || d > 16 || r < 1 || r > kMaxR || hidden < 1 || hidden > 4096)
      return invalid("need 1 <= d <= 16, 1 <= r <= 64, 1 <= hidden <= 4096");
    const int64_t nw = int64_t(hidden) * d + hidden + int64_t(hidden) * hidden + hidden + int64_t(r) * hidden + r;
    if (!all_finite(w, nw)) return invalid("weights have non-finite entries");
    subap_surrogate_s* h = new (std::nothrow) subap_surrogate_s{nullptr};
    if (!h) return SUBAP_E_NOMEM;
    subap_status rc = surrogate_create(d, r, hidden, w, &h->impl);
    if (rc != SUBAP_OK) {
      delete h;
      return rc;
    }
    *out = h;
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

int64_t subap_surrogate_nparams(subap_surrogate s) {
  return (s && s->impl) ? surrogate_nparams(s->impl) : -1;
}

subap_status subap_surrogate_weights(subap_surrogate s, double* w) {
  try {
    clear_error();
    if (!s || !s->impl || !w) return invalid("surrogate and weights must not be NULL");
    return surrogate_weights(s->impl, w);
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_surrogate_gradient(subap_surrogate s, const double* P, const double* T, int64_t m, double* g,
                                      double* loss, void* hip_stream) {
  try {
    clear_error();
    if (!s || !s->impl || !P || !T || !g || !loss) return invalid("arguments must not be NULL");
    if (m < 1 || m > 65536) return invalid("m must be in [1, 65536]");
    return surrogate_gradient(s->impl, P, T, m, g, loss, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_surrogate_train(subap_surrogate s, const double* P, const double* Y, int64_t m,
                                   const subap_train_opts* o, double* loss, void* hip_stream) {
  try {
    clear_error();
    if (!s || !s->impl || !P || !Y || !o) return invalid("arguments must not be NULL");
    if (m < 1 || m > (int64_t(1) << 31) - 1) return invalid("m must be in [1, 2^31)");
    if (o->epochs < 1) return invalid("epochs must be >= 1");
    const int batch = o->batch == 0 ? 4096 : o->batch;
    if (batch < 1 || batch > 65536) return invalid("batch must be in [1, 65536]");
    const double lr = o->lr == 0.0 ? 1e-3 : o->lr;
    if (!(lr > 0.0) || !(o->lr_min >= 0.0) || !std::isfinite(lr)) return invalid("learning rates must be finite, lr > 0");
    return surrogate_train(s->impl, P, Y, m, o->epochs, batch, lr, o->lr_min, o->seed, loss,
                           static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_surrogate_predict(subap_surrogate s, const double* P, int64_t m, double* y, void* hip_stream) {
  try {
    clear_error();
    if (!s || !s->impl) return invalid("surrogate must not be NULL");
    if (m < 0) return invalid("m must be >= 0");
    if (m == 0) return SUBAP_OK;
    if (!P || !y) return invalid("params and y must not be NULL");
    return surrogate_predict(s->impl, P, m, y, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return host_exception();
  }
}

static subap_status surrogate_solve_checked(subap_model M, subap_surrogate s, const double* P, int64_t m,
                                            double tol, double* y, uint8_t* accepted, int32_t* status,
                                            const subap_solve_opts* fb, int64_t* n_acc, void* hip_stream,
                                            double sigma_min) {
  try {
    clear_error();
    if (!M || !s || !s->impl || !n_acc) return invalid("model, surrogate and n_accepted must not be NULL");
    if (m < 0) return invalid("m must be >= 0");
    *n_acc = 0;
    if (m == 0) return SUBAP_OK;
    if (!P || !y) return invalid("params and y must not be NULL");
    if (!(tol >= 0.0)) return invalid("accept_tol must be >= 0");
    int sd_ = 0, sr_ = 0;
    surrogate_shape(s->impl, &sd_, &sr_);
    if (M->d != sd_ || M->r != sr_) return invalid("surrogate shape does not match the model");
    const int prec = fb ? fb->contraction : SUBAP_FP64;
    const int refine = fb ? fb->refine_steps : 0;
    const int csne = fb ? fb->refine_csne : 0;
    if (prec < SUBAP_FP64 || prec > SUBAP_FP16X3 || refine < 0 || refine > 4 || (csne != 0 && csne != 1))
      return invalid("bad fallback options");
    if (M->family != SUBAP_FAMILY_KRR && (prec == SUBAP_BF16X3 || prec == SUBAP_FP16X3))
      return invalid("split 16-bit fallback is for the kernel family only");
    if (rhs_varies(M->family)) {
      set_error("the surrogate's acceptance test is implemented for right-hand sides independent of p");
      return SUBAP_E_UNSUPPORTED;
    }
    if (m > (int64_t(1) << 31) / 64) return invalid("m too large for one call");
    return surrogate_solve(M, s->impl, P, m, tol, y, accepted, status, prec, refine, csne != 0, n_acc,
                           static_cast<hipStream_t>(hip_stream), sigma_min);
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_surrogate_solve_batch(subap_model M, subap_surrogate s, const double* P, int64_t m, double tol,
                                         double* y, uint8_t* accepted, int32_t* status,
                                         const subap_solve_opts* fb, int64_t* n_acc, void* hip_stream) {
  return surrogate_solve_checked(M, s, P, m, tol, y, accepted, status, fb, n_acc, hip_stream, 0.0);
}

subap_status subap_surrogate_solve_batch_excess(subap_model M, subap_surrogate s, const double* P, int64_t m,
                                                double sigma_min, double tol, double* y, uint8_t* accepted,
                                                int32_t* status, const subap_solve_opts* fb, int64_t* n_acc,
                                                void* hip_stream) {
  if (!(sigma_min > 0.0) || !std::isfinite(sigma_min)) {
    clear_error();
    return invalid("sigma_min must be finite and > 0");
  }
  return surrogate_solve_checked(M, s, P, m, tol, y, accepted, status, fb, n_acc, hip_stream, sigma_min);
}

subap_status subap_surrogate_free(subap_surrogate s) {
  try {
    clear_error();
    if (!s) return SUBAP_OK;
    (void)hipDeviceSynchronize();
    surrogate_free(s->impl);
    delete s;
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_exp2_rate(int32_t form, int64_t evals, double* evals_per_s, void* hip_stream) {
  try {
    clear_error();
    if (!evals_per_s) return invalid("evals_per_s must not be NULL");
    if (form != 0 && form != 7 && form != 9 && form != 11) return invalid("form must be 0, 7, 9 or 11");
    if (evals < 1 || evals > (int64_t(1) << 40)) return invalid("evals must be in [1, 2^40]");
    return exp2_rate(form, evals, evals_per_s, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_profile_enable(int32_t on) {
  try {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_profile_reset(void) {
  try {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_drain();
    g_prof_totals.clear();
    g_prof_names.clear();
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

int32_t subap_profile_count(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  prof_drain();
  return static_cast<int32_t>(g_prof_names.size());
}

subap_status subap_profile_entry(int32_t i, const char** name, int64_t* calls, double* total_ms) {
  try {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (i < 0 || i >= static_cast<int32_t>(g_prof_names.size())) {
      set_error("profile entry index out of range");
      return SUBAP_E_INVALID;
    }
    const std::string& nm = g_prof_names[i];
    const ProfTotal& t = g_prof_totals[nm];
    if (name) *name = nm.c_str();
    if (calls) *calls = t.calls;
    if (total_ms) *total_ms = t.ms;
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

subap_status subap_model_free(subap_model M) {
  try {
    clear_error();
    if (!M) return SUBAP_OK;
    (void)hipDeviceSynchronize();
    free_model(M);
    return SUBAP_OK;
  } catch (...) {
    return host_exception();
  }
}

}  // extern "C"
