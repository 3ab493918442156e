// Batched online solve over many finite-difference models of uneven size in
// one persistent launch.  Each block repeatedly takes the next work item (one
// parameter of one instance) from a global counter, generates its s rows
// (face coefficients), forms S A(p) Q (eq. (3.4)) in LDS, solves the least
// squares problem (eq. (3.3)) by Householder QR in LDS, optionally refines in
// FP64, and writes y.  The LDS formulation handles any s <= 256, r <= 64, so
// instances of every shape share one kernel; items are ordered largest
// instance first so the long solves start early.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <numeric>
#include <sstream>
#include <sys/stat.h>
#include <string>
#include <vector>

#include "common.h"
#include "profile.h"

namespace subap {

struct MultiInst {
  int r, s, F, DP;
  const double* phi;
  const double* delta64;
  const float* delta32;
  const double* bS;
  double inv_h2, bS_norm;
  const double* params;
  int64_t m;
  double* y;
  double* rho;
  int32_t* status;
  int64_t begin;  // first global item index of this instance
};

namespace {

constexpr int kMT = 256;  // threads per block (upper bound; launch may use 128)

struct MultiArgs {
  const MultiInst* inst;
  int k;
  int64_t total;
  unsigned long long* counter;
  int prec;
  int refine;
  int lds_r;  // leading dimension of G in LDS (max r + 1)
  int lds_s;  // rows of G in LDS (max s)
};

// block-wide sum; every thread returns the same value (fixed order)
__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x / 64;
  __syncthreads();
  if (threadIdx.x % 64 == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x / 64;
  for (int i = 0; i < nw; ++i) t += red[i];
  return t;
}

__global__ void k_reset(unsigned long long* c) { *c = 0ull; }

__global__ __launch_bounds__(kMT) void k_fd_multi(MultiArgs A) {
  extern __shared__ double lds[];
  const int LD = A.lds_r;
  double* G = lds;                              // lds_s x LD
  double* bv = G + A.lds_s * LD;                // lds_s
  double* b0 = bv + A.lds_s;                    // lds_s
  double* af = b0 + A.lds_s;                    // lds_s x 6
  double* tau = af + A.lds_s * 6;               // 64
  double* yv = tau + kMaxR;                     // 64
  double* wv = yv + kMaxR;                      // 65
  double* red = wv + kMaxR + 1;                 // 4
  long long* item_s = reinterpret_cast<long long*>(red + 4);
  const int tid = threadIdx.x, nt = blockDim.x;

  while (true) {
    __syncthreads();
    if (tid == 0) {
      const long long it = static_cast<long long>(atomicAdd(A.counter, 1ull));
      int lo = 0, hi = A.k - 1;  // instance with begin <= it (begins are increasing)
      while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (A.inst[mid].begin <= it) lo = mid;
        else hi = mid - 1;
      }
      item_s[0] = it;
      item_s[1] = lo;
    }
    __syncthreads();
    const long long item = item_s[0];
    if (item >= A.total) return;  // uniform: every wave leaves the loop
    const MultiInst I = A.inst[item_s[1]];
    const int64_t p = item - I.begin;
    const int r = I.r, s = I.s, F = I.F, DP = I.DP;
    double pv[4] = {0.0, 0.0, 0.0, 0.0};
    bool finite = true;
    for (int q = 0; q < DP; ++q) {
      pv[q] = I.params[p * DP + q];
      finite = finite && isfinite(pv[q]);
    }
    // A1: face coefficients
    for (int idx = tid; idx < s * F; idx += nt) {
      const int k = idx / F, f = idx % F;
      double t = 0.0;
      for (int q = 0; q < DP; ++q) t += pv[q] * I.phi[(f * DP + q) * s + k];
      af[k * 6 + f] = exp(t) * I.inv_h2;
    }
    __syncthreads();
    // A2: S A(p) Q into LDS (threads walk k fastest: coalesced table reads)
    for (int idx = tid; idx < s * r; idx += nt) {
      const int c = idx / s, k = idx % s;
      double g;
      if (A.prec == SUBAP_FP64) {
        g = 0.0;
        for (int f = 0; f < F; ++f) g += af[k * 6 + f] * I.delta64[(f * r + c) * s + k];
      } else {
        float g32 = 0.0f;
        for (int f = 0; f < F; ++f)
          g32 = fmaf(static_cast<float>(af[k * 6 + f]), I.delta32[(f * r + c) * s + k], g32);
        g = g32;
      }
      G[k * LD + c] = g;
    }
    for (int k = tid; k < s; k += nt) {
      b0[k] = I.bS[k];
      bv[k] = I.bS[k];
    }
    __syncthreads();
    // A3: Householder QR in LDS, applied to bv as well
    bool full_rank = true;
    double r00 = 0.0;
    for (int j = 0; j < r; ++j) {
      double ss = 0.0;
      for (int i = j + 1 + tid; i < s; i += nt) ss += G[i * LD + j] * G[i * LD + j];
      ss = block_sum(ss, red);
      const double alpha = G[j * LD + j];
      double tj = 0.0, scale = 0.0, beta = alpha;
      if (ss > 0.0) {
        const double norm = sqrt(alpha * alpha + ss);
        beta = alpha >= 0.0 ? -norm : norm;
        tj = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      __syncthreads();
      for (int i = j + 1 + tid; i < s; i += nt) G[i * LD + j] *= scale;
      __syncthreads();
      // w_c = v^T G[:, c] for c in (j, r) and for b (c == r); 4 lanes per column
      const int ncol = r - j;  // columns j+1..r-1 plus b
      for (int cc = tid / 4; cc < ncol; cc += nt / 4) {
        const int c = j + 1 + cc;  // c == r means b
        double t = 0.0;
        for (int i = j + (tid & 3); i < s; i += 4) {
          const double v = (i == j) ? 1.0 : G[i * LD + j];
          t += v * (c < r ? G[i * LD + c] : bv[i]);
        }
        t += __shfl_xor(t, 1, 64);
        t += __shfl_xor(t, 2, 64);
        if ((tid & 3) == 0) wv[cc] = t;
      }
      __syncthreads();
      for (int idx = tid; idx < (s - j) * ncol; idx += nt) {
        const int i = j + idx / ncol, cc = idx % ncol, c = j + 1 + cc;
        const double v = (i == j) ? 1.0 : G[i * LD + j];
        const double d = tj * wv[cc] * v;
        if (c < r) G[i * LD + c] -= d;
        else bv[i] -= d;
      }
      __syncthreads();
      if (tid == 0) {
        G[j * LD + j] = beta;
        tau[j] = tj;
      }
      const double ab = fabs(beta);
      if (j == 0) r00 = ab;
      if (!(ab > kRankTol * r00)) full_rank = false;
    }
    __syncthreads();
    double tail = 0.0;
    {
      double t = 0.0;
      for (int i = r + tid; i < s; i += nt) t += bv[i] * bv[i];
      tail = sqrt(block_sum(t, red));
    }
    // back substitution R y = (Q^T b)[0:r], overwriting bv
    for (int c = r - 1; c >= 0; --c) {
      const double yc = bv[c] / G[c * LD + c];
      __syncthreads();
      for (int i = tid; i < c; i += nt) bv[i] -= G[i * LD + c] * yc;
      if (tid == 0) yv[c] = yc;
      __syncthreads();
    }
    // A4: FP64 refinement with the same factorisation; residual in bv
    auto residual = [&]() {
      for (int k = tid; k < s; k += nt) {
        double t = 0.0;
        for (int f = 0; f < F; ++f) {
          double u = 0.0;
          for (int c = 0; c < r; ++c) u += I.delta64[(f * r + c) * s + k] * yv[c];
          t += af[k * 6 + f] * u;
        }
        bv[k] = t - b0[k];
      }
      __syncthreads();
    };
    for (int it = 0; it < A.refine; ++it) {
      residual();
      for (int j = 0; j < r; ++j) {
        double t = 0.0;
        for (int i = j + tid; i < s; i += nt) t += ((i == j) ? 1.0 : G[i * LD + j]) * bv[i];
        t = block_sum(t, red) * tau[j];
        for (int i = j + tid; i < s; i += nt) bv[i] -= t * ((i == j) ? 1.0 : G[i * LD + j]);
        __syncthreads();
      }
      for (int c = r - 1; c >= 0; --c) {
        const double dc = bv[c] / G[c * LD + c];
        __syncthreads();
        for (int i = tid; i < c; i += nt) bv[i] -= G[i * LD + c] * dc;
        if (tid == 0) yv[c] -= dc;
        __syncthreads();
      }
    }
    double rho = tail;
    if (A.refine > 0 || A.prec != SUBAP_FP64) {
      residual();
      double t = 0.0;
      for (int k = tid; k < s; k += nt) t += bv[k] * bv[k];
      rho = sqrt(block_sum(t, red));
    }
    __syncthreads();
    bool yfin = true;
    for (int c = 0; c < r; ++c) yfin = yfin && isfinite(yv[c]);
    int32_t code = SUBAP_OK;
    if (!finite) code = SUBAP_E_NONFINITE;
    else if (!full_rank) code = SUBAP_E_RANK;
    else if (!yfin) code = SUBAP_E_NONFINITE;
    for (int c = tid; c < r; c += nt)
      I.y[p * r + c] = code == SUBAP_OK ? yv[c] : __longlong_as_double(0x7ff8000000000000LL);
    if (tid == 0) {
      if (I.rho) I.rho[p] = rho / I.bS_norm;
      if (I.status) I.status[p] = code;
    }
  }
}

size_t lds_bytes(int max_s, int max_r) {
  const int LD = max_r + 1;
  return sizeof(double) * (static_cast<size_t>(max_s) * LD + 2 * max_s + 6 * max_s + kMaxR + kMaxR +
                           (kMaxR + 1) + 4) + 2 * sizeof(long long);
}

}  // namespace

// ---------------------------------------------------------------------------
// plans: instance table, launch shape (autotuned, cached), hipGraph
// ---------------------------------------------------------------------------
struct PlanImpl {
  std::vector<MultiInst> inst;   // host copy, largest first
  MultiInst* inst_d = nullptr;
  unsigned long long* counter = nullptr;
  int64_t total = 0;
  int max_s = 0, max_r = 0;
  int prec = 0, refine = 0;
  int threads = 256, blocks = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string key;
};

namespace {

subap_status launch_plan(PlanImpl* P, hipStream_t st) {
  MultiArgs a{P->inst_d, static_cast<int>(P->inst.size()), P->total, P->counter, P->prec, P->refine,
              P->max_r + 1, P->max_s};
  ProfScope prof("fd_multi_persistent", st);
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, st, P->counter);
  hipLaunchKernelGGL(k_fd_multi, dim3(P->blocks), dim3(P->threads), lds_bytes(P->max_s, P->max_r), st, a);
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

std::string cache_path() {
  const char* e = std::getenv("SUBAP_AUTOTUNE_CACHE");
  if (e && *e) return e;
  const char* h = std::getenv("HOME");
  return std::string(h ? h : "/tmp") + "/.cache/subap_autotune.txt";
}

bool cache_lookup(const std::string& key, int* threads, int* blocks) {
  std::ifstream f(cache_path());
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string k;
    int t, b;
    if (is >> k >> t >> b && k == key) {
      *threads = t;
      *blocks = b;
      return true;
    }
  }
  return false;
}

void cache_store(const std::string& key, int threads, int blocks) {
  const std::string path = cache_path();
  const size_t slash = path.find_last_of('/');
  if (slash != std::string::npos && slash > 0) (void)::mkdir(path.substr(0, slash).c_str(), 0755);
  std::ofstream f(path, std::ios::app);
  if (f) f << key << ' ' << threads << ' ' << blocks << '\n';
}

}  // namespace

subap_status plan_build(subap_model_s* const* models, int k, const double* const* params, const int64_t* m,
                        double* const* y, double* const* rho, int32_t* const* status, int prec, int refine,
                        int flags, hipStream_t st, PlanImpl** out) {
  PlanImpl* P = new (std::nothrow) PlanImpl();
  if (!P) return SUBAP_E_NOMEM;
  auto fail = [&](subap_status rc) {
    dfree(P->inst_d);
    dfree(P->counter);
    delete P;
    return rc;
  };
  std::vector<int> order(k);
  std::iota(order.begin(), order.end(), 0);
  // largest per-item cost first (s r^2 dominates)
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const double ca = double(models[a]->s) * models[a]->r * models[a]->r;
    const double cb = double(models[b]->s) * models[b]->r * models[b]->r;
    return ca > cb;
  });
  std::ostringstream key;
  key << "fd_multi/p" << prec << "/f" << refine;
  int64_t begin = 0;
  for (int oi : order) {
    const subap_model_s* M = models[oi];
    MultiInst I{M->r, M->s, M->F, M->d, M->phi, M->delta64, M->delta32, M->bS, M->inv_h2, M->bS_norm,
                params[oi], m[oi], y[oi], rho ? rho[oi] : nullptr, status ? status[oi] : nullptr, begin};
    P->inst.push_back(I);
    begin += m[oi];
    P->max_s = std::max(P->max_s, M->s);
    P->max_r = std::max(P->max_r, M->r);
    key << '/' << M->s << 'x' << M->r << 'x' << m[oi];
  }
  P->total = begin;
  P->prec = prec;
  P->refine = refine;
  P->key = key.str();
  subap_status rc = dalloc(&P->inst_d, P->inst.size());
  if (rc != SUBAP_OK) return fail(rc);
  rc = dalloc(&P->counter, 1);
  if (rc != SUBAP_OK) return fail(rc);
  if (hipMemcpyAsync(P->inst_d, P->inst.data(), sizeof(MultiInst) * P->inst.size(), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    set_error("copying the instance table failed");
    return fail(SUBAP_E_HIP);
  }
  const size_t lds = lds_bytes(P->max_s, P->max_r);
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(k_fd_multi), hipFuncAttributeMaxDynamicSharedMemorySize,
                          static_cast<int>(lds)) != hipSuccess) {
    set_error("cannot reserve LDS for the persistent kernel");
    return fail(SUBAP_E_HIP);
  }
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int per_cu = std::max(1, static_cast<int>((160 * 1024) / std::max<size_t>(lds, 1)));
  P->threads = 256;
  P->blocks = cus * std::min(per_cu, 4);
  const bool tune = flags & SUBAP_PLAN_AUTOTUNE;
  int t_c, b_c;
  if (cache_lookup(P->key, &t_c, &b_c)) {
    P->threads = t_c;
    P->blocks = b_c;
  } else if (tune) {
    // time every candidate launch shape twice on the real plan, keep the fastest
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    int bt = P->threads, bb = P->blocks;
    for (int th : {128, 256}) {
      for (int mult : {1, 2, 4, 8}) {
        if (mult > per_cu * 2) continue;
        P->threads = th;
        P->blocks = cus * mult;
        float tot = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {
          (void)hipEventRecord(e0, st);
          rc = launch_plan(P, st);
          if (rc != SUBAP_OK) return fail(rc);
          (void)hipEventRecord(e1, st);
          (void)hipEventSynchronize(e1);
          float ms = 0.0f;
          (void)hipEventElapsedTime(&ms, e0, e1);
          if (rep == 1) tot = ms;  // first run warms up
        }
        if (tot < best) {
          best = tot;
          bt = th;
          bb = P->blocks;
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P->threads = bt;
    P->blocks = bb;
    cache_store(P->key, bt, bb);
  }
  if (flags & SUBAP_PLAN_GRAPH) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
      set_error("cannot create the capture stream");
      return fail(SUBAP_E_HIP);
    }
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      MultiArgs a{P->inst_d, static_cast<int>(P->inst.size()), P->total, P->counter, P->prec, P->refine,
                  P->max_r + 1, P->max_s};
      hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, cs, P->counter);
      hipLaunchKernelGGL(k_fd_multi, dim3(P->blocks), dim3(P->threads), lds, cs, a);
      ok = hipStreamEndCapture(cs, &P->graph) == hipSuccess;
    }
    ok = ok && hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0) == hipSuccess;
    (void)hipStreamDestroy(cs);
    if (!ok) {
      (void)hipGetLastError();
      if (P->graph) (void)hipGraphDestroy(P->graph);
      P->graph = nullptr;
      set_error("hipGraph capture of the persistent launch failed");
      return fail(SUBAP_E_HIP);
    }
  }
  *out = P;
  return SUBAP_OK;
}

subap_status plan_execute(PlanImpl* P, hipStream_t st) {
  if (P->exec) {
    ProfScope prof("fd_multi_persistent", st);
    SUBAP_HIP_TRY(hipGraphLaunch(P->exec, st));
    return SUBAP_OK;
  }
  return launch_plan(P, st);
}

void plan_free(PlanImpl* P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  dfree(P->inst_d);
  dfree(P->counter);
  delete P;
}

// Single-model solve through the LDS kernel, for (s, r) shapes the register
// kernel is not instantiated for.  The one-entry instance table and the work
// counter are allocated once per model.
subap_status fd_solve_lds(subap_model_s* M, const double* params, int64_t m, double* y, double* rho,
                          int32_t* status, int prec, int refine, hipStream_t st) {
  if (!M->lds_inst) {
    SUBAP_TRY(dalloc(reinterpret_cast<MultiInst**>(&M->lds_inst), 1));
    SUBAP_TRY(dalloc(reinterpret_cast<unsigned long long**>(&M->lds_counter), 1));
  }
  MultiInst I{M->r, M->s, M->F, M->d, M->phi, M->delta64, M->delta32, M->bS, M->inv_h2, M->bS_norm,
              params, m, y, rho, status, 0};
  // pageable source: the copy is staged before hipMemcpyAsync returns
  SUBAP_HIP_TRY(hipMemcpyAsync(M->lds_inst, &I, sizeof(I), hipMemcpyHostToDevice, st));
  const size_t lds = lds_bytes(M->s, M->r);
  SUBAP_HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(k_fd_multi),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int per_cu = std::max(1, std::min(4, static_cast<int>((160 * 1024) / lds)));
  const int64_t blocks = std::min<int64_t>(m, static_cast<int64_t>(cus) * per_cu);
  MultiArgs a{static_cast<const MultiInst*>(M->lds_inst), 1, m,
              static_cast<unsigned long long*>(M->lds_counter), prec, refine, M->r + 1, M->s};
  ProfScope prof("fd_solve_lds", st);
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(1), 0, st, static_cast<unsigned long long*>(M->lds_counter));
  hipLaunchKernelGGL(k_fd_multi, dim3(static_cast<unsigned>(blocks)), dim3(256), lds, st, a);
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

void plan_shape(const PlanImpl* P, int* threads, int* blocks) {
  *threads = P->threads;
  *blocks = P->blocks;
}

}  // namespace subap
