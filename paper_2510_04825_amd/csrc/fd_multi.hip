// Batched online solve over many finite-difference models of uneven size in
// one persistent launch.  Each wavefront repeatedly takes the next work item
// (one parameter of one instance) from a work counter and solves it with the
// column-per-lane Householder routine of fd_cols.h (rows generated on the
// fly, eq. (3.4) contraction in FP64 or FP32, eq. (3.3) least squares,
// optional FP64 refinement).  Every instance with r <= 64 and s <= 256 shares
// the kernel.
//
// The instances are split into kXcds groups of about equal work (largest
// first, each to the least-loaded group), one group per XCD: workgroups are
// dispatched to the XCDs in turn (block b to XCD b mod 8), and a wavefront
// takes items from its own XCD's counter first, so each XCD's L2 holds the
// tables of its own instances.  When its group is done it takes items from
// the other groups' counters in turn, and it leaves once every counter has
// passed the end of its group.  Within a group, the largest instances come
// first so the long solves start early.  The FP64 kernel is built for two
// waves per SIMD; the refining kernel, whose solver needs more registers,
// for one.  Both are instantiated per set of model dimensions (2-D, 3-D,
// both), so a plan of one kind carries one solver.
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
#include "fd_cols.h"
#include "profile.h"

namespace subap {

struct MultiInst {
  int r, s, F, DP;
  const double* phi;
  const double* delta64T;
  const float* delta32T;
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

constexpr int kMT = 256;  // threads per block (upper bound; launch may use 64 or 128)
constexpr int kXcds = 8;  // XCDs of the device: one work group each

// waves per CU the kernel is built for: two per SIMD, one when refining
constexpr int waves_per_cu(bool ref) { return ref ? 4 : 8; }

struct MultiArgs {
  const MultiInst* inst;
  int k;
  int64_t total;
  unsigned long long* counter;  // kXcds counters
  int64_t group[kXcds + 1];     // items [group[x], group[x + 1]) belong to XCD x
  int prec;
  int refine;
  int ldsw;  // LDS doubles per wavefront
  bool csne;  // refinement by the corrected semi-normal equations
};

__global__ void k_reset(unsigned long long* c) {
  if (threadIdx.x < kXcds) c[threadIdx.x] = 0ull;
}

template <int F, int DP, bool REF>
__device__ __forceinline__ void multi_item(const MultiInst& I, int64_t p, int prec, int refine, bool csne,
                                           double* lds, int lane) {
  const ColsModel M{I.r, I.s, I.phi, I.delta64T, I.delta32T, I.bS, I.inv_h2, I.bS_norm};
  double* yo = I.y + p * I.r;
  double* ro = I.rho ? I.rho + p : nullptr;
  int32_t* so = I.status ? I.status + p : nullptr;
  if (I.r == 64) cols_solve<F, DP, true, REF>(M, I.params + p * DP, prec, refine, csne, lds, I.s, lane, yo, ro, so);
  else cols_solve<F, DP, false, REF>(M, I.params + p * DP, prec, refine, csne, lds, I.s, lane, yo, ro, so);
}

// REF: FP32 contraction or refinement steps (uniform over the launch).
// DIMS: bit 0 = the plan holds 2-D models, bit 1 = 3-D models; a kernel that
// serves one kind only carries one solver and needs fewer registers.
template <bool REF, int DIMS>
__global__ __launch_bounds__(kMT, REF ? 1 : 2) void k_fd_multi(MultiArgs A) {
  extern __shared__ double lds[];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  double* mine = lds + static_cast<int64_t>(wave) * A.ldsw;
  const int home = static_cast<int>(blockIdx.x % kXcds);
  int d = 0;  // groups passed: own first, then the others in turn
  while (d < kXcds) {
    const int x = (home + d) % kXcds;
    unsigned long long c = 0;
    if (lane == 0) c = atomicAdd(A.counter + x, 1ull);
    c = (static_cast<unsigned long long>(static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(c >> 32))))
         << 32) |
        static_cast<unsigned>(__builtin_amdgcn_readfirstlane(static_cast<int>(c & 0xffffffffull)));
    const int64_t it = A.group[x] + static_cast<int64_t>(c);
    if (it >= A.group[x + 1]) {  // uniform per wavefront
      ++d;
      continue;
    }
    int lo = 0, hi = A.k - 1;  // instance with begin <= it (begins are increasing)
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (A.inst[mid].begin <= it) lo = mid;
      else hi = mid - 1;
    }
    const MultiInst I = A.inst[lo];
    const int64_t p = it - I.begin;
    if constexpr (DIMS == 1) multi_item<4, 2, REF>(I, p, A.prec, A.refine, A.csne, mine, lane);
    else if constexpr (DIMS == 2) multi_item<6, 4, REF>(I, p, A.prec, A.refine, A.csne, mine, lane);
    else if (I.F == 4) multi_item<4, 2, REF>(I, p, A.prec, A.refine, A.csne, mine, lane);
    else multi_item<6, 4, REF>(I, p, A.prec, A.refine, A.csne, mine, lane);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// plans: instance table, launch shape (autotuned, cached), hipGraph
// ---------------------------------------------------------------------------
// A plan member that the persistent kernel does not take: a model of another
// family (the kernel family, the delay system, eq. (5.7), the identity
// family, the affine family), or a diffusion model whose form fd_solve gives
// to the matrix-core semi-normal solve (FP64 without refinement, s >= 96,
// 16 <= r <= 47) with a batch that fills that kernel's first round on the
// device (two parameters per wavefront, eight wavefronts per CU); smaller
// ones stay in the persistent launch, where they overlap the other members
// instead of adding an underfilled launch after it.  Each is solved by its
// family's batched solver, enqueued after the persistent kernel on the same
// stream.
struct OtherInst {
  subap_model_s* M;
  const double* params;
  int64_t m;
  double* y;
  double* rho;
  int32_t* status;
};

struct PlanImpl {
  std::vector<MultiInst> inst;   // host copy of the diffusion members, largest first
  MultiInst* inst_d = nullptr;
  std::vector<OtherInst> other;  // the other members, in the caller's order
  void* work = nullptr;          // workspace of the kernel-family members (the largest one's)
  unsigned long long* counter = nullptr;
  int64_t total = 0;
  int max_s = 0, max_r = 0;
  int prec = 0, refine = 0;
  bool csne = false;
  int dims = 0;  // bit 0: some model is 2-D, bit 1: some model is 3-D
  int64_t group[kXcds + 1] = {};  // item range of each XCD's group
  int threads = 256, blocks = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::string key;
};

namespace {

bool plan_ref(const PlanImpl* P);

size_t plan_lds(const PlanImpl* P, int threads) {
  return sizeof(double) * static_cast<size_t>(threads / 64) * cols_lds_doubles(P->max_r, P->max_s, plan_ref(P));
}

bool plan_ref(const PlanImpl* P) { return P->refine > 0 || P->prec != SUBAP_FP64; }

using MultiKernel = void (*)(MultiArgs);

MultiKernel plan_kernel(bool ref, int dims) {
  static const MultiKernel tab[2][3] = {
      {k_fd_multi<false, 1>, k_fd_multi<false, 2>, k_fd_multi<false, 3>},
      {k_fd_multi<true, 1>, k_fd_multi<true, 2>, k_fd_multi<true, 3>}};
  return tab[ref ? 1 : 0][dims - 1];
}

// counter reset + the persistent kernel, then the other members' solves, on
// st (also used under capture; nothing here allocates or synchronizes)
subap_status enqueue_plan(const PlanImpl* P, hipStream_t st, bool others = true) {
  if (!P->inst.empty()) {
  MultiArgs a{};
  a.inst = P->inst_d;
  a.k = static_cast<int>(P->inst.size());
  a.total = P->total;
  a.counter = P->counter;
  for (int x = 0; x <= kXcds; ++x) a.group[x] = P->group[x];
  a.prec = P->prec;
  a.refine = P->refine;
  a.ldsw = cols_lds_doubles(P->max_r, P->max_s, plan_ref(P));
  a.csne = P->csne;
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, st, P->counter);
  hipLaunchKernelGGL(plan_kernel(plan_ref(P), P->dims), dim3(P->blocks), dim3(P->threads),
                     plan_lds(P, P->threads), st, a);
  }
  if (!others) return SUBAP_OK;
  for (const OtherInst& o : P->other) {
    if (o.m == 0) continue;
    if (o.M->family == SUBAP_FAMILY_KRR)
      SUBAP_TRY(krr_solve_ws(o.M, o.params, o.m, o.y, o.rho, o.status, P->prec, P->refine, P->csne, P->work, st));
    else
      SUBAP_TRY(fd_solve(o.M, o.params, o.m, o.y, o.rho, o.status, P->prec, P->refine, P->csne, st));
  }
  return SUBAP_OK;
}

subap_status launch_plan(PlanImpl* P, hipStream_t st, bool others = true) {
  ProfScope prof("fd_multi_persistent", st);
  SUBAP_TRY(enqueue_plan(P, st, others));
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
                        bool csne, int flags, hipStream_t st, PlanImpl** out) {
  PlanImpl* P = new (std::nothrow) PlanImpl();
  if (!P) return SUBAP_E_NOMEM;
  auto fail = [&](subap_status rc) {
    dfree(P->inst_d);
    dfree(P->counter);
    dfree(P->work);
    delete P;
    return rc;
  };
  P->prec = prec;
  P->refine = refine;
  P->csne = csne && refine > 0;
  // members the persistent kernel takes (diffusion models) and the others
  std::vector<int> order;
  size_t work_bytes = 0;
  int cus = 256;
  {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  }
  const int64_t gram_min_m = int64_t(16) * cus;
  for (int i = 0; i < k; ++i) {
    subap_model_s* M = models[i];
    if ((M->family == SUBAP_FAMILY_DIFF2D || M->family == SUBAP_FAMILY_DIFF3D) &&
        !(m[i] >= gram_min_m && fd_solve_on_matrix_cores(M, prec, refine))) {
      order.push_back(i);
      continue;
    }
    P->other.push_back(OtherInst{M, params[i], m[i], y[i], rho ? rho[i] : nullptr, status ? status[i] : nullptr});
    if (M->family == SUBAP_FAMILY_KRR && m[i] > 0) {
      const size_t b = krr_work_bytes(M, m[i], prec, refine, P->csne);
      if (b == 0) {
        set_error("no least-squares kernel for a kernel-family member's (s, r)");
        return fail(SUBAP_E_UNSUPPORTED);
      }
      work_bytes = std::max(work_bytes, b);
    }
  }
  if (work_bytes > 0) {
    char* w = nullptr;
    subap_status rw = dalloc(&w, work_bytes);
    if (rw != SUBAP_OK) return fail(rw);
    P->work = w;
  }
  // largest per-item cost first (s r^2 dominates)
  auto item_cost = [&](int a) { return double(models[a]->s) * models[a]->r * models[a]->r; };
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return item_cost(a) > item_cost(b); });
  // instances to XCD groups: largest total work first, each to the group with
  // the least work so far; then group by group, largest items first
  std::vector<int> by_work(order);
  std::stable_sort(by_work.begin(), by_work.end(),
                   [&](int a, int b) { return item_cost(a) * m[a] > item_cost(b) * m[b]; });
  std::vector<int> grp(k, 0);
  double load[kXcds] = {};
  for (int oi : by_work) {
    const int g = static_cast<int>(std::min_element(load, load + kXcds) - load);
    grp[oi] = g;
    load[g] += item_cost(oi) * m[oi];
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return grp[a] < grp[b]; });
  std::ostringstream key;
  key << "fd_multi/p" << prec << "/f" << refine << (csne ? "c" : "");
  int64_t begin = 0;
  for (int x = 0; x <= kXcds; ++x) P->group[x] = 0;
  for (int oi : order) {
    for (int x = grp[oi] + 1; x <= kXcds; ++x) P->group[x] += m[oi];
    const subap_model_s* M = models[oi];
    MultiInst I{M->r, M->s, M->F, M->d, M->phi, M->delta64T, M->delta32T, M->bS, M->inv_h2, M->bS_norm,
                params[oi], m[oi], y[oi], rho ? rho[oi] : nullptr, status ? status[oi] : nullptr, begin};
    P->inst.push_back(I);
    begin += m[oi];
    P->max_s = std::max(P->max_s, M->s);
    P->max_r = std::max(P->max_r, M->r);
    P->dims |= M->F == 4 ? 1 : 2;
    key << '/' << (M->F == 4 ? 2 : 3) << 'd' << M->s << 'x' << M->r << 'x' << m[oi];
  }
  P->total = begin;
  P->key = key.str();
  subap_status rc = SUBAP_OK;
  if (!P->inst.empty()) {
  rc = dalloc(&P->inst_d, P->inst.size());
  if (rc != SUBAP_OK) return fail(rc);
  rc = dalloc(&P->counter, kXcds);
  if (rc != SUBAP_OK) return fail(rc);
  if (hipMemcpyAsync(P->inst_d, P->inst.data(), sizeof(MultiInst) * P->inst.size(), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    set_error("copying the instance table failed");
    return fail(SUBAP_E_HIP);
  }
  const size_t lds_max = plan_lds(P, kMT);
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(plan_kernel(plan_ref(P), P->dims)),
                          hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds_max)) != hipSuccess) {
    set_error("cannot reserve LDS for the persistent kernel");
    return fail(SUBAP_E_HIP);
  }
  // blocks of th threads that fit one CU: LDS (160 KiB) and the waves per
  // SIMD the kernel is built for
  auto per_cu = [&](int th) {
    const int by_lds = static_cast<int>((160 * 1024) / std::max<size_t>(plan_lds(P, th), 1));
    return std::max(1, std::min(by_lds, waves_per_cu(plan_ref(P)) / (th / 64)));
  };
  P->threads = 128;
  P->blocks = cus * per_cu(128);
  const bool tune = flags & SUBAP_PLAN_AUTOTUNE;
  int t_c, b_c;
  // a cached shape is used only if it is one this plan could have chosen
  const bool cached = cache_lookup(P->key, &t_c, &b_c) && (t_c == 64 || t_c == 128 || t_c == 256) && b_c >= 1 &&
                      b_c <= cus * per_cu(t_c);
  if (cached) {
    P->threads = t_c;
    P->blocks = b_c;
  } else if (tune) {
    // time every candidate launch shape twice on the real plan, keep the fastest
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 1e30f;
    int bt = P->threads, bb = P->blocks;
    for (int th : {64, 128, 256}) {
      for (int mult = 1; mult <= per_cu(th); ++mult) {
        P->threads = th;
        P->blocks = cus * mult;
        float tot = 0.0f;
        for (int rep = 0; rep < 2; ++rep) {
          (void)hipEventRecord(e0, st);
          rc = launch_plan(P, st, false);  // the persistent kernel alone
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
  }  // diffusion members
  if (flags & SUBAP_PLAN_GRAPH) {
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
      set_error("cannot create the capture stream");
      return fail(SUBAP_E_HIP);
    }
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      const subap_status er = enqueue_plan(P, cs);
      ok = hipStreamEndCapture(cs, &P->graph) == hipSuccess && er == SUBAP_OK;
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
  dfree(P->work);
  delete P;
}

void plan_shape(const PlanImpl* P, int* threads, int* blocks) {
  *threads = P->threads;
  *blocks = P->blocks;
}

}  // namespace subap
