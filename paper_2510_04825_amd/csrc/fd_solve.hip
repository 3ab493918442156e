// Online solve for the finite-difference diffusion families, fully fused:
// one team of lanes per parameter p* generates the s selected rows of A(p*)
// (face coefficients a_f = exp(sum_q p_q phi_q) at the s x F faces, Section
// 3.1 "Computing S A(p*) X"), contracts them with the face-difference table
// Delta_{k,f} = Q[i_k] - Q[nb_f(i_k)] into S A(p*) Q (eq. (3.4)), solves the
// s x r least-squares problem (eq. (3.3)) by Householder QR in registers and
// optionally refines in FP64.  Row k of S A(p) Q is sum_f a_f Delta_{k,f} / h^2
// because the diagonal of row i_k is the sum of its face coefficients.
#include <hip/hip_runtime.h>

#include "common.h"
#include "profile.h"
#include "fd_cols.h"
#include "fd_gram.h"
#include "team_qr.h"

namespace subap {
namespace {

struct FDArgs {
  const double* params;
  int64_t m;
  int r, s;
  const double* phi;
  const double* delta64;
  const float* delta32;
  const double* delta64T;
  const float* delta32T;
  const double* bS;
  double inv_h2, bS_norm;
  double* y;
  double* rho;
  int32_t* status;
  int prec;
  int refine;
  double aff_c0, aff_tau;  // delay family only
  bool csne;               // refinement by the corrected semi-normal equations
  const double* wS;        // row weights and per-row data of right-hand sides
  const double* rowdat;    // that vary with p (eq. (5.7), identity family)
};

template <int TEAM, int R, int RM, int F, int DP>
__global__ __launch_bounds__(256) void k_fd_solve(FDArgs A) {
  constexpr int TEAMS = 256 / TEAM;
  __shared__ double s_tau[TEAMS][RM];
  __shared__ double s_y[TEAMS][RM];
  __shared__ double s_dy[TEAMS][RM];
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * TEAMS + team;
  if (p >= A.m) return;  // uniform across the team
  const int r = A.r, s = A.s;
  double* tau = s_tau[team];
  double* yv = s_y[team];
  double* dy = s_dy[team];

  double pv[DP];
  bool finite = true;
#pragma unroll
  for (int q = 0; q < DP; ++q) {
    pv[q] = A.params[p * DP + q];
    finite = finite && isfinite(pv[q]);
  }
  // A1: face coefficients of my rows (scaled by 1/h^2)
  double af[R][F];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = lane + TEAM * q;
#pragma unroll
    for (int f = 0; f < F; ++f) {
      double t = 0.0;
      if (k < s) {
#pragma unroll
        for (int qq = 0; qq < DP; ++qq) t += pv[qq] * A.phi[(f * DP + qq) * s + k];
      }
      af[q][f] = (k < s) ? exp(t) * A.inv_h2 : 0.0;
    }
  }
  // A2: S A(p) Q from the face differences
  TeamQR<TEAM, R, RM> qr;
  double b0[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = lane + TEAM * q;
#pragma unroll
    for (int c = 0; c < RM; ++c) qr.a[q][c] = 0.0;
    if (k < s) {
      if (A.prec == SUBAP_FP64) {
#pragma unroll 1
        for (int f = 0; f < F; ++f)
#pragma unroll
          for (int c = 0; c < RM; ++c)
            if (c < r) qr.a[q][c] += af[q][f] * A.delta64[(f * r + c) * s + k];
      } else {
        float acc[RM];
#pragma unroll
        for (int c = 0; c < RM; ++c) acc[c] = 0.0f;
#pragma unroll 1
        for (int f = 0; f < F; ++f) {
          const float a32 = static_cast<float>(af[q][f]);
#pragma unroll
          for (int c = 0; c < RM; ++c)
            if (c < r) acc[c] = fmaf(a32, A.delta32[(f * r + c) * s + k], acc[c]);
        }
#pragma unroll
        for (int c = 0; c < RM; ++c) qr.a[q][c] = acc[c];
      }
    }
    b0[q] = (k < s) ? A.bS[k] : 0.0;
    qr.b[q] = b0[q];
  }
  // A3: Householder least squares
  qr.factor(r, lane, tau);
  const double tail = qr.tail_norm(qr.b, r, lane);
  {
    double x[R];
#pragma unroll
    for (int q = 0; q < R; ++q) x[q] = qr.b[q];
    qr.back_substitute(x, r, lane, yv);
  }
  // FP64 residual S(A(p) Q y - b) of the current y, distributed like b
  auto residual = [&](double (&res)[R]) {
    // Re-read the table on every use: an opaque copy of the pointer stops the
    // compiler from hoisting F x r loads per row into registers across the
    // factorisation and the refinement loop.
    const double* D64 = A.delta64;
    asm volatile("" : "+s"(D64));
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int k = lane + TEAM * q;
      double t = 0.0;
      if (k < s) {
#pragma unroll 1
        for (int f = 0; f < F; ++f) {
          double u = 0.0;
#pragma unroll
          for (int c = 0; c < RM; ++c)
            if (c < r) u += D64[(f * r + c) * s + k] * yv[c];
          t += af[q][f] * u;
        }
      }
      res[q] = t - b0[q];
    }
  };
  // A4: refinement steps with the same factorisation
  for (int it = 0; it < A.refine; ++it) {
    double res[R];
    residual(res);
    qr.apply_qt(res, r, lane, tau);
    qr.back_substitute(res, r, lane, dy);
#pragma unroll
    for (int c = 0; c < RM; ++c)
      if (c < r) yv[c] -= dy[c];
  }
  double rho;
  if (A.refine > 0 || A.prec != SUBAP_FP64) {
    double res[R];
    residual(res);
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) t += res[q] * res[q];
    rho = sqrt(team_sum<TEAM>(t));
  } else {
    rho = tail;
  }
  bool yfin = true;
  for (int c = 0; c < r; ++c) yfin = yfin && isfinite(yv[c]);
  int32_t code = SUBAP_OK;
  if (!finite) code = SUBAP_E_NONFINITE;
  else if (!qr.full_rank) code = SUBAP_E_RANK;
  else if (!yfin) code = SUBAP_E_NONFINITE;
  for (int c = lane; c < r; c += TEAM) A.y[p * r + c] = (code == SUBAP_OK) ? yv[c] : __longlong_as_double(0x7ff8000000000000LL);
  if (lane == 0) {
    if (A.rho) A.rho[p] = rho / A.bS_norm;
    if (A.status) A.status[p] = code;
  }
}

// Column-per-lane solve (fd_cols.h): one wavefront per parameter, two per block.
template <int F, int DP, bool BRED, bool REF, int COEF, int RB = kColsRB>
__global__ __launch_bounds__(128, REF ? 1 : (BRED ? 2 : 4)) void k_fd_cols(FDArgs A, int ldsw) {
  extern __shared__ double lds_cols[];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * 2 + wave;
  if (p >= A.m) return;  // uniform per wavefront; no block-level barrier follows
  const ColsModel M{A.r, A.s, A.phi, A.delta64T, A.delta32T, A.bS, A.inv_h2, A.bS_norm, A.aff_c0, A.aff_tau,
                    A.wS, A.rowdat};
  cols_solve<F, DP, BRED, REF, COEF, RB>(M, A.params + p * DP, A.prec, A.refine, A.csne,
                                         lds_cols + static_cast<int64_t>(wave) * ldsw, A.s,
                          lane, A.y + p * A.r, A.rho ? A.rho + p : nullptr, A.status ? A.status + p : nullptr);
}

// Semi-normal equations on the matrix cores (fd_gram.h): P parameters per
// wavefront, two wavefronts per block.
template <int F, int DP, int T, int P>
__global__ __launch_bounds__(128, 2) void k_fd_gram(FDArgs A, int ldsw) {
  extern __shared__ double lds_gram[];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t p0 = (static_cast<int64_t>(blockIdx.x) * 2 + wave) * P;
  if (p0 >= A.m) return;  // uniform per wavefront; no block-level barrier follows
  const ColsModel M{A.r, A.s, A.phi, A.delta64T, A.delta32T, A.bS, A.inv_h2, A.bS_norm, A.aff_c0, A.aff_tau,
                    A.wS, A.rowdat};
  gram_solve<F, DP, T, P>(M, A.params, A.m, p0, lds_gram + static_cast<int64_t>(wave) * ldsw, lane, A.y, A.rho,
                          A.status);
}

// The parameters the matrix-core solve deferred (first coefficient
// kGramDefer), solved by column-per-lane Householder.  Each wavefront checks
// 64 parameters with one load per lane and solves the marked ones in turn
// (usually none); a grid-stride loop covers any batch.  Its occupancy does
// not matter (it solves few parameters), so it takes the registers that keep
// the solver from spilling.
template <int F, int DP>
__global__ __launch_bounds__(128, 1) void k_fd_gram_fixup(FDArgs A, int ldsw) {
  extern __shared__ double lds_fix[];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const ColsModel M{A.r, A.s, A.phi, A.delta64T, A.delta32T, A.bS, A.inv_h2, A.bS_norm, A.aff_c0, A.aff_tau,
                    A.wS, A.rowdat};
  const int64_t stride = static_cast<int64_t>(gridDim.x) * 128;
  for (int64_t base = (static_cast<int64_t>(blockIdx.x) * 2 + wave) * 64; base < A.m; base += stride) {
    const int64_t p = base + lane;
    const bool mark =
        p < A.m && static_cast<unsigned long long>(__double_as_longlong(A.y[p * A.r])) == kGramDefer;
    unsigned long long todo = __ballot(mark);  // wave-uniform
    while (todo != 0) {
      const int64_t q = base + __builtin_ctzll(todo);
      todo &= todo - 1;
      cols_solve<F, DP, false, false>(M, A.params + q * DP, SUBAP_FP64, 0, false,
                                      lds_fix + static_cast<int64_t>(wave) * ldsw, A.s, lane, A.y + q * A.r,
                                      A.rho ? A.rho + q : nullptr, A.status ? A.status + q : nullptr);
    }
  }
}

// Column-per-lane solve with four parameters per wavefront (r <= 15, FP64
// without refinement, fd_cols.h): eight parameters per block of two waves.
template <int F, int DP, int COEF, int RB>
__global__ __launch_bounds__(128, 2) void k_fd_cols_packed(FDArgs A, int ldsw) {
  extern __shared__ double lds_cols[];
  const int grp = threadIdx.x / kPackLanes, lane = threadIdx.x % 64;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * (128 / kPackLanes) + grp;
  const bool in = p < A.m;
  const ColsModel M{A.r, A.s, A.phi, A.delta64T, A.delta32T, A.bS, A.inv_h2, A.bS_norm, A.aff_c0, A.aff_tau,
                    A.wS, A.rowdat};
  cols_solve_packed<F, DP, COEF, RB>(M, in ? A.params + p * DP : nullptr, lds_cols + static_cast<int64_t>(grp) * ldsw,
                                     lane, in ? A.y + p * A.r : nullptr, (in && A.rho) ? A.rho + p : nullptr,
                                     (in && A.status) ? A.status + p : nullptr);
}

// Sketched residual S(A(p) Q y - b) of given coefficients, FP64: one
// wavefront per parameter, lanes over the selected rows.
template <int F, int DP, int COEF>
__global__ __launch_bounds__(256) void k_fd_resid(const double* params, int64_t m, int r, int s,
                                                   const double* phi, const double* delta64, const double* bS,
                                                   double inv_h2, double bS_norm, double aff_c0, double aff_tau,
                                                   const double* wS, const double* rowdat,
                                                   const double* y, double* res, double* norm) {
  ColsModel CM{r, s, phi, nullptr, nullptr, bS, inv_h2, bS_norm, aff_c0, aff_tau, wS, rowdat};
  const int64_t p = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (p >= m) return;
  double pv[DP];
  bool finite = true;
  for (int q = 0; q < DP; ++q) {
    pv[q] = params[p * DP + q];
    finite = finite && isfinite(pv[q]);
  }
  double ss = 0.0, bb = 0.0;
  for (int k = lane; k < s; k += 64) {
    double t = 0.0;
    for (int f = 0; f < F; ++f) {
      double u = 0.0;
      for (int c = 0; c < r; ++c) u += delta64[(f * r + c) * s + k] * y[p * r + c];
      t += cols_coef<F, DP, COEF>(CM, pv, f, k) * u;
    }
    const double bk = cols_rhs<COEF>(CM, pv, k);
    t -= bk;
    bb += bk * bk;
    if (!finite) t = __longlong_as_double(0x7ff8000000000000LL);
    if (res) res[p * s + k] = t;
    ss += t * t;
  }
  ss = team_sum<64>(ss);
  if constexpr (coef_rhs_varies<COEF>()) bb = team_sum<64>(bb);
  if (lane == 0 && norm) norm[p] = sqrt(ss) / (coef_rhs_varies<COEF>() ? sqrt(bb) : bS_norm);
}

// A posteriori bound on the distance of given coefficients to the SubApSnap
// solution (the normal-equation excess): with G = S A(p) Q and r_S = G y - S b,
// G^T r_S = G^T G (y - y*), so |G (y - y*)| <= |G^T r_S| / sigma_min(G).
// out[p] = |G^T r_S| / (sigma_min |S b(p)|), FP64 from the generated rows: one
// wavefront per parameter, first lanes over rows (r_S and the term
// coefficients of every row into LDS), then lanes over columns.
template <int F, int DP, int COEF>
__global__ __launch_bounds__(128) void k_fd_excess(const double* params, int64_t m, int r, int s, const double* phi,
                                                   const double* delta64, const double* delta64T, const double* bS,
                                                   double inv_h2, double bS_norm, double aff_c0, double aff_tau,
                                                   const double* wS, const double* rowdat, const double* y,
                                                   double sigma_min, double* out) {
  __shared__ double sh[2][kMaxS * (F + 1)];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * 2 + wave;
  if (p >= m) return;  // uniform per wavefront; no block-level barrier follows
  ColsModel CM{r, s, phi, nullptr, nullptr, bS, inv_h2, bS_norm, aff_c0, aff_tau, wS, rowdat};
  double* rs = sh[wave];          // s residual entries
  double* af = rs + kMaxS;        // s x F term coefficients
  double pv[DP];
  bool finite = true;
  for (int q = 0; q < DP; ++q) {
    pv[q] = params[p * DP + q];
    finite = finite && isfinite(pv[q]);
  }
  double bb = 0.0;
  for (int k = lane; k < s; k += 64) {
    double t = 0.0;
    for (int f = 0; f < F; ++f) {
      const double a = cols_coef<F, DP, COEF>(CM, pv, f, k);
      af[k * F + f] = a;
      double u = 0.0;
      for (int c = 0; c < r; ++c) u = fma(delta64[(f * r + c) * s + k], y[p * r + c], u);
      t = fma(a, u, t);
    }
    const double bk = cols_rhs<COEF>(CM, pv, k);
    rs[k] = t - bk;
    bb = fma(bk, bk, bb);
  }
  wave_sync_lds();
  double g = 0.0;
  if (lane < r) {
    for (int k = 0; k < s; ++k) {
      double gk = 0.0;
      for (int f = 0; f < F; ++f) gk = fma(af[k * F + f], delta64T[(static_cast<int64_t>(f) * s + k) * r + lane], gk);
      g = fma(gk, rs[k], g);
    }
  }
  const double gg = team_sum<64>(g * g);
  if constexpr (coef_rhs_varies<COEF>()) bb = team_sum<64>(bb);
  if (lane == 0) {
    const double den = sigma_min * (coef_rhs_varies<COEF>() ? sqrt(bb) : bS_norm);
    out[p] = finite ? sqrt(gg) / den : __longlong_as_double(0x7ff8000000000000LL);
  }
}

// G = S A(p) Q in FP64 (s x r row-major per parameter) from the term tables.
template <int F, int DP, int COEF>
__global__ __launch_bounds__(256) void k_fd_gmat(const double* params, int64_t m, int r, int s, const double* phi,
                                                 const double* delta64T, double inv_h2, double aff_c0, double aff_tau,
                                                 double* G) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m * s * r) return;
  const int64_t p = e / (static_cast<int64_t>(s) * r);
  const int k = static_cast<int>((e / r) % s), c = static_cast<int>(e % r);
  ColsModel CM{r, s, phi, nullptr, nullptr, nullptr, inv_h2, 0.0, aff_c0, aff_tau};
  double pv[DP];
  for (int q = 0; q < DP; ++q) pv[q] = params[p * DP + q];
  double t = 0.0;
  for (int f = 0; f < F; ++f)
    t = fma(cols_coef<F, DP, COEF>(CM, pv, f, k), delta64T[(static_cast<int64_t>(f) * s + k) * r + c], t);
  G[e] = t;
}

template <int TEAM, int R, int RM, int F, int DP>
subap_status launch(const FDArgs& a, hipStream_t st) {
  constexpr int TEAMS = 256 / TEAM;
  const int64_t nb = (a.m + TEAMS - 1) / TEAMS;
  if (nb > 0x7fffffff) {
    set_error("batch too large");
    return SUBAP_E_INVALID;
  }
  ProfScope prof("fd_solve", st);
  hipLaunchKernelGGL((k_fd_solve<TEAM, R, RM, F, DP>), dim3(static_cast<unsigned>(nb)), dim3(256), 0, st, a);
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

constexpr int kGramP = 2;  // parameters per wavefront: they share every table load

template <int F, int DP, int T>
subap_status launch_gram_t(const FDArgs& a, hipStream_t st) {
  const int64_t waves = (a.m + kGramP - 1) / kGramP;
  const int64_t nb = (waves + 1) / 2;
  if (nb > 0x7fffffff) {
    set_error("batch too large");
    return SUBAP_E_INVALID;
  }
  const int ldsw = gram_lds_doubles(a.r, kGramP, F);
  const size_t lds = sizeof(double) * 2 * static_cast<size_t>(ldsw);
  {
    ProfScope prof("fd_gram", st);
    hipLaunchKernelGGL((k_fd_gram<F, DP, T, kGramP>), dim3(static_cast<unsigned>(nb)), dim3(128), lds, st, a,
                       ldsw);
    SUBAP_HIP_TRY(hipGetLastError());
  }
  const int ldsc = cols_lds_doubles(a.r, a.s, false);
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>((a.m + 127) / 128, 2048));  // 64 per wave
  ProfScope prof("fd_gram_fixup", st);
  hipLaunchKernelGGL((k_fd_gram_fixup<F, DP>), dim3(grid), dim3(128), sizeof(double) * 2 * static_cast<size_t>(ldsc),
                     st, a, ldsc);
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

// The FP64 form without refinement of tall row sets (s >= 96) at
// 16 <= r <= 47 (G~ = [G | S b] fits three 16-column tiles).
bool gram_form(int prec, int refine, int r, int s) {
  return s >= 96 && prec == SUBAP_FP64 && refine == 0 && r > kPackMaxR && r + 1 <= 48;
}

// T is the least number of 16-column tiles holding the r + 1 columns of
// [G | S b] (r >= 16 here), so S b always sits in tile T - 1
template <int F, int DP>
subap_status launch_gram(const FDArgs& a, hipStream_t st) {
  if (a.r + 1 <= 32) return launch_gram_t<F, DP, 2>(a, st);
  return launch_gram_t<F, DP, 3>(a, st);
}

// Column-per-lane launch.  RB is the row block of the FP64 form without
// refinement at r < 64; the other forms keep blocks of kColsRB rows (their
// residual slices of 64 rows hold whole blocks).
template <int F, int DP, int COEF = kCoefDiffusion, int RB = kColsRB>
subap_status launch_cols(const FDArgs& a, hipStream_t st) {
  const int64_t nb = (a.m + 1) / 2;
  if (nb > 0x7fffffff) {
    set_error("batch too large");
    return SUBAP_E_INVALID;
  }
  const bool ref = a.refine > 0 || a.prec != SUBAP_FP64;
  const bool own_rb = !ref && a.r < 64;
  const int ldsw = cols_lds_doubles(a.r, a.s, ref, own_rb ? RB : kColsRB);
  ProfScope prof("fd_solve", st);
  if (!ref && a.r <= kPackMaxR) {  // four parameters per wavefront
    constexpr int per_block = 128 / kPackLanes;
    const int64_t nbp = (a.m + per_block - 1) / per_block;
    const size_t ldsp = sizeof(double) * per_block * static_cast<size_t>(ldsw);
    hipLaunchKernelGGL((k_fd_cols_packed<F, DP, COEF, RB>), dim3(static_cast<unsigned>(nbp)), dim3(128), ldsp, st, a,
                       ldsw);
    SUBAP_HIP_TRY(hipGetLastError());
    return SUBAP_OK;
  }
  const size_t lds = sizeof(double) * 2 * static_cast<size_t>(ldsw);
  const dim3 grid(static_cast<unsigned>(nb)), block(128);
  if (a.r == 64) {
    if (ref) hipLaunchKernelGGL((k_fd_cols<F, DP, true, true, COEF>), grid, block, lds, st, a, ldsw);
    else hipLaunchKernelGGL((k_fd_cols<F, DP, true, false, COEF>), grid, block, lds, st, a, ldsw);
  } else {
    if (ref) hipLaunchKernelGGL((k_fd_cols<F, DP, false, true, COEF>), grid, block, lds, st, a, ldsw);
    else hipLaunchKernelGGL((k_fd_cols<F, DP, false, false, COEF, RB>), grid, block, lds, st, a, ldsw);
  }
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

// Instantiated shapes: (TEAM, R) from s, RM from r.
template <int F, int DP>
subap_status dispatch(const FDArgs& a, hipStream_t st) {
  const int s = a.s, r = a.r;
  // tall problems: column-per-lane Householder (any precision and refinement).
  // The corrected semi-normal equations need R^T R solves, which only the
  // column-per-lane solver does.
  if (gram_form(a.prec, a.refine, r, s)) return launch_gram<F, DP>(a, st);
  if (s >= 96 || (a.csne && a.refine > 0)) return launch_cols<F, DP>(a, st);
#define SUBAP_FD(TEAM, R, RM) \
  if (s <= TEAM * R && r <= RM) return launch<TEAM, R, RM, F, DP>(a, st);
  // s <= 16 / 32 / 64 / 128 / 192 rows; r up to 40 columns
  SUBAP_FD(16, 1, 8) SUBAP_FD(32, 1, 8) SUBAP_FD(32, 1, 16)
  SUBAP_FD(64, 1, 16) SUBAP_FD(64, 2, 32) SUBAP_FD(64, 3, 40)
#undef SUBAP_FD
  return launch_cols<F, DP>(a, st);  // shapes without a register-resident team instantiation
}

}  // namespace

subap_status fd_solve(subap_model_s* M, const double* params, int64_t m, double* y, double* rho,
                      int32_t* status, int prec, int refine, bool csne, hipStream_t st) {
  FDArgs a{params, m, M->r, M->s, M->phi, M->delta64, M->delta32, M->delta64T, M->delta32T, M->bS, M->inv_h2,
           M->bS_norm, y, rho, status, prec, refine, M->aff_c0, M->tau, csne, M->wS, M->rowdat};
  // eq. (5.7) and the identity family: their affine pieces (two and one) and
  // p-dependent right-hand sides, column-per-lane solver
  // the affine family: S A(theta) Q = sum_q theta_q S A_q Q from its pieces
  if (M->family == SUBAP_FAMILY_AFFINE) {
    switch (M->F) {
      case 1: return launch_cols<1, 1, kCoefAffine>(a, st);
      case 2: return launch_cols<2, 2, kCoefAffine>(a, st);
      case 3: return launch_cols<3, 3, kCoefAffine>(a, st);
      default: return launch_cols<4, 4, kCoefAffine>(a, st);
    }
  }
  if (M->family == SUBAP_FAMILY_TRIDIAG_SHIFT) return launch_cols<2, 1, kCoefTridiag>(a, st);
  if (M->family == SUBAP_FAMILY_IDENTITY) return launch_cols<1, 1, kCoefIdentity>(a, st);
  // the delay family's two affine terms: column-per-lane solver for every
  // shape.  Its FP64 form fits blocks of 40 rows in registers (no spills at
  // F = 2), which shortens the reflector chain when that saves a block: at
  // s = 40, one block of 40 rows instead of 32 + 8 (padded to 32).  Short
  // row sets take one block of 24 or 28 rows, which pads less than 32.
  if (M->family == SUBAP_FAMILY_DELAY) {
    if (a.s <= 24) return launch_cols<2, 1, kCoefDelay, 24>(a, st);
    if (a.s <= 28) return launch_cols<2, 1, kCoefDelay, 28>(a, st);
    if ((a.s + 39) / 40 < (a.s + 31) / 32) return launch_cols<2, 1, kCoefDelay, 40>(a, st);
    return launch_cols<2, 1, kCoefDelay>(a, st);
  }
  return M->dimx == 2 ? dispatch<4, 2>(a, st) : dispatch<6, 4>(a, st);
}

bool fd_solve_on_matrix_cores(const subap_model_s* M, int prec, int refine) {
  return (M->family == SUBAP_FAMILY_DIFF2D || M->family == SUBAP_FAMILY_DIFF3D) &&
         gram_form(prec, refine, M->r, M->s);
}

subap_status fd_residual(subap_model_s* M, const double* params, int64_t m, const double* y, double* res,
                         double* norm, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>((m + 3) / 4);
  ProfScope prof("fd_residual", st);
#define SUBAP_RESID(F_, DP_, COEF_)                                                                              \
  hipLaunchKernelGGL((k_fd_resid<F_, DP_, COEF_>), dim3(grid), dim3(256), 0, st, params, m, M->r, M->s, M->phi, \
                     M->delta64, M->bS, M->inv_h2, M->bS_norm, M->aff_c0, M->tau, M->wS, M->rowdat, y, res, norm)
  if (M->family == SUBAP_FAMILY_AFFINE) {
    if (M->F == 1) SUBAP_RESID(1, 1, kCoefAffine);
    else if (M->F == 2) SUBAP_RESID(2, 2, kCoefAffine);
    else if (M->F == 3) SUBAP_RESID(3, 3, kCoefAffine);
    else SUBAP_RESID(4, 4, kCoefAffine);
  } else if (M->family == SUBAP_FAMILY_DELAY) SUBAP_RESID(2, 1, kCoefDelay);
  else if (M->family == SUBAP_FAMILY_TRIDIAG_SHIFT) SUBAP_RESID(2, 1, kCoefTridiag);
  else if (M->family == SUBAP_FAMILY_IDENTITY) SUBAP_RESID(1, 1, kCoefIdentity);
  else if (M->dimx == 2) SUBAP_RESID(4, 2, kCoefDiffusion);
  else SUBAP_RESID(6, 4, kCoefDiffusion);
#undef SUBAP_RESID
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

subap_status fd_excess(subap_model_s* M, const double* params, int64_t m, const double* y, double sigma_min,
                       double* out, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>((m + 1) / 2);
  ProfScope prof("fd_excess", st);
#define SUBAP_EXC(F_, DP_, COEF_)                                                                                  \
  hipLaunchKernelGGL((k_fd_excess<F_, DP_, COEF_>), dim3(grid), dim3(128), 0, st, params, m, M->r, M->s, M->phi,   \
                     M->delta64, M->delta64T, M->bS, M->inv_h2, M->bS_norm, M->aff_c0, M->tau, M->wS, M->rowdat, y, \
                     sigma_min, out)
  if (M->family == SUBAP_FAMILY_AFFINE) {
    if (M->F == 1) SUBAP_EXC(1, 1, kCoefAffine);
    else if (M->F == 2) SUBAP_EXC(2, 2, kCoefAffine);
    else if (M->F == 3) SUBAP_EXC(3, 3, kCoefAffine);
    else SUBAP_EXC(4, 4, kCoefAffine);
  } else if (M->family == SUBAP_FAMILY_DELAY) SUBAP_EXC(2, 1, kCoefDelay);
  else if (M->family == SUBAP_FAMILY_TRIDIAG_SHIFT) SUBAP_EXC(2, 1, kCoefTridiag);
  else if (M->family == SUBAP_FAMILY_IDENTITY) SUBAP_EXC(1, 1, kCoefIdentity);
  else if (M->dimx == 2) SUBAP_EXC(4, 2, kCoefDiffusion);
  else SUBAP_EXC(6, 4, kCoefDiffusion);
#undef SUBAP_EXC
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

subap_status fd_reduced_matrix(subap_model_s* M, const double* params, int64_t m, double* G, hipStream_t st) {
  const int64_t len = m * M->s * M->r;
  const unsigned grid = static_cast<unsigned>((len + 255) / 256);
#define SUBAP_GM(F_, DP_, COEF_)                                                                                  \
  hipLaunchKernelGGL((k_fd_gmat<F_, DP_, COEF_>), dim3(grid), dim3(256), 0, st, params, m, M->r, M->s, M->phi,    \
                     M->delta64T, M->inv_h2, M->aff_c0, M->tau, G)
  if (M->family == SUBAP_FAMILY_AFFINE) {
    if (M->F == 1) SUBAP_GM(1, 1, kCoefAffine);
    else if (M->F == 2) SUBAP_GM(2, 2, kCoefAffine);
    else if (M->F == 3) SUBAP_GM(3, 3, kCoefAffine);
    else SUBAP_GM(4, 4, kCoefAffine);
  } else if (M->family == SUBAP_FAMILY_DELAY) SUBAP_GM(2, 1, kCoefDelay);
  else if (M->family == SUBAP_FAMILY_TRIDIAG_SHIFT) SUBAP_GM(2, 1, kCoefTridiag);
  else if (M->family == SUBAP_FAMILY_IDENTITY) SUBAP_GM(1, 1, kCoefIdentity);
  else if (M->dimx == 2) SUBAP_GM(4, 2, kCoefDiffusion);
  else SUBAP_GM(6, 4, kCoefDiffusion);
#undef SUBAP_GM
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

}  // namespace subap
