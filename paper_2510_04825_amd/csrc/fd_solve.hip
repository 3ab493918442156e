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
  const double* bS;
  double inv_h2, bS_norm;
  double* y;
  double* rho;
  int32_t* status;
  int prec;
  int refine;
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

// Column-per-lane Householder least squares, FP64 contraction, no refinement.
// One wavefront per parameter; lane c < r owns column c of S A(p) Q and lane r
// owns S b, so no dot product needs a cross-lane reduction.  The s rows arrive
// in blocks of RB held in registers.  Each block is merged into the running
// triangular factor by Householder reflections of the stacked matrix
// [R; block] (reflector j acts on row j of R and on all block rows): this is
// Householder QR of S A(p) Q applied in block order, the same R up to
// rounding.  R (with Q^T b as column r) lives in wave-private LDS, packed by
// rows, so that step j reads row j across the lanes without bank conflicts
// and the registers hold only the block.  The pivot lane's block column is
// broadcast into scalar registers by v_readlane (no LDS round trip in the
// step); the squared norm each column needs for its own reflector is
// accumulated while the previous reflector is applied.  After a
// block, the block part of the b column is orthogonal to the range of the
// first r columns, so its squared norm adds to the sketched residual.  No
// block-level barrier is used: the waves of a block are independent.
template <int RM>
__device__ __forceinline__ int packed_row(int j) {
  return j * (RM + 1) - j * (j - 1) / 2;  // row j holds columns j..RM
}

template <int RM, int RB, int F, int DP>
__global__ __launch_bounds__(128) void k_fd_cols(FDArgs A) {
  constexpr int W = 2;  // wavefronts per block
  constexpr int RP = (RM + 1) * (RM + 2) / 2;
  struct Smem {
    double R[RP];      // packed rows of [R | Q^T b]
    double a[RB][F];   // face coefficients / h^2 of the current rows
    double y[RM];
  };
  __shared__ Smem sm_all[W];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * W + wave;
  if (p >= A.m) return;  // uniform per wavefront
  Smem& sm = sm_all[wave];
  const int r = A.r, s = A.s;
  const bool col = lane <= r;  // lane r carries b
  double pv[DP];
  bool finite = true;
#pragma unroll
  for (int q = 0; q < DP; ++q) {
    pv[q] = A.params[p * DP + q];
    finite = finite && isfinite(pv[q]);
  }
  for (int idx = lane; idx < RP; idx += 64) sm.R[idx] = 0.0;
  double rho2 = 0.0, r00 = 0.0;
  bool full_rank = true;
  for (int k0 = 0; k0 < s; k0 += RB) {
    for (int idx = lane; idx < RB * F; idx += 64) {
      const int i = idx / F, f = idx % F;
      const int k = k0 + i;
      double t = 0.0;
      if (k < s) {
#pragma unroll
        for (int q = 0; q < DP; ++q) t += pv[q] * A.phi[(f * DP + q) * s + k];
      }
      sm.a[i][f] = (k < s) ? exp(t) * A.inv_h2 : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // this block's rows of my column, and their squared norm
    double B[RB];
    double ss = 0.0;
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int k = k0 + i;
      double t = 0.0;
      if (k < s) {
        if (lane < r) {
#pragma unroll
          for (int f = 0; f < F; ++f)
            t = fma(sm.a[i][f], A.delta64T[(static_cast<int64_t>(f) * s + k) * r + lane], t);
        } else if (lane == r) {
          t = A.bS[k];
        }
      }
      B[i] = t;
      ss = fma(t, t, ss);
    }
    const bool last = k0 + RB >= s;  // the pivots of the last block are final
    for (int j = 0; j < r; ++j) {
      const int rowj = packed_row<RM>(j);
      const double alpha = (col && lane >= j) ? sm.R[rowj + (lane - j)] : 0.0;
      // reflector of column j from (R[j][j], block column j): lane j's values count
      double tau = 0.0, scale = 0.0, beta = alpha;
      if (ss > 0.0) {
        const double nrm = sqrt(alpha * alpha + ss);
        beta = (alpha >= 0.0) ? -nrm : nrm;
        const double d = alpha - beta;
        tau = -d / beta;
        scale = 1.0 / d;
      }
      if (lane == j) sm.R[rowj] = beta;
      const double tauj = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(tau), j),
                                           __builtin_amdgcn_readlane(__double2loint(tau), j));
      const double betaj = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(beta), j),
                                            __builtin_amdgcn_readlane(__double2loint(beta), j));
      const double scalej = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(scale), j),
                                             __builtin_amdgcn_readlane(__double2loint(scale), j));
      // lane j's block column, broadcast into scalar registers
      double vj[RB];
#pragma unroll
      for (int i = 0; i < RB; ++i)
        vj[i] = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(B[i]), j),
                                 __builtin_amdgcn_readlane(__double2loint(B[i]), j));
      if (lane > j && col) {
        double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
#pragma unroll
        for (int i = 0; i < RB; i += 4) {
          w0 = fma(vj[i], B[i], w0);
          if (i + 1 < RB) w1 = fma(vj[i + 1], B[i + 1], w1);
          if (i + 2 < RB) w2 = fma(vj[i + 2], B[i + 2], w2);
          if (i + 3 < RB) w3 = fma(vj[i + 3], B[i + 3], w3);
        }
        const double w = tauj * fma(scalej, (w0 + w1) + (w2 + w3), alpha);
        sm.R[rowj + (lane - j)] = alpha - w;
        const double ws = w * scalej;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int i = 0; i < RB; ++i) {
          B[i] = fma(-ws, vj[i], B[i]);
          if (i % 2 == 0) s0 = fma(B[i], B[i], s0);
          else s1 = fma(B[i], B[i], s1);
        }
        ss = s0 + s1;
      }
      if (last) {
        const double ab = fabs(betaj);
        if (j == 0) r00 = ab;
        if (!(ab > kRankTol * r00)) full_rank = false;
      }
    }
    if (lane == r) rho2 += ss;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  // back substitution R y = (Q^T b)[0..r-1], redundantly in every lane
  for (int j = r - 1; j >= 0; --j) {
    const int rowj = packed_row<RM>(j);
    double t = sm.R[rowj + (r - j)];
    for (int c = j + 1; c < r; ++c) t = fma(-sm.R[rowj + (c - j)], sm.y[c], t);
    const double yj = t / sm.R[rowj];
    if (lane == 0) sm.y[j] = yj;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  const double yc = lane < r ? sm.y[lane] : 0.0;
  bool yfin = lane >= r || isfinite(yc);
  yfin = __all(yfin);
  int32_t code = SUBAP_OK;
  if (!finite) code = SUBAP_E_NONFINITE;
  else if (!full_rank) code = SUBAP_E_RANK;
  else if (!yfin) code = SUBAP_E_NONFINITE;
  if (lane < r) A.y[p * r + lane] = (code == SUBAP_OK) ? yc : __longlong_as_double(0x7ff8000000000000LL);
  const double rho = sqrt(__hiloint2double(__builtin_amdgcn_readlane(__double2hiint(rho2), r),
                                           __builtin_amdgcn_readlane(__double2loint(rho2), r)));
  if (lane == 0) {
    if (A.rho) A.rho[p] = rho / A.bS_norm;
    if (A.status) A.status[p] = code;
  }
}

// Sketched residual S(A(p) Q y - b) of given coefficients, FP64: one
// wavefront per parameter, lanes over the selected rows.
template <int F, int DP>
__global__ __launch_bounds__(256) void k_fd_resid(const double* params, int64_t m, int r, int s,
                                                   const double* phi, const double* delta64, const double* bS,
                                                   double inv_h2, double bS_norm, const double* y, double* res,
                                                   double* norm) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (p >= m) return;
  double pv[DP];
  bool finite = true;
  for (int q = 0; q < DP; ++q) {
    pv[q] = params[p * DP + q];
    finite = finite && isfinite(pv[q]);
  }
  double ss = 0.0;
  for (int k = lane; k < s; k += 64) {
    double t = 0.0;
    for (int f = 0; f < F; ++f) {
      double arg = 0.0;
      for (int q = 0; q < DP; ++q) arg += pv[q] * phi[(f * DP + q) * s + k];
      double u = 0.0;
      for (int c = 0; c < r; ++c) u += delta64[(f * r + c) * s + k] * y[p * r + c];
      t += exp(arg) * inv_h2 * u;
    }
    t -= bS[k];
    if (!finite) t = __longlong_as_double(0x7ff8000000000000LL);
    if (res) res[p * s + k] = t;
    ss += t * t;
  }
  ss = team_sum<64>(ss);
  if (lane == 0 && norm) norm[p] = sqrt(ss) / bS_norm;
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

// Instantiated shapes: (TEAM, R) from s, RM from r.
template <int RM, int F, int DP>
subap_status launch_cols(const FDArgs& a, hipStream_t st) {
  constexpr int W = 2;
  const int64_t nb = (a.m + W - 1) / W;
  if (nb > 0x7fffffff) {
    set_error("batch too large");
    return SUBAP_E_INVALID;
  }
  ProfScope prof("fd_solve", st);
  hipLaunchKernelGGL((k_fd_cols<RM, 32, F, DP>), dim3(static_cast<unsigned>(nb)), dim3(64 * W), 0, st, a);
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

template <int F, int DP>
subap_status dispatch(const FDArgs& a, hipStream_t st) {
  const int s = a.s, r = a.r;
  // FP64 without refinement on tall problems: column-per-lane Householder
  if (a.prec == SUBAP_FP64 && a.refine == 0 && s >= 96 && r < 64) {
    if (r <= 16) return launch_cols<16, F, DP>(a, st);
    if (r <= 32) return launch_cols<32, F, DP>(a, st);
    if (r <= 40) return launch_cols<40, F, DP>(a, st);
  }
#define SUBAP_FD(TEAM, R, RM) \
  if (s <= TEAM * R && r <= RM) return launch<TEAM, R, RM, F, DP>(a, st);
  // s <= 16 / 32 / 64 / 128 / 192 rows; r up to 40 columns
  SUBAP_FD(16, 1, 8) SUBAP_FD(32, 1, 8) SUBAP_FD(32, 1, 16)
  SUBAP_FD(64, 1, 16) SUBAP_FD(64, 2, 32) SUBAP_FD(64, 3, 40)
#undef SUBAP_FD
  return SUBAP_E_UNSUPPORTED;  // the caller falls back to the LDS kernel
}

}  // namespace

subap_status fd_solve(subap_model_s* M, const double* params, int64_t m, double* y, double* rho,
                      int32_t* status, int prec, int refine, hipStream_t st) {
  FDArgs a{params, m, M->r, M->s, M->phi, M->delta64, M->delta32, M->delta64T, M->bS, M->inv_h2, M->bS_norm,
           y, rho, status, prec, refine};
  const subap_status rc = M->dimx == 2 ? dispatch<4, 2>(a, st) : dispatch<6, 4>(a, st);
  if (rc != SUBAP_E_UNSUPPORTED) return rc;
  // shapes without a register-resident instantiation: Householder in LDS
  return fd_solve_lds(M, params, m, y, rho, status, prec, refine, st);
}

subap_status fd_residual(subap_model_s* M, const double* params, int64_t m, const double* y, double* res,
                         double* norm, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>((m + 3) / 4);
  ProfScope prof("fd_residual", st);
  if (M->dimx == 2)
    hipLaunchKernelGGL((k_fd_resid<4, 2>), dim3(grid), dim3(256), 0, st, params, m, M->r, M->s, M->phi, M->delta64,
                       M->bS, M->inv_h2, M->bS_norm, y, res, norm);
  else
    hipLaunchKernelGGL((k_fd_resid<6, 4>), dim3(grid), dim3(256), 0, st, params, m, M->r, M->s, M->phi, M->delta64,
                       M->bS, M->inv_h2, M->bS_norm, y, res, norm);
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

}  // namespace subap
