// Column-per-lane Householder solve of one finite-difference parameter
// (Section 3.1 rows, eq. (3.4) contraction, eq. (3.3) least squares) by one
// wavefront.
//
// Lane c < r owns column c of G = S A(p) Q; S b is owned by lane r when
// r < 64 and carried identically by every lane when r = 64.  No dot product
// needs a cross-lane reduction.  The s rows arrive in blocks of RB rows
// (kColsRB unless the caller picks another multiple of 4) held in registers;
// each block is merged into the running triangular factor by
// Householder reflections of the stacked matrix [R; block] (reflector j acts
// on row j of R and on all block rows).  This is Householder QR of G applied
// in block order: the same R up to rounding.  R, with Q^T b as its last
// column, lives in wave-private LDS packed by rows, so that step j reads row
// j across the lanes without bank conflicts.  The pivot lane's block column
// is broadcast into scalar registers by v_readlane.  The squared block norm
// each column needs for its own reflector is downdated when a reflector is
// applied (|x - t v|^2 = |x|^2 - 2 t v.x + t^2 |v|^2, from the dot product the
// step already has) and recomputed once it has lost three quarters of its
// last exact value.  After a block, the block part of the b column is
// orthogonal to the range of the first r columns, so its squared norm adds to
// the sketched residual.
//
// Refinement (FP64) does not need the reflectors: with r_S = S(A(p) Q y - b)
// from the FP64 difference table, the correction solves R^T R dy = G^T r_S.
// Simple refinement takes G^T r_S with the G that was factorised (recomputed
// in the same arithmetic), which equals R^{-1} Q^T r_S; its fixed point is the
// least-squares solution of that rounded G.  The corrected semi-normal
// equations (csne) take G^T r_S with G from the FP64 table, whose fixed point
// is the exact solution of eq. (3.3).
//
// The caller gives each wavefront cols_lds_doubles(rmax, smax, REF) doubles of LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace subap {

constexpr int kColsRB = 32;  // rows per block

struct ColsModel {
  int r, s;
  const double* phi;    // [(f * DP + q) * s + k]
  const double* d64T;   // [(f * s + k) * r + c]
  const float* d32T;    // [(f * s + k) * r + c]
  const double* bS;
  double inv_h2, bS_norm;
  double aff_c0 = 0.0, aff_tau = 0.0;  // delay family: A(p) = p I - (c0 + e^{tau p}) A_1
  const double* wS = nullptr;          // row weights (right-hand sides that vary with p)
  const double* rowdat = nullptr;      // per-row data of those right-hand sides
};

// Coefficients of the term form G_k = sum_f a_f(p, k) Delta_{k,f} that every
// family here shares:
//   kCoefDiffusion  a_f = exp(sum_q p_q phi_{f,q}(face of row k)) / h^2, the
//                   face coefficients of the diffusion stencil;
//   kCoefDelay      F = 2, DP = 1: a_0 = p, a_1 = -(c0 + e^{tau p}), the
//                   affine weights of S Q and S A_1 Q (Section 3.1, computing
//                   S A(p*) X from precomputed pieces; Section 6.2.2);
//   kCoefTridiag    F = 2, DP = 1: a_0 = -p, a_1 = 1, the pieces S Q and
//                   S A_0 Q of A(p) = A_0 - p I (eq. (5.7));
//   kCoefIdentity   F = 1, DP = 1: a_0 = 1, A(p) = I (DEIM, eq. (3.5));
//   kCoefAffine     DP = F: a_q = theta_q, the weights of the pieces S A_q Q
//                   of a general affine family (Section 3.1).
// Tridiag and identity have right-hand sides that depend on p (cols_rhs).
constexpr int kCoefDiffusion = 0, kCoefDelay = 1, kCoefTridiag = 2, kCoefIdentity = 3, kCoefAffine = 4;

template <int COEF>
constexpr bool coef_rhs_varies() {
  return COEF == kCoefTridiag || COEF == kCoefIdentity;
}

// entry k of W S b(p): the stored table for a fixed b; for eq. (5.7)
// b_i(p) = exp(b0_i sin(p / 10) p) with rowdat[k] = b0 at row i_k; for the
// identity family b_i(p) = 1 / (1 + 25 (t_i - p)^2) with rowdat[k] = t at i_k
template <int COEF>
__device__ __forceinline__ double cols_rhs(const ColsModel& M, const double* pv, int k) {
  if constexpr (COEF == kCoefTridiag) {
    return M.wS[k] * exp(M.rowdat[k] * sin(pv[0] / 10.0) * pv[0]);
  } else if constexpr (COEF == kCoefIdentity) {
    const double t = M.rowdat[k] - pv[0];
    return M.wS[k] / (1.0 + 25.0 * (t * t));
  } else {
    return M.bS[k];
  }
}

template <int F, int DP, int COEF>
__device__ __forceinline__ double cols_coef(const ColsModel& M, const double* pv, int f, int k) {
  if constexpr (COEF == kCoefDelay) {
    return f == 0 ? pv[0] : -(M.aff_c0 + exp(M.aff_tau * pv[0]));
  } else if constexpr (COEF == kCoefTridiag) {
    return f == 0 ? -pv[0] : 1.0;
  } else if constexpr (COEF == kCoefIdentity) {
    return 1.0;
  } else if constexpr (COEF == kCoefAffine) {
    return pv[f];
  } else {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < DP; ++q) t += pv[q] * M.phi[(f * DP + q) * M.s + k];
    return exp(t) * M.inv_h2;
  }
}

__host__ __device__ inline int cols_lds_doubles(int rmax, int smax, bool ref, int rb = kColsRB) {
  return (rmax + 1) * (rmax + 2) / 2         // packed [R | Q^T b]
         + rb * 6                            // face coefficients of a block
         + kMaxR                             // y
         + (ref ? kMaxR : 0);                // correction, or 64 residual rows (refinement)
}

// start of packed row j (columns j..r1-1) for r1 = r + 1 columns
__device__ __forceinline__ int cols_row(int j, int r1) { return j * r1 - j * (j - 1) / 2; }

__device__ __forceinline__ double lane_bcast(double v, int src) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), src),
                          __builtin_amdgcn_readlane(__double2loint(v), src));
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// term coefficients of rows k0 .. k0 + RB - 1 into a[i * F + f]
template <int F, int DP, int COEF, int RB = kColsRB>
__device__ __forceinline__ void cols_faces(const ColsModel& M, const double* pv, int k0, double* a, int lane) {
  for (int idx = lane; idx < RB * F; idx += 64) {
    const int i = idx / F, f = idx % F;
    const int k = k0 + i;
    a[idx] = (k < M.s) ? cols_coef<F, DP, COEF>(M, pv, f, k) : 0.0;
  }
  wave_sync_lds();
}

// this block's rows of column `lane` of G in the contraction precision
template <int F, int RB = kColsRB>
__device__ __forceinline__ void cols_block(const ColsModel& M, int prec, int k0, const double* a, int lane,
                                           double (&B)[RB]) {
#pragma unroll
  for (int i = 0; i < RB; ++i) {
    const int k = k0 + i;
    double t = 0.0;
    if (k < M.s && lane < M.r) {
      if (prec == SUBAP_FP64) {
#pragma unroll
        for (int f = 0; f < F; ++f) t = fma(a[i * F + f], M.d64T[(static_cast<int64_t>(f) * M.s + k) * M.r + lane], t);
      } else {
        float t32 = 0.0f;
#pragma unroll
        for (int f = 0; f < F; ++f)
          t32 = fmaf(static_cast<float>(a[i * F + f]), M.d32T[(static_cast<int64_t>(f) * M.s + k) * M.r + lane], t32);
        t = t32;
      }
    }
    B[i] = t;
  }
}

// FP64 residual r_k = (S A(p) Q y - b)_k of row k (0 for k >= s); y in LDS.
// The rows are taken 64 at a time, one per lane.
template <int F, int DP, int COEF>
__device__ __forceinline__ double cols_residual_row(const ColsModel& M, const double* pv, const double* y, int k) {
  const int r = M.r, s = M.s;
  if (k >= s) return 0.0;
  double t = 0.0;
#pragma unroll
  for (int f = 0; f < F; ++f) {
    const double* d = M.d64T + (static_cast<int64_t>(f) * s + k) * r;
    double u0 = 0.0, u1 = 0.0;
    int c = 0;
    for (; c + 1 < r; c += 2) {
      u0 = fma(d[c], y[c], u0);
      u1 = fma(d[c + 1], y[c + 1], u1);
    }
    if (c < r) u0 = fma(d[c], y[c], u0);
    t = fma(cols_coef<F, DP, COEF>(M, pv, f, k), u0 + u1, t);
  }
  return t - cols_rhs<COEF>(M, pv, k);
}

// y <- R^{-1} v in place (v in LDS, every lane computes the same values)
__device__ __forceinline__ void cols_back_solve(const double* R, int r1, int r, double* v) {
  for (int j = r - 1; j >= 0; --j) {
    const int rowj = cols_row(j, r1);
    double t = v[j];
    for (int c = j + 1; c < r; ++c) t = fma(-R[rowj + (c - j)], v[c], t);
    t /= R[rowj];
    wave_sync_lds();
    v[j] = t;  // identical in every lane
    wave_sync_lds();
  }
}

// v <- R^{-T} v in place
__device__ __forceinline__ void cols_forward_solve(const double* R, int r1, int r, double* v) {
  for (int j = 0; j < r; ++j) {
    double t = v[j];
    for (int i = 0; i < j; ++i) t = fma(-R[cols_row(i, r1) + (j - i)], v[i], t);
    t /= R[cols_row(j, r1)];
    wave_sync_lds();
    v[j] = t;
    wave_sync_lds();
  }
}

// One parameter.  BRED: r == 64 (S b carried by every lane).  REF: an FP32
// contraction or refinement steps (FP64 residuals); without it prec must be
// FP64 and refine 0.  csne: refinement steps use the FP64 G^T r_S.  Writes y
// (r values), rho and status when the pointers are not NULL.
template <int F, int DP, bool BRED, bool REF, int COEF = kCoefDiffusion, int RB = kColsRB>
__device__ void cols_solve(const ColsModel& M, const double* params, int prec, int refine, bool csne, double* lds,
                           int smax, int lane, double* y_out, double* rho_out, int32_t* status_out) {
  static_assert(RB % 4 == 0, "the dot products run four rows at a time");
  static_assert(!REF || 64 % RB == 0, "the refinement's 64-row residual slices hold whole blocks");
  const int r = M.r, s = M.s, r1 = r + 1;
  double* R = lds;                     // r1 (r1 + 1) / 2 doubles
  double* a = R + r1 * (r1 + 1) / 2;
  double* yv = a + RB * 6;
  double* cv = yv + kMaxR;  // refinement: 64 residual rows, then the correction
  double* res = cv;
  (void)smax;
  const bool col = lane < r || (!BRED && lane == r);
  double pv[DP];
  bool finite = true;
#pragma unroll
  for (int q = 0; q < DP; ++q) {
    pv[q] = params[q];
    finite = finite && isfinite(pv[q]);
  }
  for (int idx = lane; idx < r1 * (r1 + 1) / 2; idx += 64) R[idx] = 0.0;
  wave_sync_lds();
  double rho2 = 0.0, r00 = 0.0;
  double bn2 = 0.0;  // |W S b(p)|^2 (the same in every lane)
  bool full_rank = true;
  for (int k0 = 0; k0 < s; k0 += RB) {
    cols_faces<F, DP, COEF, RB>(M, pv, k0, a, lane);
    double B[RB];
    cols_block<F, RB>(M, REF ? prec : SUBAP_FP64, k0, a, lane, B);
    double Bb[BRED ? RB : 1];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const double bk = (k0 + i < s) ? cols_rhs<COEF>(M, pv, k0 + i) : 0.0;
      if constexpr (coef_rhs_varies<COEF>()) bn2 = fma(bk, bk, bn2);
      if constexpr (BRED) Bb[i] = bk;
      else if (lane == r) B[i] = bk;
    }
    double ss = 0.0;
#pragma unroll
    for (int i = 0; i < RB; ++i) ss = fma(B[i], B[i], ss);
    double ss_ref = ss;  // the last exactly computed value
    const bool last = k0 + RB >= s;  // the pivots of the last block are final
    for (int j = 0; j < r; ++j) {
      const int rowj = cols_row(j, r1);
      const double alpha = (col && lane >= j) ? R[rowj + (lane - j)] : 0.0;
      // reflector of column j from (R[j][j], block column j): lane j's values
      // count.  u = [alpha - beta; block column]; H = I - 2 u u^T / u^T u with
      // u^T u = -2 beta (alpha - beta), so one division gives the coefficient.
      double dd = 0.0, coef = 0.0, beta = alpha;
      if (ss > 0.0) {
        const double nrm = sqrt(alpha * alpha + ss);
        beta = (alpha >= 0.0) ? -nrm : nrm;
        dd = alpha - beta;
        coef = -1.0 / (beta * dd);
      }
      if (lane == j) R[rowj] = beta;
      const double dj = lane_bcast(dd, j);
      const double cj = lane_bcast(coef, j);
      const double betaj = lane_bcast(beta, j);
      const double ssj = lane_bcast(ss, j);
      double vj[RB];
#pragma unroll
      for (int i = 0; i < RB; ++i) vj[i] = lane_bcast(B[i], j);
      if (lane > j && col) {
        double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
#pragma unroll
        for (int i = 0; i < RB; i += 4) {
          w0 = fma(vj[i], B[i], w0);
          w1 = fma(vj[i + 1], B[i + 1], w1);
          w2 = fma(vj[i + 2], B[i + 2], w2);
          w3 = fma(vj[i + 3], B[i + 3], w3);
        }
        // t = coef u^T x for this column: x <- x - t u
        const double dot = (w0 + w1) + (w2 + w3);
        const double t = cj * fma(dj, alpha, dot);
        R[rowj + (lane - j)] = fma(-t, dj, alpha);
#pragma unroll
        for (int i = 0; i < RB; ++i) B[i] = fma(-t, vj[i], B[i]);
        // |x - t v|^2 = |x|^2 - 2 t (v.x) + t^2 |v|^2, recomputed when it has
        // lost more than three quarters of its last exact value
        const double down = fma(t * t, ssj, fma(-2.0 * t, dot, ss));
        if (down >= 0.25 * ss_ref) {
          ss = down;
        } else {
          double s0 = 0.0, s1 = 0.0;
#pragma unroll
          for (int i = 0; i < RB; i += 2) {
            s0 = fma(B[i], B[i], s0);
            s1 = fma(B[i + 1], B[i + 1], s1);
          }
          ss = s0 + s1;
          ss_ref = ss;
        }
      }
      if constexpr (BRED) {
        const double alpha_b = R[rowj + (r - j)];
        double w0 = 0.0, w1 = 0.0;
#pragma unroll
        for (int i = 0; i < RB; i += 2) {
          w0 = fma(vj[i], Bb[i], w0);
          w1 = fma(vj[i + 1], Bb[i + 1], w1);
        }
        const double tb = cj * fma(dj, alpha_b, w0 + w1);
        wave_sync_lds();  // every lane has read R[j][r] before lane 0 overwrites it
        if (lane == 0) R[rowj + (r - j)] = fma(-tb, dj, alpha_b);
#pragma unroll
        for (int i = 0; i < RB; ++i) Bb[i] = fma(-tb, vj[i], Bb[i]);
      }
      if (last) {
        const double ab = fabs(betaj);
        if (j == 0) r00 = ab;
        if (!(ab > kRankTol * r00)) full_rank = false;
      }
    }
    if constexpr (BRED) {
      double t = 0.0;
#pragma unroll
      for (int i = 0; i < RB; ++i) t = fma(Bb[i], Bb[i], t);
      rho2 += t;
    } else {
      rho2 += lane_bcast(ss, r);
    }
    wave_sync_lds();
  }
  // y = R^{-1} (Q^T b)[0..r-1]
  for (int j = lane; j < r; j += 64) yv[j] = R[cols_row(j, r1) + (r - j)];
  wave_sync_lds();
  cols_back_solve(R, r1, r, yv);
  // FP64 refinement: R^T R dy = G^T r_S with the factorised G, or with the
  // FP64 G (corrected semi-normal equations)
  const int gprec = csne ? SUBAP_FP64 : prec;
  for (int it = 0; it < (REF ? refine : 0); ++it) {
    double g = 0.0;
    for (int k0 = 0; k0 < s; k0 += RB) {
      if (k0 % 64 == 0) {  // the next 64 residual rows (the previous ones are read)
        const double v = cols_residual_row<F, DP, COEF>(M, pv, yv, k0 + lane);
        res[lane] = v;
        wave_sync_lds();
      }
      cols_faces<F, DP, COEF, RB>(M, pv, k0, a, lane);
      double B[RB];
      cols_block<F, RB>(M, gprec, k0, a, lane, B);
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        const double rk = res[k0 % 64 + i];  // 0 beyond s
        g = fma(B[i], rk, g);
      }
      wave_sync_lds();  // the next block's face coefficients overwrite a
    }
    if (lane < r) cv[lane] = g;
    wave_sync_lds();
    cols_forward_solve(R, r1, r, cv);
    cols_back_solve(R, r1, r, cv);
    for (int j = lane; j < r; j += 64) yv[j] -= cv[j];
    wave_sync_lds();
  }
  double rho;
  if (REF && (refine > 0 || prec != SUBAP_FP64)) {
    double t = 0.0;
    for (int k0 = 0; k0 < s; k0 += 64) {
      const double v = cols_residual_row<F, DP, COEF>(M, pv, yv, k0 + lane);
      t = fma(v, v, t);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    rho = sqrt(t);
  } else {
    rho = sqrt(rho2);
  }
  const double yc = lane < r ? yv[lane] : 0.0;
  const bool yfin = __all(lane >= r || isfinite(yc));
  int32_t code = SUBAP_OK;
  if (!finite) code = SUBAP_E_NONFINITE;
  else if (!full_rank) code = SUBAP_E_RANK;
  else if (!yfin) code = SUBAP_E_NONFINITE;
  if (lane < r) y_out[lane] = (code == SUBAP_OK) ? yc : __longlong_as_double(0x7ff8000000000000LL);
  if (lane == 0) {
    if (rho_out) *rho_out = rho / (coef_rhs_varies<COEF>() ? sqrt(bn2) : M.bS_norm);
    if (status_out) *status_out = code;
  }
  wave_sync_lds();  // the region is reused by the next item
}


// ---------------------------------------------------------------------------
// Four parameters per wavefront for r <= 15 (FP64, no refinement): lane l
// serves parameter l / 16 of the wave with local lane c = l % 16 in the role
// that lane c has above (column c < r, S b at c = r).  A 16-lane group is one
// DPP row, so the pivot's values reach its group with one row_newbcast move
// per 32-bit half; the reflector loop is unrolled so that the pivot index is
// a constant of the instruction.  Each group has its own LDS region (R, the
// block's term coefficients, y) and writes only its own parameter.
// ---------------------------------------------------------------------------
template <int J>
__device__ __forceinline__ double row_bcast(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x150 + J, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x150 + J, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

constexpr int kPackLanes = 16;  // lanes per parameter
constexpr int kPackMaxR = kPackLanes - 1;

// one reflector step of the packed solver (pivot column J of this block)
template <int J, int RB>
__device__ __forceinline__ void packed_step(double* R, int r1, int c, bool col, double (&B)[RB], double& ss,
                                            double& ss_ref, bool last, double& r00, bool& full_rank) {
  const int rowj = cols_row(J, r1);
  const double alpha = (col && c >= J) ? R[rowj + (c - J)] : 0.0;
  double dd = 0.0, coef = 0.0, beta = alpha;
  if (ss > 0.0) {
    const double nrm = sqrt(alpha * alpha + ss);
    beta = (alpha >= 0.0) ? -nrm : nrm;
    dd = alpha - beta;
    coef = -1.0 / (beta * dd);
  }
  if (c == J) R[rowj] = beta;
  const double dj = row_bcast<J>(dd);
  const double cj = row_bcast<J>(coef);
  const double betaj = row_bcast<J>(beta);
  const double ssj = row_bcast<J>(ss);
  double vj[RB];
#pragma unroll
  for (int i = 0; i < RB; ++i) vj[i] = row_bcast<J>(B[i]);
  if (c > J && col) {
    double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
#pragma unroll
    for (int i = 0; i < RB; i += 4) {
      w0 = fma(vj[i], B[i], w0);
      w1 = fma(vj[i + 1], B[i + 1], w1);
      w2 = fma(vj[i + 2], B[i + 2], w2);
      w3 = fma(vj[i + 3], B[i + 3], w3);
    }
    const double dot = (w0 + w1) + (w2 + w3);
    const double t = cj * fma(dj, alpha, dot);
    R[rowj + (c - J)] = fma(-t, dj, alpha);
#pragma unroll
    for (int i = 0; i < RB; ++i) B[i] = fma(-t, vj[i], B[i]);
    const double down = fma(t * t, ssj, fma(-2.0 * t, dot, ss));
    if (down >= 0.25 * ss_ref) {
      ss = down;
    } else {
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int i = 0; i < RB; i += 2) {
        s0 = fma(B[i], B[i], s0);
        s1 = fma(B[i + 1], B[i + 1], s1);
      }
      ss = s0 + s1;
      ss_ref = ss;
    }
  }
  if (last) {
    const double ab = fabs(betaj);
    if (J == 0) r00 = ab;
    if (!(ab > kRankTol * r00)) full_rank = false;
  }
}

template <int J, int RB>
__device__ __forceinline__ void packed_steps(int r, double* R, int r1, int c, bool col, double (&B)[RB], double& ss,
                                             double& ss_ref, bool last, double& r00, bool& full_rank) {
  if constexpr (J < kPackMaxR) {
    if (J < r) {
      packed_step<J, RB>(R, r1, c, col, B, ss, ss_ref, last, r00, full_rank);
      packed_steps<J + 1, RB>(r, R, r1, c, col, B, ss, ss_ref, last, r00, full_rank);
    }
  }
}

// One parameter per 16-lane group.  params: this group's parameter (or
// nullptr for a group past the end of the batch, which computes on zeros and
// writes nothing); lds: this group's region of cols_lds_doubles(r, s, false, RB).
template <int F, int DP, int COEF, int RB>
__device__ void cols_solve_packed(const ColsModel& M, const double* params, double* lds, int lane, double* y_out,
                                  double* rho_out, int32_t* status_out) {
  static_assert(RB % 4 == 0, "the dot products run four rows at a time");
  constexpr int L = kPackLanes;
  const int c = lane % L;
  const int r = M.r, s = M.s, r1 = r + 1;
  double* R = lds;
  double* a = R + r1 * (r1 + 1) / 2;
  double* yv = a + RB * 6;
  const bool col = c <= r;
  double pv[DP];
  bool finite = true;
#pragma unroll
  for (int q = 0; q < DP; ++q) {
    pv[q] = params ? params[q] : 0.0;
    finite = finite && isfinite(pv[q]);
  }
  for (int idx = c; idx < r1 * (r1 + 1) / 2; idx += L) R[idx] = 0.0;
  double rho2 = 0.0, r00 = 0.0, bn2 = 0.0;
  bool full_rank = true;
  for (int k0 = 0; k0 < s; k0 += RB) {
    for (int idx = c; idx < RB * F; idx += L) {
      const int i = idx / F, f = idx % F;
      a[idx] = (k0 + i < s) ? cols_coef<F, DP, COEF>(M, pv, f, k0 + i) : 0.0;
    }
    wave_sync_lds();
    double B[RB];
#pragma unroll
    for (int i = 0; i < RB; ++i) {
      const int k = k0 + i;
      double t = 0.0;
      if (k < s && c < r) {
#pragma unroll
        for (int f = 0; f < F; ++f) t = fma(a[i * F + f], M.d64T[(static_cast<int64_t>(f) * s + k) * r + c], t);
      }
      const double bk = k < s ? cols_rhs<COEF>(M, pv, k) : 0.0;
      if constexpr (coef_rhs_varies<COEF>()) bn2 = fma(bk, bk, bn2);
      B[i] = (c == r) ? bk : t;
    }
    double ss = 0.0;
#pragma unroll
    for (int i = 0; i < RB; ++i) ss = fma(B[i], B[i], ss);
    double ss_ref = ss;
    const bool last = k0 + RB >= s;
    packed_steps<0, RB>(r, R, r1, c, col, B, ss, ss_ref, last, r00, full_rank);
    if (c == r) rho2 += ss;  // the b column's part outside the range of the first r columns
    wave_sync_lds();  // the next block's term coefficients overwrite a
  }
  for (int j = c; j < r; j += L) yv[j] = R[cols_row(j, r1) + (r - j)];
  wave_sync_lds();
  cols_back_solve(R, r1, r, yv);
  const double yc = c < r ? yv[c] : 0.0;
  // lanes of this group holding a non-finite coefficient
  const uint64_t bad = __ballot(c < r && !isfinite(yc));
  const bool yfin = ((bad >> (lane - c)) & 0xffffull) == 0;
  int32_t code = SUBAP_OK;
  if (!finite) code = SUBAP_E_NONFINITE;
  else if (!full_rank) code = SUBAP_E_RANK;
  else if (!yfin) code = SUBAP_E_NONFINITE;
  if (params) {
    if (c < r) y_out[c] = (code == SUBAP_OK) ? yc : __longlong_as_double(0x7ff8000000000000LL);
    if (c == r) {
      if (rho_out) *rho_out = sqrt(rho2) / (coef_rhs_varies<COEF>() ? sqrt(bn2) : M.bS_norm);
      if (status_out) *status_out = code;
    }
  }
  wave_sync_lds();
}

}  // namespace subap
