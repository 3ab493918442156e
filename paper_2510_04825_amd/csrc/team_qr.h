// Team-level FP64 Householder least squares for the s x r problem of
// eq. (3.3): min_y |G y - b|, G = S A(p) Q.
//
// A "team" is TEAM consecutive lanes of one wavefront (TEAM in {16, 32, 64});
// one team owns one parameter p.  Lane t of the team holds rows
// i = t + TEAM * q, q = 0..R-1, of G and b in registers (rows >= s are zero).
// Column loops are unrolled up to RM >= r (columns >= r are zero), so every
// register index is a compile-time constant.  Dot products over rows are
// team reductions by xor-butterfly shuffles; IEEE addition is commutative,
// so every lane ends with a bitwise identical sum.
//
// Factorisation (LAPACK dgeqr2 convention): step j builds the reflector
// H_j = I - tau_j v_j v_j^T with v_j = 1 at row j and v_j = 0 above it, so
// that H_j G[:, j] = beta_j e_j.  Afterwards a[q][c] holds R above and on
// the diagonal and v below it; tau lives in team-private LDS.  Values kept
// in that LDS (tau, y) are team-uniform and every lane stores them, so no
// lane ever reads a value that only another lane wrote.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace subap {

template <int TEAM>
__device__ __forceinline__ double team_sum(double v) {
#pragma unroll
  for (int off = TEAM / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, TEAM);
  return v;
}

template <int TEAM>
__device__ __forceinline__ double team_bcast(double v, int src) {
  return __shfl(v, src, TEAM);
}

template <int TEAM, int R, int RM>
struct TeamQR {
  double a[R][RM];   // rows of G, then R and the reflectors
  double b[R];       // right-hand side, then Q^T b
  double r00;        // |R_11|
  bool full_rank;

  __device__ __forceinline__ int row(int lane, int q) const { return lane + TEAM * q; }

  // Householder QR of a, applied to b at the same time.  tau_s: RM doubles of
  // team-private LDS.
  __device__ __forceinline__ void factor(int r, int lane, double* tau_s) {
    full_rank = true;
    r00 = 0.0;
#pragma unroll
    for (int j = 0; j < RM; ++j) {
      if (j < r) {
        const int qj = j / TEAM, lj = j % TEAM;
        double ss = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const double x = (row(lane, q) > j) ? a[q][j] : 0.0;
          ss += x * x;
        }
        ss = team_sum<TEAM>(ss);
        const double alpha = team_bcast<TEAM>(a[qj][j], lj);
        double tau = 0.0, scale = 0.0, beta = alpha;
        if (ss > 0.0) {
          const double norm = sqrt(alpha * alpha + ss);
          beta = (alpha >= 0.0) ? -norm : norm;
          tau = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
        double v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = row(lane, q);
          v[q] = (i > j) ? a[q][j] * scale : (i == j ? 1.0 : 0.0);
        }
        // Trailing columns c > j (and b as column RM) in groups of 8:
        // w_c = v^T a[:, c] by one batched butterfly per group, then the
        // rank-1 update.  Grouping bounds the live registers while keeping
        // 8 independent shuffle chains in flight.
#pragma unroll
        for (int c0 = 0; c0 <= RM; c0 += 8) {
          if (c0 + 7 > j) {
            double w[8];
#pragma unroll
            for (int g = 0; g < 8; ++g) {
              const int c = c0 + g;
              w[g] = 0.0;
              if (c > j && c <= RM) {
#pragma unroll
                for (int q = 0; q < R; ++q) w[g] += v[q] * (c < RM ? a[q][c] : b[q]);
              }
            }
#pragma unroll
            for (int off = TEAM / 2; off > 0; off >>= 1) {
#pragma unroll
              for (int g = 0; g < 8; ++g)
                if (c0 + g > j && c0 + g <= RM) w[g] += __shfl_xor(w[g], off, TEAM);
            }
#pragma unroll
            for (int g = 0; g < 8; ++g) {
              const int c = c0 + g;
              if (c > j && c <= RM) {
                const double tw = tau * w[g];
#pragma unroll
                for (int q = 0; q < R; ++q) {
                  if (c < RM) a[q][c] -= tw * v[q];
                  else b[q] -= tw * v[q];
                }
              }
            }
          }
        }
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = row(lane, q);
          if (i == j) a[q][j] = beta;
          else if (i > j) a[q][j] = v[q];
        }
        tau_s[j] = tau;  // every lane stores the same value: no cross-lane hazard
        const double ab = fabs(beta);
        if (j == 0) r00 = ab;
        if (!(ab > kRankTol * r00)) full_rank = false;
      }
    }
  }

  // x <- Q^T x using the stored reflectors (x distributed like b).
  __device__ __forceinline__ void apply_qt(double (&x)[R], int r, int lane, const double* tau_s) const {
#pragma unroll
    for (int j = 0; j < RM; ++j) {
      if (j < r) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = row(lane, q);
          const double v = (i > j) ? a[q][j] : (i == j ? 1.0 : 0.0);
          t += v * x[q];
        }
        t = team_sum<TEAM>(t) * tau_s[j];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const int i = row(lane, q);
          const double v = (i > j) ? a[q][j] : (i == j ? 1.0 : 0.0);
          x[q] -= t * v;
        }
      }
    }
  }

  // Solve R y = x[0:r] (x distributed like b, already multiplied by Q^T).
  // y_s: RM doubles of team-private LDS receiving y (every lane may read it
  // after the call; the team is one wavefront or part of one).
  __device__ __forceinline__ void back_substitute(double (&x)[R], int r, int lane, double* y_s) const {
#pragma unroll
    for (int c = RM - 1; c >= 0; --c) {
      if (c < r) {
        const int qc = c / TEAM, lc = c % TEAM;
        const double yc = team_bcast<TEAM>(x[qc], lc) / team_bcast<TEAM>(a[qc][c], lc);
#pragma unroll
        for (int q = 0; q < R; ++q)
          if (row(lane, q) < c) x[q] -= a[q][c] * yc;
        y_s[c] = yc;  // team-uniform value, stored by every lane
      }
    }
  }

  // Solve R^T z = x[0:r] in place (x distributed like b; rows >= r are left
  // alone).  Row j needs sum_{i<j} R[i][j] z_i, a team reduction over the
  // lanes that own rows i < j.
  __device__ __forceinline__ void forward_substitute_t(double (&x)[R], int r, int lane) const {
#pragma unroll
    for (int j = 0; j < RM; ++j) {
      if (j < r) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q)
          if (row(lane, q) < j) t = fma(a[q][j], x[q], t);
        t = team_sum<TEAM>(t);
#pragma unroll
        for (int q = 0; q < R; ++q)
          if (row(lane, q) == j) x[q] = (x[q] - t) / a[q][j];
      }
    }
  }

  // |x[r:s]|_2 for x distributed like b (x = Q^T b gives the LSQ residual).
  __device__ __forceinline__ double tail_norm(const double (&x)[R], int r, int lane) const {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) t += (row(lane, q) >= r) ? x[q] * x[q] : 0.0;
    return sqrt(team_sum<TEAM>(t));
  }
};

}  // namespace subap
