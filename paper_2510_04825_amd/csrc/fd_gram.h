// FP64 least squares of one finite-difference parameter (eq. (3.3)) by the
// semi-normal equations on the FP64 matrix cores, with corrected semi-normal
// steps (Bjorck) for full FP64 accuracy.
//
// With G~ = [G | S b] (G = S A(p) Q, s x r, Section 3.1 rows contracted as in
// eq. (3.4)), the upper Cholesky factor of G~^T G~ is [[R, z], [0, rho]] with
// R^T R = G^T G, R^T z = G^T S b and rho = min |G y - S b|.  y0 = R^{-1} z is
// the semi-normal solution; its error grows like kappa(G)^2 eps.  Each
// corrected step takes the residual res = G y - S b in FP64 from freshly
// generated rows, g = G^T res, and solves R^T R dy = -g; the error then
// contracts by about kappa^2 eps per step down to the kappa eps level of a
// backward-stable solver, to the exact least-squares solution of the FP64 rows.
//
// Layout (one wavefront, lane l = 16 g + c): a group of four rows
// k = 4 q + g is generated with lane l holding column 16 I + c of row k for
// each 16-column tile I, which is the operand layout of
// v_mfma_f64_16x16x4f64 (A[m][kk] and B[kk][n] at lane 16 kk + m / n), so
// G~^T G~ accumulates with no data movement: one MFMA per tile pair (I <= J)
// per four rows.  The face coefficients of 64 rows at a time are computed
// with lanes over rows into LDS (in each pass: the LDS holds the two factors
// and one 64-row chunk, which keeps four blocks per CU) and read back as
// broadcasts.  P parameters share every load of the difference table.
//
// The Cholesky factorisation runs with lanes over columns (column c of the
// Gram matrix in registers of lane c), one pivot row per parameter broadcast
// through LDS per step; the P factorisations advance together.  The pivots
// take the hardware reciprocal square root with Newton corrections.  The
// triangular solves keep vectors distributed one entry per lane: each lane
// loads its column (R^T w = v) or its row (R y = v) of R, scaled by its own
// 1 / R_jj, into registers eight entries ahead, so a step is one lane
// broadcast and one FMA, and the P parameters' solves interleave.  The residual pass reduces each row over its 16 lanes with DPP
// row rotations; wave-wide sums add the four row sums by lane reads.
//
// A parameter whose Cholesky pivot falls below kGramPivTol times the largest
// column norm (kappa beyond about 1e6), whose Gram diagonal leaves [1e-200,
// 1e200], whose corrected steps do not settle, or whose result is not finite
// is left to the column-per-lane Householder
// solver: its first output coefficient is set to kGramDefer and no status or
// residual is written.  Non-finite parameters get SUBAP_E_NONFINITE directly.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"
#include "fd_cols.h"

namespace subap {

typedef double gram_v4d __attribute__((ext_vector_type(4)));

constexpr double kGramPivTol = 1e-6;
constexpr double kGramConv = 1e-14;  // estimated relative error at which the corrected steps stop
constexpr int kGramMaxSteps = 3;
constexpr unsigned long long kGramDefer = 0x7ffc5ab0a9f00001ULL;  // a quiet NaN no arithmetic produces

// Doubles of LDS per wavefront: P packed triangular factors of r + 1
// columns, then one region that holds the face coefficients of a 64-row
// chunk for P parameters during the passes over the rows and the P broadcast
// rows during the Cholesky factorisation.  At two wavefronts per SIMD a
// wavefront may take 160 KiB / 8 = 2560 doubles: r = 40, F = 6, P = 2 takes
// 2490.
__host__ __device__ inline int gram_lds_doubles(int r, int P, int F) {
  const int r1 = r + 1, npk = r1 * (r1 + 1) / 2;
  const int cf = P * 64 * F > 64 * P ? P * 64 * F : 64 * P;
  return ((P * npk + 1) & ~1) + cf;
}

template <int N>
__device__ __forceinline__ double gram_row_ror(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x120 + N, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x120 + N, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

// sum over the 16 lanes of a DPP row, in every lane of the row
__device__ __forceinline__ double gram_row_sum(double v) {
  v += gram_row_ror<8>(v);
  v += gram_row_ror<4>(v);
  v += gram_row_ror<2>(v);
  v += gram_row_ror<1>(v);
  return v;
}

// sum and maximum over the wavefront, in every lane (the four row results
// read from lanes 0, 16, 32, 48)
__device__ __forceinline__ double gram_wave_sum(double v) {
  v = gram_row_sum(v);
  return (lane_bcast(v, 0) + lane_bcast(v, 16)) + (lane_bcast(v, 32) + lane_bcast(v, 48));
}

__device__ __forceinline__ double gram_wave_max(double v) {
  v = fmax(v, gram_row_ror<8>(v));
  v = fmax(v, gram_row_ror<4>(v));
  v = fmax(v, gram_row_ror<2>(v));
  v = fmax(v, gram_row_ror<1>(v));
  return fmax(fmax(lane_bcast(v, 0), lane_bcast(v, 16)), fmax(lane_bcast(v, 32), lane_bcast(v, 48)));
}

// sqrt(d) and 1 / sqrt(d) for d > 0 (both 0 otherwise): the hardware
// reciprocal square root, one Goldschmidt step on the pair (g ~ sqrt(d),
// h ~ 1 / (2 sqrt(d))), a Newton correction of g against d and one of 1 / g.
// Each result is within a few ulp, which a Cholesky pivot needs (no correct
// rounding).  The caller keeps d inside [1e-212, 1e200], where the hardware
// estimate needs no rescaling.
__device__ __forceinline__ void gram_sqrt_rsqrt(double d, double& sq, double& inv) {
  const double y = __builtin_amdgcn_rsq(d);
  double g = d * y, h = 0.5 * y;
  const double e = fma(-g, h, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  g = fma(fma(-g, g, d), h, g);
  double w = 2.0 * h;
  w = fma(w, fma(-g, w, 1.0), w);
  const bool pos = d > 0.0;
  sq = pos ? g : 0.0;
  inv = pos ? w : 0.0;
}

// Buffer resource over a table of `bytes` bytes (raw, stride 0; the gfx9
// word 3), read with a per-lane voffset and a wave-uniform soffset.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t gram_rsrc(const double* p, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), 0, static_cast<int>(bytes), 0x00020000);
}

__device__ __forceinline__ double gram_bload(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
}

// The F x T table entries of one row group for this lane: face f's rows of
// the group start at the wave-uniform byte offset soff + f fbytes, and the
// lane adds its own loop-invariant offset (row g of the group, column
// 16 I + c), so no vector address arithmetic is needed per group.  A lane
// whose column is past r has an offset beyond the table: the buffer's range
// check returns 0 without a memory access.  Rows past s read the next face
// or the zero rows after the table (kRowPad), which the zero coefficients of
// those rows cancel.
template <int F, int T>
__device__ __forceinline__ void gram_load(__amdgpu_buffer_rsrc_t rs, unsigned soff, unsigned fbytes,
                                          const unsigned (&vo)[T], double (&d)[F][T]) {
#pragma unroll
  for (int f = 0; f < F; ++f)
#pragma unroll
    for (int I = 0; I < T; ++I) d[f][I] = gram_bload(rs, vo[I], soff + f * fbytes);
}

// Face coefficients a_f(p_u, k) of rows c0 .. c0 + 63 for the P parameters
// into coef[(u 64 + k - c0) F + f] (rows past s are 0), lanes over rows.
// The phi values of a row are loaded once for all P parameters, all before
// the exponentials.
template <int F, int DP, int P>
__device__ __forceinline__ void gram_coefs(const ColsModel& M, const double (&pv)[P][DP], double* coef, int c0,
                                           int lane) {
  const int s = M.s, k = c0 + lane, kc = k < s ? k : 0;
  double ph[F][DP];
#pragma unroll
  for (int f = 0; f < F; ++f)
#pragma unroll
    for (int q = 0; q < DP; ++q) ph[f][q] = M.phi[(f * DP + q) * s + kc];
#pragma unroll
  for (int u = 0; u < P; ++u)
#pragma unroll
    for (int f = 0; f < F; ++f) {
      double t = 0.0;
#pragma unroll
      for (int q = 0; q < DP; ++q) t += pv[u][q] * ph[f][q];
      coef[(u * 64 + lane) * F + f] = k < s ? exp(t) * M.inv_h2 : 0.0;
    }
  wave_sync_lds();
}

// the coefficients of chunk row kr for the P parameters
template <int F, int P>
__device__ __forceinline__ void gram_coef_load(const double* coef, int kr, double (&a)[P][F]) {
#pragma unroll
  for (int u = 0; u < P; ++u)
#pragma unroll
    for (int f = 0; f < F; ++f) a[u][f] = coef[(u * 64 + kr) * F + f];
}

// the rows of one group (lane row g of rows 4 qq .. 4 qq + 3) for the P
// parameters; S b is column r, in the last tile (T is the least number of
// 16-column tiles that hold r + 1 columns), and bk is 0 in the other lanes
template <int F, int T, int P, bool GRAM>
__device__ __forceinline__ void gram_group(const double (&d)[F][T], double bk, const double (&a)[P][F],
                                           gram_v4d (&acc)[P][T * (T + 1) / 2], const double (&yreg)[P][T],
                                           double (&gacc)[P][T], double (&rr)[P]) {
#pragma unroll
  for (int u = 0; u < P; ++u) {
    double Gv[T];
#pragma unroll
    for (int I = 0; I < T; ++I) {
      double t = 0.0;
#pragma unroll
      for (int f = 0; f < F; ++f) t = fma(a[u][f], d[f][I], t);
      Gv[I] = t;
    }
    Gv[T - 1] += bk;
    if constexpr (GRAM) {
      int t = 0;
#pragma unroll
      for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = I; J < T; ++J, ++t)
          acc[u][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(Gv[I], Gv[J], acc[u][t], 0, 0, 0);
    } else {
      double dot = 0.0;
#pragma unroll
      for (int I = 0; I < T; ++I) dot = fma(Gv[I], yreg[u][I], dot);
      const double res = gram_row_sum(dot);
#pragma unroll
      for (int I = 0; I < T; ++I) gacc[u][I] = fma(Gv[I], res, gacc[u][I]);
      rr[u] = fma(res, res, rr[u]);  // in all 16 lanes of the row
    }
  }
}

// one pass over the s rows in 64-row chunks of groups of four.  GRAM:
// accumulate G~^T G~ tiles.  Otherwise res_k = G~_k (y, -1) (= (G y - S
// b)_k), gacc += G~^T res per lane column, rr += |res|^2 (in each of the 16
// lanes of the row: a wave sum of rr counts every row 16 times, exactly).  The table loads of a group issue
// together, unconditionally, one group ahead: two register buffers
// alternate.  (With one parameter per wavefront the second buffer
// cost a wavefront per SIMD of occupancy and measured slower; with two, the
// kernel sits at two wavefronts per SIMD either way.)
template <int F, int DP, int T, int P, bool GRAM>
__device__ __forceinline__ void gram_pass(const ColsModel& M, const double (&pv)[P][DP], double* coef, int lane,
                                          gram_v4d (&acc)[P][T * (T + 1) / 2], const double (&yreg)[P][T],
                                          double (&gacc)[P][T], double (&rr)[P]) {
  const int r = M.r, s = M.s, g = lane >> 4, c16 = lane & 15;
  const unsigned fbytes = 8u * static_cast<unsigned>(s) * r, gbytes = 32u * r;  // a face, a row group
  const __amdgpu_buffer_rsrc_t rs = gram_rsrc(M.d64T, fbytes * F + 8u * kRowPad * r);
  unsigned vo[T];
#pragma unroll
  for (int I = 0; I < T; ++I)  // past the table for columns >= r (the range check gives 0)
    vo[I] = (16 * I + c16 < r) ? 8u * static_cast<unsigned>(g * r + 16 * I + c16) : 0x80000000u;
  const double bm = (c16 == (r & 15)) ? 1.0 : 0.0;
  for (int c0 = 0; c0 < s; c0 += 64) {
    gram_coefs<F, DP, P>(M, pv, coef, c0, lane);
    // the group after a chunk's last reads table rows up to s + 6 (the next
    // face, or the kRowPad zero rows) and S b the same (padded alike); it is
    // not used
    const int nq = min(16, (s - c0 + 3) / 4);
    const unsigned s0 = 8u * static_cast<unsigned>(c0) * r;
    double dA[F][T], dB[F][T], a[P][F];
    gram_load<F, T>(rs, s0, fbytes, vo, dA);
    double bA = M.bS[c0 + g], bB;
    for (int qq = 0; qq < nq; qq += 2) {
      const int k = c0 + 4 * qq + g;
      gram_load<F, T>(rs, s0 + (qq + 1) * gbytes, fbytes, vo, dB);
      bB = M.bS[k + 4];
      // keep these loads here (no instruction, no wait): otherwise they are
      // moved to their use in the next group
      asm volatile("" ::: "memory");
      gram_coef_load<F, P>(coef, 4 * qq + g, a);
      gram_group<F, T, P, GRAM>(dA, (k < s ? bm : 0.0) * bA, a, acc, yreg, gacc, rr);
      if (qq + 1 < nq) {
        gram_load<F, T>(rs, s0 + (qq + 2) * gbytes, fbytes, vo, dA);
        bA = M.bS[k + 8];
        asm volatile("" ::: "memory");
        gram_coef_load<F, P>(coef, 4 * qq + 4 + g, a);
        gram_group<F, T, P, GRAM>(dB, (k + 4 < s ? bm : 0.0) * bB, a, acc, yreg, gacc, rr);
      }
    }
    wave_sync_lds();  // the next chunk's coefficients overwrite these
  }
}

// Triangular solves of the P parameters together, vectors distributed one
// entry per lane (entry j in lane j < r, lanes >= r ignored).  Factor u is
// packed column-major at Rb + u npk (column c at c (c + 1) / 2), dinv[u] =
// 1 / R_jj in lane j < r.  Eight register entries per lane and parameter are
// loaded while the previous eight steps run.

// v <- R^{-T} v.  Lane c keeps w_c = v_c / R_cc and, at step i < c, takes
// the final w_i of lane i: w_c -= (R_ic / R_cc) w_i.  Its column R_0c ..
// R_{c-1,c} is contiguous.  Chunk q covers steps 8 q .. 8 q + 7; chunks
// past r - 1 are not run.
template <int T, int P>
__device__ __forceinline__ void gram_forward(const double* Rb, int npk, int r, const double (&dinv)[P],
                                             double (&v)[P], int lane) {
  constexpr int K = 8, NQ = 2 * T;
  const int lim = lane < r ? lane : 0;  // entries i < lim are R_{i,lane}
  const double* col = Rb + lim * (lim + 1) / 2;
  const int qend = (r - 1) / K;
  double w[P], b[2][P][K];
#pragma unroll
  for (int u = 0; u < P; ++u) w[u] = lane < r ? v[u] * dinv[u] : 0.0;
  auto load = [&](double (&bq)[P][K], int q) {
#pragma unroll
    for (int u = 0; u < P; ++u)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        // inside the factor for every lane: lim (lim + 1) / 2 + 16 T - 1 <
        // npk whenever r + 1 > 16 (T - 1) and T >= 2
        const double x = col[u * npk + q * K + k];
        bq[u][k] = (q * K + k < lim) ? x * dinv[u] : 0.0;
      }
  };
  load(b[0], 0);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    if (q > qend) break;
    if (q + 1 < NQ && q + 1 <= qend) load(b[(q + 1) & 1], q + 1);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int u = 0; u < P; ++u) w[u] = fma(-b[q & 1][u][k], lane_bcast(w[u], q * K + k), w[u]);
  }
#pragma unroll
  for (int u = 0; u < P; ++u) v[u] = w[u];
}

// v <- R^{-1} v.  Lane i keeps w_i = v_i / R_ii and, at step c > i (from
// c = r - 1 down), takes the final w_c of lane c: w_i -= (R_ic / R_ii) w_c.
// Its row entries sit at c (c + 1) / 2 + i; the entries a lane does not use
// (i >= c, or c >= r in the top chunk) are read at a clamped address inside
// the factor and dropped.  Chunks run from the one holding column r - 1 down.
template <int T, int P>
__device__ __forceinline__ void gram_backward(const double* Rb, int npk, int r, const double (&dinv)[P],
                                              double (&v)[P], int lane) {
  constexpr int K = 8, NQ = 2 * T;
  const int qtop = (r - 1) / K;
  double w[P], b[2][P][K];
#pragma unroll
  for (int u = 0; u < P; ++u) w[u] = lane < r ? v[u] * dinv[u] : 0.0;
  // entry k of chunk q: column q K + K - 1 - k
  auto load = [&](double (&bq)[P][K], int q) {
#pragma unroll
    for (int u = 0; u < P; ++u)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const int c = q * K + K - 1 - k;
        const int cc = c < r ? c : r - 1;
        const double x = Rb[u * npk + cc * (cc + 1) / 2 + (lane < cc ? lane : cc)];
        bq[u][k] = (lane < c && c < r) ? x * dinv[u] : 0.0;
      }
  };
#pragma unroll
  for (int q = NQ - 1; q >= 0; --q) {
    if (q > qtop) continue;
    if (q == qtop) load(b[q & 1], q);
    if (q >= 1) load(b[(q - 1) & 1], q - 1);
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int u = 0; u < P; ++u) w[u] = fma(-b[q & 1][u][k], lane_bcast(w[u], q * K + K - 1 - k), w[u]);
  }
#pragma unroll
  for (int u = 0; u < P; ++u) v[u] = w[u];
}

// Parameters p0 .. p0 + P - 1 (those < m) of one wavefront; r + 1 <= 16 T.
template <int F, int DP, int T, int P>
__device__ __forceinline__ void gram_solve(const ColsModel& M, const double* params, int64_t m, int64_t p0, double* lds, int lane,
                           double* y, double* rho, int32_t* status) {
  constexpr int NT = T * (T + 1) / 2;
  const int r = M.r, r1 = r + 1;
  const int npk = r1 * (r1 + 1) / 2;
  double* Rbase = lds;
  double* coef = lds + ((P * npk + 1) & ~1);  // 16-byte aligned
  double* rowbuf = coef;                      // the Cholesky's broadcast rows (no coefficients live then)
  const int g = lane >> 4, c16 = lane & 15;

  double pv[P][DP];
  bool finite[P], valid[P];
#pragma unroll
  for (int u = 0; u < P; ++u) {
    valid[u] = p0 + u < m;
    finite[u] = true;
#pragma unroll
    for (int q = 0; q < DP; ++q) {
      pv[u][q] = valid[u] ? params[(p0 + u) * DP + q] : 0.0;
      finite[u] = finite[u] && isfinite(pv[u][q]);
    }
    if (!finite[u]) {  // keep the arithmetic finite; the result is replaced
#pragma unroll
      for (int q = 0; q < DP; ++q) pv[u][q] = 0.0;
    }
  }

  // G~^T G~ on the matrix cores
  {
    gram_v4d acc[P][NT];
#pragma unroll
    for (int u = 0; u < P; ++u)
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[u][t] = gram_v4d{0.0, 0.0, 0.0, 0.0};
    double yreg[P][T], gacc[P][T], rr[P];
    gram_pass<F, DP, T, P, true>(M, pv, coef, lane, acc, yreg, gacc, rr);
    // upper triangle, packed column-major; of each 16 x 16 result tile,
    // lane l = 16 g + c holds rows g, g + 4, g + 8, g + 12 of column c
#pragma unroll
    for (int u = 0; u < P; ++u) {
      double* R = Rbase + u * npk;
      int t = 0;
#pragma unroll
      for (int I = 0; I < T; ++I)
#pragma unroll
        for (int J = I; J < T; ++J, ++t) {
          const int col = 16 * J + c16;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = 16 * I + g + 4 * i;
            if (col < r1 && row <= col) R[col * (col + 1) / 2 + row] = acc[u][t][i];
          }
        }
    }
    wave_sync_lds();
  }

  // Cholesky, lanes over columns; the P factorisations advance together, so
  // each step's broadcast, pivot and update chains overlap
  double dinv[P], yv[P];
  bool ok[P];
  {
    double colv[P][16 * T], thr2[P];
    // column `lane` of the Gram matrix; lanes past r read column 0.  The
    // loads of column r reach at most 16 T - 1 - r <= 15 doubles past the
    // factor: into the next factor or the coefficient region
    const int lc = lane < r1 ? lane : 0;
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const double* gc = Rbase + u * npk + lc * (lc + 1) / 2;
#pragma unroll
      for (int i = 0; i < 16 * T; ++i) {
        const double x = gc[i];
        colv[u][i] = (i <= lc && lane < r1) ? x : 0.0;
      }
      const double dmax = gram_wave_max(lane < r ? gc[lc] : 0.0);
      thr2[u] = kGramPivTol * kGramPivTol * dmax;
      // the pivots then lie in [1e-12 dmax, dmax], where gram_sqrt_rsqrt holds
      ok[u] = dmax > 1e-200 && dmax < 1e200;
      dinv[u] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < 16 * T; ++j) {
      if (j < r1) {
#pragma unroll
        for (int u = 0; u < P; ++u) {
          const double djj = lane_bcast(colv[u][j], j);
          if (j < r) ok[u] = ok[u] && (djj > thr2[u]);
          double piv, inv;
          gram_sqrt_rsqrt(djj, piv, inv);
          if (lane == j) dinv[u] = inv;
          colv[u][j] = lane > j ? colv[u][j] * inv : (lane == j ? piv : colv[u][j]);
          rowbuf[u * 64 + lane] = colv[u][j];
        }
        wave_sync_lds();
        // entries beyond column r are zero in every lane and stay zero, so
        // the update runs over the whole register column without a guard
#pragma unroll
        for (int u = 0; u < P; ++u)
#pragma unroll
          for (int i = (j + 1) & ~1; i < 16 * T; i += 2) {
            const double2 rb = *reinterpret_cast<const double2*>(rowbuf + u * 64 + i);
            if (i > j) colv[u][i] = fma(-rb.x, colv[u][j], colv[u][i]);
            colv[u][i + 1] = fma(-rb.y, colv[u][j], colv[u][i + 1]);
          }
        wave_sync_lds();
      }
    }
#pragma unroll
    for (int u = 0; u < P; ++u)
#pragma unroll
      for (int i = 0; i < 16 * T; ++i)
        if (lane < r1 && i <= lane) Rbase[u * npk + lane * (lane + 1) / 2 + i] = colv[u][i];
    wave_sync_lds();
  }
  // z = column r of each factor
#pragma unroll
  for (int u = 0; u < P; ++u) yv[u] = lane < r ? Rbase[u * npk + r * (r + 1) / 2 + lane] : 0.0;
  // semi-normal solutions y0 = R^{-1} z
  gram_backward<T, P>(Rbase, npk, r, dinv, yv, lane);

  // corrected semi-normal steps
  double rho2[P], rate[P];
  bool done[P];
#pragma unroll
  for (int u = 0; u < P; ++u) {
    rho2[u] = 0.0;
    rate[u] = 1.0;
    done[u] = !ok[u];
  }
  for (int step = 0; step < kGramMaxSteps; ++step) {
    bool all = true;
#pragma unroll
    for (int u = 0; u < P; ++u) all = all && done[u];
    if (all) break;
    double yreg[P][T], gacc[P][T], rr[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      const double yt = lane < r ? yv[u] : (lane == r ? -1.0 : 0.0);
#pragma unroll
      for (int I = 0; I < T; ++I) {
        yreg[u][I] = __shfl(yt, 16 * I + c16, 64);
        gacc[u][I] = 0.0;
      }
      rr[u] = 0.0;
    }
    gram_v4d acc[P][NT];
    gram_pass<F, DP, T, P, false>(M, pv, coef, lane, acc, yreg, gacc, rr);
    // w = -R^{-T} g and dy = R^{-1} w for every parameter (those already
    // done discard theirs)
    double w[P], dy[P];
#pragma unroll
    for (int u = 0; u < P; ++u) {
      double gsel = 0.0;
#pragma unroll
      for (int I = 0; I < T; ++I) {
        double v = gacc[u][I];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (g == I) gsel = v;
      }
      w[u] = lane < r ? -gsel : 0.0;
    }
    gram_forward<T, P>(Rbase, npk, r, dinv, w, lane);
#pragma unroll
    for (int u = 0; u < P; ++u) dy[u] = w[u];
    gram_backward<T, P>(Rbase, npk, r, dinv, dy, lane);
#pragma unroll
    for (int u = 0; u < P; ++u) {
      if (done[u]) continue;
      if (lane < r) yv[u] += dy[u];
      const double rrs = gram_wave_sum(rr[u]) * 0.0625;  // every row counted by its 16 lanes
      const double ww = gram_wave_sum(lane < r ? w[u] * w[u] : 0.0);
      const double ndy = sqrt(gram_wave_sum(lane < r ? dy[u] * dy[u] : 0.0));
      const double ny = sqrt(gram_wave_sum(lane < r ? yv[u] * yv[u] : 0.0));
      rho2[u] = fmax(rrs - ww, 0.0);  // |res(y + dy)|^2 = |res(y)|^2 - |R dy|^2
      // the first step's size relative to y estimates the contraction rate;
      // the error left after a step is about rate times that step
      if (step == 0) rate[u] = ny > 0.0 ? fmin(ndy / ny, 1.0) : 1.0;
      done[u] = rate[u] * ndy <= kGramConv * ny;
      if (rate[u] > 0.5) {  // no contraction: leave it to Householder
        ok[u] = false;
        done[u] = true;
      }
    }
  }

#pragma unroll
  for (int u = 0; u < P; ++u) {
    if (!valid[u]) continue;
    const int64_t p = p0 + u;
    const bool yfin = __all(lane >= r || isfinite(yv[u]));
    if (!finite[u]) {
      if (lane < r) y[p * r + lane] = __longlong_as_double(0x7ff8000000000000LL);
      if (lane == 0) {
        if (rho) rho[p] = __longlong_as_double(0x7ff8000000000000LL);
        if (status) status[p] = SUBAP_E_NONFINITE;
      }
    } else if (!ok[u] || !done[u] || !yfin) {
      if (lane == 0) y[p * r] = __longlong_as_double(static_cast<long long>(kGramDefer));
    } else {
      if (lane < r) y[p * r + lane] = yv[u];
      if (lane == 0) {
        if (rho) rho[p] = sqrt(rho2[u]) / M.bS_norm;
        if (status) status[p] = SUBAP_OK;
      }
    }
  }
}

}  // namespace subap
