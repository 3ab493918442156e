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
// with lanes over rows into LDS and read back as broadcasts.  P parameters
// share every load of the difference table.
//
// The Cholesky factorisation runs with lanes over columns (column c of the
// Gram matrix in registers of lane c), one pivot row broadcast through LDS
// per step; the triangular solves keep vectors distributed one entry per
// lane and read R column-major from LDS.  The residual pass reduces each row
// over its 16 lanes with DPP row rotations.
//
// A parameter whose Cholesky pivot falls below kGramPivTol times the largest
// column norm (kappa beyond about 1e6), whose corrected steps do not settle,
// or whose result is not finite is left to the column-per-lane Householder
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

// doubles of LDS per wavefront: face coefficients of 64 rows for P
// parameters, one broadcast row, P packed triangular factors of r + 1 columns
__host__ __device__ inline int gram_lds_doubles(int r, int P, int F) {
  const int r1 = r + 1;
  const int n = P * 64 * F + 64 + P * (r1 * (r1 + 1) / 2);
  return (n + 1) & ~1;
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

__device__ __forceinline__ double gram_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double gram_wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
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

// the rows of one group (4 qq + g of the chunk) for the P parameters
template <int F, int T, int P, bool GRAM>
__device__ __forceinline__ void gram_group(const double (&d)[F][T], double bk, const double* coef, int kr, int bI,
                                           int c16, gram_v4d (&acc)[P][T * (T + 1) / 2],
                                           const double (&yreg)[P][T], double (&gacc)[P][T], double (&rr)[P]) {
#pragma unroll
  for (int u = 0; u < P; ++u) {
    double a[F];  // zero beyond row s
#pragma unroll
    for (int f = 0; f < F; ++f) a[f] = coef[(u * 64 + kr) * F + f];
    double Gv[T];
#pragma unroll
    for (int I = 0; I < T; ++I) {
      double t = 0.0;
#pragma unroll
      for (int f = 0; f < F; ++f) t = fma(a[f], d[f][I], t);
      Gv[I] = (I == bI) ? t + bk : t;
    }
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
      rr[u] = fma(res * (c16 == 0 ? 1.0 : 0.0), res, rr[u]);
    }
  }
}

// one pass over the s rows.  GRAM: accumulate G~^T G~ tiles.  Otherwise
// res_k = G~_k (y, -1) (= (G y - S b)_k), gacc += G~^T res per lane column,
// rr += |res|^2 (counted once per row, by the lanes with c = 0).  The T F
// loads of a group issue together, unconditionally, and two register
// buffers alternate: the next group's loads are in flight while one
// computes.  (With one parameter per wavefront the second buffer cost a
// wavefront per SIMD of occupancy and measured slower; with two, the
// kernel sits at two wavefronts per SIMD either way.)
template <int F, int DP, int T, int P, bool GRAM>
__device__ __forceinline__ void gram_pass(const ColsModel& M, const double (&pv)[P][DP], double* coef, int lane,
                                          gram_v4d (&acc)[P][T * (T + 1) / 2], const double (&yreg)[P][T],
                                          double (&gacc)[P][T], double (&rr)[P]) {
  const int r = M.r, s = M.s, g = lane >> 4, c16 = lane & 15;
  const int bI = r >> 4;  // tile of S b
  const unsigned fbytes = 8u * static_cast<unsigned>(s) * r, gbytes = 32u * r;  // a face, a row group
  const __amdgpu_buffer_rsrc_t rs = gram_rsrc(M.d64T, fbytes * F + 8u * kRowPad * r);
  unsigned vo[T];
#pragma unroll
  for (int I = 0; I < T; ++I)  // past the table for columns >= r (the range check gives 0)
    vo[I] = (16 * I + c16 < r) ? 8u * static_cast<unsigned>(g * r + 16 * I + c16) : 0x80000000u;
  const double bm = (c16 == (r & 15)) ? 1.0 : 0.0;
  for (int c0 = 0; c0 < s; c0 += 64) {
    {
      const int k = c0 + lane;
#pragma unroll
      for (int u = 0; u < P; ++u)
#pragma unroll
        for (int f = 0; f < F; ++f)
          coef[(u * 64 + lane) * F + f] = (k < s) ? cols_coef<F, DP, kCoefDiffusion>(M, pv[u], f, k) : 0.0;
    }
    wave_sync_lds();
    const int nq = min(16, (s - c0 + 3) / 4);
    const unsigned s0 = 8u * static_cast<unsigned>(c0) * r;
    double dA[F][T], dB[F][T];
    gram_load<F, T>(rs, s0, fbytes, vo, dA);
    double bA = M.bS[c0 + g], bB;
    for (int qq = 0; qq < nq; qq += 2) {
      const int k = c0 + 4 * qq + g;
      gram_load<F, T>(rs, s0 + (qq + 1) * gbytes, fbytes, vo, dB);
      bB = M.bS[k + 4];
      // keep these loads here (no instruction, no wait): otherwise they are
      // moved to their use in the next group
      asm volatile("" ::: "memory");
      gram_group<F, T, P, GRAM>(dA, (k < s ? bm : 0.0) * bA, coef, 4 * qq + g, bI, c16, acc, yreg, gacc, rr);
      if (qq + 1 < nq) {
        gram_load<F, T>(rs, s0 + (qq + 2) * gbytes, fbytes, vo, dA);
        bA = M.bS[k + 8];
        asm volatile("" ::: "memory");
        gram_group<F, T, P, GRAM>(dB, (k + 4 < s ? bm : 0.0) * bB, coef, 4 * qq + 4 + g, bI, c16, acc, yreg,
                                  gacc, rr);
      }
    }
    wave_sync_lds();  // the next chunk's coefficients overwrite these
  }
}

// v <- R^{-T} v with v distributed (entry j in lane j, j < r); R packed
// column-major in LDS (column c at c (c + 1) / 2), dinv = 1 / R_jj in lane j.
__device__ __forceinline__ double gram_forward(const double* R, int r, double dinv, double v, int lane) {
  double out = 0.0;
  for (int i = 0; i < r; ++i) {
    const double wi = lane_bcast(v * dinv, i);
    if (lane == i) out = wi;
    if (lane > i && lane < r) v = fma(-R[lane * (lane + 1) / 2 + i], wi, v);
  }
  return out;
}

// v <- R^{-1} v, same layout
__device__ __forceinline__ double gram_backward(const double* R, int r, double dinv, double v, int lane) {
  double out = 0.0;
  for (int c = r - 1; c >= 0; --c) {
    const double yc = lane_bcast(v * dinv, c);
    if (lane == c) out = yc;
    if (lane < c) v = fma(-R[c * (c + 1) / 2 + lane], yc, v);
  }
  return out;
}

// Parameters p0 .. p0 + P - 1 (those < m) of one wavefront; r + 1 <= 16 T.
template <int F, int DP, int T, int P>
__device__ __forceinline__ void gram_solve(const ColsModel& M, const double* params, int64_t m, int64_t p0, double* lds, int lane,
                           double* y, double* rho, int32_t* status) {
  constexpr int NT = T * (T + 1) / 2;
  const int r = M.r, r1 = r + 1;
  const int npk = r1 * (r1 + 1) / 2;
  double* coef = lds;
  double* rowbuf = coef + P * 64 * F;  // 16-byte aligned: P 64 F is even
  double* Rbase = rowbuf + 64;
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

  // Cholesky, lanes over columns
  double dinv[P], yv[P];
  bool ok[P];
#pragma unroll
  for (int u = 0; u < P; ++u) {
    double* R = Rbase + u * npk;
    double colv[16 * T];
#pragma unroll
    for (int i = 0; i < 16 * T; ++i) colv[i] = (lane < r1 && i <= lane) ? R[lane * (lane + 1) / 2 + i] : 0.0;
    const double dmax = gram_wave_max(lane < r ? R[lane * (lane + 1) / 2 + lane] : 0.0);
    const double thr2 = kGramPivTol * kGramPivTol * dmax;
    bool good = dmax > 0.0;
    dinv[u] = 0.0;
#pragma unroll
    for (int j = 0; j < 16 * T; ++j) {
      if (j < r1) {
        const double djj = lane_bcast(colv[j], j);
        if (j < r) good = good && (djj > thr2);
        const double piv = sqrt(fmax(djj, 0.0));
        const double inv = piv > 0.0 ? 1.0 / piv : 0.0;
        if (lane == j) dinv[u] = inv;
        colv[j] = lane > j ? colv[j] * inv : (lane == j ? piv : colv[j]);
        rowbuf[lane] = colv[j];
        wave_sync_lds();
        // entries beyond column r are zero in every lane and stay zero, so
        // the update runs over the whole register column without a guard
#pragma unroll
        for (int i = (j + 1) & ~1; i < 16 * T; i += 2) {
          const double2 rb = *reinterpret_cast<const double2*>(rowbuf + i);
          if (i > j) colv[i] = fma(-rb.x, colv[j], colv[i]);
          colv[i + 1] = fma(-rb.y, colv[j], colv[i + 1]);
        }
        wave_sync_lds();
      }
    }
#pragma unroll
    for (int i = 0; i < 16 * T; ++i)
      if (lane < r1 && i <= lane) R[lane * (lane + 1) / 2 + i] = colv[i];
    wave_sync_lds();
    ok[u] = good;
    // semi-normal solution y0 = R^{-1} z, z = column r of the factor
    const double z = lane < r ? R[r * (r + 1) / 2 + lane] : 0.0;
    yv[u] = gram_backward(R, r, dinv[u], z, lane);
  }

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
#pragma unroll
    for (int u = 0; u < P; ++u) {
      if (done[u]) continue;
      double gsel = 0.0;
#pragma unroll
      for (int I = 0; I < T; ++I) {
        double v = gacc[u][I];
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
        if (g == I) gsel = v;
      }
      if (lane >= r) gsel = 0.0;
      const double* R = Rbase + u * npk;
      const double w = gram_forward(R, r, dinv[u], -gsel, lane);
      const double dy = gram_backward(R, r, dinv[u], w, lane);
      if (lane < r) yv[u] += dy;
      const double rrs = gram_wave_sum(rr[u]);
      const double ww = gram_wave_sum(lane < r ? w * w : 0.0);
      const double ndy = sqrt(gram_wave_sum(lane < r ? dy * dy : 0.0));
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
