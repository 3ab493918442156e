// Online solve for kernel ridge regression (Section 6.3): A(p) = K_p + lambda I,
// K_p[i, j] = exp(-|t_i - t_j|^2 / (2 p^2)).  Only the s selected rows of K_p
// are generated (Section 3.1 "Computing S A(p*) X"), on the fly from the
// precomputed squared distances D[k, j] = |t_{i_k} - t_j|^2, and contracted
// with Q:  S A(p) Q = K_S(p) Q + lambda Q_S  (eq. (3.4)).
//
// Contraction forms:
//   FP64      exp and products in FP64 (vector ALU);
//   FP32      v_exp_f32 rows, FP32 MFMA 32x32x2, FP32 accumulation;
//   BF16X3    v_exp_f32 rows split as bf16 hi + lo, Q split likewise, three
//             MFMA 32x32x16 products hi*hi + hi*lo + lo*hi, FP32 accumulation;
//   FP16X3    the same with fp16 halves (Q columns scaled by powers of two).
// Then the FP64 Householder least squares (team_qr.h), and optional FP64
// refinement: r_S = K_S(p) (Q y) + lambda (Q y)_S - b_S with FP64-accurate
// kernel entries, correction from the stored factorisation (simple
// refinement) or from the corrected semi-normal equations with an FP64
// G^T r_S (a second pass over the kernel rows).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.h"
#include "family.h"
#include "profile.h"
#include "team_qr.h"

namespace subap {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr double kLog2e = 1.4426950408889634074;

__device__ __forceinline__ bool krr_param_ok(double sig) { return isfinite(sig) && sig > 0.0; }


// ---------------------------------------------------------------------------
// FP64 contraction, many parameters: lanes = parameters, one wave per KR rows.
// G[(p s + k) r + c] = sum_j exp(-D[k, j] / (2 p^2)) Q[j, c]
// ---------------------------------------------------------------------------
constexpr int kJC = 64;  // points per LDS chunk

template <int KR, int RM>
__global__ __launch_bounds__(256) void k_contract_f64(const double* params, int64_t m, int64_t n, int r,
                                                       int s, const double* Dt64, const double* Qrm,
                                                       double* G) {
  __shared__ double s_q[kJC][RM];
  __shared__ double s_d[kJC][4 * KR];
  const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * 64 + l;
  const int kbase = blockIdx.y * 4 * KR;
  const double sig = p < m ? params[p] : 1.0;
  const double cexp = krr_param_ok(sig) ? -0.5 * kLog2e / (sig * sig) : 0.0;
  double acc[KR][RM];
#pragma unroll
  for (int kr = 0; kr < KR; ++kr)
#pragma unroll
    for (int c = 0; c < RM; ++c) acc[kr][c] = 0.0;
  for (int64_t j0 = 0; j0 < n; j0 += kJC) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < kJC * RM; idx += 256) {
      const int jj = idx / RM, c = idx % RM;
      const int64_t j = j0 + jj;
      s_q[jj][c] = (j < n && c < r) ? Qrm[j * r + c] : 0.0;
    }
    for (int idx = threadIdx.x; idx < kJC * 4 * KR; idx += 256) {
      const int jj = idx / (4 * KR), kk = idx % (4 * KR);
      const int64_t j = j0 + jj;
      const int k = kbase + kk;
      s_d[jj][kk] = (j < n && k < s) ? Dt64[j * s + k] : 1e300;
    }
    __syncthreads();
    const int cnt = static_cast<int>(std::min<int64_t>(kJC, n - j0));
    for (int jj = 0; jj < cnt; ++jj) {
#pragma unroll
      for (int kr = 0; kr < KR; ++kr) {
        const double e = exp2_any<11>(cexp * s_d[jj][wave * KR + kr]);
#pragma unroll
        for (int c = 0; c < RM; ++c) acc[kr][c] = fma(e, s_q[jj][c], acc[kr][c]);
      }
    }
  }
  if (p < m) {
#pragma unroll
    for (int kr = 0; kr < KR; ++kr) {
      const int k = kbase + wave * KR + kr;
      if (k < s)
#pragma unroll
        for (int c = 0; c < RM; ++c)
          if (c < r) G[(p * s + k) * r + c] = acc[kr][c];
    }
  }
}

// FP64 contraction for few parameters (the per-p plain solve): one block per
// (p, k), threads split the points, block reduction of the r sums.
template <int RM>
__global__ __launch_bounds__(256) void k_contract_f64_small(const double* params, int64_t n, int r, int s,
                                                             const double* Dt64, const double* Qrm, double* G) {
  __shared__ double s_red[4][RM];
  const int64_t p = blockIdx.x;
  const int k = blockIdx.y;
  const double sig = params[p];
  const double cexp = krr_param_ok(sig) ? -0.5 * kLog2e / (sig * sig) : 0.0;
  double acc[RM];
#pragma unroll
  for (int c = 0; c < RM; ++c) acc[c] = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += 256) {
    const double e = exp2_any<11>(cexp * Dt64[j * s + k]);
#pragma unroll
    for (int c = 0; c < RM; ++c)
      if (c < r) acc[c] = fma(e, Qrm[j * r + c], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < RM; ++c) acc[c] = team_sum<64>(acc[c]);
  const int wave = threadIdx.x / 64;
  if (threadIdx.x % 64 == 0)
#pragma unroll
    for (int c = 0; c < RM; ++c) s_red[wave][c] = acc[c];
  __syncthreads();
  for (int c = threadIdx.x; c < r; c += 256)
    G[(p * s + k) * r + c] = (s_red[0][c] + s_red[1][c]) + (s_red[2][c] + s_red[3][c]);
}

// ---------------------------------------------------------------------------
// MFMA contraction with fused row generation.  A wave owns 32 rows of S
// (k0..k0+31) and PW parameters; per 16 points it loads its 32 x 16 distance
// tile once and the 16 x 32 tile of Q per column block once, and reuses both
// for all PW parameters.  MFMA 32x32 operand layout (64 lanes): lane l holds
// row/column (l mod 32) and the 8 (16-bit) or 1 (fp32) reduction indices of
// half (l / 32); A and B use the same reduction index for the same element.
// Accumulator element i of lane l is (row 8 (i/4) + 4 (l/32) + i mod 4,
// column l mod 32).
//
// The points are split into kSplit contiguous ranges (grid.z); each range is
// accumulated in FP32 and written as its own partial, and the least-squares
// kernel sums the partials in FP64, which keeps the FP32 accumulation error
// to that of n / kSplit terms.
//
// 16-bit split forms: K = 2^(c D) from v_exp_f32 is split as hi = t16(K),
// lo = t16(K - hi) and multiplied with the precomputed split of Q by three
// MFMAs (hi*hi + hi*lo + lo*hi).  t16 is bf16 (BF16X3) or fp16 (FP16X3); the
// fp16 split of Q is taken on the column scaled by a power of two so that its
// largest entry is near 2^14, and the scale is undone in FP64 afterwards.
// ---------------------------------------------------------------------------
constexpr int kSplit = 4;

struct MArgs {
  const double* params;
  int64_t m, n;
  int r, s;
  const float* D32;       // s x n
  const uint16_t* Qh;     // n x r col-major, bf16 or fp16 bits (scaled columns)
  const uint16_t* Ql;
  const float* Q32;       // n x r col-major fp32
  float* G;               // kSplit x m x s x r partials
};

__device__ __forceinline__ void load_dist8(const float* Drow, int64_t j, int64_t jend, bool vec, float (&dv)[8]) {
  if (vec && j + 8 <= jend) {
    const f32x4 a = *reinterpret_cast<const f32x4*>(Drow + j);
    const f32x4 b = *reinterpret_cast<const f32x4*>(Drow + j + 4);
    dv[0] = a[0]; dv[1] = a[1]; dv[2] = a[2]; dv[3] = a[3];
    dv[4] = b[0]; dv[5] = b[1]; dv[6] = b[2]; dv[7] = b[3];
  } else {
#pragma unroll
    for (int e = 0; e < 8; ++e) dv[e] = (j + e < jend) ? Drow[j + e] : __builtin_inff();
  }
}

template <typename T16>
struct Vec8;
template <>
struct Vec8<__bf16> {
  typedef __bf16 type __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ f32x16 mfma(type a, type b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  // hi = nearest bf16 of v, lo = nearest bf16 of v - hi
  static __device__ __forceinline__ void split(float v, __bf16* h, __bf16* l) {
    const __bf16 hh = static_cast<__bf16>(v);
    *h = hh;
    *l = static_cast<__bf16>(v - static_cast<float>(hh));
  }
};
template <>
struct Vec8<_Float16> {
  typedef _Float16 type __attribute__((ext_vector_type(8)));
  static __device__ __forceinline__ f32x16 mfma(type a, type b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
  // hi = v with its mantissa cut to fp16's 10 bits (a mask, exact in fp16 for
  // v >= 2^-14; below that the conversion rounds to the subnormal grid),
  // lo = nearest fp16 of v - hi, which is exact in FP32.
  static __device__ __forceinline__ void split(float v, _Float16* h, _Float16* l) {
    const float hf = __uint_as_float(__float_as_uint(v) & 0xFFFFE000u);
    *h = static_cast<_Float16>(hf);
    *l = static_cast<_Float16>(v - hf);
  }
};

// (j range of split z)
__device__ __forceinline__ void split_range(int64_t n, int z, int64_t* jb, int64_t* je) {
  const int64_t per = ((n + kSplit - 1) / kSplit + 15) / 16 * 16;
  *jb = z * per;
  *je = n < (z + 1) * per ? n : (z + 1) * per;
}

// Block -> (parameter block, point range).  Consecutive block indices go
// round-robin over the 8 XCDs; each point range is given to kXcd / kSplit
// XCDs so that every XCD's L2 holds one range of D and Q instead of all of
// them.  The grid has ceil(parameter blocks / (kXcd / kSplit)) * kXcd blocks
// along x; blocks past the last parameter block return at once.
constexpr int kXcd = 8;
static_assert(kXcd % kSplit == 0, "point ranges must divide the XCD count");

__device__ __forceinline__ void xcd_block(int64_t* pb, int* z) {
  constexpr unsigned per = kXcd / kSplit;
  const unsigned id = blockIdx.x, x = id % kXcd;
  *z = static_cast<int>(x / per);
  *pb = static_cast<int64_t>(id / kXcd) * per + x % per;
}

inline unsigned xcd_grid(int64_t blocks) {
  constexpr int64_t per = kXcd / kSplit;
  return static_cast<unsigned>((blocks + per - 1) / per * kXcd);
}

template <typename T16, int PW, int NB>
__global__ __launch_bounds__(256) void k_contract_x3(MArgs A) {
  typedef typename Vec8<T16>::type v8;
  const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
  const int k0 = (blockIdx.y * 4 + wave) * 32;
  int64_t pb;
  int z;
  xcd_block(&pb, &z);
  const int64_t p0 = pb * PW;
  if (k0 >= A.s || p0 >= A.m) return;  // uniform per wave
  int64_t jb, je;
  split_range(A.n, z, &jb, &je);
  const int row = k0 + (l & 31);
  const bool row_ok = row < A.s;
  const float* Drow = A.D32 + static_cast<int64_t>(row_ok ? row : 0) * A.n;
  const int jo = 8 * (l >> 5);
  const bool vec = (A.n & 7) == 0;
  float cexp[PW];
#pragma unroll
  for (int w = 0; w < PW; ++w) {
    const int64_t p = p0 + w;
    const double sig = p < A.m ? A.params[p] : 1.0;
    cexp[w] = krr_param_ok(sig) ? static_cast<float>(-0.5 * kLog2e / (sig * sig)) : 0.0f;
  }
  f32x16 acc[PW][NB];
#pragma unroll
  for (int w = 0; w < PW; ++w)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[w][nb][i] = 0.0f;
  for (int64_t j0 = jb; j0 < je; j0 += 16) {
    const int64_t j = j0 + jo;
    float dv[8];
    load_dist8(Drow, j, je, vec, dv);
    if (!row_ok)
#pragma unroll
      for (int e = 0; e < 8; ++e) dv[e] = __builtin_inff();
    v8 qh[NB], ql[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = nb * 32 + (l & 31);
      if (c < A.r && vec && j + 8 <= je) {
        qh[nb] = *reinterpret_cast<const v8*>(A.Qh + static_cast<int64_t>(c) * A.n + j);
        ql[nb] = *reinterpret_cast<const v8*>(A.Ql + static_cast<int64_t>(c) * A.n + j);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const bool ok = c < A.r && j + e < je;
          const uint16_t hb = ok ? A.Qh[static_cast<int64_t>(c) * A.n + j + e] : 0;
          const uint16_t lb = ok ? A.Ql[static_cast<int64_t>(c) * A.n + j + e] : 0;
          qh[nb][e] = __builtin_bit_cast(T16, hb);
          ql[nb][e] = __builtin_bit_cast(T16, lb);
        }
      }
    }
#pragma unroll
    for (int w = 0; w < PW; ++w) {
      v8 kh, kl;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        T16 h, lo;
        Vec8<T16>::split(__builtin_amdgcn_exp2f(cexp[w] * dv[e]), &h, &lo);
        kh[e] = h;
        kl[e] = lo;
      }
#pragma unroll
      for (int nb = 0; nb < NB; ++nb) {
        acc[w][nb] = Vec8<T16>::mfma(kh, qh[nb], acc[w][nb]);
        acc[w][nb] = Vec8<T16>::mfma(kh, ql[nb], acc[w][nb]);
        acc[w][nb] = Vec8<T16>::mfma(kl, qh[nb], acc[w][nb]);
      }
    }
  }
  float* Gz = A.G + static_cast<int64_t>(z) * A.m * A.s * A.r;
#pragma unroll
  for (int w = 0; w < PW; ++w) {
    const int64_t p = p0 + w;
    if (p >= A.m) continue;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = nb * 32 + (l & 31);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int rr = k0 + 8 * (i / 4) + 4 * (l >> 5) + (i & 3);
        if (rr < A.s && c < A.r) Gz[(p * A.s + rr) * A.r + c] = acc[w][nb][i];
      }
    }
  }
}

template <int PW, int NB>
__global__ __launch_bounds__(256) void k_contract_f32(MArgs A) {
  const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
  const int k0 = (blockIdx.y * 4 + wave) * 32;
  int64_t pb;
  int z;
  xcd_block(&pb, &z);
  const int64_t p0 = pb * PW;
  if (k0 >= A.s || p0 >= A.m) return;  // uniform per wave
  int64_t jb, je;
  split_range(A.n, z, &jb, &je);
  const int row = k0 + (l & 31);
  const bool row_ok = row < A.s;
  const float* Drow = A.D32 + static_cast<int64_t>(row_ok ? row : 0) * A.n;
  const int jo = 8 * (l >> 5);
  const bool vec = (A.n & 7) == 0;
  float cexp[PW];
#pragma unroll
  for (int w = 0; w < PW; ++w) {
    const int64_t p = p0 + w;
    const double sig = p < A.m ? A.params[p] : 1.0;
    cexp[w] = krr_param_ok(sig) ? static_cast<float>(-0.5 * kLog2e / (sig * sig)) : 0.0f;
  }
  f32x16 acc[PW][NB];
#pragma unroll
  for (int w = 0; w < PW; ++w)
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[w][nb][i] = 0.0f;
  for (int64_t j0 = jb; j0 < je; j0 += 16) {
    const int64_t j = j0 + jo;
    float dv[8];
    load_dist8(Drow, j, je, vec, dv);
    if (!row_ok)
#pragma unroll
      for (int e = 0; e < 8; ++e) dv[e] = __builtin_inff();
    float qv[NB][8];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = nb * 32 + (l & 31);
      const float* qc = A.Q32 + static_cast<int64_t>(c < A.r ? c : 0) * A.n;
      float tmp[8];
      load_dist8(qc, j, je, vec, tmp);
#pragma unroll
      for (int e = 0; e < 8; ++e) qv[nb][e] = (c < A.r && j + e < je) ? tmp[e] : 0.0f;
    }
#pragma unroll
    for (int w = 0; w < PW; ++w) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const float kv = __builtin_amdgcn_exp2f(cexp[w] * dv[e]);
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
          acc[w][nb] = __builtin_amdgcn_mfma_f32_32x32x2f32(kv, qv[nb][e], acc[w][nb], 0, 0, 0);
      }
    }
  }
  float* Gz = A.G + static_cast<int64_t>(z) * A.m * A.s * A.r;
#pragma unroll
  for (int w = 0; w < PW; ++w) {
    const int64_t p = p0 + w;
    if (p >= A.m) continue;
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) {
      const int c = nb * 32 + (l & 31);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int rr = k0 + 8 * (i / 4) + 4 * (l >> 5) + (i & 3);
        if (rr < A.s && c < A.r) Gz[(p * A.s + rr) * A.r + c] = acc[w][nb][i];
      }
    }
  }
}

// Sum of the kSplit FP32 partials in FP64, with the column scale undone:
// G64[e] = colscale[c] * sum_z G32[z][e], e = (p s + k) r + c.  Coalesced.
__global__ void k_reduce_partials(const float* G32, int64_t len, int r, const double* colscale, double* G64) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double g = 0.0;
#pragma unroll
  for (int z = 0; z < kSplit; ++z) g += static_cast<double>(G32[z * len + e]);
  if (colscale) g *= colscale[e % r];
  G64[e] = g;
}

// ---------------------------------------------------------------------------
// Least squares from a contraction in global memory: one team per p.
// G_full = G + lambda Q_S.  Stores the factorisation for refinement.
// ---------------------------------------------------------------------------
struct LArgs {
  const double* params;
  int64_t m;
  int r, s;
  const void* G;          // double m x s x r, or float nsplit x m x s x r partials
  int nsplit;             // number of float partials to add (1 for double)
  const double* colscale; // r: multiply column c of the sum by colscale[c] (or nullptr)
  const double* wS;       // s row weights of the kernel part (QS, bS carry theirs)
  const double* QS;       // s x r
  const double* bS;
  double lambda, bS_norm;
  double* y;
  double* rho;
  int32_t* status;
  double* fac;            // m x fac_stride, or nullptr
  int fac_stride;
};

template <int TEAM, int R, int RM>
__device__ __forceinline__ int fac_index(int q, int c, int lane) {
  return (q * RM + c) * TEAM + lane;
}

template <int TEAM, int R, int RM, typename GT>
__global__ __launch_bounds__(256) void k_lsq(LArgs A) {
  constexpr int TEAMS = 256 / TEAM;
  __shared__ double s_tau[TEAMS][RM];
  __shared__ double s_y[TEAMS][RM];
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * TEAMS + team;
  if (p >= A.m) return;
  const int r = A.r, s = A.s;
  const GT* G = static_cast<const GT*>(A.G);
  TeamQR<TEAM, R, RM> qr;
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = lane + TEAM * q;
#pragma unroll
    for (int c = 0; c < RM; ++c) {
      double g = 0.0;
      if (k < s && c < r) {
        for (int z = 0; z < A.nsplit; ++z)
          g += static_cast<double>(G[((z * A.m + p) * s + k) * r + c]);
        if (A.colscale) g *= A.colscale[c];
        g = fma(A.wS[k], g, A.lambda * A.QS[k * r + c]);
      }
      qr.a[q][c] = g;
    }
    qr.b[q] = k < s ? A.bS[k] : 0.0;
  }
  qr.factor(r, lane, s_tau[team]);
  const double tail = qr.tail_norm(qr.b, r, lane);
  double x[R];
#pragma unroll
  for (int q = 0; q < R; ++q) x[q] = qr.b[q];
  qr.back_substitute(x, r, lane, s_y[team]);
  const double sig = A.params[p];
  bool yfin = true;
  for (int c = 0; c < r; ++c) yfin = yfin && isfinite(s_y[team][c]);
  int32_t code = SUBAP_OK;
  if (!krr_param_ok(sig)) code = SUBAP_E_NONFINITE;
  else if (!qr.full_rank) code = SUBAP_E_RANK;
  else if (!yfin) code = SUBAP_E_NONFINITE;
  for (int c = lane; c < r; c += TEAM)
    A.y[p * r + c] = code == SUBAP_OK ? s_y[team][c] : __longlong_as_double(0x7ff8000000000000LL);
  if (lane == 0) {
    if (A.rho) A.rho[p] = tail / A.bS_norm;
    if (A.status) A.status[p] = code;
  }
  if (A.fac) {
    double* f = A.fac + p * A.fac_stride;
#pragma unroll
    for (int q = 0; q < R; ++q)
#pragma unroll
      for (int c = 0; c < RM; ++c) f[fac_index<TEAM, R, RM>(q, c, lane)] = qr.a[q][c];
    for (int j = lane; j < RM; j += TEAM) f[TEAM * R * RM + j] = s_tau[team][j];
  }
}

// ---------------------------------------------------------------------------
// Refinement, part 1: partial sums of K_S(p) z, z = Q y, over a range of
// points.  Block: PB parameters x one point range; thread = selected row k.
// Kernel entries 2^(c_p D) with the degree-DEG polynomial of exp2_poly.h:
// DEG = 7 (relative error 5.5e-11) in the first refinement step, DEG = 11
// (FP64 rounding) in later steps and in the sketched residual.  The range
// index is the block index mod 8, so with round-robin dispatch over the 8
// XCDs each XCD reads one eighth of D through its L2.
// ---------------------------------------------------------------------------
constexpr int kRefPB = 16;     // parameters per block
constexpr int kRefNJ = 128;    // points per LDS chunk
constexpr int kRefSplit = 8;   // point ranges

template <int RM, int DEG>
__global__ __launch_bounds__(256, 4) void k_refine_partial(const double* params, int64_t m, int64_t n, int r,
                                                         int s, double dmax, const double* Dt64,
                                                         const double* Qrm, const double* y, double* part) {
  __shared__ double s_y[RM][kRefPB];
  __shared__ double s_z[kRefNJ][kRefPB];
  const int t = threadIdx.x;
  const int split = blockIdx.x % kRefSplit;
  const int64_t p0 = static_cast<int64_t>(blockIdx.x / kRefSplit) * kRefPB;
  for (int idx = t; idx < kRefPB * RM; idx += blockDim.x) {
    const int w = idx / RM, c = idx % RM;
    s_y[c][w] = (p0 + w < m && c < r) ? y[(p0 + w) * r + c] : 0.0;
  }
  // per-parameter factor: entry = 2^(cv D), cv = -log2(e) / (2 p^2)
  // (the same for every thread of the block: kept in scalar registers, which
  // leaves the vector registers to the accumulators)
  double cv[kRefPB];
  double cmax = 0.0;
#pragma unroll
  for (int w = 0; w < kRefPB; ++w) {
    const double sig = p0 + w < m ? params[p0 + w] : 1.0;
    const double c = krr_param_ok(sig) ? -0.5 * kLog2e / (sig * sig) : 0.0;
    cv[w] = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(c)),
                             __builtin_amdgcn_readfirstlane(__double2loint(c)));
    cmax = fmax(cmax, -cv[w]);
  }
  // every |cv D| of the block below 2^30: unclamped reduction (uniform branch)
  const bool direct = cmax * dmax < kExp2Range;
  double acc[kRefPB];
#pragma unroll
  for (int w = 0; w < kRefPB; ++w) acc[w] = 0.0;
  const int64_t per = (n + kRefSplit - 1) / kRefSplit;
  const int64_t jb = split * per, je = std::min<int64_t>(n, jb + per);
  for (int64_t j0 = jb; j0 < je; j0 += kRefNJ) {
    __syncthreads();
    // z for this chunk: thread = point, all PB parameters
    for (int jj = t; jj < kRefNJ; jj += blockDim.x) {
      const int64_t j = j0 + jj;
      double z[kRefPB];
#pragma unroll
      for (int w = 0; w < kRefPB; ++w) z[w] = 0.0;
      if (j < je)
        for (int c = 0; c < r; ++c) {
          const double q = Qrm[j * r + c];
#pragma unroll
          for (int w = 0; w < kRefPB; ++w) z[w] = fma(q, s_y[c][w], z[w]);
        }
#pragma unroll
      for (int w = 0; w < kRefPB; ++w) s_z[jj][w] = z[w];
    }
    __syncthreads();
    if (t < s) {
      const int cnt = static_cast<int>(std::min<int64_t>(kRefNJ, je - j0));
      const double* Dp = Dt64 + j0 * s + t;
      double dn = cnt > 0 ? Dp[0] : 0.0;
      if (direct) {
        for (int jj = 0; jj < cnt; ++jj) {
          const double d = dn;
          if (jj + 1 < cnt) dn = Dp[(jj + 1) * s];  // prefetch the next distance
#pragma unroll
          for (int w = 0; w < kRefPB; ++w) acc[w] = fma(exp2_mul<DEG>(cv[w], d), s_z[jj][w], acc[w]);
        }
      } else {
        for (int jj = 0; jj < cnt; ++jj) {
          const double d = dn;
          if (jj + 1 < cnt) dn = Dp[(jj + 1) * s];
#pragma unroll
          for (int w = 0; w < kRefPB; ++w) acc[w] = fma(exp2_any<DEG>(cv[w] * d), s_z[jj][w], acc[w]);
        }
      }
    }
  }
  if (t < s)
#pragma unroll
    for (int w = 0; w < kRefPB; ++w)
      if (p0 + w < m) part[(static_cast<int64_t>(split) * m + p0 + w) * s + t] = acc[w];
}

// Refinement, part 2: r_S = sum of partials + lambda Q_S y - b_S; y -= R^{-1} Q^T r_S.
struct CArgs {
  int64_t m;
  int r, s;
  const double* part;
  const double* wS;
  const double* QS;
  const double* bS;
  double lambda, bS_norm;
  const double* fac;
  int fac_stride;
  double* y;
  double* rho;
  const int32_t* status;
};

template <int TEAM, int R, int RM>
__global__ __launch_bounds__(256) void k_correct(CArgs A) {
  constexpr int TEAMS = 256 / TEAM;
  __shared__ double s_tau[TEAMS][RM];
  __shared__ double s_y[TEAMS][RM];
  __shared__ double s_dy[TEAMS][RM];
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * TEAMS + team;
  if (p >= A.m) return;
  if (A.status && A.status[p] != SUBAP_OK) return;  // y already NaN
  const int r = A.r, s = A.s;
  TeamQR<TEAM, R, RM> qr;
  const double* f = A.fac + p * A.fac_stride;
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int c = 0; c < RM; ++c) qr.a[q][c] = f[fac_index<TEAM, R, RM>(q, c, lane)];
  for (int j = 0; j < RM; ++j) s_tau[team][j] = f[TEAM * R * RM + j];
  for (int c = 0; c < RM; ++c) s_y[team][c] = c < r ? A.y[p * r + c] : 0.0;
  double res[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = lane + TEAM * q;
    double t = 0.0;
    if (k < s) {
      for (int sp = 0; sp < kRefSplit; ++sp) t += A.part[(static_cast<int64_t>(sp) * A.m + p) * s + k];
      double zs = 0.0;
      for (int c = 0; c < r; ++c) zs = fma(A.QS[k * r + c], s_y[team][c], zs);
      t = A.wS[k] * t + (A.lambda * zs - A.bS[k]);
    }
    res[q] = k < s ? t : 0.0;
  }
  qr.apply_qt(res, r, lane, s_tau[team]);
  const double tail = qr.tail_norm(res, r, lane);
  qr.back_substitute(res, r, lane, s_dy[team]);
  for (int c = lane; c < r; c += TEAM) A.y[p * r + c] = s_y[team][c] - s_dy[team][c];
  if (lane == 0 && A.rho) A.rho[p] = tail / A.bS_norm;
}

// Sketched residual from the partial sums: one wavefront per parameter.
__global__ __launch_bounds__(256) void k_resid_finish(const double* params, int64_t m, int r, int s,
                                                       const double* part, const double* wS, const double* QS,
                                                       const double* bS,
                                                       double lambda, double bS_norm, const double* y,
                                                       double* res, double* norm) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (p >= m) return;
  const bool ok = krr_param_ok(params[p]);
  double ss = 0.0;
  for (int k = lane; k < s; k += 64) {
    double t = 0.0;
    for (int sp = 0; sp < kRefSplit; ++sp) t += part[(static_cast<int64_t>(sp) * m + p) * s + k];
    double zs = 0.0;
    for (int c = 0; c < r; ++c) zs = fma(QS[k * r + c], y[p * r + c], zs);
    t = wS[k] * t + (lambda * zs - bS[k]);
    if (!ok) t = __longlong_as_double(0x7ff8000000000000LL);
    if (res) res[p * s + k] = t;
    ss += t * t;
  }
  ss = team_sum<64>(ss);
  if (lane == 0 && norm) norm[p] = sqrt(ss) / bS_norm;
}

// ---------------------------------------------------------------------------
// Corrected semi-normal equations (Bjorck): the correction of a refinement
// step solves R^T R dy = G^T r_S with R from the rounded contraction and
//   G^T r_S = Q^T (K_S(p)^T (w o r_S)) + lambda Q_S^T r_S
// in FP64 (G = W S A(p) Q; w the row weights, carried by Q_S already).  The
// fixed point is G^T r_S = 0, the exact solution of eq. (3.3), where simple
// refinement stops at the least-squares solution of the rounded G.
//
// Adjoint, part 1: partial sums of Q^T K_S(p)^T (w o r_S) over a range of
// points.  Block: PB parameters x one point range (block index mod 8, the
// same XCD split as the residual).  Thread = point j of a chunk of 256:
//   u_j = sum_k 2^(c_p D[j, k]) w_k r_k       (kernel entries as in the residual)
// then the block adds u_j Q[j, :] over the chunk, (parameter, column) pairs
// over the threads.  Split 0 also adds lambda Q_S^T r_S.
// ---------------------------------------------------------------------------
constexpr int kAdjNJ = 256;  // points per chunk (one per thread)

template <int RM, int DEG>
__global__ __launch_bounds__(256) void k_adjoint_partial(const double* params, int64_t m, int64_t n, int r, int s,
                                                         double dmax, const double* Dt64, const double* Qrm,
                                                         const double* wS, const double* QS, double lambda,
                                                         const double* rvec, double* gpart) {
  extern __shared__ double adj_lds[];
  double* s_t = adj_lds;                    // s x PB: w_k r_k of each parameter
  double* s_u = adj_lds + s * kRefPB;       // kAdjNJ x PB
  constexpr int NP = (kRefPB * RM + 255) / 256;  // (parameter, column) pairs per thread
  const int t = threadIdx.x;
  const int split = blockIdx.x % kRefSplit;
  const int64_t p0 = static_cast<int64_t>(blockIdx.x / kRefSplit) * kRefPB;
  for (int idx = t; idx < s * kRefPB; idx += 256) {
    const int k = idx / kRefPB, w = idx % kRefPB;
    s_t[idx] = (p0 + w < m) ? wS[k] * rvec[(p0 + w) * s + k] : 0.0;
  }
  double cv[kRefPB];
  double cmax = 0.0;
#pragma unroll
  for (int w = 0; w < kRefPB; ++w) {
    const double sig = p0 + w < m ? params[p0 + w] : 1.0;
    const double c = krr_param_ok(sig) ? -0.5 * kLog2e / (sig * sig) : 0.0;
    cv[w] = __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(c)),
                             __builtin_amdgcn_readfirstlane(__double2loint(c)));
    cmax = fmax(cmax, -cv[w]);
  }
  const bool direct = cmax * dmax < kExp2Range;
  double acc[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) acc[i] = 0.0;
  const int64_t per = (n + kRefSplit - 1) / kRefSplit;
  const int64_t jb = split * per, je = std::min<int64_t>(n, jb + per);
  for (int64_t j0 = jb; j0 < je; j0 += kAdjNJ) {
    __syncthreads();  // s_t is written; the previous chunk's s_u is consumed
    const int64_t j = j0 + t;
    double u[kRefPB];
#pragma unroll
    for (int w = 0; w < kRefPB; ++w) u[w] = 0.0;
    if (j < je) {
      const double* Dp = Dt64 + j * s;
      double dn = Dp[0];
      if (direct) {
        for (int k = 0; k < s; ++k) {
          const double d = dn;
          if (k + 1 < s) dn = Dp[k + 1];
#pragma unroll
          for (int w = 0; w < kRefPB; ++w) u[w] = fma(exp2_mul<DEG>(cv[w], d), s_t[k * kRefPB + w], u[w]);
        }
      } else {
        for (int k = 0; k < s; ++k) {
          const double d = dn;
          if (k + 1 < s) dn = Dp[k + 1];
#pragma unroll
          for (int w = 0; w < kRefPB; ++w) u[w] = fma(exp2_any<DEG>(cv[w] * d), s_t[k * kRefPB + w], u[w]);
        }
      }
    }
#pragma unroll
    for (int w = 0; w < kRefPB; ++w) s_u[t * kRefPB + w] = u[w];
    __syncthreads();
    const int cnt = static_cast<int>(std::min<int64_t>(kAdjNJ, je - j0));
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int pair = t + 256 * i, w = pair / RM, c = pair % RM;
      if (w < kRefPB && c < r) {
        double a0 = 0.0, a1 = 0.0;
        int jj = 0;
        for (; jj + 1 < cnt; jj += 2) {
          a0 = fma(s_u[jj * kRefPB + w], Qrm[(j0 + jj) * r + c], a0);
          a1 = fma(s_u[(jj + 1) * kRefPB + w], Qrm[(j0 + jj + 1) * r + c], a1);
        }
        if (jj < cnt) a0 = fma(s_u[jj * kRefPB + w], Qrm[(j0 + jj) * r + c], a0);
        acc[i] += a0 + a1;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    const int pair = t + 256 * i, w = pair / RM, c = pair % RM;
    if (w < kRefPB && c < r && p0 + w < m) {
      double g = acc[i];
      if (split == 0) {  // lambda Q_S^T r_S (Q_S carries the row weights)
        double l = 0.0;
        for (int k = 0; k < s; ++k) l = fma(QS[k * r + c], rvec[(p0 + w) * s + k], l);
        g = fma(lambda, l, g);
      }
      gpart[(static_cast<int64_t>(split) * m + p0 + w) * r + c] = g;
    }
  }
}

// Adjoint, part 2: g = sum of the partials; y -= R^{-1} R^{-T} g with R from
// the stored factorisation; rho from the part of the FP64 residual r_S outside
// the range of the computed Q factor (as in k_correct).
template <int TEAM, int R, int RM>
__global__ __launch_bounds__(256) void k_csne_correct(CArgs A, const double* rvec, const double* gpart) {
  constexpr int TEAMS = 256 / TEAM;
  __shared__ double s_tau[TEAMS][RM];
  __shared__ double s_dy[TEAMS][RM];
  const int team = threadIdx.x / TEAM, lane = threadIdx.x % TEAM;
  const int64_t p = static_cast<int64_t>(blockIdx.x) * TEAMS + team;
  if (p >= A.m) return;
  if (A.status && A.status[p] != SUBAP_OK) return;  // y already NaN
  const int r = A.r, s = A.s;
  TeamQR<TEAM, R, RM> qr;
  const double* f = A.fac + p * A.fac_stride;
#pragma unroll
  for (int q = 0; q < R; ++q)
#pragma unroll
    for (int c = 0; c < RM; ++c) qr.a[q][c] = f[fac_index<TEAM, R, RM>(q, c, lane)];
  for (int j = 0; j < RM; ++j) s_tau[team][j] = f[TEAM * R * RM + j];
  double g[R], res[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int k = lane + TEAM * q;
    double t = 0.0;
    if (k < r)
      for (int sp = 0; sp < kRefSplit; ++sp) t += gpart[(static_cast<int64_t>(sp) * A.m + p) * r + k];
    g[q] = t;
    res[q] = k < s ? rvec[p * s + k] : 0.0;
  }
  qr.forward_substitute_t(g, r, lane);
  qr.back_substitute(g, r, lane, s_dy[team]);
  for (int c = lane; c < r; c += TEAM) A.y[p * r + c] -= s_dy[team][c];
  qr.apply_qt(res, r, lane, s_tau[team]);
  const double tail = qr.tail_norm(res, r, lane);
  if (lane == 0 && A.rho) A.rho[p] = tail / A.bS_norm;
}

// ---------------------------------------------------------------------------
// dispatch helpers
// ---------------------------------------------------------------------------
struct Shape {
  int team, R, RM;
};

bool pick_shape(int s, int r, Shape* out) {
  static const Shape kShapes[] = {
      {16, 1, 8}, {16, 1, 16}, {32, 1, 8}, {32, 1, 16}, {32, 1, 32}, {64, 1, 16},
      {64, 1, 32}, {64, 1, 40}, {64, 2, 16}, {64, 2, 32}, {64, 2, 40}, {64, 3, 32}, {64, 3, 40},
      {64, 4, 40}};
  for (const Shape& sh : kShapes)
    if (s <= sh.team * sh.R && r <= sh.RM) {
      *out = sh;
      return true;
    }
  return false;
}

template <typename GT>
subap_status launch_lsq(const Shape& sh, const LArgs& a, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>((a.m * sh.team + 255) / 256);
#define SUBAP_LSQ(T_, R_, M_)                                                              \
  if (sh.team == T_ && sh.R == R_ && sh.RM == M_) {                                      \
    hipLaunchKernelGGL((k_lsq<T_, R_, M_, GT>), dim3(grid), dim3(256), 0, st, a);        \
    SUBAP_HIP_TRY(hipGetLastError());                                                    \
    return SUBAP_OK;                                                                     \
  }
  SUBAP_LSQ(16, 1, 8) SUBAP_LSQ(16, 1, 16) SUBAP_LSQ(32, 1, 8) SUBAP_LSQ(32, 1, 16) SUBAP_LSQ(32, 1, 32)
  SUBAP_LSQ(64, 1, 16) SUBAP_LSQ(64, 1, 32) SUBAP_LSQ(64, 1, 40)
  SUBAP_LSQ(64, 2, 16) SUBAP_LSQ(64, 2, 32) SUBAP_LSQ(64, 2, 40)
  SUBAP_LSQ(64, 3, 32) SUBAP_LSQ(64, 3, 40) SUBAP_LSQ(64, 4, 40)
#undef SUBAP_LSQ
  set_error("no least-squares kernel for this (s, r)");
  return SUBAP_E_UNSUPPORTED;
}

subap_status launch_correct(const Shape& sh, const CArgs& a, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>((a.m * sh.team + 255) / 256);
#define SUBAP_COR(T_, R_, M_)                                                        \
  if (sh.team == T_ && sh.R == R_ && sh.RM == M_) {                                \
    hipLaunchKernelGGL((k_correct<T_, R_, M_>), dim3(grid), dim3(256), 0, st, a);  \
    SUBAP_HIP_TRY(hipGetLastError());                                              \
    return SUBAP_OK;                                                               \
  }
  SUBAP_COR(16, 1, 8) SUBAP_COR(16, 1, 16) SUBAP_COR(32, 1, 8) SUBAP_COR(32, 1, 16) SUBAP_COR(32, 1, 32)
  SUBAP_COR(64, 1, 16) SUBAP_COR(64, 1, 32) SUBAP_COR(64, 1, 40)
  SUBAP_COR(64, 2, 16) SUBAP_COR(64, 2, 32) SUBAP_COR(64, 2, 40)
  SUBAP_COR(64, 3, 32) SUBAP_COR(64, 3, 40) SUBAP_COR(64, 4, 40)
#undef SUBAP_COR
  set_error("no correction kernel for this (s, r)");
  return SUBAP_E_UNSUPPORTED;
}

subap_status launch_csne_correct(const Shape& sh, const CArgs& a, const double* rvec, const double* gpart,
                                 hipStream_t st) {
  const unsigned grid = static_cast<unsigned>((a.m * sh.team + 255) / 256);
#define SUBAP_CSNE(T_, R_, M_)                                                                          \
  if (sh.team == T_ && sh.R == R_ && sh.RM == M_) {                                                     \
    hipLaunchKernelGGL((k_csne_correct<T_, R_, M_>), dim3(grid), dim3(256), 0, st, a, rvec, gpart);    \
    SUBAP_HIP_TRY(hipGetLastError());                                                                   \
    return SUBAP_OK;                                                                                    \
  }
  SUBAP_CSNE(16, 1, 8) SUBAP_CSNE(16, 1, 16) SUBAP_CSNE(32, 1, 8) SUBAP_CSNE(32, 1, 16) SUBAP_CSNE(32, 1, 32)
  SUBAP_CSNE(64, 1, 16) SUBAP_CSNE(64, 1, 32) SUBAP_CSNE(64, 1, 40)
  SUBAP_CSNE(64, 2, 16) SUBAP_CSNE(64, 2, 32) SUBAP_CSNE(64, 2, 40)
  SUBAP_CSNE(64, 3, 32) SUBAP_CSNE(64, 3, 40) SUBAP_CSNE(64, 4, 40)
#undef SUBAP_CSNE
  set_error("no correction kernel for this (s, r)");
  return SUBAP_E_UNSUPPORTED;
}

int rm_of(int r) { return r <= 8 ? 8 : r <= 16 ? 16 : r <= 32 ? 32 : r <= 40 ? 40 : 64; }

template <int DEG>
void launch_adjoint_deg(subap_model_s* M, const double* params, int64_t m, const double* rvec, double* gpart,
                        hipStream_t st) {
  const int r = M->r, s = M->s;
  const int64_t n = M->n;
  const dim3 grid(static_cast<unsigned>((m + kRefPB - 1) / kRefPB * kRefSplit));
  const size_t lds = sizeof(double) * kRefPB * (static_cast<size_t>(s) + kAdjNJ);
#define SUBAP_ADJ(RM_)                                                                                      \
  hipLaunchKernelGGL((k_adjoint_partial<RM_, DEG>), grid, dim3(256), lds, st, params, m, n, r, s, M->dmax,  \
                     M->Dt64, M->Qrm, M->wS, M->QS, M->lambda, rvec, gpart)
  switch (rm_of(r)) {
    case 8: SUBAP_ADJ(8); break;
    case 16: SUBAP_ADJ(16); break;
    case 32: SUBAP_ADJ(32); break;
    case 40: SUBAP_ADJ(40); break;
    default: SUBAP_ADJ(64); break;
  }
#undef SUBAP_ADJ
}

// FP64 G^T r_S partials for the corrected semi-normal equations; the first
// step's kernel entries use the degree-7 polynomial like its residual.
subap_status launch_adjoint(subap_model_s* M, const double* params, int64_t m, const double* rvec, double* gpart,
                            bool exact, hipStream_t st) {
  {
    ProfScope prof(exact ? "krr_adjoint_partial_exact" : "krr_adjoint_partial", st);
    if (exact) launch_adjoint_deg<11>(M, params, m, rvec, gpart, st);
    else launch_adjoint_deg<7>(M, params, m, rvec, gpart, st);
  }
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

}  // namespace

subap_status launch_refine_partial(subap_model_s* M, const double* params, int64_t m, const double* y,
                                   double* part, bool exact, hipStream_t st);

namespace {

// Workspace of one krr_solve call, in bytes, laid out as consecutive
// 256-byte-aligned pieces: G (FP64, plus the FP32 split partials of the MFMA
// forms), the stored factorisation and the residual partials (refinement),
// the status fallback, and for the corrected semi-normal equations the
// residual vectors and the G^T r_S partials.
struct KrrWork {
  size_t g, f, p, st, rv, a;
  static size_t al(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }
  size_t total() const { return al(g) + al(f) + al(p) + al(st) + al(rv) + al(a); }
};

KrrWork krr_work(const subap_model_s* M, const Shape& sh, int64_t m, int prec, int refine, bool csne) {
  const int r = M->r, s = M->s;
  const bool cs = csne && refine > 0;
  const int fac_stride = sh.team * sh.R * sh.RM + sh.RM;
  KrrWork w;
  w.g = static_cast<size_t>(m) * s * r * (prec == SUBAP_FP64 ? 8 : 8 + 4 * kSplit);
  w.f = refine > 0 ? static_cast<size_t>(m) * fac_stride * 8 : 0;
  w.p = refine > 0 ? static_cast<size_t>(kRefSplit) * m * s * 8 : 0;
  w.st = static_cast<size_t>(m) * 4;
  w.rv = cs ? static_cast<size_t>(m) * s * 8 : 0;
  w.a = cs ? static_cast<size_t>(kRefSplit) * m * r * 8 : 0;
  return w;
}

}  // namespace

int64_t krr_chunk(const subap_model_s* M, int prec, int refine, bool csne, size_t bytes) {
  Shape sh;
  if (!pick_shape(M->s, M->r, &sh)) return 0;
  // parameters in multiples of the refinement's block of kRefPB, so that a
  // chunked batch groups its parameters into blocks as one call would
  int64_t lo = 0, hi = int64_t(1) << 26;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (krr_work(M, sh, mid * kRefPB, prec, refine, csne).total() <= bytes) lo = mid;
    else hi = mid - 1;
  }
  return lo * kRefPB;
}

size_t krr_work_bytes(const subap_model_s* M, int64_t m, int prec, int refine, bool csne) {
  Shape sh;
  if (!pick_shape(M->s, M->r, &sh)) return 0;
  return krr_work(M, sh, m, prec, refine, csne).total();
}

subap_status krr_solve(subap_model_s* M, const double* params, int64_t m, double* y, double* rho,
                       int32_t* status, int prec, int refine, bool csne, hipStream_t st) {
  Shape sh;
  if (!pick_shape(M->s, M->r, &sh)) {
    set_error("no least-squares kernel for this (s, r)");
    return SUBAP_E_UNSUPPORTED;
  }
  SUBAP_TRY(ensure_work(M, krr_work(M, sh, m, prec, refine, csne).total()));
  return krr_solve_ws(M, params, m, y, rho, status, prec, refine, csne, M->work, st);
}

subap_status krr_solve_ws(subap_model_s* M, const double* params, int64_t m, double* y, double* rho,
                          int32_t* status, int prec, int refine, bool csne, void* work, hipStream_t st) {
  const int r = M->r, s = M->s;
  const int64_t n = M->n;
  Shape sh;
  if (!pick_shape(s, r, &sh)) {
    set_error("no least-squares kernel for this (s, r)");
    return SUBAP_E_UNSUPPORTED;
  }
  const int RM = rm_of(r);
  const KrrWork kw = krr_work(M, sh, m, prec, refine, csne);
  const size_t gbytes = kw.g, fbytes = kw.f, pbytes = kw.p, stbytes = kw.st, rbytes = kw.rv;
  const int fac_stride = sh.team * sh.R * sh.RM + sh.RM;
  const bool cs = csne && refine > 0;
  auto al = KrrWork::al;
  char* w = static_cast<char*>(work);
  void* G = w;
  double* fac = refine > 0 ? reinterpret_cast<double*>(w + al(gbytes)) : nullptr;
  double* part = refine > 0 ? reinterpret_cast<double*>(w + al(gbytes) + al(fbytes)) : nullptr;
  int32_t* stat = status ? status : reinterpret_cast<int32_t*>(w + al(gbytes) + al(fbytes) + al(pbytes));
  char* wc = w + al(gbytes) + al(fbytes) + al(pbytes) + al(stbytes);
  double* rvec = cs ? reinterpret_cast<double*>(wc) : nullptr;
  double* gpart = cs ? reinterpret_cast<double*>(wc + al(rbytes)) : nullptr;

  // A1 + A2: rows and contraction
  if (prec == SUBAP_FP64) {
    double* Gd = static_cast<double*>(G);
    if (m >= 32) {
      ProfScope prof("krr_contract_fp64", st);
      constexpr int KR = 2;
      dim3 grid(static_cast<unsigned>((m + 63) / 64), static_cast<unsigned>((s + 4 * KR - 1) / (4 * KR)));
      switch (RM) {
        case 8: hipLaunchKernelGGL((k_contract_f64<KR, 8>), grid, dim3(256), 0, st, params, m, n, r, s, M->Dt64, M->Qrm, Gd); break;
        case 16: hipLaunchKernelGGL((k_contract_f64<KR, 16>), grid, dim3(256), 0, st, params, m, n, r, s, M->Dt64, M->Qrm, Gd); break;
        case 32: hipLaunchKernelGGL((k_contract_f64<KR, 32>), grid, dim3(256), 0, st, params, m, n, r, s, M->Dt64, M->Qrm, Gd); break;
        case 40: hipLaunchKernelGGL((k_contract_f64<1, 40>), dim3(grid.x, (s + 3) / 4), dim3(256), 0, st, params, m, n, r, s, M->Dt64, M->Qrm, Gd); break;
        default: hipLaunchKernelGGL((k_contract_f64<1, 64>), dim3(grid.x, (s + 3) / 4), dim3(256), 0, st, params, m, n, r, s, M->Dt64, M->Qrm, Gd); break;
      }
    } else {
      ProfScope prof("krr_contract_fp64_small", st);
      dim3 grid(static_cast<unsigned>(m), static_cast<unsigned>(s));
      switch (RM) {
        case 8: hipLaunchKernelGGL((k_contract_f64_small<8>), grid, dim3(256), 0, st, params, n, r, s, M->Dt64, M->Qrm, Gd); break;
        case 16: hipLaunchKernelGGL((k_contract_f64_small<16>), grid, dim3(256), 0, st, params, n, r, s, M->Dt64, M->Qrm, Gd); break;
        case 32: hipLaunchKernelGGL((k_contract_f64_small<32>), grid, dim3(256), 0, st, params, n, r, s, M->Dt64, M->Qrm, Gd); break;
        case 40: hipLaunchKernelGGL((k_contract_f64_small<40>), grid, dim3(256), 0, st, params, n, r, s, M->Dt64, M->Qrm, Gd); break;
        default: hipLaunchKernelGGL((k_contract_f64_small<64>), grid, dim3(256), 0, st, params, n, r, s, M->Dt64, M->Qrm, Gd); break;
      }
    }
  } else {
    const bool f16 = prec == SUBAP_FP16X3;
    float* G32 = reinterpret_cast<float*>(static_cast<double*>(G) + static_cast<size_t>(m) * s * r);
    MArgs a{params, m, n, r, s, M->D32, f16 ? M->Qh16 : M->Qhi, f16 ? M->Ql16 : M->Qlo, M->Q32, G32};
    constexpr int PW = 8;
    const unsigned gy = static_cast<unsigned>((s + 127) / 128);
    const dim3 g8(xcd_grid((m + PW - 1) / PW), gy);
    const dim3 g4(xcd_grid((m + 3) / 4), gy);
    if (prec == SUBAP_BF16X3) {
      ProfScope prof("krr_contract_bf16x3", st);
      if (r <= 32) hipLaunchKernelGGL((k_contract_x3<__bf16, PW, 1>), g8, dim3(256), 0, st, a);
      else hipLaunchKernelGGL((k_contract_x3<__bf16, 4, 2>), g4, dim3(256), 0, st, a);
    } else if (prec == SUBAP_FP16X3) {
      ProfScope prof("krr_contract_fp16x3", st);
      if (r <= 32) hipLaunchKernelGGL((k_contract_x3<_Float16, PW, 1>), g8, dim3(256), 0, st, a);
      else hipLaunchKernelGGL((k_contract_x3<_Float16, 4, 2>), g4, dim3(256), 0, st, a);
    } else {
      ProfScope prof("krr_contract_fp32", st);
      if (r <= 32) hipLaunchKernelGGL((k_contract_f32<PW, 1>), g8, dim3(256), 0, st, a);
      else hipLaunchKernelGGL((k_contract_f32<4, 2>), g4, dim3(256), 0, st, a);
    }
    const int64_t len = m * s * r;
    ProfScope prof("reduce_partials", st);
    hipLaunchKernelGGL(k_reduce_partials, dim3(static_cast<unsigned>((len + 255) / 256)), dim3(256), 0, st, G32,
                       len, r, f16 ? M->colscale_inv : nullptr, static_cast<double*>(G));
  }
  SUBAP_HIP_TRY(hipGetLastError());
  // A3: least squares
  LArgs la{params, m, r, s, G, 1, nullptr, M->wS, M->QS, M->bS, M->lambda, M->bS_norm, y, rho, stat, fac, fac_stride};
  {
    ProfScope prof("lsq_householder", st);
    SUBAP_TRY(launch_lsq<double>(sh, la, st));
  }
  // A4: refinement
  for (int it = 0; it < refine; ++it) {
    // degree-7 kernel entries only in the first step from a reduced contraction,
    // whose own error is far larger; FP64-rounding entries otherwise
    const bool exact = it > 0 || prec == SUBAP_FP64;
    SUBAP_TRY(launch_refine_partial(M, params, m, y, part, exact, st));
    CArgs ca{m, r, s, part, M->wS, M->QS, M->bS, M->lambda, M->bS_norm, fac, fac_stride, y, rho, stat};
    if (cs) {
      {
        ProfScope prof("krr_resid_finish", st);
        hipLaunchKernelGGL(k_resid_finish, dim3(static_cast<unsigned>((m + 3) / 4)), dim3(256), 0, st, params, m,
                           r, s, part, M->wS, M->QS, M->bS, M->lambda, M->bS_norm, y, rvec, nullptr);
        SUBAP_HIP_TRY(hipGetLastError());
      }
      SUBAP_TRY(launch_adjoint(M, params, m, rvec, gpart, exact, st));
      ProfScope prof("lsq_csne_correct", st);
      SUBAP_TRY(launch_csne_correct(sh, ca, rvec, gpart, st));
    } else {
      ProfScope prof("lsq_correct", st);
      SUBAP_TRY(launch_correct(sh, ca, st));
    }
  }
  return SUBAP_OK;
}

subap_status krr_residual(subap_model_s* M, const double* params, int64_t m, const double* y, double* res,
                          double* norm, hipStream_t st) {
  const int s = M->s;
  SUBAP_TRY(ensure_work(M, static_cast<size_t>(kRefSplit) * m * s * 8));
  double* part = static_cast<double*>(M->work);
  SUBAP_TRY(launch_refine_partial(M, params, m, y, part, true, st));
  ProfScope prof("krr_resid_finish", st);
  hipLaunchKernelGGL(k_resid_finish, dim3(static_cast<unsigned>((m + 3) / 4)), dim3(256), 0, st, params, m,
                     M->r, s, part, M->wS, M->QS, M->bS, M->lambda, M->bS_norm, y, res, norm);
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

// (refinement partial-sum launcher, shared by the solve and the residual.
// exact selects the FP64-rounding polynomial (degree 11): the sketched
// residual and every refinement step after the first.  The first step uses
// degree 7 (relative error 5.5e-11 per entry): its result is limited by the
// contraction it corrects (errors near 1e-7), so the entries' share of its
// error stays four orders below that while the evaluation takes 12 VALU
// instructions instead of 16.)
template <int DEG>
static void launch_refine_deg(subap_model_s* M, const double* params, int64_t m, const double* y, double* part,
                              hipStream_t st) {
  const int r = M->r, s = M->s;
  const int64_t n = M->n;
  const dim3 grid(static_cast<unsigned>((m + kRefPB - 1) / kRefPB * kRefSplit));
  const dim3 block(static_cast<unsigned>(std::max(64, (s + 63) / 64 * 64)));
  const double dmax = M->dmax;
  switch (rm_of(r)) {
    case 8: hipLaunchKernelGGL((k_refine_partial<8, DEG>), grid, block, 0, st, params, m, n, r, s, dmax, M->Dt64, M->Qrm, y, part); break;
    case 16: hipLaunchKernelGGL((k_refine_partial<16, DEG>), grid, block, 0, st, params, m, n, r, s, dmax, M->Dt64, M->Qrm, y, part); break;
    case 32: hipLaunchKernelGGL((k_refine_partial<32, DEG>), grid, block, 0, st, params, m, n, r, s, dmax, M->Dt64, M->Qrm, y, part); break;
    case 40: hipLaunchKernelGGL((k_refine_partial<40, DEG>), grid, block, 0, st, params, m, n, r, s, dmax, M->Dt64, M->Qrm, y, part); break;
    default: hipLaunchKernelGGL((k_refine_partial<64, DEG>), grid, block, 0, st, params, m, n, r, s, dmax, M->Dt64, M->Qrm, y, part); break;
  }
}

subap_status launch_refine_partial(subap_model_s* M, const double* params, int64_t m, const double* y,
                                   double* part, bool exact, hipStream_t st) {
  {
    ProfScope prof(exact ? "krr_refine_partial_exact" : "krr_refine_partial", st);
    if (exact)
      launch_refine_deg<11>(M, params, m, y, part, st);
    else
      launch_refine_deg<7>(M, params, m, y, part, st);
  }
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

namespace {

// |G^T r_S| / den from the adjoint partials (one thread per parameter)
__global__ void k_excess_finish(const double* gpart, int64_t m, int r, double den, double* out) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= m) return;
  double gg = 0.0;
  for (int c = 0; c < r; ++c) {
    double g = 0.0;
    for (int sp = 0; sp < kRefSplit; ++sp) g += gpart[(static_cast<int64_t>(sp) * m + p) * r + c];
    gg = fma(g, g, gg);
  }
  out[p] = sqrt(gg) / den;
}

// G[(p s + k) r + c] <- w_k G + lambda Q_S[k, c]: the FP64 contraction of the
// kernel part plus the ridge, as the least-squares kernels form it
__global__ void k_krr_gfinish(double* G, int64_t m, int r, int s, const double* wS, const double* QS,
                              double lambda) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= m * s * r) return;
  const int k = static_cast<int>((e / r) % s), c = static_cast<int>(e % r);
  G[e] = fma(wS[k], G[e], lambda * QS[k * r + c]);
}

}  // namespace

// Normal-equation excess |G^T (G y - S b)| / (sigma_min |S b|) in FP64: the
// residual pass, the adjoint pass of the corrected semi-normal equations, and
// the norm.
subap_status krr_excess(subap_model_s* M, const double* params, int64_t m, const double* y, double sigma_min,
                        double* out, hipStream_t st) {
  const int r = M->r, s = M->s;
  const size_t np = static_cast<size_t>(kRefSplit) * m * s, nr = static_cast<size_t>(m) * s,
               na = static_cast<size_t>(kRefSplit) * m * r;
  SUBAP_TRY(ensure_work(M, 8 * (np + nr + na)));
  double* part = static_cast<double*>(M->work);
  double* rvec = part + np;
  double* gpart = rvec + nr;
  SUBAP_TRY(launch_refine_partial(M, params, m, y, part, true, st));
  {
    ProfScope prof("krr_resid_finish", st);
    hipLaunchKernelGGL(k_resid_finish, dim3(static_cast<unsigned>((m + 3) / 4)), dim3(256), 0, st, params, m, r, s,
                       part, M->wS, M->QS, M->bS, M->lambda, M->bS_norm, y, rvec, nullptr);
    SUBAP_HIP_TRY(hipGetLastError());
  }
  SUBAP_TRY(launch_adjoint(M, params, m, rvec, gpart, true, st));
  hipLaunchKernelGGL(k_excess_finish, dim3(static_cast<unsigned>((m + 255) / 256)), dim3(256), 0, st, gpart, m, r,
                     sigma_min * M->bS_norm, out);
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

// G = S A(p) Q in FP64 for m parameters (s x r row-major each)
subap_status krr_reduced_matrix(subap_model_s* M, const double* params, int64_t m, double* G, hipStream_t st) {
  const int r = M->r, s = M->s;
  const int64_t n = M->n;
  const int RM = rm_of(r);
  {
    ProfScope prof("krr_contract_fp64", st);
    constexpr int KR = 2;
    const dim3 grid(static_cast<unsigned>((m + 63) / 64), static_cast<unsigned>((s + 4 * KR - 1) / (4 * KR)));
    switch (RM) {
      case 8: hipLaunchKernelGGL((k_contract_f64<KR, 8>), grid, dim3(256), 0, st, params, m, n, r, s, M->Dt64, M->Qrm, G); break;
      case 16: hipLaunchKernelGGL((k_contract_f64<KR, 16>), grid, dim3(256), 0, st, params, m, n, r, s, M->Dt64, M->Qrm, G); break;
      case 32: hipLaunchKernelGGL((k_contract_f64<KR, 32>), grid, dim3(256), 0, st, params, m, n, r, s, M->Dt64, M->Qrm, G); break;
      case 40: hipLaunchKernelGGL((k_contract_f64<1, 40>), dim3(grid.x, (s + 3) / 4), dim3(256), 0, st, params, m, n, r, s, M->Dt64, M->Qrm, G); break;
      default: hipLaunchKernelGGL((k_contract_f64<1, 64>), dim3(grid.x, (s + 3) / 4), dim3(256), 0, st, params, m, n, r, s, M->Dt64, M->Qrm, G); break;
    }
  }
  const int64_t len = m * s * r;
  hipLaunchKernelGGL(k_krr_gfinish, dim3(static_cast<unsigned>((len + 255) / 256)), dim3(256), 0, st, G, m, r, s, M->wS,
                     M->QS, M->lambda);
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

// ---------------------------------------------------------------------------
// Transcendental-rate microbenchmark: 2^(c d) evaluations per second as the
// refinement issues them (16 independent evaluations per lane and point,
// accumulated), for the FP64 polynomial forms and for v_exp_f32.
namespace {

constexpr int kRateChains = 16;

template <int DEG>
__global__ __launch_bounds__(256) void k_exp2_rate(int64_t iters, double* out) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double c[kRateChains], acc[kRateChains];
#pragma unroll
  for (int w = 0; w < kRateChains; ++w) {
    c[w] = -0.05 - 0.01 * w;
    acc[w] = 0.0;
  }
  double d = 0.5 + 1e-6 * static_cast<double>(t & 1023);
  for (int64_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int w = 0; w < kRateChains; ++w) {
      if constexpr (DEG == 0)
        acc[w] += static_cast<double>(__builtin_amdgcn_exp2f(static_cast<float>(c[w] * d)));
      else
        acc[w] = fma(exp2_mul<DEG>(c[w], d), 0.5, acc[w]);
    }
    d += 0.001;
  }
  double sum = 0.0;
#pragma unroll
  for (int w = 0; w < kRateChains; ++w) sum += acc[w];
  out[t] = sum;
}

}  // namespace

subap_status exp2_rate(int form, int64_t evals, double* rate, hipStream_t st) {
  constexpr int kThreads = 256, kBlocks = 256 * 16;
  const int64_t lanes = static_cast<int64_t>(kThreads) * kBlocks;
  const int64_t iters = std::max<int64_t>(1, evals / (lanes * kRateChains));
  struct Buf {
    double* p = nullptr;
    ~Buf() { dfree(p); }
  } out;
  SUBAP_TRY(dalloc(&out.p, static_cast<size_t>(lanes)));
  hipEvent_t e0, e1;
  SUBAP_HIP_TRY(hipEventCreate(&e0));
  SUBAP_HIP_TRY(hipEventCreate(&e1));
  struct Ev {
    hipEvent_t a, b;
    ~Ev() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } ev{e0, e1};
  auto launch = [&](int64_t it) {
    switch (form) {
      case 0: hipLaunchKernelGGL(k_exp2_rate<0>, dim3(kBlocks), dim3(kThreads), 0, st, it, out.p); break;
      case 7: hipLaunchKernelGGL(k_exp2_rate<7>, dim3(kBlocks), dim3(kThreads), 0, st, it, out.p); break;
      case 9: hipLaunchKernelGGL(k_exp2_rate<9>, dim3(kBlocks), dim3(kThreads), 0, st, it, out.p); break;
      default: hipLaunchKernelGGL(k_exp2_rate<11>, dim3(kBlocks), dim3(kThreads), 0, st, it, out.p); break;
    }
  };
  launch(1);  // warm-up
  SUBAP_HIP_TRY(hipEventRecord(e0, st));
  launch(iters);
  SUBAP_HIP_TRY(hipEventRecord(e1, st));
  SUBAP_HIP_TRY(hipGetLastError());
  SUBAP_HIP_TRY(hipEventSynchronize(e1));
  float ms = 0.0f;
  SUBAP_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
  *rate = static_cast<double>(lanes) * kRateChains * static_cast<double>(iters) / (ms * 1e-3);
  return SUBAP_OK;
}

}  // namespace subap
