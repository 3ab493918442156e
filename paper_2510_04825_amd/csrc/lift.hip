// Lift x = Q y (Algorithm 3.1 step 4 outputs X c) for k coefficient vectors;
// x is column-major with leading dimension ld >= n (rows n..ld-1 untouched).
//
// FP64 output: each thread owns one row j of Q, keeps Q[j, :] in registers
// and streams x[j, i] for all i (FP64 FMAs).
//
// FP32 output: a split-bf16 MFMA product.  Q (rounded to FP32) and the y
// vectors (rounded to FP32) are each written exactly as hi + mid + lo bf16
// parts; the six products hi.hi, hi.mid, mid.hi, hi.lo, mid.mid, lo.hi are
// accumulated in FP32 by v_mfma_f32_32x32x16_bf16, so the dropped terms are
// below 2^-23 of |Q||y| and x carries FP32-level error.  The MFMA tile is
// x^T: M = 32 output vectors, N = 32 rows of Q, K = 16 of the r columns, so
// each store instruction writes two 128-byte runs of one column of x (whole
// cache lines when ld is a multiple of 32).  The y operands of the next group
// of 32 vectors are loaded before the stores of the current group are
// issued: loads and stores share one completion counter, so waiting for
// loads issued after the stores would also wait for the stores.  The kernel
// is bound by the HBM write of x (4 n k bytes).
#include <hip/hip_runtime.h>

#include "common.h"
#include "profile.h"

namespace subap {
namespace {

constexpr int kLiftChunk = 64;

template <int RM, typename OT>
__global__ __launch_bounds__(256) void k_lift(const double* Q, int64_t n, int r, const double* y, int64_t k,
                                               OT* x, int64_t ld) {
  __shared__ double s_y[kLiftChunk][RM];
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  double q[RM];
#pragma unroll
  for (int c = 0; c < RM; ++c) q[c] = (j < n && c < r) ? Q[static_cast<int64_t>(c) * n + j] : 0.0;
  for (int64_t i0 = 0; i0 < k; i0 += kLiftChunk) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < kLiftChunk * RM; idx += 256) {
      const int ii = idx / RM, c = idx % RM;
      s_y[ii][c] = (i0 + ii < k && c < r) ? y[(i0 + ii) * r + c] : 0.0;
    }
    __syncthreads();
    if (j < n) {
      const int cnt = static_cast<int>(k - i0 < kLiftChunk ? k - i0 : kLiftChunk);
      for (int ii = 0; ii < cnt; ++ii) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < RM; ++c) acc = fma(q[c], s_y[ii][c], acc);
        x[(i0 + ii) * ld + j] = static_cast<OT>(acc);
      }
    }
  }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// v = hi + mid + lo exactly (each part the nearest bf16 of what remains;
// FP32 has 24 significant bits and each bf16 part takes 8 of them).
__device__ __forceinline__ void split3(float v, __bf16* hi, __bf16* mid, __bf16* lo) {
  const __bf16 h = static_cast<__bf16>(v);
  const float r1 = v - static_cast<float>(h);
  const __bf16 m = static_cast<__bf16>(r1);
  *hi = h;
  *mid = m;
  *lo = static_cast<__bf16>(r1 - static_cast<float>(m));
}

// y (k x r, FP64 row-major) -> A operands: Ys[((ic * NKB + kb) * 3 + part) * 64 + lane]
// holds part of y[32 ic + lane % 32][16 kb + 8 (lane / 32) + e], e = 0..7
// (zero past k or r).
__global__ __launch_bounds__(64) void k_lift_split_y(const double* y, int64_t k, int r, int nkb, bf16x8* Ys) {
  const int lane = threadIdx.x;
  const int64_t ic = blockIdx.x / nkb;
  const int kb = blockIdx.x % nkb;
  const int64_t i = ic * 32 + lane % 32;
  bf16x8 h, m, l;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int c = kb * 16 + 8 * (lane / 32) + e;
    const float v = (i < k && c < r) ? static_cast<float>(y[i * r + c]) : 0.0f;
    __bf16 a, b, d;
    split3(v, &a, &b, &d);
    h[e] = a;
    m[e] = b;
    l[e] = d;
  }
  bf16x8* out = Ys + (static_cast<int64_t>(blockIdx.x) * 3) * 64 + lane;
  out[0] = h;
  out[64] = m;
  out[128] = l;
}

__device__ __forceinline__ f32x16 mfma(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// 32-row tiles of Q per wave: four tiles (1 wave per SIMD) write 512-byte runs
// of each column per wave and beat two tiles (2 waves per SIMD) by about 9%
constexpr int kLiftTiles = 4;
constexpr int kLiftRowsPerBlock = 4 * kLiftTiles * 32;

template <int NKB>
__device__ __forceinline__ void load_y_ops(const bf16x8* Ys, int64_t ic, int lane, bf16x8 (&ya)[NKB][3]) {
  const bf16x8* src = Ys + (ic * NKB * 3) * 64 + lane;
#pragma unroll
  for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
    for (int part = 0; part < 3; ++part) ya[kb][part] = src[(kb * 3 + part) * 64];
}

// Block: 4 waves x kLiftTiles tiles of 32 consecutive rows; every output vector.
template <int NKB>
__global__ __launch_bounds__(256) void k_lift_x6(const double* Q, int64_t n, int r, const bf16x8* Ys, int64_t k,
                                                  float* x, int64_t ld) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t jw = static_cast<int64_t>(blockIdx.x) * kLiftRowsPerBlock + wave * kLiftTiles * 32;
  // B operands: split rows of Q, kept for the whole sweep over the vectors
  bf16x8 qb[kLiftTiles][NKB][3];
#pragma unroll
  for (int t = 0; t < kLiftTiles; ++t) {
    const int64_t j = jw + t * 32 + lane % 32;
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb) {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int c = kb * 16 + 8 * (lane / 32) + e;
        const float v = (j < n && c < r) ? static_cast<float>(Q[static_cast<int64_t>(c) * n + j]) : 0.0f;
        __bf16 a, b, d;
        split3(v, &a, &b, &d);
        qb[t][kb][0][e] = a;
        qb[t][kb][1][e] = b;
        qb[t][kb][2][e] = d;
      }
    }
  }
  const int64_t nic = (k + 31) / 32;
  bf16x8 ya[NKB][3], yn[NKB][3];
  load_y_ops<NKB>(Ys, 0, lane, yn);
  for (int64_t ic = 0; ic < nic; ++ic) {
#pragma unroll
    for (int kb = 0; kb < NKB; ++kb)
#pragma unroll
      for (int part = 0; part < 3; ++part) ya[kb][part] = yn[kb][part];
    if (ic + 1 < nic) load_y_ops<NKB>(Ys, ic + 1, lane, yn);  // before this group's stores
    f32x16 acc[kLiftTiles];
#pragma unroll
    for (int t = 0; t < kLiftTiles; ++t) {
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[t][v] = 0.0f;
      // smallest terms first
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        acc[t] = mfma(ya[kb][2], qb[t][kb][0], acc[t]);
        acc[t] = mfma(ya[kb][1], qb[t][kb][1], acc[t]);
        acc[t] = mfma(ya[kb][0], qb[t][kb][2], acc[t]);
      }
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) {
        acc[t] = mfma(ya[kb][1], qb[t][kb][0], acc[t]);
        acc[t] = mfma(ya[kb][0], qb[t][kb][1], acc[t]);
      }
#pragma unroll
      for (int kb = 0; kb < NKB; ++kb) acc[t] = mfma(ya[kb][0], qb[t][kb][0], acc[t]);
    }
#pragma unroll
    for (int t = 0; t < kLiftTiles; ++t) {
      const int64_t j = jw + t * 32 + lane % 32;
      if (j < n) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t i = ic * 32 + 8 * (v / 4) + 4 * (lane / 32) + (v % 4);
          if (i < k) x[i * ld + j] = acc[t][v];
        }
      }
    }
  }
}

template <typename OT>
subap_status launch_fma(const subap_model_s* M, const double* y, int64_t k, OT* x, int64_t ld, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>((M->n + 255) / 256);
  const int r = M->r;
  ProfScope prof("lift", st);
  if (r <= 8) hipLaunchKernelGGL((k_lift<8, OT>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, y, k, x, ld);
  else if (r <= 16) hipLaunchKernelGGL((k_lift<16, OT>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, y, k, x, ld);
  else if (r <= 32) hipLaunchKernelGGL((k_lift<32, OT>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, y, k, x, ld);
  else if (r <= 40) hipLaunchKernelGGL((k_lift<40, OT>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, y, k, x, ld);
  else hipLaunchKernelGGL((k_lift<64, OT>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, y, k, x, ld);
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

subap_status launch_x6(subap_model_s* M, const double* y, int64_t k, float* x, int64_t ld, hipStream_t st) {
  const int r = M->r;
  const int nkb = (r + 15) / 16;
  const int64_t nic = (k + 31) / 32;
  SUBAP_TRY(ensure_work(M, static_cast<size_t>(nic) * nkb * 3 * 64 * sizeof(bf16x8)));
  bf16x8* Ys = static_cast<bf16x8*>(M->work);
  const unsigned grid = static_cast<unsigned>((M->n + kLiftRowsPerBlock - 1) / kLiftRowsPerBlock);
  ProfScope prof("lift", st);
  hipLaunchKernelGGL(k_lift_split_y, dim3(static_cast<unsigned>(nic * nkb)), dim3(64), 0, st, y, k, r, nkb, Ys);
  switch (nkb) {
    case 1: hipLaunchKernelGGL((k_lift_x6<1>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, Ys, k, x, ld); break;
    case 2: hipLaunchKernelGGL((k_lift_x6<2>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, Ys, k, x, ld); break;
    case 3: hipLaunchKernelGGL((k_lift_x6<3>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, Ys, k, x, ld); break;
    default: hipLaunchKernelGGL((k_lift_x6<4>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, Ys, k, x, ld); break;
  }
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

}  // namespace

subap_status lift(subap_model_s* M, const double* y, int64_t k, void* x, int64_t ldx, int prec, hipStream_t st) {
  if (k == 0) return SUBAP_OK;
  if (prec == SUBAP_FP64) return launch_fma(M, y, k, static_cast<double*>(x), ldx, st);
  return launch_x6(M, y, k, static_cast<float*>(x), ldx, st);
}

}  // namespace subap
