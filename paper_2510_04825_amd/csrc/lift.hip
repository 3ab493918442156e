// Lift x = Q y (Algorithm 3.1 step 4 outputs X c) for k coefficient vectors.
// Each thread owns one row j of Q, keeps Q[j, :] in registers, and streams
// x[j, i] for all i, so Q is read once and x is written once, coalesced.
#include <hip/hip_runtime.h>

#include "common.h"
#include "profile.h"

namespace subap {
namespace {

constexpr int kLiftChunk = 64;

template <int RM, typename OT>
__global__ __launch_bounds__(256) void k_lift(const double* Q, int64_t n, int r, const double* y, int64_t k,
                                               OT* x) {
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
        x[(i0 + ii) * n + j] = static_cast<OT>(acc);
      }
    }
  }
}

template <typename OT>
subap_status launch(const subap_model_s* M, const double* y, int64_t k, OT* x, hipStream_t st) {
  const unsigned grid = static_cast<unsigned>((M->n + 255) / 256);
  const int r = M->r;
  ProfScope prof("lift", st);
  if (r <= 8) hipLaunchKernelGGL((k_lift<8, OT>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, y, k, x);
  else if (r <= 16) hipLaunchKernelGGL((k_lift<16, OT>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, y, k, x);
  else if (r <= 32) hipLaunchKernelGGL((k_lift<32, OT>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, y, k, x);
  else if (r <= 40) hipLaunchKernelGGL((k_lift<40, OT>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, y, k, x);
  else hipLaunchKernelGGL((k_lift<64, OT>), dim3(grid), dim3(256), 0, st, M->Q, M->n, r, y, k, x);
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

}  // namespace

subap_status lift(subap_model_s* M, const double* y, int64_t k, void* x, int prec, hipStream_t st) {
  if (prec == SUBAP_FP64) return launch(M, y, k, static_cast<double*>(x), st);
  return launch(M, y, k, static_cast<float*>(x), st);
}

}  // namespace subap
