// Learned surrogate p -> y: a multilayer perceptron d -> H -> H -> r with
// GELU activations, trained on (p, y) pairs produced by the SubApSnap solve,
// with hand-written forward, backward and Adam kernels.  Matrix products run
// on BF16 MFMA with FP32 accumulation (the output layer splits both operands
// into bf16 hi + lo for three products so the prediction is not limited to
// bf16 precision); master weights and Adam moments are FP32.
//
// Layout: weights in one FP32 buffer [W1 (H x d) | b1 | W2 (H x H) | b2 |
// W3 (r x H) | b3], W row-major (fan_out x fan_in); activations batch-major.
// Targets are standardised per component with the training mean and
// standard deviation, and predictions are mapped back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "profile.h"

namespace subap {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));

enum Epi { EPI_NONE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3 };

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

struct GemmArgs {
  int M, N, K;
  const float* A;
  long a_i, a_k;   // A(i, k) = A[i a_i + k a_k]
  const float* B;
  long b_k, b_j;   // B(k, j) = B[k b_k + j b_j]
  float* C;        // C[i ldc + j]
  long ldc;
  const float* bias;   // N (EPI_BIAS, EPI_BIAS_GELU)
  float* Z;            // pre-activation out (EPI_BIAS_GELU) / in (EPI_GELU_GRAD), ld = ldc
  int epi;
};

// C = op(A) op(B) on a 64 x 64 tile per block, 32 x 32 per wave, MFMA
// 32x32x16 bf16.  SPLIT: both operands as bf16 hi + lo, three products.
template <bool SPLIT>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
  const int wave = threadIdx.x / 64, l = threadIdx.x % 64;
  const int i0 = blockIdx.y * 64 + (wave / 2) * 32;
  const int j0 = blockIdx.x * 64 + (wave % 2) * 32;
  const int ia = i0 + (l & 31);   // A row of this lane
  const int jb = j0 + (l & 31);   // B column of this lane
  const int ko = 8 * (l >> 5);
  f32x16_t acc;
  for (int t = 0; t < 16; ++t) acc[t] = 0.0f;
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    bf16x8_t ah, al, bh, bl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + ko + e;
      const float av = (ia < g.M && k < g.K) ? g.A[ia * g.a_i + k * g.a_k] : 0.0f;
      const float bv = (jb < g.N && k < g.K) ? g.B[k * g.b_k + jb * g.b_j] : 0.0f;
      const __bf16 ahe = static_cast<__bf16>(av), bhe = static_cast<__bf16>(bv);
      ah[e] = ahe;
      bh[e] = bhe;
      if (SPLIT) {
        al[e] = static_cast<__bf16>(av - static_cast<float>(ahe));
        bl[e] = static_cast<__bf16>(bv - static_cast<float>(bhe));
      }
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
    if (SPLIT) {
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    const int i = i0 + 8 * (t / 4) + 4 * (l >> 5) + (t & 3);
    const int j = j0 + (l & 31);
    if (i >= g.M || j >= g.N) continue;
    float v = acc[t];
    const long o = i * g.ldc + j;
    switch (g.epi) {
      case EPI_BIAS: v += g.bias[j]; break;
      case EPI_BIAS_GELU:
        v += g.bias[j];
        g.Z[o] = v;
        v = gelu_f(v);
        break;
      case EPI_GELU_GRAD: v *= gelu_grad_f(g.Z[o]); break;
      default: break;
    }
    g.C[o] = v;
  }
}

subap_status gemm(const GemmArgs& a, bool split, hipStream_t st) {
  dim3 grid((a.N + 63) / 64, (a.M + 63) / 64);
  if (split) hipLaunchKernelGGL(k_gemm<true>, grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL(k_gemm<false>, grid, dim3(256), 0, st, a);
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

// out[j] = sum_i X[i ld + j], i < M (column sums for bias gradients)
__global__ void k_colsum(const float* X, int M, int N, long ld, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  double t = 0.0;
  for (int i = 0; i < M; ++i) t += X[i * ld + j];
  out[j] = static_cast<float>(t);
}

// batch gather: Pb[b] = float(P[idx_b]), Tb[b] = standardised y[idx_b];
// idx_b = (stride * (start + b) + offset) mod m, an affine permutation
__global__ void k_gather(const double* P, const double* Y, int64_t m, int d, int r, int64_t start, int Bt,
                         int64_t stride, int64_t offset, const double* mu, const double* sd, float* Pb,
                         float* Tb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= Bt) return;
  // stride < m and start + b < m with m < 2^31, so the product fits in 64 bits
  const int64_t idx = static_cast<int64_t>(
      (static_cast<uint64_t>(stride) * static_cast<uint64_t>(start + b) + static_cast<uint64_t>(offset)) %
      static_cast<uint64_t>(m));
  for (int q = 0; q < d; ++q) Pb[b * d + q] = static_cast<float>(P[idx * d + q]);
  if (Y)
    for (int c = 0; c < r; ++c) Tb[b * r + c] = static_cast<float>((Y[idx * r + c] - mu[c]) / sd[c]);
}

// dOut = 2 (out - T) / (Bt r); per-block partial of sum (out - T)^2
__global__ void k_mse(const float* out, const float* T, int n, float scale, float* dout, double* part) {
  __shared__ double sh[256];
  double t = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const float e = out[i] - T[i];
    dout[i] = scale * e;
    t += static_cast<double>(e) * e;
  }
  sh[threadIdx.x] = t;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_adam(float* w, const float* g, float* m1, float* m2, long n, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
  const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.0f - b1) * gi;
  const float v = b2 * m2[i] + (1.0f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = v;
  w[i] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
}

// per-component mean and standard deviation of Y (m x r), FP64
__global__ void k_moments(const double* Y, int64_t m, int r, double* mu, double* sd) {
  __shared__ double s1[256], s2[256];
  const int c = blockIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const double v = Y[i * r + c];
    a += v;
  }
  s1[threadIdx.x] = a;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) s1[threadIdx.x] += s1[threadIdx.x + s];
    __syncthreads();
  }
  const double mean = s1[0] / static_cast<double>(m);
  for (int64_t i = threadIdx.x; i < m; i += 256) {
    const double v = Y[i * r + c] - mean;
    b += v * v;
  }
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) s2[threadIdx.x] += s2[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mu[c] = mean;
    const double v = sqrt(s2[0] / static_cast<double>(m));
    sd[c] = v > 0.0 ? v : 1.0;
  }
}

__global__ void k_destandardise(const float* out, int64_t rows, int r, const double* mu, const double* sd,
                                double* y) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= rows * r) return;
  const int c = static_cast<int>(i % r);
  y[i] = static_cast<double>(out[i]) * sd[c] + mu[c];
}

// ---------------------------------------------------------------------------
struct Surrogate {
  int d = 0, r = 0, H = 0;
  long nw = 0;
  float* w = nullptr;      // master weights
  float* m1 = nullptr;     // Adam moments
  float* m2 = nullptr;
  float* g = nullptr;      // gradient
  double* mu = nullptr;    // target standardisation
  double* sd = nullptr;
  long step = 0;
  // activation workspace for a batch of up to cap rows
  int cap = 0;
  float* act = nullptr;
  double* part = nullptr;

  long oW1() const { return 0; }
  long ob1() const { return static_cast<long>(H) * d; }
  long oW2() const { return ob1() + H; }
  long ob2() const { return oW2() + static_cast<long>(H) * H; }
  long oW3() const { return ob2() + H; }
  long ob3() const { return oW3() + static_cast<long>(r) * H; }
};

namespace {

constexpr int kPartBlocks = 256;

struct Act {
  float *Pb, *Tb, *Z1, *H1, *Z2, *H2, *Out, *dOut, *dZ2, *dZ1;
};

Act carve(Surrogate* S, int Bt) {
  Act a;
  float* p = S->act;
  const long H = S->H;
  a.Pb = p; p += static_cast<long>(Bt) * S->d;
  a.Tb = p; p += static_cast<long>(Bt) * S->r;
  a.Z1 = p; p += Bt * H;
  a.H1 = p; p += Bt * H;
  a.Z2 = p; p += Bt * H;
  a.H2 = p; p += Bt * H;
  a.Out = p; p += static_cast<long>(Bt) * S->r;
  a.dOut = p; p += static_cast<long>(Bt) * S->r;
  a.dZ2 = p; p += Bt * H;
  a.dZ1 = p;
  return a;
}

subap_status ensure_act(Surrogate* S, int Bt) {
  if (S->cap >= Bt) return SUBAP_OK;
  dfree(S->act);
  S->act = nullptr;
  S->cap = 0;
  const long per = 2L * S->d + 3L * S->r + 6L * S->H;
  SUBAP_TRY(dalloc(&S->act, per * Bt + 64));
  S->cap = Bt;
  return SUBAP_OK;
}

// forward on Pb (Bt rows) into Out; keeps Z1, H1, Z2, H2
subap_status forward(Surrogate* S, const Act& a, int Bt, hipStream_t st) {
  const int d = S->d, H = S->H, r = S->r;
  const float* w = S->w;
  SUBAP_TRY(gemm({Bt, H, d, a.Pb, d, 1, w + S->oW1(), 1, d, a.H1, H, w + S->ob1(), a.Z1, EPI_BIAS_GELU}, false, st));
  SUBAP_TRY(gemm({Bt, H, H, a.H1, H, 1, w + S->oW2(), 1, H, a.H2, H, w + S->ob2(), a.Z2, EPI_BIAS_GELU}, false, st));
  SUBAP_TRY(gemm({Bt, r, H, a.H2, H, 1, w + S->oW3(), 1, H, a.Out, r, w + S->ob3(), nullptr, EPI_BIAS}, true, st));
  return SUBAP_OK;
}

// loss partials in S->part[0..kPartBlocks), gradient into S->g
subap_status backward(Surrogate* S, const Act& a, int Bt, hipStream_t st) {
  const int d = S->d, H = S->H, r = S->r;
  const float* w = S->w;
  float* g = S->g;
  const int n = Bt * r;
  hipLaunchKernelGGL(k_mse, dim3(kPartBlocks), dim3(256), 0, st, a.Out, a.Tb, n, 2.0f / n, a.dOut, S->part);
  // output layer
  SUBAP_TRY(gemm({r, H, Bt, a.dOut, 1, r, a.H2, H, 1, g + S->oW3(), H, nullptr, nullptr, EPI_NONE}, false, st));
  hipLaunchKernelGGL(k_colsum, dim3((r + 63) / 64), dim3(64), 0, st, a.dOut, Bt, r, static_cast<long>(r), g + S->ob3());
  SUBAP_TRY(gemm({Bt, H, r, a.dOut, r, 1, w + S->oW3(), H, 1, a.dZ2, H, nullptr, a.Z2, EPI_GELU_GRAD}, false, st));
  // hidden layer 2
  SUBAP_TRY(gemm({H, H, Bt, a.dZ2, 1, H, a.H1, H, 1, g + S->oW2(), H, nullptr, nullptr, EPI_NONE}, false, st));
  hipLaunchKernelGGL(k_colsum, dim3((H + 63) / 64), dim3(64), 0, st, a.dZ2, Bt, H, static_cast<long>(H), g + S->ob2());
  SUBAP_TRY(gemm({Bt, H, H, a.dZ2, H, 1, w + S->oW2(), H, 1, a.dZ1, H, nullptr, a.Z1, EPI_GELU_GRAD}, false, st));
  // hidden layer 1
  SUBAP_TRY(gemm({H, d, Bt, a.dZ1, 1, H, a.Pb, d, 1, g + S->oW1(), d, nullptr, nullptr, EPI_NONE}, false, st));
  hipLaunchKernelGGL(k_colsum, dim3((H + 63) / 64), dim3(64), 0, st, a.dZ1, Bt, H, static_cast<long>(H), g + S->ob1());
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

double read_loss(Surrogate* S, int n, hipStream_t st) {
  std::vector<double> h(kPartBlocks);
  (void)hipMemcpyAsync(h.data(), S->part, sizeof(double) * kPartBlocks, hipMemcpyDeviceToHost, st);
  (void)hipStreamSynchronize(st);
  double t = 0.0;
  for (double v : h) t += v;
  return t / n;
}

int64_t gcd64(int64_t a, int64_t b) {
  while (b) {
    const int64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

}  // namespace

subap_status surrogate_create(int d, int r, int H, const double* wh, Surrogate** out) {
  Surrogate* S = new (std::nothrow) Surrogate();
  if (!S) return SUBAP_E_NOMEM;
  S->d = d;
  S->r = r;
  S->H = H;
  S->nw = static_cast<long>(H) * d + H + static_cast<long>(H) * H + H + static_cast<long>(r) * H + r;
  auto fail = [&](subap_status rc) {
    surrogate_free(S);
    return rc;
  };
  subap_status rc;
  if ((rc = dalloc(&S->w, S->nw)) != SUBAP_OK) return fail(rc);
  if ((rc = dalloc(&S->m1, S->nw)) != SUBAP_OK) return fail(rc);
  if ((rc = dalloc(&S->m2, S->nw)) != SUBAP_OK) return fail(rc);
  if ((rc = dalloc(&S->g, S->nw)) != SUBAP_OK) return fail(rc);
  if ((rc = dalloc(&S->mu, r)) != SUBAP_OK) return fail(rc);
  if ((rc = dalloc(&S->sd, r)) != SUBAP_OK) return fail(rc);
  if ((rc = dalloc(&S->part, kPartBlocks)) != SUBAP_OK) return fail(rc);
  std::vector<float> hw(S->nw);
  for (long i = 0; i < S->nw; ++i) hw[i] = static_cast<float>(wh[i]);
  std::vector<float> zeros(S->nw, 0.0f);
  std::vector<double> mu0(r, 0.0), sd0(r, 1.0);
  if (hipMemcpy(S->w, hw.data(), sizeof(float) * S->nw, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(S->m1, zeros.data(), sizeof(float) * S->nw, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(S->m2, zeros.data(), sizeof(float) * S->nw, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(S->mu, mu0.data(), sizeof(double) * r, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(S->sd, sd0.data(), sizeof(double) * r, hipMemcpyHostToDevice) != hipSuccess) {
    set_error("uploading surrogate weights failed");
    return fail(SUBAP_E_HIP);
  }
  *out = S;
  return SUBAP_OK;
}

void surrogate_free(Surrogate* S) {
  if (!S) return;
  for (void* p : {static_cast<void*>(S->w), static_cast<void*>(S->m1), static_cast<void*>(S->m2),
                  static_cast<void*>(S->g), static_cast<void*>(S->mu), static_cast<void*>(S->sd),
                  static_cast<void*>(S->act), static_cast<void*>(S->part)})
    dfree(p);
  delete S;
}

long surrogate_nparams(const Surrogate* S) { return S->nw; }

void surrogate_shape(const Surrogate* S, int* d, int* r) {
  *d = S->d;
  *r = S->r;
}

subap_status surrogate_weights(Surrogate* S, double* host) {
  std::vector<float> hw(S->nw);
  SUBAP_HIP_TRY(hipDeviceSynchronize());
  SUBAP_HIP_TRY(hipMemcpy(hw.data(), S->w, sizeof(float) * S->nw, hipMemcpyDeviceToHost));
  for (long i = 0; i < S->nw; ++i) host[i] = hw[i];
  return SUBAP_OK;
}

subap_status surrogate_gradient(Surrogate* S, const double* P, const double* T, int64_t m, double* grad_host,
                                double* loss, hipStream_t st) {
  const int Bt = static_cast<int>(m);
  SUBAP_TRY(ensure_act(S, Bt));
  Act a = carve(S, Bt);
  // targets are given standardised: gather with mu = 0, sd = 1
  double* unit = nullptr;
  SUBAP_TRY(dalloc(&unit, 2 * S->r));
  std::vector<double> hu(2 * S->r);
  for (int c = 0; c < S->r; ++c) {
    hu[c] = 0.0;
    hu[S->r + c] = 1.0;
  }
  (void)hipMemcpy(unit, hu.data(), sizeof(double) * 2 * S->r, hipMemcpyHostToDevice);
  hipLaunchKernelGGL(k_gather, dim3((Bt + 255) / 256), dim3(256), 0, st, P, T, m, S->d, S->r, int64_t(0), Bt,
                     int64_t(1), int64_t(0), unit, unit + S->r, a.Pb, a.Tb);
  subap_status rc = forward(S, a, Bt, st);
  if (rc == SUBAP_OK) rc = backward(S, a, Bt, st);
  if (rc == SUBAP_OK) {
    *loss = read_loss(S, Bt * S->r, st);
    std::vector<float> hg(S->nw);
    if (hipMemcpy(hg.data(), S->g, sizeof(float) * S->nw, hipMemcpyDeviceToHost) != hipSuccess) rc = SUBAP_E_HIP;
    for (long i = 0; i < S->nw; ++i) grad_host[i] = hg[i];
  }
  dfree(unit);
  return rc;
}

subap_status surrogate_train(Surrogate* S, const double* P, const double* Y, int64_t m, int epochs, int batch,
                             double lr, double lr_min, uint64_t seed, double* loss_out, hipStream_t st) {
  const int Bt = static_cast<int>(std::min<int64_t>(batch, m));
  SUBAP_TRY(ensure_act(S, Bt));
  Act a = carve(S, Bt);
  hipLaunchKernelGGL(k_moments, dim3(S->r), dim3(256), 0, st, Y, m, S->r, S->mu, S->sd);
  const int64_t steps_per_epoch = m / Bt;  // whole batches; the stride permutation moves every epoch
  const int64_t total = steps_per_epoch * epochs;
  int64_t step = 0;
  for (int e = 0; e < epochs; ++e) {
    // epoch permutation i -> (stride i + offset) mod m, stride coprime to m
    int64_t stride = static_cast<int64_t>((seed * 0x9E3779B97F4A7C15ull + 2654435761ull * (e + 1)) % m) | 1;
    while (gcd64(stride, m) != 1) stride += 2;
    stride %= m;
    if (stride == 0) stride = 1;
    const int64_t offset = static_cast<int64_t>((seed + 0x632BE59BD9B4E019ull * (e + 7)) % m);
    double loss_sum = 0.0;
    for (int64_t b = 0; b < steps_per_epoch; ++b, ++step) {
      hipLaunchKernelGGL(k_gather, dim3((Bt + 255) / 256), dim3(256), 0, st, P, Y, m, S->d, S->r, b * Bt, Bt,
                         stride, offset, S->mu, S->sd, a.Pb, a.Tb);
      SUBAP_TRY(forward(S, a, Bt, st));
      SUBAP_TRY(backward(S, a, Bt, st));
      const double cosw =
          0.5 * (1.0 + std::cos(3.14159265358979323846 * static_cast<double>(step) / std::max<int64_t>(total, 1)));
      const double lr_t = lr_min + (lr - lr_min) * cosw;
      S->step += 1;
      const float c1 = static_cast<float>(1.0 - std::pow(0.9, static_cast<double>(S->step)));
      const float c2 = static_cast<float>(1.0 - std::pow(0.999, static_cast<double>(S->step)));
      hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((S->nw + 255) / 256)), dim3(256), 0, st, S->w, S->g,
                         S->m1, S->m2, S->nw, static_cast<float>(lr_t), 0.9f, 0.999f, c1, c2, 1e-8f);
      if (loss_out && b == steps_per_epoch - 1) loss_sum = read_loss(S, Bt * S->r, st);
    }
    SUBAP_HIP_TRY(hipGetLastError());
    if (loss_out) loss_out[e] = loss_sum;
  }
  SUBAP_HIP_TRY(hipStreamSynchronize(st));
  return SUBAP_OK;
}

subap_status surrogate_predict(Surrogate* S, const double* P, int64_t m, double* y, hipStream_t st) {
  const int chunk = 16384;
  SUBAP_TRY(ensure_act(S, chunk));
  Act a = carve(S, chunk);
  ProfScope prof("mlp_predict", st);
  for (int64_t c0 = 0; c0 < m; c0 += chunk) {
    const int Bt = static_cast<int>(std::min<int64_t>(chunk, m - c0));
    hipLaunchKernelGGL(k_gather, dim3((Bt + 255) / 256), dim3(256), 0, st, P + c0 * S->d, nullptr, Bt, S->d,
                       S->r, int64_t(0), Bt, int64_t(1), int64_t(0), S->mu, S->sd, a.Pb, a.Tb);
    SUBAP_TRY(forward(S, a, Bt, st));
    hipLaunchKernelGGL(k_destandardise, dim3(static_cast<unsigned>((static_cast<int64_t>(Bt) * S->r + 255) / 256)),
                       dim3(256), 0, st, a.Out, Bt, S->r, S->mu, S->sd, y + c0 * S->r);
  }
  SUBAP_HIP_TRY(hipGetLastError());
  return SUBAP_OK;
}

// acceptance of predicted coefficients and compaction of the rejected ones
__global__ void k_accept(const double* norm, int64_t m, double tol, uint8_t* accepted, int32_t* status,
                         int64_t* rej_idx, unsigned long long* rej_count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double v = norm[i];
  const bool ok = isfinite(v) && v <= tol;
  if (accepted) accepted[i] = ok ? 1 : 0;
  if (ok) {
    if (status) status[i] = SUBAP_OK;
  } else {
    const unsigned long long k = atomicAdd(rej_count, 1ull);
    rej_idx[k] = i;
  }
}

__global__ void k_gather_rows_by_index(const double* src, int w, const int64_t* idx, int64_t k, double* dst) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= k * w) return;
  const int64_t i = t / w, c = t % w;
  dst[t] = src[idx[i] * w + c];
}

__global__ void k_scatter_results(const double* ys, const int32_t* sts, int r, const int64_t* idx, int64_t k,
                                  double* y, int32_t* status) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= k * r) return;
  const int64_t i = t / r, c = t % r;
  y[idx[i] * r + c] = ys[t];
  if (c == 0 && status) status[idx[i]] = sts[i];
}

__global__ void k_zero_u64(unsigned long long* c) { *c = 0ull; }

subap_status surrogate_solve(subap_model_s* M, Surrogate* S, const double* P, int64_t m, double tol, double* y,
                             uint8_t* accepted, int32_t* status, int prec, int refine, bool csne,
                             int64_t* n_acc, hipStream_t st, double sigma_min) {
  // workspace: norms (m), rejected indices (m), count, compact params (m d), y (m r), status (m)
  const size_t bytes = 8 * static_cast<size_t>(m) * (2 + M->d + M->r + 1) + 64;
  char* buf = nullptr;
  SUBAP_TRY(dalloc(&buf, bytes));
  struct Free {
    char* p;
    ~Free() { dfree(p); }
  } fr{buf};
  double* norm = reinterpret_cast<double*>(buf);
  int64_t* rej = reinterpret_cast<int64_t*>(norm + m);
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(rej + m);
  double* Pc = reinterpret_cast<double*>(cnt + 8);
  double* Yc = Pc + m * M->d;
  int32_t* Sc = reinterpret_cast<int32_t*>(Yc + m * M->r);
  SUBAP_TRY(surrogate_predict(S, P, m, y, st));
  if (sigma_min > 0.0) {  // the normal-equation excess bound
    ProfScope prof("surrogate_excess", st);
    if (M->family == SUBAP_FAMILY_KRR) SUBAP_TRY(krr_excess(M, P, m, y, sigma_min, norm, st));
    else SUBAP_TRY(fd_excess(M, P, m, y, sigma_min, norm, st));
  } else {               // the sketched relative residual
    ProfScope prof("surrogate_residual", st);
    if (M->family == SUBAP_FAMILY_KRR) SUBAP_TRY(krr_residual(M, P, m, y, nullptr, norm, st));
    else SUBAP_TRY(fd_residual(M, P, m, y, nullptr, norm, st));
  }
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, cnt);
  hipLaunchKernelGGL(k_accept, dim3(static_cast<unsigned>((m + 255) / 256)), dim3(256), 0, st, norm, m, tol,
                     accepted, status, rej, cnt);
  unsigned long long h = 0;
  SUBAP_HIP_TRY(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, st));
  SUBAP_HIP_TRY(hipStreamSynchronize(st));
  const int64_t k = static_cast<int64_t>(h);
  *n_acc = m - k;
  if (k == 0) return SUBAP_OK;
  hipLaunchKernelGGL(k_gather_rows_by_index, dim3(static_cast<unsigned>((k * M->d + 255) / 256)), dim3(256), 0, st,
                     P, M->d, rej, k, Pc);
  if (M->family == SUBAP_FAMILY_KRR) SUBAP_TRY(krr_solve(M, Pc, k, Yc, nullptr, Sc, prec, refine, csne, st));
  else SUBAP_TRY(fd_solve(M, Pc, k, Yc, nullptr, Sc, prec, refine, csne, st));
  hipLaunchKernelGGL(k_scatter_results, dim3(static_cast<unsigned>((k * M->r + 255) / 256)), dim3(256), 0, st, Yc,
                     Sc, M->r, rej, k, y, status);
  SUBAP_HIP_TRY(hipGetLastError());
  SUBAP_HIP_TRY(hipStreamSynchronize(st));
  return SUBAP_OK;
}

}  // namespace subap
