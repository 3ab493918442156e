// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "subap.h"

namespace subap {

void set_error(const std::string& msg);
void clear_error();

#define SUBAP_HIP_TRY(expr)                                                        \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess) {                                                        \
      subap::set_error(std::string(#expr) + ": " + hipGetErrorString(e_));       \
      return SUBAP_E_HIP;                                                          \
    }                                                                              \
  } while (0)

#define SUBAP_TRY(expr)                 \
  do {                                  \
    subap_status s_ = (expr);           \
    if (s_ != SUBAP_OK) return s_;      \
  } while (0)

constexpr int kMaxR = 64;
constexpr int kMaxS = 256;
constexpr int kMaxAffineTerms = 4;  // terms of the affine family
constexpr int kRowPad = 8;  // zero rows after the s rows of bS and of the diffusion delta64T
constexpr double kRankTol = 1e-13;   // |R_jj| <= kRankTol |R_11| -> rank deficient
constexpr double kTieRtol = 1e-6;    // pivot tie window

// Device allocation with the library's error convention.
subap_status dmalloc(void** p, size_t bytes);
template <class T>
subap_status dalloc(T** p, size_t count) {
  return dmalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}
void dfree(void* p);

}  // namespace subap

// The opaque model.  All device pointers are owned by the model.
struct subap_model_s {
  int family = 0;
  int N = 0;          // FD: nodes per axis
  int dimx = 0;       // FD: spatial dimension (2/3); KRR: point dimension
  int64_t n = 0;
  int r = 0, s = 0, d = 0;
  int F = 0;          // FD: faces per row (2 * dimx)
  double h = 0.0, inv_h2 = 0.0;
  double lambda = 0.0;
  double tau = 0.0, kappa = 0.0;      // delay family
  double aff_c0 = 0.0;                // delay family: A_0 = aff_c0 A_1 (3)
  double bS_norm = 0.0;               // |S b|_2, or |b|_2 with weighted rows (b is p-independent in every family)
  double b_norm = 0.0;                // |b|_2
  int selection = 0;                  // subap_selection
  std::vector<double> weights;        // host copy of wS
  double dmax = 0.0;                  // KRR: upper bound on every squared distance D[k, j]
  std::vector<int64_t> rows;          // host copy, selection order

  // basis and selection (device)
  double* Q = nullptr;                // n x r col-major, orthonormal
  int* rows_d = nullptr;              // s
  double* wS = nullptr;               // s row weights (1 for pivoted-QR rows)
  double* bS = nullptr;               // s: w_k b[rows[k]]
  double* QS = nullptr;               // s x r row-major: w_k Q[rows[k], c]
  double* rhs = nullptr;              // n (device copy of b)
  double* cQ = nullptr;               // r: c^T Q (models built with an output vector)
  double* rowdat = nullptr;           // s: per-row data of a p-dependent b (eq. (5.7): b0[i_k];
                                      //    identity family: t at i_k)

  // finite-difference tables, layouts [(f * r + c) * s + k] and [(f * d + q) * s + k]
  double* phi = nullptr;              // s x F x d  mode values at face midpoints
  double* delta64 = nullptr;          // s x F x r  w_k (Q[i_k] - Q[nb_f(i_k)]) (0 outside)
  float* delta32 = nullptr;
  double* delta64T = nullptr;         // the same at [(f * s + k) * r + c] (lanes = columns)
  float* delta32T = nullptr;

  // affine family: the nterms (= F) terms, CSR, concatenated; term q's row i
  // holds entries [aff_rp[q (n + 1) + i], aff_rp[q (n + 1) + i + 1])
  int64_t* aff_rp = nullptr;
  int* aff_ci = nullptr;
  double* aff_v = nullptr;

  // kernel ridge regression tables
  double* points = nullptr;           // n x dimx row-major
  double* Dt64 = nullptr;             // n x s: |t_j - t_{i_k}|^2 at [j * s + k]
  float* D32 = nullptr;               // s x n: same, FP32, at [k * n + j]
  double* Qrm = nullptr;              // n x r row-major FP64 copy of Q
  float* Q32 = nullptr;               // n x r col-major FP32
  uint16_t* Qhi = nullptr;            // n x r col-major bf16 (round to nearest even)
  uint16_t* Qlo = nullptr;            // bf16(Q32 - hi)
  uint16_t* Qh16 = nullptr;           // n x r col-major fp16 of Q[:, c] * 2^e_c
  uint16_t* Ql16 = nullptr;           // fp16 of the remainder
  double* colscale_inv = nullptr;     // r: 2^-e_c

  // online workspaces (grown on demand)
  void* work = nullptr;
  size_t work_bytes = 0;
};

namespace subap {

// families whose right-hand side b depends on p
inline bool rhs_varies(int family) {
  return family == SUBAP_FAMILY_TRIDIAG_SHIFT || family == SUBAP_FAMILY_IDENTITY;
}

// ---- offline (offline.hip) ----
subap_status offline_build(const subap_problem_desc* pd, const subap_offline_opts* o,
                           hipStream_t st, subap_model_s* M);
subap_status build_tables(subap_model_s* M, hipStream_t st);
subap_status residual_bounds(const double* rho, int64_t m, double eps, double* lo, double* hi, hipStream_t st);
subap_status output_apply(const subap_model_s* M, const double* y, int64_t m, double* out, hipStream_t st);
subap_status restore_model(subap_model_s* M, const double* Q, const int64_t* rows, const double* weights,
                           const double* rhs, const double* points, const double* cQ, hipStream_t st);
subap_status full_residual(subap_model_s* M, const double* params, int64_t m, const double* x, double* res,
                           hipStream_t st);
subap_status delta_residual(subap_model_s* M, const double* params, int64_t m, const double* y1, const double* y2,
                            double* res, hipStream_t st);
subap_status apsnap_solve(subap_model_s* M, const double* params, int64_t m, double* y, double* rho,
                          hipStream_t st);
subap_status polish(subap_model_s* M, const double* params, int64_t m, double* x, int max_iter, double tol,
                    double* res, hipStream_t st);

// ---- online ----
// refine: FP64 refinement steps; csne: each step solves the corrected
// semi-normal equations R^T R dy = G^T r_S with an FP64 G^T r_S instead of
// applying the stored factorisation of the rounded G.
subap_status fd_solve(subap_model_s* M, const double* params, int64_t m, double* y,
                      double* rho, int32_t* status, int prec, int refine, bool csne, hipStream_t st);
// true when fd_solve takes the matrix-core semi-normal solve for this model
// and form (a diffusion model, FP64 without refinement, s >= 96, 16 <= r <= 47)
bool fd_solve_on_matrix_cores(const subap_model_s* M, int prec, int refine);
subap_status exp2_rate(int form, int64_t evals, double* rate, hipStream_t st);
subap_status krr_solve(subap_model_s* M, const double* params, int64_t m, double* y,
                       double* rho, int32_t* status, int prec, int refine, bool csne, hipStream_t st);
// krr_solve with a caller-given device workspace of at least the bytes the
// call needs (no allocation); krr_chunk: the largest batch, a multiple of
// the refinement's parameter block, whose workspace fits in `bytes`.
subap_status krr_solve_ws(subap_model_s* M, const double* params, int64_t m, double* y, double* rho,
                          int32_t* status, int prec, int refine, bool csne, void* work, hipStream_t st);
int64_t krr_chunk(const subap_model_s* M, int prec, int refine, bool csne, size_t bytes);
// workspace bytes of krr_solve_ws for m parameters (0: no least-squares kernel for (s, r))
size_t krr_work_bytes(const subap_model_s* M, int64_t m, int prec, int refine, bool csne);
subap_status lift(subap_model_s* M, const double* y, int64_t k, void* x, int64_t ldx, int prec,
                  hipStream_t st);
subap_status fd_residual(subap_model_s* M, const double* params, int64_t m, const double* y, double* res,
                         double* norm, hipStream_t st);
subap_status krr_residual(subap_model_s* M, const double* params, int64_t m, const double* y, double* res,
                          double* norm, hipStream_t st);
// normal-equation excess |G^T (G y - S b)| / (sigma_min |S b|) and the FP64
// reduced matrix G = S A(p) Q (s x r row-major per parameter)
subap_status fd_excess(subap_model_s* M, const double* params, int64_t m, const double* y, double sigma_min,
                       double* out, hipStream_t st);
subap_status krr_excess(subap_model_s* M, const double* params, int64_t m, const double* y, double sigma_min,
                        double* out, hipStream_t st);
subap_status fd_reduced_matrix(subap_model_s* M, const double* params, int64_t m, double* G, hipStream_t st);
subap_status krr_reduced_matrix(subap_model_s* M, const double* params, int64_t m, double* G, hipStream_t st);

subap_status ensure_work(subap_model_s* M, size_t bytes);

// ---- batched plans (fd_multi.hip) ----
struct PlanImpl;
subap_status plan_build(subap_model_s* const* models, int k, const double* const* params, const int64_t* m,
                        double* const* y, double* const* rho, int32_t* const* status, int prec, int refine,
                        bool csne, int flags, hipStream_t st, PlanImpl** out);
subap_status plan_execute(PlanImpl* P, hipStream_t st);
void plan_free(PlanImpl* P);
void plan_shape(const PlanImpl* P, int* threads, int* blocks);
// ---- learned surrogate (mlp.hip) ----
struct Surrogate;
subap_status surrogate_create(int d, int r, int H, const double* weights, Surrogate** out);
void surrogate_free(Surrogate* S);
long surrogate_nparams(const Surrogate* S);
void surrogate_shape(const Surrogate* S, int* d, int* r);
subap_status surrogate_weights(Surrogate* S, double* host);
subap_status surrogate_gradient(Surrogate* S, const double* P, const double* T, int64_t m, double* grad_host,
                                double* loss, hipStream_t st);
subap_status surrogate_train(Surrogate* S, const double* P, const double* Y, int64_t m, int epochs, int batch,
                             double lr, double lr_min, uint64_t seed, double* loss_out, hipStream_t st);
subap_status surrogate_predict(Surrogate* S, const double* P, int64_t m, double* y, hipStream_t st);
subap_status surrogate_solve(subap_model_s* M, Surrogate* S, const double* P, int64_t m, double tol, double* y,
                             uint8_t* accepted, int32_t* status, int prec, int refine, bool csne,
                             int64_t* n_acc, hipStream_t st, double sigma_min = 0.0);

}  // namespace subap

struct subap_surrogate_s {
  subap::Surrogate* impl;
};

struct subap_plan_s {
  subap::PlanImpl* impl;
};
