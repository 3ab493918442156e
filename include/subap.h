/*
 * subap.h -- C ABI of the MI355X (gfx950) SubApSnap library.
 *
 * SubApSnap (Jones & Nakatsukasa, arXiv 2510.04825) solves the family of
 * linear systems A(p) x(p) = b(p), p in Omega (Section 1, eq. (1.1)), for
 * many parameters p* by (Algorithm 3.1):
 *   offline  1. snapshots X = [x(p_1) ... x(p_r)];
 *            2. orthonormalise X <- Q (Section 3.1, thin QR);
 *            3. choose s >= r rows S by pivoting on (A(p_sel) X)^T (Section 5.3);
 *   online   4. for each p*: form S A(p*) X (s x r, eq. (3.4)) from the s
 *               selected rows only, solve min_c |S A(p*) X c - S b(p*)|
 *               (eq. (3.3)) and output x = X c.
 *
 * The problem is never given as a matrix: the library generates the rows it
 * needs (Section 3.1, "Computing S A(p*) X") for one of these families:
 *   SUBAP_FAMILY_DIFF2D   -div(a grad u) = f on (0,1)^2, 5-point finite
 *                         differences, N x N interior nodes, Dirichlet 0,
 *                         a = exp(p1 sin 2 pi x + p2 cos 2 pi y), d = 2;
 *   SUBAP_FAMILY_DIFF3D   same on (0,1)^3, 7-point stencil, d = 4,
 *                         a = exp(p1 s_x c_y + p2 s_y c_z + p3 s_z c_x + p4 c_x c_y c_z)
 *                         with s_x = sin 2 pi x, c_x = cos 2 pi x, ...;
 *   SUBAP_FAMILY_KRR      kernel ridge regression (Section 6.3, eqs.
 *                         (6.3)-(6.4)): A(p) = K_p + lambda I,
 *                         K_p[i,j] = exp(-|t_i - t_j|^2 / (2 p^2)), d = 1;
 *   SUBAP_FAMILY_DELAY    the delay system of Section 6.2.2 with a real
 *                         parameter: A(p) = p I - A_0 - e^{tau p} A_1,
 *                         A_1 = (T - kappa I) / tau, A_0 = 3 A_1, T the n x n
 *                         matrix with ones on the first off-diagonals and at
 *                         T[0,0] and T[n-1,n-1], d = 1.  Symmetric positive
 *                         definite for p > -3 (kappa - 2) / tau.  The online
 *                         solve assembles S A(p) X = p S X - (3 + e^{tau p})
 *                         S A_1 X from the two precomputed s x r pieces
 *                         (Section 3.1, "Computing S A(p*) X").
 *   SUBAP_FAMILY_TRIDIAG_SHIFT  the example of eq. (5.7): A(p) = A_0 - p I with
 *                         A_0 = tridiag(-1, 2, -1) (n x n) and the
 *                         p-dependent right-hand side b_i(p) =
 *                         exp(b0_i sin(p / 10) p), b0 = problem->rhs; d = 1.
 *                         Online S A(p) X = S A_0 X - p S X from the two
 *                         precomputed pieces.  The snapshot solves (conjugate
 *                         gradients) need A(p_i) positive definite, i.e. p_i <
 *                         2 - 2 cos(pi / (n + 1)); other snapshot points need
 *                         basis_in.
 *   SUBAP_FAMILY_IDENTITY  A(p) = I with b_i(p) = 1 / (1 + 25 (t_i - p)^2) on
 *                         t_i = i / (n - 1): SubApSnap is then DEIM (eq.
 *                         (3.5)); d = 1, problem->rhs ignored.
 *   For these two families the right-hand side varies with p: the sketched
 *   residual of subap_solve_batch and subap_sketched_residual is relative to
 *   |S b(p)| and subap_delta_residual to |b(p)|.  Leverage-score selection,
 *   subap_apsnap_solve, subap_polish and the surrogate are not available for
 *   them (SUBAP_E_UNSUPPORTED).
 *   SUBAP_FAMILY_AFFINE   a general affine family (Section 3.1, "Computing
 *                         S A(p*) X"): A(theta) = sum_q theta_q A_q with
 *                         nterms (1..4) given sparse n x n terms and a fixed
 *                         b = problem->rhs; the parameter is theta itself,
 *                         d = nterms (a caller with a physical parameter p
 *                         evaluates theta_q(p)).  The offline phase stores the
 *                         s x r pieces S A_q X, and the online solve assembles
 *                         S A(theta) X = sum_q theta_q S A_q X in O(nterms s r).
 *                         The snapshot solver needs symmetric positive
 *                         definite systems, so this family takes its basis
 *                         from basis_in (SUBAP_E_UNSUPPORTED without it);
 *                         rows come from rows_in or any selection at
 *                         select_param (theta).  subap_polish and
 *                         subap_model_save are not available for it.
 * Finite-difference layout: node (ix, iy[, iz]) sits at ((ix+1) h, ...),
 * h = 1/(N+1), index ix + N iy (+ N^2 iz); the face coefficient is a at
 * the face midpoint; row i holds sum_f a_f / h^2 on the diagonal and
 * -a_f / h^2 for each in-domain neighbour.
 *
 * Conventions for every entry point
 *   - Return value: SUBAP_OK or an error code; arguments are validated
 *     before any device work, and on error nothing has been enqueued.
 *     subap_last_error() gives a message for the calling thread.
 *   - "host" pointers are read during the call and may be freed after it.
 *     "device" pointers are HIP device memory owned by the caller.
 *   - Device work is enqueued on the given HIP stream (NULL = default
 *     stream) and is asynchronous unless stated otherwise.  One model must
 *     not be used by two streams at once.
 *   - Matrices are FP64 unless stated; "col-major n x r" means element
 *     (i, c) at [i + n c]; "row-major m x d" means (k, q) at [k d + q].
 *   - The library never prints and never aborts.
 */
#ifndef SUBAP_H
#define SUBAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define SUBAP_API __attribute__((visibility("default")))
#else
#define SUBAP_API
#endif

typedef enum {
  SUBAP_OK = 0,
  SUBAP_E_INVALID = 1,     /* bad argument (NULL, size, range)               */
  SUBAP_E_NOMEM = 2,       /* device or host allocation failed               */
  SUBAP_E_HIP = 3,         /* a HIP runtime call failed                      */
  SUBAP_E_RANK = 4,        /* per-p: S A(p) X numerically rank deficient     */
  SUBAP_E_NOCONV = 5,      /* snapshot solver did not reach its tolerance    */
  SUBAP_E_NONFINITE = 6,   /* per-p: non-finite parameter or coefficient     */
  SUBAP_E_UNSUPPORTED = 7  /* valid request this library does not implement  */
} subap_status;

typedef enum {
  SUBAP_FAMILY_DIFF2D = 1,
  SUBAP_FAMILY_DIFF3D = 2,
  SUBAP_FAMILY_KRR = 3,
  SUBAP_FAMILY_DELAY = 4,
  SUBAP_FAMILY_TRIDIAG_SHIFT = 5,
  SUBAP_FAMILY_IDENTITY = 6,
  SUBAP_FAMILY_AFFINE = 7
} subap_family;

/* Arithmetic of the bulk contraction S A(p) X.  The least-squares solve is
 * always FP64 Householder QR. */
typedef enum {
  SUBAP_FP64 = 0,    /* FP64 rows, FP64 contraction                           */
  SUBAP_FP32 = 1,    /* FP32 rows and contraction (FP32 MFMA for KRR)          */
  SUBAP_BF16X3 = 2,  /* KRR only: bf16 hi/lo split operands, three MFMA
                        products hi*hi + hi*lo + lo*hi, FP32 accumulation     */
  SUBAP_FP16X3 = 3   /* KRR only: as BF16X3 with fp16 halves (11-bit
                        significands; Q columns scaled by powers of two)      */
} subap_precision;

typedef struct {
  int32_t family;          /* subap_family                                   */
  int32_t grid;            /* DIFF2D/3D: interior nodes per axis N (>= 2)    */
  int64_t n;               /* KRR: number of points (ignored for DIFF*)       */
  int32_t dim;             /* KRR: point dimension (1..16)                    */
  const double* points;    /* KRR: host, n x dim row-major                    */
  const double* rhs;       /* host, n entries; NULL = all ones (DIFF* only);
                              TRIDIAG_SHIFT: b0 of b_i(p) (required)        */
  double lambda;           /* KRR ridge parameter (> 0)                       */
  double tau;              /* DELAY: delay tau (> 0)                          */
  double kappa;            /* DELAY: shift kappa (> 2)                        */
  const double* c_out;     /* optional host n entries: output vector c of
                              subap_output (the transfer function's c)        */
  /* AFFINE: nterms (1..4) terms A_q in CSR form, host arrays: row offsets
   * term_rowptr[q] (n + 1 entries, term_rowptr[q][0] = 0, non-decreasing),
   * column indices term_cols[q] and values term_vals[q]
   * (term_rowptr[q][n] entries each, columns in [0, n)).                      */
  int32_t nterms;
  const int64_t* const* term_rowptr;
  const int32_t* const* term_cols;
  const double* const* term_vals;
} subap_problem_desc;

typedef struct subap_model_s* subap_model;   /* opaque; owns device buffers */

/* How the s rows are chosen (Section 5.3). */
typedef enum {
  SUBAP_SELECT_CPQR = 0,     /* rounds of column-pivoted QR on (A(p_sel) X)^T  */
  SUBAP_SELECT_LEVERAGE = 1, /* leverage-score sampling with weights           */
  SUBAP_SELECT_LU = 2        /* rounds of LU with partial pivoting on A(p_sel) X */
} subap_selection;

typedef struct {
  int32_t r;                   /* snapshots / basis columns (1..64)           */
  int32_t s;                   /* selected rows, r <= s <= min(n, 256)        */
  const double* snap_params;   /* host, r x d row-major (ignored with basis_in) */
  const double* select_param;  /* host, d: p at which rows are selected       */
  double snap_tol;             /* snapshot solver relative residual; 0 = 1e-12 */
  int32_t snap_maxiter;        /* snapshot solver iteration cap; 0 = default  */
  const double* basis_in;      /* optional host n x r col-major: use instead of
                                  snapshot solves (still orthonormalised)     */
  const int64_t* rows_in;      /* optional host s row indices: use instead of
                                  pivoted-QR selection                        */
  int32_t selection;           /* subap_selection (ignored with rows_in)      */
  const double* sample_u;      /* LEVERAGE: host, s uniforms in [0, 1), one
                                  per sampled row (the caller owns the random
                                  stream, so a selection is reproducible)     */
  int32_t n_select;            /* CPQR / LU: > 1 selects the union of the r
                                  pivots found at each of n_select points
                                  (Section 5.3.2); 0 or 1 = one point         */
  const double* select_params; /* host, n_select x d row-major (n_select > 1) */
} subap_offline_opts;

/*
 * subap_offline -- Algorithm 3.1 steps 1-3 on the GPU.
 *   1. Snapshot solves A(p_i) x_i = b(p_i) by conjugate gradients (all
 *      three families are symmetric positive definite) to relative residual
 *      snap_tol; the paper allows approximate snapshots (Algorithm 3.1).
 *   2. Householder QR of X with diag(R) > 0; X <- Q (Section 3.1).
 *   3. Rows: rounds of column-pivoted QR on M = (A(select_param) Q)^T (r x n),
 *      each round a fresh pivoted QR over the rows not chosen yet, taking
 *      min(r, s - chosen) pivots; pivot = smallest index whose residual norm
 *      is >= (1 - 1e-6) max (Section 5.3 names pivoted QR on (A(p_i) X)^T;
 *      the round and tie rules are this library's reading for s > r).
 *      With selection = SUBAP_SELECT_LEVERAGE instead (Section 5.3, the
      selector the paper recommends with oversampling, and Section 5.3.1):
      B = [A(select_param) Q, b] (n x (r+1)) is orthonormalised by
      Householder QR; leverage score l_i = squared norm of row i of that
      factor (of its first r columns when |R[r,r]| <= 1e-8 |b|: b then lies
      in span(A Q) and its direction is rounding noise); draw k takes the first row i whose running sum
      l_0 + ... + l_i exceeds sample_u[k] * sum(l) (sums in a fixed
      chunked order), with replacement; row k is weighted by
      w_k = 1 / sqrt(s l_i / sum(l)).  Every row of S A(p) X and entry of
      S b is multiplied by its weight, and rho (subap_solve_batch) becomes
      |W S (A(p) X y - b)| / |b|, an estimate of the full relative residual
      (subap_residual_bounds).  Duplicate rows are allowed.
      With selection = SUBAP_SELECT_LU the rounds run LU with partial
      pivoting on W = A(select_param) Q (n x r) instead (Section 5.3): pivot
      of column j = smallest free row index with |W[i,j]| >= (1 - 1e-6) max,
      then every free row i loses W[i,j] / W[piv,j] times the pivot row.
      With n_select > 1 (CPQR or LU) the rows are the union, in order of
      first appearance, of the r pivots found at each of select_params
      (Section 5.3.2); the model's s is then the union's size (r..256, read it
      with subap_model_dims) and opts->s is ignored.
   Then builds the per-row tables the online kernels read.
 * Blocks until the model is complete.  On success *out owns device memory;
 * release it with subap_model_free.  SUBAP_E_NOCONV if a snapshot solve
 * stalls (the model is not created).
 */
SUBAP_API subap_status subap_offline(const subap_problem_desc* problem,
                           const subap_offline_opts* opts,
                           void* hip_stream, subap_model* out);

typedef struct {
  int32_t contraction;   /* subap_precision of S A(p) X                        */
  int32_t refine_steps;  /* FP64 refinement steps after the solve (0..4): the
                            residual r_S = S(A(p) X y - b) is re-evaluated in
                            FP64 and a correction dy subtracted from y        */
  int32_t refine_csne;   /* 0: simple refinement, dy = R^{-1} Q_G^T r_S with
                            the QR of the contraction-precision S A(p) X; its
                            fixed point is the least-squares solution of that
                            rounded matrix, off the exact one by about
                            (contraction error) x cond x (sketched residual)
                            when s > r.
                            1: corrected semi-normal equations (Bjorck):
                            R^T R dy = G^T r_S with G^T r_S = X^T A(p)_S^T r_S
                            evaluated in FP64 from the generated rows, whose
                            fixed point is the exact eq. (3.3) solution.
                            Costs a second pass over the rows per step.      */
} subap_solve_opts;

/*
 * subap_solve_batch -- Algorithm 3.1 step 4 for m parameters.
 *   params_dev  device, m x d row-major FP64 parameters p*;
 *   y_dev       device, m x r row-major FP64 output coefficients c(p*)
 *               in the orthonormal basis Q (x = Q c);
 *   rho_dev     device or NULL, m: sketched relative residual
 *               |S(A(p) Q y - b)|_2 / |S b|_2 in FP64 after the last step;
 *   status_dev  device or NULL, m int32: SUBAP_OK, SUBAP_E_RANK (some
 *               |R_jj| <= 1e-13 |R_11| in the QR of S A(p) Q; y is NaN) or
 *               SUBAP_E_NONFINITE (non-finite p or coefficient; y is NaN).
 *   opts        host or NULL (= FP64, no refinement).
 * m = 0 is a no-op.  Asynchronous on hip_stream.
 */
SUBAP_API subap_status subap_solve_batch(subap_model model, const double* params_dev, int64_t m,
                               double* y_dev, double* rho_dev, int32_t* status_dev,
                               const subap_solve_opts* opts, void* hip_stream);

/*
 * subap_solve_batch_noalloc -- subap_solve_batch without any device
 * allocation, for callers that cannot allocate: code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that
 * forbid it.  Same arguments, layouts, statuses and results (bitwise) as
 * subap_solve_batch.  The finite-difference and delay solves need no
 * workspace.  The kernel ridge solve takes its workspace from a fixed 64 MiB
 * device array inside the library (one per GPU, held until the process
 * ends) and solves a batch larger than fits in consecutive chunks (about 650
 * parameters per chunk at n = 16384, r = 32, s = 128 with a split contraction
 * and one CSNE step).  Every call on one GPU shares that array: calls that
 * overlap on one GPU (two streams, two threads) race and give undefined
 * results.  SUBAP_E_UNSUPPORTED if a single block of 16 parameters would need
 * more than 64 MiB (not reachable with r <= 64, s <= 256).  Asynchronous on
 * hip_stream; the model must be on the current device.
 */
SUBAP_API subap_status subap_solve_batch_noalloc(subap_model model, const double* params_dev, int64_t m,
                                                 double* y_dev, double* rho_dev, int32_t* status_dev,
                                                 const subap_solve_opts* opts, void* hip_stream);

/*
 * subap_lift -- x = Q y (Algorithm 3.1 step 4, output X c) for k coefficient
 * vectors.
 *   y_dev      device k x r row-major FP64.
 *   x_dev      device, column i (i < k) at x_dev + i * ldx, rows 0..n-1 written,
 *              rows n..ldx-1 untouched; FP64 (precision = SUBAP_FP64) or FP32
 *              (SUBAP_FP32, split-bf16 MFMA with FP32-level error).
 *   ldx        leading dimension in elements, 0 (= n) or >= n.  For FP32 output
 *              an ldx that is a multiple of 32 with x_dev 128-byte aligned lets
 *              every column start on a cache line (full-line stores; about twice
 *              the write bandwidth of an odd n).
 * k = 0 is a no-op.  SUBAP_E_INVALID for k < 0, 0 < ldx < n, NULL pointers or
 * another precision.  Asynchronous on hip_stream.
 */
SUBAP_API subap_status subap_lift(subap_model model, const double* y_dev, int64_t k,
                        void* x_dev, int64_t ldx, int32_t precision, void* hip_stream);

/*
 * subap_sketched_residual -- FP64 sketched residual of given coefficients,
 * from the s selected rows only (Section 5.3.1 uses |S(B c - b)| as the
 * estimate of the full residual):
 *   res_dev[p s + k] = (A(p) Q y_p - b(p))_{i_k}        (device, m x s, or NULL)
 *   norm_dev[p]      = |res_p|_2 / |S b|_2               (device, m, or NULL)
 * Rows are generated with FP64-accurate entries and applied to z = Q y_p, an
 * s x n matrix-vector product per parameter; S A(p) Q is never formed.  This
 * is the acceptance test of a predicted y and the reference for comparing
 * two coefficient vectors: |res(y1) - res(y2)| = |S A(p) Q (y1 - y2)|.
 * At least one output must be given.  Asynchronous on hip_stream.
 */
SUBAP_API subap_status subap_sketched_residual(subap_model model, const double* params_dev, int64_t m,
                                               const double* y_dev, double* res_dev, double* norm_dev,
                                               void* hip_stream);

/*
 * subap_excess_bound -- an a posteriori bound on how far given coefficients
 * are from the SubApSnap solution, without solving: with G = S A(p) Q
 * (weighted rows for leverage-score models) and r_S = G y - S b,
 *   out[k] = |G^T r_S| / (sigma_min |S b|)
 * (|S b| as in the sketched residual).  Since G^T r_S = G^T G (y - y*),
 * out[k] >= |G (y_k - y*_k)| / |S b| whenever sigma_min <= sigma_min(G_k): the
 * normal-equation excess over the method's own residual floor, which the
 * sketched residual |r_S| alone cannot show (its minimum is that floor,
 * Section 5.3.1).  Evaluated in FP64 from the generated rows: an s x n
 * matrix-vector product and its adjoint (kernel family) or the face tables
 * (stencil families); no contraction of S A(p) Q with Q is formed for the
 * kernel family.  sigma_min is the caller's (e.g. a fraction of the smallest
 * sigma_min(G) over training parameters, from subap_reduced_matrix).
 *   y_dev device m x r; out_dev device m.  Asynchronous.
 * subap_reduced_matrix -- G_k = S A(p_k) Q in FP64, device m x s x r (row k of
 * G_k at G_dev + (k_param s + k) r), for calibration and analysis.
 */
SUBAP_API subap_status subap_excess_bound(subap_model model, const double* params_dev, int64_t m, const double* y_dev,
                                          double sigma_min, double* out_dev, void* hip_stream);
SUBAP_API subap_status subap_reduced_matrix(subap_model model, const double* params_dev, int64_t m, double* G_dev,
                                            void* hip_stream);

/*
 * Batched solve over many models.  A plan fixes the models, the parameter
 * counts and the device buffers; executing it runs Algorithm 3.1 step 4 for
 * every parameter of every model.  The diffusion models share one persistent
 * launch, except those that subap_solve_batch gives to the matrix-core
 * semi-normal solve (FP64 without refinement, s >= 96, 16 <= r <= 47) with
 * at least 16 parameters per compute unit (4096 on MI355X); those and every
 * other member (the kernel family, the delay system, eq. (5.7),
 * the identity and affine families) are solved by their family's batched
 * solver after it, on the same stream, with a workspace the plan owns.  All
 * buffers keep the layouts of subap_solve_batch, one per model (rho_dev and
 * status_dev may be NULL, or contain NULL entries); a member's results equal
 * those of subap_solve_batch with the same options, bit for bit, except the
 * diffusion members of the persistent launch, which it solves by Householder
 * QR.
 *   flags  SUBAP_PLAN_GRAPH:    capture the launch in a hipGraph once and
 *                               replay it on every execute;
 *          SUBAP_PLAN_AUTOTUNE: time the candidate launch shapes (threads per
 *                               block, resident blocks) on the plan and keep
 *                               the fastest; the choice is cached in the file
 *                               named by $SUBAP_AUTOTUNE_CACHE (default
 *                               ~/.cache/subap_autotune.txt) under a key made
 *                               of the shapes, and reused when the key recurs.
 * Work items (one parameter each) are taken from a device counter, largest
 * instances first.  Autotuning runs the plan, so it writes the outputs.
 * Contraction FP64 or FP32; refine_steps 0..4.  The models and buffers must
 * outlive the plan.  subap_solve_multi is create + execute + free.
 */
typedef struct subap_plan_s* subap_plan;
#define SUBAP_PLAN_GRAPH 1
#define SUBAP_PLAN_AUTOTUNE 2
SUBAP_API subap_status subap_plan_create(const subap_model* models, int32_t k, const double* const* params_dev,
                                         const int64_t* m, double* const* y_dev, double* const* rho_dev,
                                         int32_t* const* status_dev, const subap_solve_opts* opts,
                                         int32_t flags, void* hip_stream, subap_plan* out);
SUBAP_API subap_status subap_plan_execute(subap_plan plan, void* hip_stream);
/* Launch shape of the persistent launch in use (after autotuning): threads
 * per block, blocks; blocks is 0 when no member takes the persistent launch. */
SUBAP_API subap_status subap_plan_shape(subap_plan plan, int32_t* threads, int32_t* blocks);
SUBAP_API subap_status subap_plan_free(subap_plan plan);
SUBAP_API subap_status subap_solve_multi(const subap_model* models, int32_t k, const double* const* params_dev,
                                         const int64_t* m, double* const* y_dev, double* const* rho_dev,
                                         int32_t* const* status_dev, const subap_solve_opts* opts,
                                         void* hip_stream);

/*
 * Learned surrogate p -> y (not in the paper): a multilayer perceptron
 * d -> hidden -> hidden -> r with GELU activations, trained on (p, y) pairs
 * produced by subap_solve_batch, with the library's own forward, backward and
 * Adam kernels (BF16 MFMA products with FP32 accumulation, FP32 master
 * weights; the output layer uses split bf16 hi/lo products).  Targets are
 * standardised per component with the training mean and deviation.
 *
 * Weights (host, FP64, caller-drawn initial values) are laid out as
 * [W1 (hidden x d) | b1 | W2 (hidden x hidden) | b2 | W3 (r x hidden) | b3],
 * each W row-major (fan_out x fan_in); subap_surrogate_nparams gives the
 * total length.
 */
typedef struct subap_surrogate_s* subap_surrogate;
typedef struct {
  int32_t epochs;    /* passes over the pairs (>= 1)                              */
  int32_t batch;     /* mini-batch rows (1..65536); 0 = 4096                      */
  double lr;         /* peak Adam step (betas 0.9, 0.999, eps 1e-8); 0 = 1e-3     */
  double lr_min;     /* floor of the cosine decay over all steps                   */
  uint64_t seed;     /* selects the per-epoch affine permutations of the pairs    */
} subap_train_opts;
SUBAP_API subap_status subap_surrogate_create(int32_t d, int32_t r, int32_t hidden, const double* weights_host,
                                              subap_surrogate* out);
SUBAP_API int64_t subap_surrogate_nparams(subap_surrogate s);
/* Current master weights as FP64 (blocking). */
SUBAP_API subap_status subap_surrogate_weights(subap_surrogate s, double* weights_host);
/* Gradient of the mean-squared error of the network on (params, targets),
 * targets already standardised (device, m x d and m x r; m <= 65536).  The
 * weights are not changed.  Blocking; host outputs. */
SUBAP_API subap_status subap_surrogate_gradient(subap_surrogate s, const double* params_dev,
                                                const double* targets_dev, int64_t m, double* grad_host,
                                                double* loss_host, void* hip_stream);
/* Train on m pairs (device, m x d params and m x r coefficients from
 * subap_solve_batch).  loss_host: optional, one mean-squared error per epoch
 * (of the last mini-batch).  Blocking. */
SUBAP_API subap_status subap_surrogate_train(subap_surrogate s, const double* params_dev, const double* y_dev,
                                             int64_t m, const subap_train_opts* opts, double* loss_host,
                                             void* hip_stream);
/* Predicted coefficients (device, m x r FP64).  Asynchronous. */
SUBAP_API subap_status subap_surrogate_predict(subap_surrogate s, const double* params_dev, int64_t m,
                                               double* y_dev, void* hip_stream);
/*
 * Surrogate with fallback: predict y for every p, evaluate its FP64 sketched
 * relative residual |S(A(p) Q y - b)| / |S b| (subap_sketched_residual) and
 * accept the prediction when it is <= accept_tol; the rejected parameters
 * are gathered and solved by subap_solve_batch with fallback_opts (NULL =
 * FP64), and their results scattered back.  accepted_dev (m bytes) and
 * status_dev (m) may be NULL.  *n_accepted receives the accepted count.
 * Blocking (the host needs the rejected count).
 */
SUBAP_API subap_status subap_surrogate_solve_batch(subap_model model, subap_surrogate s, const double* params_dev,
                                                   int64_t m, double accept_tol, double* y_dev,
                                                   uint8_t* accepted_dev, int32_t* status_dev,
                                                   const subap_solve_opts* fallback_opts, int64_t* n_accepted,
                                                   void* hip_stream);
/*
 * As subap_surrogate_solve_batch, with the normal-equation excess bound of
 * subap_excess_bound (sigma_min > 0, finite) as the acceptance measure: a
 * prediction is accepted when |G^T r_S| / (sigma_min |S b|) <= accept_tol,
 * which, for sigma_min <= sigma_min(S A(p) Q), guarantees
 * |S A(p) Q (y - y*)| / |S b| <= accept_tol for the SubApSnap solution y*
 * (Section 5.3.1 takes the sketched residual as an estimate of the full one;
 * the bound measures the distance to y* itself, which the sketched residual
 * cannot show below its own floor).  Blocking.
 */
SUBAP_API subap_status subap_surrogate_solve_batch_excess(subap_model model, subap_surrogate s,
                                                          const double* params_dev, int64_t m, double sigma_min,
                                                          double accept_tol, double* y_dev, uint8_t* accepted_dev,
                                                          int32_t* status_dev, const subap_solve_opts* fallback_opts,
                                                          int64_t* n_accepted, void* hip_stream);
SUBAP_API subap_status subap_surrogate_free(subap_surrogate s);

/*
 * subap_exp2_rate -- transcendental-rate microbenchmark for the kernel family's
 * entries K = 2^(c D) (eq. (6.4) with c = -log2(e) / (2 p^2)): times about
 * `evals` evaluations on the whole device, 16 independent ones per lane as the
 * refinement issues them, each accumulated in FP64, and writes evaluations
 * per second to *evals_per_s (host).  form 7, 9 or 11: the FP64 polynomial
 * of that degree after exact range reduction (relative error 5.5e-11,
 * 1.9e-14, 2.2e-16); form 0: the FP32 hardware v_exp_f32 that the 16-bit and
 * FP32 contractions use.  Blocking; allocates a small device buffer.
 */
SUBAP_API subap_status subap_exp2_rate(int32_t form, int64_t evals, double* evals_per_s, void* hip_stream);

/*
 * Per-kernel timing for benchmarks.  While enabled, the library records a
 * HIP event pair on the launching stream around every kernel it enqueues.
 * subap_profile_count() waits for the recorded events and returns the
 * number of distinct kernel names; subap_profile_entry(i, ...) gives the
 * name (valid until the next profile call), the number of launches and
 * their total duration in milliseconds.  Process-wide; thread-safe.
 */
SUBAP_API subap_status subap_profile_enable(int32_t on);
SUBAP_API subap_status subap_profile_reset(void);
SUBAP_API int32_t subap_profile_count(void);
SUBAP_API subap_status subap_profile_entry(int32_t i, const char** name, int64_t* calls,
                                           double* total_ms);

/* Model queries (blocking, host outputs). */
SUBAP_API subap_status subap_model_dims(subap_model model, int64_t* n, int32_t* r,
                              int32_t* s, int32_t* d);
/* rows_host: s indices in selection order. */
SUBAP_API subap_status subap_model_rows(subap_model model, int64_t* rows_host);
/*
 * subap_output -- the linear output c^T x of x = X y without forming x
 * (Section 6.2.2: H(p*) ~ (c^T X) c_hat with c^T X precomputed offline):
 *   y_dev    device, m x r row-major coefficients (subap_solve_batch);
 *   out_dev  device, m values (written): out[k] = sum_c (c^T Q)_c y[k, c].
 * SUBAP_E_INVALID if the model was built without c_out.
 */
SUBAP_API subap_status subap_output(subap_model model, const double* y_dev, int64_t m, double* out_dev,
                                    void* hip_stream);
/*
 * Full-size reference paths (all n rows; meant for checking a method's
 * quality on a few parameters, not for throughput).  Each blocks until done.
 *
 * subap_full_residual -- res[k] = |A(p_k) x_k - b| / |b| (the measure of the
 *   paper's Tables 3-4) for full vectors x_dev (device, n x m col-major,
 *   column k = x_k, e.g. from subap_lift).
 * subap_delta_residual -- res[k] = |A(p_k) Q (y1_k - y2_k)| / |b| over all n
 *   rows: the distance between two coefficient vectors in the residual norm
 *   of the paper's Tables 3-4 (|res(y1) - res(y2)| with res(y) = A Q y - b).
 *   y1_dev, y2_dev (device, m x r row-major), res_dev (device, m).  Used to
 *   hold a reduced-precision form to the FP64 one.
 * subap_apsnap_solve -- ApSnap (eq. (3.1)): y_k = argmin_c |A(p_k) X c - b|
 *   over all n rows, by Householder QR of the n x r matrix A(p_k) Q.
 *   y_dev (device, m x r row-major), rho_dev (device, m, or NULL): the full
 *   relative residual of y_k.
 * subap_polish -- conjugate gradients on A(p_k) x = b warm-started from
 *   x_dev (device, n x m col-major, overwritten with the iterate): the
 *   polishing from the SubApSnap solution that Section 3.1 mentions (CG,
 *   Jacobi-preconditioned for the stencil families, since every family here
 *   is symmetric positive definite).  Stops a column once |b - A x| <= tol
 *   |b| (checked every 16 iterations and at the end) or after max_iter
 *   iterations; reaching max_iter is not an error.  res_dev (device, m, or
 *   NULL): the final relative residuals.
 */
SUBAP_API subap_status subap_full_residual(subap_model model, const double* params_dev, int64_t m,
                                           const double* x_dev, double* res_dev, void* hip_stream);
SUBAP_API subap_status subap_delta_residual(subap_model model, const double* params_dev, int64_t m,
                                            const double* y1_dev, const double* y2_dev, double* res_dev,
                                            void* hip_stream);
SUBAP_API subap_status subap_apsnap_solve(subap_model model, const double* params_dev, int64_t m, double* y_dev,
                                          double* rho_dev, void* hip_stream);
SUBAP_API subap_status subap_polish(subap_model model, const double* params_dev, int64_t m, double* x_dev,
                                    int32_t max_iter, double tol, double* res_dev, void* hip_stream);
/* Row weights (host, s values): 1 for pivoted-QR rows, 1/sqrt(s pi_i) for
 * leverage-score rows. */
SUBAP_API subap_status subap_model_weights(subap_model model, double* weights_host);
/*
 * subap_residual_bounds -- Section 5.3.1: with leverage-score rows the
 * weighted sketch of span([A X, b]) satisfies, with high probability at
 * select_param, (1 - eps) |v| <= |W S v| <= (1 + eps) |v| for every v in that
 * span, so the full relative residual lies in
 * [rho / (1 + eps), rho / (1 - eps)] (upper bound +inf when eps >= 1).  At
 * other parameters the bounds are the paper's heuristic estimate.
 *   rho_dev   device, m relative sketched residuals (rho of subap_solve_batch);
 *   eps       > 0, or <= 0 for the default k ln(k) / s with k = r + 1;
 *   lo_dev, hi_dev  device, m values each (written).
 * SUBAP_E_INVALID if the model's rows are not leverage-score rows.
 */
SUBAP_API subap_status subap_residual_bounds(subap_model model, const double* rho_dev, int64_t m, double eps,
                                             double* lo_dev, double* hi_dev, void* hip_stream);
/* Q_host: n x r col-major orthonormal basis. */
SUBAP_API subap_status subap_model_basis(subap_model model, double* Q_host);

SUBAP_API subap_status subap_model_free(subap_model model);
/*
 * subap_model_save / subap_model_load -- keep the offline result (Algorithm
 * 3.1 steps 1-3) for later sessions: the file holds the problem data (b,
 * KRR points, family constants), the basis Q, the rows, their weights and
 * c^T Q.  Loading uploads them and rebuilds the per-row tables on the GPU,
 * so a loaded model solves bit-identically to the saved one.  Both block.
 * The file uses the host's byte order.  SUBAP_E_INVALID for a path that
 * cannot be opened, a file that is not a model file, or a truncated or
 * inconsistent one (nothing is allocated on the device then).
 */
SUBAP_API subap_status subap_model_save(subap_model model, const char* path);
SUBAP_API subap_status subap_model_load(const char* path, void* hip_stream, subap_model* out);

SUBAP_API const char* subap_status_string(subap_status status);
/* Message of the last failing call on this thread ("" if none). */
SUBAP_API const char* subap_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SUBAP_H */
