/*
 * mrcqr.h - C ABI of the MI355X (gfx950) MRCQR library.
 *
 * MRCQR computes the thin QR factorization A = Q R of a tall-skinny float64
 * matrix A (m x n, m >= n, rank n) with an explicit Q (Q^T Q = I_n) and an
 * upper-triangular R with positive diagonal. It follows Algorithm 2 of
 * Garrison, Chen and Ipsen, "Numerically Stable Cholesky-QR on GPU via
 * Mixed-Precision Randomized Preconditioning" (arXiv 2606.18411):
 *   Stage 1 (sketch precision p): Rademacher signs D, a subsampled DCT-II
 *           along the rows (the sketch Y = S F D A, s rows), Householder QR
 *           of Y giving the preconditioner Rs;
 *   Stage 2 (float64): B = A Rs^{-1}, then Cholesky-QR of B (Algorithm 1):
 *           G = B^T B, G = Rc^T Rc, Q = B Rc^{-1};
 *           B = A Rs^{-1} is a block substitution (Rs may be as ill
 *           conditioned as A, so Rs itself is never inverted; only its
 *           16 x 16 diagonal blocks are, as GPU triangular solves do); Q is
 *           the product of B with the explicit inverse of Rc, whose
 *           condition number is that of B, a small constant;
 *   Stage 3: R = Rc Rs.
 *
 * Conventions for every entry point:
 *   - all matrices are column-major float64 with a leading dimension
 *     (element (i, j) of X is X[i + j * ldx]); ld >= number of rows;
 *   - every matrix/array pointer is a DEVICE pointer (hipMalloc'd or
 *     torch-allocated memory on the current device); the library never
 *     frees or retains caller memory past the call;
 *   - `stream` is a hipStream_t (NULL = the legacy default stream); all
 *     work is enqueued asynchronously on it; no entry point waits for the
 *     device, except mrcqr_factor_batched (blocking argument copy) and
 *     mrcqr_release_cache. A fixed-precision factorization with n > 128
 *     (mrcqr_factor, mrcqr_execute) runs its posterior check on a second
 *     stream that the library keeps per (device, stream), forked from
 *     `stream` after Rc^{-1} and joined back before the info is written,
 *     so that it overlaps the product Q = B Rc^{-1}; work enqueued on
 *     `stream` after the call is ordered after all of it (under stream
 *     capture both become graph nodes; a stream first seen under capture
 *     takes the serial sequence);
 *   - argument errors are returned synchronously (MRCQR_ERR_ARG /
 *     MRCQR_ERR_UNSUPPORTED) before anything is launched; numeric outcomes
 *     (non-finite sketch, Cholesky breakdown, singular sketch, posterior
 *     warning) are written
 *     asynchronously to a device-resident mrcqr_info that the caller reads
 *     after synchronizing the stream;
 *   - results are deterministic: the same inputs, seed and device give
 *     bitwise-identical outputs (no floating-point atomics).
 * Limits of this library: n <= s <= m, m < 2^28, and
 *   - the factorization (mrcqr_factor, the plan API, the no-allocation
 *     entry point) and the steps mrcqr_sketch, mrcqr_trsm, mrcqr_gram,
 *     mrcqr_tri_inverse, mrcqr_form_q, mrcqr_trmm and mrcqr_posterior_kappa
 *     take 1 <= n <= 512; for 128 < n <= 512 they run a column-panel path
 *     (128-column panels of the solve, the Gram, the Cholesky and the
 *     product; a blocked Householder QR of the sketch, s <= 1024);
 *   - for n <= 128 the sketch must fit the one-workgroup Householder QR:
 *     s <= 2048 for n <= 16, s <= 1024 for n <= 32, s <= 512 for n <= 64,
 *     s <= 256 for n <= 128 (the default s = 2n always fits);
 *   - batches, CholQR2, mrcqr_sketch_qr, mrcqr_cholesky, mrcqr_condest and
 *     the estimators take n <= 128;
 *   - larger shapes return MRCQR_ERR_UNSUPPORTED.
 */
#ifndef MRCQR_H
#define MRCQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sketch precision p of Algorithm 2 (Section "Adaptive Precision
 * Selection": half for kappa < 1e4, single below 1e8, double otherwise).
 * BF16 is an extra option (8-bit exponent, 8-bit significand).
 * AUTO starts at FP16 and escalates per call from an on-device condition
 * estimate of Rs, and reruns one precision higher when the posterior check
 * fails (see mrcqr_factor).
 * AUTO_CARRY is AUTO for a sequence of similar matrices (block Arnoldi,
 * power iterations: Section "Adaptive Precision Selection", repeated
 * calls): a call starts from the precision that the previous AUTO_CARRY
 * call on the same workspace accepted, instead of from FP16, and escalates
 * from there as AUTO does. The record lives in the workspace on the device,
 * so it also carries across the replays of a captured graph; it never moves
 * down (mrcqr_regime_reset forgets it). A workspace without a record (all
 * zero bytes) starts from FP16. Calls sharing one workspace share its
 * record, so AUTO_CARRY needs a workspace owned by the caller: the plan and
 * batch-plan APIs accept it, mrcqr_factor and mrcqr_factor_batched (whose
 * workspaces are shared per shape) return MRCQR_ERR_ARG. */
enum mrcqr_precision {
  MRCQR_PREC_AUTO = 0,
  MRCQR_PREC_FP64 = 1,
  MRCQR_PREC_FP32 = 2,
  MRCQR_PREC_FP16 = 3,
  MRCQR_PREC_BF16 = 4,
  MRCQR_PREC_AUTO_CARRY = 5
};

enum mrcqr_status {
  MRCQR_OK = 0,
  MRCQR_ERR_ARG = 1,              /* invalid argument (synchronous)               */
  MRCQR_ERR_NONFINITE = 2,        /* the sketch Y holds inf or NaN: A has a
                                     non-finite entry, or entries beyond the
                                     range of the sketch precision (AUTO then
                                     escalates; reported at FP64 or a forced
                                     precision)                                 */
  MRCQR_ERR_CHOL_BREAKDOWN = 3,   /* Gram matrix not numerically SPD (Algorithm 1
                                     breakdown); chol_fail_index = first pivot   */
  MRCQR_ERR_SKETCH_SINGULAR = 4,  /* Rs has a zero or non-finite diagonal entry   */
  MRCQR_ERR_WORKSPACE = 5,        /* workspace missing or too small (synchronous) */
  MRCQR_ERR_DEVICE = 6,           /* a HIP runtime call failed (synchronous)      */
  MRCQR_WARN_POSTERIOR = 7,       /* Q, R produced, but the estimate of
                                     kappa(Rc) exceeds the posterior bound: the
                                     sketch precision was too low for A (Section
                                     "Adaptive Precision Selection", rerun rule)  */
  MRCQR_ERR_UNSUPPORTED = 8       /* shape outside this library's limits (synchronous) */
};

/* Per-call outcome, written by the device at the end of the call. */
typedef struct mrcqr_info {
  int32_t status;          /* mrcqr_status                                     */
  int32_t precision_used;  /* mrcqr_precision of the accepted Stage 1          */
  int32_t chol_fail_index; /* first failing pivot, or -1                       */
  int32_t escalations;     /* AUTO: number of precision escalations            */
  double kappa_rs_est;     /* ICE estimate of kappa_2(Rs) (a lower bound); only
                              AUTO computes it: NaN for a forced precision,
                              +inf when Rs was singular                      */
  double kappa_rc_est;     /* posterior estimate of kappa_2(Rc) = kappa_2(B):
                              the larger of ICE and 12 power steps on Rc and
                              Rc^{-1} (both lower bounds); +inf on breakdown */
} mrcqr_info;

typedef struct mrcqr_plan mrcqr_plan;

/* Sketch transform flags (mrcqr_plan_create_ex, mrcqr_sketch_ex). Default
 * (0): the DCT-II sketch, Y = gamma .* C fl_p(D A) with the sampled rows of
 * the DCT-II, S drawn from [0, m), default s = 2n.
 * MRCQR_SKETCH_RFFT: the paper's operator (Algorithm 2, FFT and Select):
 * the real parts of c sampled bins of the m-point DFT of fl_p(D A),
 * Y[i, :] = sqrt(c/m) sum_t cos(2 pi k_i t / m) fl_p(D A)[t, :], with S
 * drawn from the floor(m/2) + 1 distinct bins {0, ..., floor(m/2)} (Hermitian
 * symmetry), default c = 3n (the paper's default); c <= floor(m/2) + 1. Same
 * precision rules as the DCT-II sketch (coefficients rounded to p, float32
 * accumulation for p != FP64). */
#define MRCQR_SKETCH_RFFT 1

/* ---------------------------------------------------------------------
 * Whole factorization (Algorithm 2, all three stages).
 *
 * A (m x n, lda) is read only. Q (m x n, ldq) and R (n x n, ldr; the strict
 * lower triangle is set to zero) are written. Q must not overlap A.
 * s: sketch rows (0 = default 2n); n <= s <= m.
 * seed: selects D and S (counter-based SplitMix64 draw, Floyd sampling).
 * info_dev: device pointer to one mrcqr_info (may be NULL).
 * The workspace comes from a per-device cache keyed by (m, n, s), created
 * on first use with hipMalloc (no memset, no wait for the device) and kept
 * until mrcqr_release_cache; use the plan API to supply it yourself. Calls
 * of one shape are serialized on the device through an event of the cached
 * workspace (the stream of a call waits for the previous call of that
 * shape, whatever its stream or host thread), so they never race. Under
 * stream capture the event edges are left out: a captured call shares the
 * workspace with every other call of its shape, and replays must not
 * overlap them (the plan API gives a capture its own workspace).
 * AUTO: Stage 1 runs in FP16; if the ICE estimate of kappa(Rs) is >= 1e4
 * it is redone in FP32, and if that estimate is >= 1e8, in FP64. After
 * Stage 2 the posterior check (estimate of kappa(Rc) above 20, or a
 * Cholesky breakdown) reruns the factorization one precision higher, up to
 * FP64 (Section "Adaptive Precision Selection", rerun rule). All decisions
 * are taken on the device (no host round trip). AUTO_CARRY is rejected
 * (MRCQR_ERR_ARG): use the plan API.
 * Returns MRCQR_OK when the work was enqueued.
 * ------------------------------------------------------------------- */
int mrcqr_factor(const double* A, int64_t m, int64_t n, int64_t lda,
                 int sketch_precision, uint64_t seed, int64_t s,
                 double* Q, int64_t ldq, double* R, int64_t ldr,
                 void* stream, mrcqr_info* info_dev);

/* CholQR2, the unpreconditioned baseline of the paper's stability sweep
 * (Section "Numerical Stability"): Algorithm 1 applied twice, [Q1, R1] =
 * CholQR(A), [Q, R2] = CholQR(Q1), R = R2 R1, every step in float64 on the
 * library's kernels (Gram SYRK, Cholesky, block substitution Q = A R^{-1}). It
 * breaks down once the Gram matrix of A is not numerically positive definite
 * (kappa(A) past about 1e8): info->status = MRCQR_ERR_CHOL_BREAKDOWN with the
 * first failing pivot (of pass 1, else of pass 2), and Q, R unspecified.
 * Needs mrcqr_cholqr2_workspace_bytes(m, n) bytes of device workspace (Q1
 * and small n x n terms; about m n 8 bytes). Same shape limits as
 * mrcqr_factor; Q must not overlap A. info_dev may be NULL. */
size_t mrcqr_cholqr2_workspace_bytes(int64_t m, int64_t n);
int mrcqr_cholqr2(const double* A, int64_t m, int64_t n, int64_t lda, double* Q, int64_t ldq,
                  double* R, int64_t ldr, void* workspace, size_t workspace_bytes, void* stream,
                  mrcqr_info* info_dev);

/* mrcqr_factor for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results (bitwise) as mrcqr_factor; the
 * workspace is a fixed device array of
 * mrcqr_factor_noalloc_max_workspace_bytes() bytes (64 MiB) that the
 * library holds on every GPU it runs on until the process ends. It calls no
 * hipMalloc, hipFree or allocating library routine. A shape whose
 * workspace (mrcqr_plan_workspace_bytes of its plan) exceeds that size
 * returns MRCQR_ERR_WORKSPACE before anything is launched; n <= 64 with
 * m up to about 65536 fits. All calls on one GPU share the array: calls
 * that overlap on the device (other streams, other host threads, or graph
 * replays running at the same time) race and must be ordered by the caller.
 * Nothing in the array needs to start at zero, so it keeps whatever the
 * last call left. AUTO_CARRY is rejected (MRCQR_ERR_ARG). */
int mrcqr_factor_noalloc(const double* A, int64_t m, int64_t n, int64_t lda,
                         int sketch_precision, uint64_t seed, int64_t s,
                         double* Q, int64_t ldq, double* R, int64_t ldr,
                         void* stream, mrcqr_info* info_dev);
size_t mrcqr_factor_noalloc_max_workspace_bytes(void);

/* Wait for and free the workspaces cached by mrcqr_factor and
 * mrcqr_factor_batched on every device. No call of those may run
 * concurrently with it. Returns MRCQR_ERR_DEVICE if a HIP call failed. */
int mrcqr_release_cache(void);

/* mrcqr_plan_create with sketch transform flags (see MRCQR_SKETCH_RFFT); s =
 * 0 takes the transform's default sketch size. Returns MRCQR_ERR_ARG for an
 * unknown flag or a DFT sketch of more than floor(m/2) + 1 rows. */
int mrcqr_plan_create_ex(int64_t m, int64_t n, int64_t s, int flags, mrcqr_plan** out);

/* Plan API: a plan fixes (m, n, s); execute allocates nothing. Calls that
 * share a workspace must not overlap on the device (one stream, or events
 * between streams). */
int mrcqr_plan_create(int64_t m, int64_t n, int64_t s, mrcqr_plan** out);
size_t mrcqr_plan_workspace_bytes(const mrcqr_plan* plan);
int mrcqr_execute(const mrcqr_plan* plan, void* workspace, size_t workspace_bytes,
                  const double* A, int64_t lda, int sketch_precision, uint64_t seed,
                  double* Q, int64_t ldq, double* R, int64_t ldr,
                  void* stream, mrcqr_info* info_dev);
int mrcqr_plan_destroy(mrcqr_plan* plan);

/* Forget the AUTO_CARRY record of a workspace (Section "Adaptive Precision
 * Selection", repeated calls): the next AUTO_CARRY call on it starts from
 * FP16 again. Enqueued on `stream` as one small kernel (no memset, so it may
 * be captured). workspace: the plan's workspace, at least
 * mrcqr_plan_workspace_bytes bytes. Returns MRCQR_ERR_ARG for a NULL plan
 * and MRCQR_ERR_WORKSPACE for a missing or short workspace. */
int mrcqr_regime_reset(const mrcqr_plan* plan, void* workspace, size_t workspace_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Batches of independent factorizations of uneven shapes (the repeated QRs
 * of block Arnoldi or randomized-SVD power steps; each member is Algorithm 2
 * with s = 2 n). Each step of Algorithm 2 runs as one launch over every
 * member (one per kernel configuration: members are grouped by the size
 * class of n), grid (blocks per member, members), instead of one launch per
 * member and step; every member follows its own precision policy, AUTO
 * escalation and posterior rerun on the device. Member i's Q and R are
 * bitwise those of mrcqr_factor on the same A, policy and seed.
 * ------------------------------------------------------------------- */
typedef struct mrcqr_batch_plan mrcqr_batch_plan;

/* Plan for `batch` members (1 <= batch <= 65535) of shapes m[i] x n[i]
 * (HOST arrays); each shape must be valid for mrcqr_factor with s = 2 n[i].
 * The plan owns small device tables (hipMalloc at creation). Returns
 * MRCQR_ERR_ARG / MRCQR_ERR_UNSUPPORTED for a bad shape. */
int mrcqr_batch_plan_create(int32_t batch, const int64_t* m, const int64_t* n, mrcqr_batch_plan** out);
/* Workspace for one execution: the members' single-call workspaces side by
 * side (about 2 m n 8 bytes per member plus partial sums). */
size_t mrcqr_batch_plan_workspace_bytes(const mrcqr_batch_plan* plan);
int mrcqr_batch_plan_destroy(mrcqr_batch_plan* plan);

/* Enqueue the batch on `stream`; allocates nothing, launches a fixed
 * sequence (graph-capturable). Every per-member array is a DEVICE array of
 * length batch: A[i], Q[i], R[i] are device pointers to member i's
 * column-major matrices, lda/ldq/ldr its leading dimensions, precision[i]
 * its mrcqr_precision policy, seeds[i] its draw. The host checks only that
 * the arrays are non-NULL and the workspace size; the device checks every
 * member's arguments (non-NULL, A != Q, lda >= m, ldq >= m, ldr >= n, a
 * valid policy) and skips a member that fails, with status MRCQR_ERR_ARG in
 * its info. infos_dev: device array of `batch` infos, or NULL. A workspace
 * of zero bytes holds no AUTO_CARRY records. */
int mrcqr_batch_execute(const mrcqr_batch_plan* plan, void* workspace, size_t workspace_bytes,
                        const double* const* A, const int64_t* lda, const int32_t* precision,
                        const uint64_t* seeds, double* const* Q, const int64_t* ldq,
                        double* const* R, const int64_t* ldr, void* stream, mrcqr_info* infos_dev);

/* The same with HOST per-member arrays (the matrices are device memory),
 * checked synchronously like mrcqr_factor. A batch plan, its workspace
 * and the argument arrays are cached per device and shape list (freed by
 * mrcqr_release_cache); the arrays are copied to the device with a blocking
 * copy, after the previous call with the same shape list has finished
 * reading them. AUTO_CARRY members are rejected (MRCQR_ERR_ARG). Not for
 * graph capture (use mrcqr_batch_execute). infos_dev: device array of
 * `batch` infos (or NULL). */
int mrcqr_factor_batched(int32_t batch, const double* const* A, const int64_t* m,
                         const int64_t* n, const int64_t* lda, const int32_t* precision,
                         const uint64_t* seeds, double* const* Q, const int64_t* ldq,
                         double* const* R, const int64_t* ldr,
                         void* stream, mrcqr_info* infos_dev);

/* ---------------------------------------------------------------------
 * Individual steps of the path (same kernels as mrcqr_factor).
 * ------------------------------------------------------------------- */

/* Algorithm 2, Stage 1, first step: draw S (s distinct row indices of
 * [0, m), sorted ascending, int32 S_dev[s]) and, if D_dev is not NULL, the
 * Rademacher signs as int8 D_dev[m] in {+1, -1}. */
int mrcqr_draw(uint64_t seed, int64_t m, int64_t s, int32_t* S_dev, int8_t* D_dev,
               void* stream);

/* Stage 1 DiagMult + transform + Select: Y (s x n, ldy, float64 storage)
 * = gamma .* (C_p(S) * fl_p(D A)), C_p the DCT-II rows S rounded to p,
 * gamma_0 = sqrt(1/s), gamma_k = sqrt(2/s); for p != FP64 the products are
 * summed in float32 and Y holds float32 values. D is drawn from `seed`, S
 * is read from S_dev (from mrcqr_draw). precision must not be AUTO.
 * Needs mrcqr_sketch_workspace_bytes(m, n, s, precision) bytes of device
 * workspace for the per-row-chunk partial sums. */
size_t mrcqr_sketch_workspace_bytes(int64_t m, int64_t n, int64_t s, int precision);
int mrcqr_sketch(const double* A, int64_t m, int64_t n, int64_t lda,
                 const int32_t* S_dev, int64_t s, uint64_t seed, int precision,
                 double* Y, int64_t ldy, void* workspace, size_t workspace_bytes,
                 void* stream);
/* The same with transform flags: MRCQR_SKETCH_RFFT takes the real parts of
 * the DFT bins S_dev (values in [0, floor(m/2)], from mrcqr_draw with
 * floor(m/2) + 1 in place of m) scaled by sqrt(s/m). */
int mrcqr_sketch_ex(const double* A, int64_t m, int64_t n, int64_t lda,
                    const int32_t* S_dev, int64_t s, uint64_t seed, int precision, int flags,
                    double* Y, int64_t ldy, void* workspace, size_t workspace_bytes,
                    void* stream);

/* Stage 1 SketchQR: Householder thin QR of Y (s x n) in float32
 * (qr_precision = FP32) or float64 (FP64); Rs (n x n, upper, diag > 0,
 * float64) and, if kappa_dev != NULL, the ICE estimate of kappa_2(Rs). */
int mrcqr_sketch_qr(const double* Y, int64_t s, int64_t n, int64_t ldy, int qr_precision,
                    double* Rs, int64_t ldr, double* kappa_dev, void* stream);

/* Stage 2 triangular solve X = A R^{-1} (R upper, n x n), by block
 * substitution over column blocks of 16: X_J = (A_J - X_{<J} R_{<J,J})
 * inv(R_JJ). No inverse of R is formed (Section "Algorithm Description");
 * only the 16 x 16 diagonal blocks are inverted (by substitution), as GPU
 * triangular solves do. For n > 128 the columns are taken in panels of
 * 128: X_P = (A_P - X_{<P} R_{<P,P}) R_PP^{-1}, the update written into X_P
 * and solved there. X must not overlap A. Needs
 * mrcqr_trsm_workspace_bytes(n) bytes of device workspace (R staged in
 * operand order; about 75 KB at n = 128). */
size_t mrcqr_trsm_workspace_bytes(int64_t n);
int mrcqr_trsm(const double* A, int64_t m, int64_t n, int64_t lda,
               const double* R, int64_t ldr, double* X, int64_t ldx,
               void* workspace, size_t workspace_bytes, void* stream);

/* Algorithm 1 step 1: G = B^T B (n x n, both triangles written). Needs
 * mrcqr_gram_workspace_bytes(m, n) bytes of device workspace (per-row-chunk
 * partial sums, summed in a fixed order; for n > 128 also those of the
 * 128 x 128 blocks above the diagonal). */
size_t mrcqr_gram_workspace_bytes(int64_t m, int64_t n);
int mrcqr_gram(const double* B, int64_t m, int64_t n, int64_t ldb,
               double* G, int64_t ldg, void* workspace, size_t workspace_bytes,
               void* stream);

/* Algorithm 1 step 2: G = Rc^T Rc, Rc upper (lower triangle zeroed).
 * fail_dev (int32, may be NULL) receives -1 or the first failing pivot;
 * kappa_dev (may be NULL) the ICE estimate of kappa_2(Rc). */
int mrcqr_cholesky(const double* G, int64_t n, int64_t ldg, double* Rc, int64_t ldr,
                   int32_t* fail_dev, double* kappa_dev, void* stream);

/* Algorithm 1 step 3, first half: X = R^{-1} for an upper-triangular
 * n x n R (n <= 512) by column-wise back substitution, x_i = (e_j -
 * sum_{k>i} r_ik x_k)_i / r_ii. Only the upper triangle of R is read; the
 * strict lower triangle of X is written as zeros. X must not overlap R. A
 * zero or non-finite diagonal entry gives non-finite columns (no status;
 * in the factorization the Cholesky status covers it). Meant for the
 * well-conditioned Rc: the error of X grows like n u kappa(R). */
int mrcqr_tri_inverse(const double* R, int64_t n, int64_t ldr, double* X, int64_t ldx, void* stream);

/* Algorithm 1 step 3, second half: Q = B X for B (m x n) and an
 * upper-triangular X (n x n, only its upper triangle is read; X = Rc^{-1}
 * from mrcqr_tri_inverse in the factorization). Q must not overlap B. No
 * workspace. */
int mrcqr_form_q(const double* B, int64_t m, int64_t n, int64_t ldb, const double* X, int64_t ldx,
                 double* Q, int64_t ldq, void* stream);

/* Stage 3: R = R2 R1 for upper-triangular n x n factors (n <= 512). */
int mrcqr_trmm(const double* R2, int64_t ld2, const double* R1, int64_t ld1,
               int64_t n, double* R, int64_t ldr, void* stream);

/* ICE condition estimate of an upper-triangular n x n matrix. */
int mrcqr_condest(const double* R, int64_t n, int64_t ldr, double* kappa_dev, void* stream);

/* Power-step part of the posterior estimate (Section "Adaptive Precision
 * Selection", rerun rule): kappa_dev receives sigma_max(R) sigma_max(X)
 * estimated by 12 power steps on R^T R and X^T X from the normalized
 * all-ones vector, for an upper-triangular n x n R (n <= 512) and X =
 * R^{-1} (from mrcqr_tri_inverse), both with leading dimension ld. A lower
 * bound on kappa_2(R); +inf if a value is not finite.
 * workspace: device scratch of mrcqr_posterior_workspace_bytes(n) bytes
 * (zero for n <= 128, where it may be NULL; for 128 < n <= 512 the power
 * vectors, and MRCQR_ERR_WORKSPACE when it is NULL). Owned by the caller,
 * not used after the stream reaches the end of the call. */
size_t mrcqr_posterior_workspace_bytes(int64_t n);
int mrcqr_posterior_kappa(const double* R, const double* X, int64_t n, int64_t ld, double* kappa_dev,
                          void* workspace, void* stream);

/* The two other condition estimators of Section "Adaptive Precision
 * Selection" (for comparison with the ICE estimate the policy uses).
 *
 * Block 1-norm estimator (Higham and Tisseur 2000, Algorithm 2.4; t = 2
 * columns, at most 5 iterations, random +-1 columns from the counter-based
 * generator of `seed`, stream 3). With G == NULL: kappa_dev receives
 * ||R||_1 times the estimate of ||R^{-1}||_1 for an upper-triangular n x n
 * R (e.g. Rs). With G != NULL (n x n symmetric A^T A, R its Cholesky factor):
 * kappa_dev receives sqrt(n ||G||_1 est ||G^{-1}||_1), the paper's bound
 * kappa_2(A)^2 <= n ||A^T A||_1 ||(A^T A)^{-1}||_1. Both matrices share the
 * leading dimension ld; n <= 128. One wave; the estimate of the inverse's
 * norm is a lower bound (usually within a factor 3). */
int mrcqr_condest_1norm(const double* R, const double* G, int64_t n, int64_t ld, uint64_t seed,
                        double* kappa_dev, void* stream);

/* CholQR probe: one pass of Algorithm 1 on A (m x n, lda), then
 * kappa_dev = sqrt(q / (u (1 + q))) with u = 2^-53 and q = ||I - Q^T Q||_2
 * estimated by 12 power steps (a lower estimate, so the bound stays a lower
 * bound on kappa_2(A)); +inf when the pass breaks down (the Gram matrix is
 * not numerically positive definite: kappa_2(A) beyond about 1e8). Needs
 * mrcqr_cholqr_probe_workspace_bytes(m, n) bytes of device workspace (Q and
 * small terms, about m n 8 bytes). */
size_t mrcqr_cholqr_probe_workspace_bytes(int64_t m, int64_t n);
int mrcqr_cholqr_probe(const double* A, int64_t m, int64_t n, int64_t lda, void* workspace,
                       size_t workspace_bytes, double* kappa_dev, void* stream);

const char* mrcqr_status_string(int status);
/* Library version as major * 10000 + minor * 100 + patch. */
int mrcqr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MRCQR_H */
