/*
 * cqr2.h — C ABI of the MI355X (gfx950) CholeskyQR2 library (libcqr2.so).
 *
 * Computes the reduced QR factorization A = QR of an m x n matrix, m >= n,
 * with Q (m x n) having orthonormal columns and R (n x n) upper triangular
 * with a positive diagonal (unique for full-rank A).  Method: CholeskyQR2,
 * Hutter & Solomonik, "Communication-avoiding CholeskyQR2 for rectangular
 * matrices": Algorithm 4 (CQR: W = Syrk(A); Rᵀ, R^{-T} = CholInv(W);
 * Q = MM(A, R^{-1})) run twice as in Algorithm 5, then R = R2 R1.  CholInv is
 * Algorithm 2 (Cholesky factor and triangular inverse computed together).
 *
 * Conventions for every entry point:
 *  - All matrices are column-major FP64 with leading dimension >= rows.
 *    A, Q, R, work and d_info are DEVICE pointers unless stated otherwise.
 *  - Everything is enqueued on `stream` (a hipStream_t; NULL = legacy default
 *    stream).  Calls return without synchronizing; outputs are valid once the
 *    stream has reached that point.  No host synchronization happens inside.
 *  - Ownership: the caller owns A, Q, R, work and d_info.  A is read-only.
 *    Q and R must not overlap A or each other (checked on address ranges).
 *    The library never frees caller memory.
 *  - Return value: 0 = enqueued.  A negative value -i means argument i is
 *    invalid (LAPACK convention: NULL pointer, m < n, lda < m, ldq < m,
 *    ldr < n, overlapping buffers, workspace too small, misalignment,
 *    unsupported n); nothing is launched then.  CQR2_ERR_HIP means a HIP
 *    call failed.  Host argument checks run before any HIP call.
 *  - Numerical breakdown (the paper assumes symmetric positive definite Gram
 *    matrices; a non-positive or NaN Cholesky pivot) is reported on the
 *    device, LAPACK potrf style: *d_info = j (1-based column) for a failure in
 *    pass 1, n + j for pass 2, 0 on success.  Later phases then skip their
 *    work and Q is unspecified; R is filled with NaN.
 *  - Results are deterministic: the same inputs, sizes and flags give
 *    bit-identical Q and R (fixed reduction orders, no floating-point atomics).
 */
#ifndef CQR2_H
#define CQR2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CQR2_ERR_HIP (-100)
#define CQR2_ERR_UNSUPPORTED (-101)

/* flags */
#define CQR2_FP64 0u
/* Pass 1's Q1 = A R1^{-1} in FP32 arithmetic (A and R1^{-1} rounded to FP32,
 * FP32 MFMA products and sums) with an FP32 Q1 of m*n*4 bytes in the
 * workspace; the Gram matrices, CholInv and all of pass 2 stay FP64, and pass 2
 * factors the stored FP32 Q1 widened exactly.  Orthogonality is recovered by
 * pass 2 (the FP64 gate holds); the residual ||A - QR||/||A|| and R are
 * accurate to the FP32 rounding level only.  Runs the tiled path at every n.
 * Accepted by cqr2_factor_ex / cqr2_workspace_size. */
#define CQR2_MIXED_P1_FP32 1u

/* Largest n accepted (every n x n workspace block is n*n*8 bytes).  Up to
 * n = 128 the tall-skinny kernels run (split-K Gram, one-workgroup CholInv,
 * streaming Q = A R^{-1}); above, the Gram, Q formation and R2 R1 are tiled
 * GEMMs and CholInv is the recursion of Algorithm 2 with a 128 base case. */
#define CQR2_MAX_N 16384

/*
 * cqr2_factor — CholeskyQR2 of A (Algorithm 5), FP64.
 *   A   : m x n, leading dimension lda >= max(1, m); read only.
 *   Q   : m x n output, leading dimension lda (same as A).
 *   R   : n x n output, leading dimension n; upper triangle = R, strictly
 *         lower part set to 0.
 *   stream : hipStream_t to enqueue on.
 * Workspace is allocated by the library on first use per device and size
 * (hipMalloc, outside the enqueued work) and kept until process exit; calls
 * sharing a device share it, so concurrent calls on different streams must
 * use cqr2_factor_ex with their own workspace.  Breakdown: R is set to NaN.
 * Returns 0, a negative argument index, or CQR2_ERR_*.
 */
int cqr2_factor(const double* A, int64_t m, int64_t n, int64_t lda,
                double* Q, double* R, void* stream);

/* Bytes of workspace cqr2_factor_ex needs for (m, n, flags); 0 if unsupported. */
size_t cqr2_workspace_size(int64_t m, int64_t n, uint32_t flags);

/*
 * cqr2_factor_ex — as cqr2_factor with explicit leading dimensions, a
 * caller-provided device workspace (>= cqr2_workspace_size bytes, 256-byte
 * aligned) and an optional device info word (d_info may be NULL).
 * Argument indices for errors: A=1, m=2, n=3, lda=4, Q=5, ldq=6, R=7, ldr=8,
 * work=9, work_bytes=10, d_info=11, flags=12.
 */
int cqr2_factor_ex(const double* A, int64_t m, int64_t n, int64_t lda,
                   double* Q, int64_t ldq, double* R, int64_t ldr,
                   void* work, size_t work_bytes, int32_t* d_info,
                   uint32_t flags, void* stream);

/* ---- the steps of one CholeskyQR pass, exposed individually --------------
 * These are the kernels cqr2_factor chains, with their own argument checks.
 */

/* Workspace bytes of cqr2_gram for (m, n). */
size_t cqr2_gram_workspace_size(int64_t m, int64_t n);

/*
 * cqr2_gram — W = AᵀA (Syrk, paper Section "Preliminaries"; Algorithm 4
 * step 1).  Split over row blocks of A with per-block partial Grams summed
 * in a fixed order (the single-GPU form of Algorithm 6's local Syrk +
 * Allreduce).  W: n x n column-major, ldw >= n; the full symmetric matrix is
 * written.  work: >= cqr2_gram_workspace_size(m, n) bytes.
 */
int cqr2_gram(const double* A, int64_t m, int64_t n, int64_t lda,
              double* W, int64_t ldw, void* work, size_t work_bytes, void* stream);

/*
 * cqr2_cholinv — [L, Y] = CholInv(W) (Algorithm 2), returned as the
 * CholeskyQR factors R = Lᵀ and Rinv = Yᵀ = R^{-1} (both n x n upper
 * triangular, column-major, leading dimension ldr; strictly lower parts 0).
 * Reads only the lower triangle of W (n x n, ldw).  d_info (device, may be
 * NULL) receives 0 or the 1-based breakdown column; on breakdown R and Rinv
 * are NaN.
 */
int cqr2_cholinv(const double* W, int64_t n, int64_t ldw,
                 double* R, double* Rinv, int64_t ldr, int32_t* d_info, void* stream);

/*
 * cqr2_apply_rinv — Q = A U for upper-triangular U (n x n, ldu), i.e. the
 * MM(A, R^{-1}) of Algorithm 4 step 3.  Q may equal A (in place, ldq == lda);
 * otherwise they must not overlap.
 */
int cqr2_apply_rinv(const double* A, int64_t m, int64_t n, int64_t lda,
                    const double* U, int64_t ldu, double* Q, int64_t ldq, void* stream);

/*
 * cqr2_upper_product — R = R2 R1 for upper-triangular n x n factors
 * (Algorithm 5, last step).  Column-major, leading dimension ld for all three;
 * R must not overlap R2 or R1.  Strictly lower part of R set to 0.
 */
int cqr2_upper_product(const double* R2, const double* R1, double* R, int64_t n,
                       int64_t ld, void* stream);

/* Human-readable text for a return code. */
const char* cqr2_status_string(int code);

/* Library version string. */
const char* cqr2_version(void);

/* ---- timing instrumentation (used by the benchmark) ------------------------
 * When enabled, cqr2_factor/_ex record a HIP event pair around each kernel
 * they launch (on the call's stream).  cqr2_timing_read synchronizes on the
 * recorded events and returns, per kernel class, the total milliseconds and
 * launch count since the last reset.  Classes: 0 gram, 1 gram-reduce,
 * 2 cholinv, 3 apply-rinv (pass 1), 4 apply-rinv (pass 2), 5 upper-product.
 */
#define CQR2_NUM_TIMERS 6
int cqr2_timing_enable(int enable);
int cqr2_timing_reset(void);
int cqr2_timing_read(double* total_ms, int64_t* launches, int max_classes);

#ifdef __cplusplus
}
#endif

#endif /* CQR2_H */
