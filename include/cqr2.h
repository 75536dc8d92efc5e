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
 *    stream has reached that point.  No host synchronization happens inside,
 *    with two exceptions: an entry point that uses the library-cached
 *    workspace (cqr2_factor; cqr2_cholinv, cqr2_apply_rinv for n > 128;
 *    cqr2_apply_rinv_f32) synchronizes the device once when that workspace
 *    has to grow, and the batched call and the server wait for a pinned
 *    task-table staging buffer when the host runs several calls ahead.
 *    The CholInv of n >= 512 (at full inverse depth) fans its bulk products
 *    out to two streams of the library (per device, default priority, not
 *    blocking on the null stream) through events and joins them back into
 *    `stream` before any later work on it; its order on `stream` is kept.
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
 *  - Host threads: entry points may be called from several threads at once;
 *    the library's shared host state (the cached workspace, the timing
 *    records, the batched call's task-table ring) is locked.  The cached
 *    workspace is ONE device buffer per device, shared by every entry point
 *    that uses it: a call holds the lock from the lookup until its launches
 *    are enqueued, so concurrent calls on the same stream are safe, but calls
 *    on different streams would race on its contents -- they must use the
 *    entry points that take a work argument.  A server handle is not locked:
 *    each cqr2_server is used by one thread at a time.
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
/* Plain FP64 CholeskyQR2.  Pass 2's Gram is fused into pass 1's Q1 = A R1^{-1}
 * wherever that pays (64 < n <= 128: one launch forms Q1 and the partial Grams
 * of its stored values); there is no flag for it. */
#define CQR2_FP64 0u
/* Pass 1's Q1 = A R1^{-1} in FP32 arithmetic (A and R1^{-1} rounded to FP32,
 * FP32 MFMA products and sums) with an FP32 Q1 of m*n*4 bytes in the
 * workspace; the Gram matrices, CholInv and all of pass 2 stay FP64, and pass 2
 * factors the stored FP32 Q1 widened exactly.  Orthogonality is recovered by
 * pass 2 (the FP64 gate holds); the residual ||A - QR||/||A|| and R are
 * accurate to the FP32 rounding level only.  Runs the general path at every n
 * (128- or 256-column MFMA 16x16x4 kernels up to n = 256, the tiled kernels
 * above).  Accepted by cqr2_factor_ex / cqr2_workspace_size. */
#define CQR2_MIXED_P1_FP32 1u

/* Shifted CholeskyQR3, the unconditionally stable extension of CholeskyQR2
 * the paper cites (Fukaya et al.): the first CholeskyQR factors W + s I,
 * s = 11 (m n + n (n + 1)) 2^-53 trace(W) (trace W = ||A||_F^2), then
 * CholeskyQR2 of its Q; R = R3 R2 R1.  Stays as accurate as Householder QR far
 * past cond(A) ~ 1e8, where CholeskyQR2's Cholesky breaks down; costs one
 * more pass.  FP64.  Breakdown codes j, n + j, 2 n + j for the three passes.
 * Accepted by cqr2_factor_ex / cqr2_workspace_size. */
#define CQR2_SHIFTED_CQR3 2u

/* Partial inverse (the paper's alternative for 3D-CQR2, tuned in its
 * experiments as InverseDepth): OR'ed onto CQR2_FP64, CQR2_INVERSE_DEPTH(d),
 * 1 <= d <= 8, stops forming the triangular inverse in the top d levels of the
 * CholInv recursion (Algorithm 2's Y21 is skipped there), so R^{-1} is kept
 * only as inverted diagonal blocks; L21 inside the recursion and Q = A R^{-1}
 * are then formed by block substitution, one GEMM pair per block.  The
 * recursion splits at multiples of 128 and stops at n <= 128, so the blocks are
 * at least 128 wide and the flag changes nothing for n <= 128.  FP64 only
 * (not with CQR2_MIXED_P1_FP32 or CQR2_SHIFTED_CQR3).  Accepted by
 * cqr2_factor_ex / cqr2_workspace_size. */
#define CQR2_INVERSE_DEPTH(d) (((uint32_t)(d)) << 8)
#define CQR2_MAX_INVERSE_DEPTH 8

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

/*
 * cqr2_factor_noalloc — cqr2_factor for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  Same arguments, semantics and results (bit for bit) as
 * cqr2_factor, but it allocates nothing: the workspace is a static device
 * array of CQR2_NOALLOC_MAX_WORKSPACE bytes per device, part of the library's
 * code object and held until the process ends.  Every FP64 problem with
 * n <= 128 fits (any m); larger problems fit while cqr2_workspace_size(m, n,
 * CQR2_FP64) <= CQR2_NOALLOC_MAX_WORKSPACE, otherwise the call returns
 * CQR2_ERR_NOALLOC_LIMIT and launches nothing.  The first call with a device
 * current looks up that device's array address (hipGetSymbolAddress).  All
 * calls on one device share its array, which keeps the last call's contents
 * (nothing depends on them): calls that overlap in time on one device -- on
 * different streams, or from threads using different streams -- race on it and
 * must be serialized by the caller (for example, one stream).  No timing
 * records are taken.
 */
#define CQR2_NOALLOC_MAX_WORKSPACE ((size_t)20 << 20)
#define CQR2_ERR_NOALLOC_LIMIT (-103)
int cqr2_factor_noalloc(const double* A, int64_t m, int64_t n, int64_t lda,
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

/* ---- least squares on top of the factorization -----------------------------
 * cqr2_lstsq — X = argmin ||A X - B|| (the least-squares use of QR the
 * paper's Introduction names), FP64: A = QR by CholeskyQR2 (written to Q, R
 * as cqr2_factor_ex does), then X = R^{-1} (Qᵀ B) applied through the explicit
 * triangular inverses of the two passes, R^{-1} = R1^{-1} R2^{-1}.
 *   B: m x nrhs (ldb >= m), read only; X: n x nrhs (ldx >= n).
 *   work: >= cqr2_lstsq_workspace_size(m, n, nrhs) bytes, 256-byte aligned.
 *   d_info: as cqr2_factor_ex; on breakdown X and R are NaN.
 * Argument indices for errors: A=1, m=2, n=3, lda=4, B=5, ldb=6, nrhs=7, X=8,
 * ldx=9, Q=10, ldq=11, R=12, ldr=13, work=14, work_bytes=15, d_info=16.
 */
size_t cqr2_lstsq_workspace_size(int64_t m, int64_t n, int64_t nrhs);
int cqr2_lstsq(const double* A, int64_t m, int64_t n, int64_t lda,
               const double* B, int64_t ldb, int64_t nrhs, double* X, int64_t ldx,
               double* Q, int64_t ldq, double* R, int64_t ldr,
               void* work, size_t work_bytes, int32_t* d_info, void* stream);

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
 * NULL) receives 0 or the 1-based breakdown column; on breakdown the upper
 * triangles of R and Rinv (diagonal included) are NaN and their strictly lower
 * parts 0.  For n > 128 it runs on the library-cached workspace.
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
 * cqr2_apply_rinv_f32 -- the same product in the mixed-precision form's
 * arithmetic (pass 1 of CQR2_MIXED_P1_FP32): Q = fl32(A) fl32(U), both
 * operands rounded to FP32 (nearest even), every product and running sum in
 * FP32 (FP32 MFMA with FP32 accumulation, k ascending in steps of 4), Q
 * stored as FP32.  A: m x n FP64 (lda); U: upper triangular n x n FP64 (ldu,
 * strictly lower part never read); Q: m x n FP32 (ldq >= m, 4-byte aligned),
 * must not overlap A or U.  Runs on the library-cached workspace (the padded
 * image of U).  Argument indices: A=1, m=2, n=3, lda=4, U=5, ldu=6, Q=7,
 * ldq=8.
 */
int cqr2_apply_rinv_f32(const double* A, int64_t m, int64_t n, int64_t lda,
                        const double* U, int64_t ldu, float* Q, int64_t ldq, void* stream);

/*
 * cqr2_upper_product — R = R2 R1 for upper-triangular n x n factors
 * (Algorithm 5, last step).  Column-major, leading dimension ld for all three;
 * R must not overlap R2 or R1.  Strictly lower part of R set to 0.
 */
int cqr2_upper_product(const double* R2, const double* R1, double* R, int64_t n,
                       int64_t ld, void* stream);

/* ---- many problems at once ------------------------------------------------
 * The batched call takes a host array of problems and enqueues their task
 * tables itself; the serving step of the continuous-batching server
 * (cqr2_server_step) is the one-launch step over every admitted request, with
 * the task table built and uploaded by the server, so a caller never writes a
 * device task table.  Each problem's breakdown code goes to its own optional
 * device word (cqr2_problem.d_info) instead of a separate info array.
 *
 * One CholeskyQR2 problem (all pointers device, column-major FP64; same rules
 * as cqr2_factor_ex: m >= n >= 0, lda, ldq >= m, ldr >= n, Q and R must not
 * overlap A or each other).  d_info: optional device word receiving the
 * breakdown code (0, j or n + j), may be NULL.
 */
typedef struct {
  const double* A;
  double* Q;
  double* R;
  int64_t m, n, lda, ldq, ldr;
  int32_t* d_info;
} cqr2_problem;

/* 0 if *p is a valid problem, else the negative code cqr2_factor_ex would
 * return for it (A=-1, m=-2, n=-3, lda=-4, Q=-5, ldq=-6, R=-7, ldr=-8,
 * d_info=-11; CQR2_ERR_UNSUPPORTED for n > CQR2_MAX_N). */
int cqr2_problem_check(const cqr2_problem* p);

/* Bytes of device workspace cqr2_factor_batched needs (0 if any problem is
 * invalid or flags != CQR2_FP64). */
size_t cqr2_batched_workspace_size(const cqr2_problem* probs, int32_t count, uint32_t flags);

/*
 * cqr2_factor_batched — CholeskyQR2 (Algorithm 5, FP64) of `count` independent
 * problems of any shapes, enqueued on `stream`.  probs: host array, read
 * during the call only.  Problems with n <= 256 advance together: launches
 * of one multi-problem kernel, each moving every problem through one phase
 * (Gram, CholInv, Q = A R^-1; twice; R = R2 R1 with the last; six phases for
 * n <= 128, eight for 128 < n <= 256, where the sum of the partial Grams is a
 * phase of its own and CholInv splits W once at 128).  Problems with n > 256
 * run the tiled path one after another on the same stream.  work:
 * >= cqr2_batched_workspace_size bytes, 256-byte aligned, device.  The task
 * tables are staged through library-owned pinned host memory (the call may
 * wait for an earlier call's staging buffer to be consumed).  Results equal
 * those of the same problem run alone through the batched path, bit for bit.
 * Returns 0, -1 (a problem is invalid: see cqr2_problem_check), -2 (count),
 * -3 (work), -4 (work_bytes), -5 (flags) or CQR2_ERR_*.
 */
int cqr2_factor_batched(const cqr2_problem* probs, int32_t count, void* work, size_t work_bytes,
                        uint32_t flags, void* stream);

/* ---- continuous-batching server ------------------------------------------
 * A host-side scheduler over the multi-problem kernel for a stream of
 * requests of uneven m and n.  Each cqr2_server_step admits queued requests
 * (first come, first served) while an active slot is free, the workspace arena
 * has room and the in-flight footprint (bytes of A, Q, R and workspace of
 * every admitted, unfinished request) stays within the budget; then it
 * launches ONE multi-problem kernel that advances every active n <= 256
 * request by one phase, so requests admitted at different times share each
 * launch and a request finishes six (n <= 128) or eight (128 < n <= 256)
 * steps after its admission.  A step first waits (on the host) until at most
 * one of its earlier launches is still pending on the GPU, so each launch
 * carries every request admitted up to then.  Requests with n > 256 run the
 * tiled path on further streams of the server (round
 * robin) as soon as they are admitted, overlapping the steps.  There are one
 * fewer of them than the process's hardware queues (the GPU_MAX_HW_QUEUES
 * environment variable that HIP reads, default 4: three streams), so the
 * step stream keeps a queue of its own.  Apart from that wait, nothing blocks
 * on the GPU.
 * Completion times are HIP event times in milliseconds since the last
 * cqr2_server_clock call.  A, Q and R stay owned by the caller and must stay
 * valid until the request is reported done by cqr2_server_poll.  A (and B) are
 * read in the order of the server's stream: whatever the caller enqueued on
 * that stream before the cqr2_server_step call that admits a request is
 * complete before the request reads its inputs (the large-request streams
 * wait on an event recorded there).
 */
typedef struct cqr2_server cqr2_server;

/* arena_bytes: device workspace pool allocated now; footprint_budget: bytes
 * (0 = no limit beyond the arena); max_active: slots (1..4096); stream: the
 * stream steps run on.  Returns 0 and *out, or a negative argument index. */
int cqr2_server_create(size_t arena_bytes, size_t footprint_budget, int32_t max_active, void* stream,
                       cqr2_server** out);
/* Waits for all work of the server, then frees it. */
int cqr2_server_destroy(cqr2_server* s);
/* Queue a request.  Returns 0, -1 (server), -2 (invalid problem), -3 (n == 0
 * is rejected: nothing to do), or CQR2_ERR_TOO_LARGE if it could never be
 * admitted (workspace above the arena or footprint above the budget). */
int cqr2_server_submit(cqr2_server* s, const cqr2_problem* p, int64_t tag);
/* Queue a least-squares request: the factorization of p (into p->Q, p->R, as
 * cqr2_server_submit) followed, on the GPU, by X = R^{-1} (Qᵀ B) through the
 * two passes' triangular inverses -- what cqr2_lstsq computes, as one served
 * request.  B: m x nrhs (ldb >= m), read only, may alias A; X: n x nrhs
 * (ldx >= n), NaN after a breakdown.  B and X stay owned by the caller until
 * the request is reported done.  Returns 0, -1 (server), -2 (invalid problem
 * or n == 0), -3 (B null, misaligned or overlapping Q or R), -4 (ldb), -5
 * (nrhs < 1), -6 (X null, misaligned or overlapping A, B, Q or R), -7 (ldx),
 * or CQR2_ERR_TOO_LARGE. */
int cqr2_server_submit_lstsq(cqr2_server* s, const cqr2_problem* p, const double* B, int64_t ldb, int64_t nrhs,
                             double* X, int64_t ldx, int64_t tag);
/* Admit and launch one step.  n_active / n_queued (may be NULL): requests in
 * flight and waiting after the step. */
int cqr2_server_step(cqr2_server* s, int32_t* n_active, int32_t* n_queued);
/* Finished requests (their GPU work has completed): up to max_count tags and
 * completion times; *count receives the number written. */
int cqr2_server_poll(cqr2_server* s, int64_t* tags, double* done_ms, int32_t max_count, int32_t* count);
/* Records the reference event (time 0) on the server's stream and waits for it. */
int cqr2_server_clock(cqr2_server* s);

#define CQR2_ERR_TOO_LARGE (-102)

/* Human-readable text for a return code. */
const char* cqr2_status_string(int code);

/* Library version string. */
const char* cqr2_version(void);

/* ---- timing instrumentation (used by the benchmark) ------------------------
 * When enabled, cqr2_factor/_ex record a HIP event pair around each kernel
 * they launch (on the call's stream).  cqr2_timing_read synchronizes on the
 * recorded events and returns, per kernel class, the total milliseconds and
 * launch count since the last reset.  Classes: 0 Gram, 1 Gram reduction,
 * 2 CholInv, 3 pass 1's Q1 = A R1^{-1} (for 64 < n <= 128 the same launch also
 * forms pass 2's partial Grams), 4 pass 2's Q = Q1 R2^{-1} (and the shifted
 * form's later passes), 5 R = R2 R1 with the finalization.
 */
#define CQR2_NUM_TIMERS 6
int cqr2_timing_enable(int enable);
int cqr2_timing_reset(void);
int cqr2_timing_read(double* total_ms, int64_t* launches, int max_classes);

#ifdef __cplusplus
}
#endif

#endif /* CQR2_H */
