// Internal launch interface between the C ABI (cqr2_api.hip, cqr2_serve.hip)
// and the kernels (cqr2_gram.hip, cqr2_cholinv.hip, cqr2_apply.hip,
// cqr2_gemm.hip, cqr2_wide.hip, cqr2_stream16.hip, cqr2_step.hip, cqr2_driver.hip).
// Not installed; no torch types anywhere.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace cqr2 {

// Planning never depends on the device: splits and workspace layouts are a
// function of the problem shape alone, so results are bit-identical on any GPU.
constexpr int kPlanCUs = 256;

// Optional per-kernel-class timing around launches (set by the C ABI layer).
struct TimerHook {
  void (*b)(int, hipStream_t) = nullptr;
  void (*e)(int, hipStream_t) = nullptr;
  void begin(int c, hipStream_t s) const {
    if (b) b(c, s);
  }
  void end(int c, hipStream_t s) const {
    if (e) e(c, s);
  }
};

// ---- Gram (Syrk) -----------------------------------------------------------
struct GramPlan {
  int ng;        // 4-column groups the kernel instance covers (power of two, >= ceil(n/4))
  int nw;        // waves per workgroup
  int nblk;      // 4x4 blocks in the lower block triangle = ng*(ng+1)/2
  int splits;    // workgroups along m (split-K)
  int64_t stages;          // 64-row stages = ceil(m/64)
  int64_t stages_per_wg;   // contiguous stages per workgroup
  size_t partial_bytes;    // splits * nblk * 16 * 8
};
GramPlan plan_gram(int64_t m, int64_t n);

// Partial Grams of A (m x n, lda) into `partials` (plan.partial_bytes).
// reset_info != nullptr: the first kernel of a factorization; it clears
// *reset_info (and reads no info word).
hipError_t launch_gram_partials(const GramPlan& p, const double* A, int64_t m, int n, int64_t lda,
                                double* partials, const int32_t* info, hipStream_t s,
                                int32_t* reset_info = nullptr);
// Fixed-order sum of the partials into the full symmetric W (n x n, ldw).
hipError_t launch_gram_reduce(const GramPlan& p, const double* partials, int n, double* W, int64_t ldw,
                              const int32_t* info, hipStream_t s);

// ---- CholInv ---------------------------------------------------------------
// Padded order used by the triangular-inverse consumers: 32, 64 or 128.
int padded_order(int64_t n);
// W (n x n, ldw; lower triangle read) -> R = Lᵀ (col-major, ldr), optional
// Rinv = Yᵀ (col-major, ldri), optional Upad (row-major np x np, upper = R^{-1},
// identity padding).  info: device word; a nonzero value on entry means skip
// (outputs NaN); on breakdown writes info_offset + j.
hipError_t launch_cholinv(const double* W, int64_t ldw, int n, double* R, int64_t ldr, double* Rinv,
                          int64_t ldri, double* Upad, int np, int32_t* info, int info_offset,
                          hipStream_t s);


// ---- Q = A U ---------------------------------------------------------------
// U upper triangular n x n, element (i, j) at U[i*urs + j*ucs] (only i <= j < n
// is read).  Q may alias A exactly (in place).
hipError_t launch_apply_rinv(const double* A, int64_t m, int n, int64_t lda, const double* U, int64_t urs,
                             int64_t ucs, double* Q, int64_t ldq, const int32_t* info, int num_cus, hipStream_t s);

// ---- 64 < n <= 128 on MFMA 16x16x4 (cqr2_stream16.hip) ----------------------
// Row stages split over up to 256 workgroups; partial Grams are 36 lower
// 16 x 16 tiles per workgroup.  U: the padded 128 x 128 row-major image of
// R^{-1} that launch_cholinv writes (np = 128).
struct Stream16Plan {
  int64_t stages = 0, stages_per_wg = 0;
  int splits = 0;
  size_t partial_bytes = 0;
};
Stream16Plan plan_stream16(int64_t m);
// Partial Grams of A; reset_info as launch_gram_partials.
hipError_t launch_stream16_gram(const Stream16Plan& p, const double* A, int64_t m, int n, int64_t lda,
                                double* partials, const int32_t* info, hipStream_t s, int32_t* reset_info = nullptr);
// Q = A U; Q may equal A (in place, ldq == lda).
hipError_t launch_stream16_apply(const Stream16Plan& p, const double* A, int64_t m, int n, int64_t lda,
                                 const double* Upad, double* Q, int64_t ldq, const int32_t* info, hipStream_t s);
// Q = A U and the partial Grams of the stored Q; Q may equal A.
hipError_t launch_stream16_apply_gram(const Stream16Plan& p, const double* A, int64_t m, int n, int64_t lda,
                                      const double* Upad, double* Q, int64_t ldq, double* partials,
                                      const int32_t* info, hipStream_t s);
// Q = A U for n <= 256, U given as its zero-padded row-major upper image
// (ld 256, upper_image_ld).  a_f32: A is FP32 (widened exactly), FP64
// arithmetic into an FP64 Q; f32_math: FP64 A and U rounded to FP32, FP32
// products and sums into an FP32 Q; neither: FP64.  Q may equal A (same type).
hipError_t launch_apply256(int a_f32, int f32_math, const void* A, int64_t m, int n, int64_t lda,
                           const double* Uimg, void* Q, int64_t ldq, const int32_t* info, hipStream_t s);
// The same for n <= 128 (Uimg: the 256-wide image; 128-column kernel, four waves).
hipError_t launch_apply128(int a_f32, int f32_math, const void* A, int64_t m, int n, int64_t lda,
                           const double* Uimg, void* Q, int64_t ldq, const int32_t* info, hipStream_t s);
// Fixed-order sum of the partials into the symmetric W (n x n, ldw).
hipError_t launch_stream16_reduce(const Stream16Plan& p, const double* partials, int n, double* W, int64_t ldw,
                                  const int32_t* info, hipStream_t s);

// ---- general FP64 GEMM: C = alpha op(A) op(B) + beta C ----------------------
// Triangle flags are semantic: entries outside a declared triangle of A or B
// are treated as zero and never read.
enum GemmFlags {
  GEMM_A_LOWER = 1,  // op(A)(i, k) == 0 for k > i
  GEMM_A_UPPER = 2,  // op(A)(i, k) == 0 for k < i
  GEMM_B_LOWER = 4,  // op(B)(k, j) == 0 for k < j
  GEMM_B_UPPER = 8,  // op(B)(k, j) == 0 for k > j
  GEMM_C_LOWER = 16, // only C(i, j), i >= j, is computed and written
  GEMM_C_UPPER = 32, // only C(i, j), i <= j
};
// Reduction splits for a problem shape (1 = no split).
int gemm_pick_splits(int64_t M, int64_t N, int64_t K, int num_cus);
size_t gemm_workspace_bytes(int64_t M, int64_t N, int splits);
// splits > 1 needs work >= gemm_workspace_bytes(M, N, splits).
hipError_t launch_gemm(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                       int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int flags,
                       int splits, double* work, const int32_t* info, hipStream_t s);

// Same with FP32 inputs (exactly widened to FP64; a_f32 / b_f32 select float).
hipError_t launch_gemm_in32(int a_f32, int b_f32, int transA, int transB, int64_t M, int64_t N, int64_t K,
                            double alpha, const void* A, int64_t lda, const void* B, int64_t ldb, double beta,
                            double* C, int64_t ldc, int flags, int splits, double* work, const int32_t* info,
                            hipStream_t s);
// C(float) = op(fl32(A)) op(fl32(B)) with FP32 products and sums (no split).
hipError_t launch_gemm_f32(int transA, int transB, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                           const double* B, int64_t ldb, float* C, int64_t ldc, int flags, const int32_t* info,
                           hipStream_t s);

// ---- tall-skinny kernels for 128 < n <= 256 --------------------------------
constexpr int64_t kWideMaxN = 256;
struct WideGramPlan {
  int64_t stages = 0, stages_per_wg = 0;  // 32-row stages
  int splits = 0, ntiles = 0;             // lower 16 x 16 tiles per split
  size_t partial_bytes = 0;
};
// n <= 128 takes the 128-column kernel (36 tiles, up to 512 splits).
WideGramPlan plan_gram_wide(int64_t m, int64_t n);
// Lower triangle of W = AᵀA (n <= 256); A is FP64, or FP32 when a_f32.
hipError_t launch_gram_wide(const WideGramPlan& p, int a_f32, const void* A, int64_t m, int n, int64_t lda,
                            double* partials, double* W, int64_t ldw, const int32_t* info, hipStream_t s);
// Zero-padded row-major image of the upper triangle of X (n x n, column-major,
// ldx): the form of U the tall kernels read; upper_image_ld(n) = n rounded up
// to 256 is both its leading dimension and its row count.
int64_t upper_image_ld(int64_t n);
inline size_t upper_image_bytes(int64_t n) {
  const size_t ld = (size_t)((n + 255) / 256 * 256);
  return ld * ld * sizeof(double);
}
hipError_t launch_upper_image(const double* X, int64_t ldx, int n, double* T, hipStream_t s);
// R = X Y for upper-triangular X, Y (n x n): X column-major (ldx, exact zeros
// below its diagonal), Y as its upper image (launch_upper_image).  Writes R's
// upper triangle (entries below the diagonal are left alone or written as 0);
// part: upper_seg_partial_bytes(n) of scratch.
size_t upper_seg_partial_bytes(int64_t n);
hipError_t launch_upper_seg(const double* X, int n, int64_t ldx, const double* Yimg, double* R, int64_t ldr,
                            double* part, const int32_t* info, hipStream_t s);
// Q = A U (U given as its upper image); A FP64 or FP32 (a_f32), FP64
// arithmetic.  Reads rows of A across 256-column tiles: not in place for n > 256.
hipError_t launch_tall_gemm(int a_f32, const void* A, int64_t m, int n, int64_t lda, const double* Uimg, double* Q,
                            int64_t ldq, const int32_t* info, hipStream_t s);
// Q(float) = fl32(A) fl32(U) with FP32 products and sums.
hipError_t launch_tall_gemm_f32(const double* A, int64_t m, int n, int64_t lda, const double* Uimg, float* Q,
                                int64_t ldq, const int32_t* info, hipStream_t s);

// ---- Gram for n > 256 by 128 x 128 tiles --------------------------------------
struct SyrkPlan {
  int npairs = 0, splits = 0;             // lower 128 x 256 tiles, row splits
  int64_t stages = 0, stages_per_wg = 0;  // 16-row chunks
  size_t partial_bytes = 0;
};
SyrkPlan plan_syrk(int64_t m, int64_t n);
// Lower triangle of W = AᵀA (any n; A FP64, or FP32 when a_f32, widened exactly).
hipError_t launch_syrk(const SyrkPlan& p, int a_f32, const void* A, int64_t m, int n, int64_t lda, double* partials,
                       double* W, int64_t ldw, const int32_t* info, hipStream_t s);
// W(i, j) += alpha (AᵀA)(i, j) for j <= i < n, A m x n (lda), in one launch
// of 128 x 256 tiles (no partials; m is the whole reduction, meant for
// m <= a few hundred).  skip_first_block_row leaves rows 0..127 of W alone.
hipError_t launch_syrk_update(const double* A, int64_t m, int n, int64_t lda, double alpha, double* W, int64_t ldw,
                              int skip_first_block_row, const int32_t* info, hipStream_t s);

// ---- recursive CholInv and the n > 128 driver --------------------------------
int64_t cholinv_split(int64_t n);
size_t cholinv_rec_workspace(int64_t n);
// W (n x n, ldw, lower read, trailing blocks overwritten) -> R, Rinv upper.
// depth > 0: the top `depth` levels skip the off-diagonal inverse block, so
// Rinv holds only the inverses of the inverse_blocks(n, depth) diagonal
// blocks (zero elsewhere), and R12 is formed by block substitution.
hipError_t cholinv_recursive(double* W, int64_t ldw, int64_t n, double* R, int64_t ldr, double* Rinv, int64_t ldri,
                             char* work, int32_t* info, int info_offset, hipStream_t s, int depth = 0);
// R = triu(P), or NaN after a breakdown; copies the info word to user_info.
hipError_t launch_finalize_r(const double* P, int64_t ldp, double* R, int64_t ldr, int64_t n, const int32_t* info,
                             int32_t* user_info, hipStream_t s);
// R = triu(X Y) for upper-triangular n x n X, Y (ld n, n <= 128), NaN after a
// breakdown, info copied to user_info: the last step of Algorithm 5 in one
// launch.
hipError_t launch_upper_product_final(const double* X, const double* Y, int64_t n, double* R, int64_t ldr,
                                      const int32_t* info, int32_t* user_info, hipStream_t s);

// W(j, i) = W(i, j) for i > j.
hipError_t launch_mirror_lower(double* W, int64_t ldw, int64_t n, hipStream_t s);

struct GeneralPlan {
  size_t off_info = 0, off_w = 0, off_r1 = 0, off_ri1 = 0, off_r2 = 0, off_ri2 = 0, off_p = 0, off_uimg = 0,
         off_scratch = 0, off_q1 = 0, off_t = 0;
  size_t total = 0;
};
// mixed: pass 1's Q1 = A R1^-1 is formed with FP32 products and sums and kept
// as an FP32 m x n block in the workspace (everything else stays FP64).
// depth > 0: the partial inverse (inverse_blocks); the plan then holds an
// m x (widest block) FP64 buffer at off_t for the block substitution.
GeneralPlan plan_general(int64_t m, int64_t n, bool mixed, int depth = 0);
hipError_t factor_general(const double* A, int64_t m, int64_t n, int64_t lda, double* Q, int64_t ldq, double* R,
                          int64_t ldr, char* ws, const GeneralPlan& p, bool mixed, int32_t* d_info, hipStream_t s,
                          const TimerHook& th, bool shifted = false, int depth = 0);
// Diagonal blocks [start, stop) whose inverses the CholInv recursion forms
// when the top `depth` levels skip the off-diagonal inverse block (the
// recursion's own split points; depth 0 or n <= 128: one block).
struct Block {
  int64_t c0, c1;
};
int inverse_blocks(int64_t n, int depth, Block* out, int cap);
// Adds s = 11 (m n + n (n + 1)) 2^-53 trace(W) to the diagonal of W (shifted CholeskyQR).
hipError_t launch_shift_diag(double* W, int64_t ldw, int64_t n, int64_t m, const int32_t* info, hipStream_t s);

// ---- multi-problem step (batched and serving paths, n <= 256) -------------
// One launch advances every listed problem by one phase of CholeskyQR2.
// n <= 128 (six phases):
//   0 Gram(A) partials, 1 CholInv(sum of partials) -> R1, U1 = R1^-1,
//   2 Q = A U1, 3 Gram(Q) partials, 4 CholInv -> R2, U2, 5 Q = Q U2 and R = R2 R1.
// 128 < n <= 256 (eight phases):
//   0 Gram(A) partials, 1 their sum W, 2 CholInv(W) -> R1, U1, 3 Q = A U1,
//   4 Gram(Q) partials, 5 their sum, 6 CholInv -> R2, U2, 7 Q = Q U2 and
//   R = R2 R1.
// Workgroups are dealt to the problems by the table (task t owns workgroups
// [wg0, wg0 + nwg)); tasks are sorted by wg0.
constexpr int kStepThreads = 512;
constexpr int kStepStages = 64;     // 64-row stages per Gram / Q workgroup, at most (4096 rows)
constexpr int kStepMinStages = 16;  // ... and at least (1024 rows)
constexpr int kStepPhases = 6;
constexpr int kStepMaxN = 256;
constexpr int kStepWidePhases = 8;
constexpr int kStepWideStages = 64;     // 32-row stages per wide Gram / Q workgroup, at most (2048 rows)
constexpr int kStepWideMinStages = 16;  // ... and at least (512 rows)
struct StepTask {
  const double* A;
  int64_t lda;
  double* Q;
  int64_t ldq;
  double* R;
  int64_t ldr;
  int32_t* user_info;  // optional; written in the last phase
  char* ws;            // the problem's workspace (StepLayout)
  int64_t m;
  int32_t n, phase, wg0, nwg;
};
// Workspace of one problem.  n <= 128: the partial Grams in the 4x4-block
// layout, R1, R2 (n x n) and the padded images U1, U2 (np x np, row-major).
// 128 < n <= 256: the partial Grams in the 16x16-tile layout, then 256 x 256
// blocks: W, R1, R2 and R^-1 scratch (column-major, ld 256), U1, U2 (row-major
// images), and one temporary.
struct StepLayout {
  int np = 0, ng = 0, nblk = 0, splits = 0;
  size_t off_info = 0, off_part = 0, off_r1 = 0, off_r2 = 0, off_u1 = 0, off_u2 = 0, total = 0;
  size_t off_w = 0, off_ri = 0, off_t = 0;  // 128 < n <= 256 only
};
StepLayout step_layout(int64_t m, int64_t n);
// Phases of an n-column problem (n <= kStepMaxN).
int step_phases(int64_t n);
// Workgroups of phase `phase` for an m x n problem.
int step_workgroups(int64_t m, int64_t n, int phase);
// Rough duration of one workgroup of phase `phase` of an m x n problem
// (microseconds, measured on MI355X); only the order of these values is used.
double step_wg_cost(int64_t m, int64_t n, int phase);
hipError_t launch_step(const StepTask* d_tasks, int ntasks, int total_wgs, hipStream_t s);

// ---- least squares on a finished factorization ---------------------------
// X = R1^{-1} R2^{-1} Qᵀ B (n x nrhs, ldx).  U1, U2 hold R1^{-1}, R2^{-1} as
// op(U) with leading dimension ldu: utrans = 1 for the row-major padded images
// of the n <= 128 paths, 0 for the column-major inverses of the tiled path.
// work: lstsq_tail_bytes(m, n, nrhs), 256-byte aligned.  X is NaN when *info
// is nonzero.
size_t lstsq_tail_bytes(int64_t m, int64_t n, int64_t nrhs);
hipError_t lstsq_tail(const double* Q, int64_t ldq, const double* B, int64_t ldb, int64_t m, int64_t n,
                      int64_t nrhs, const double* U1, const double* U2, int64_t ldu, int utrans, double* X,
                      int64_t ldx, char* work, const int32_t* info, hipStream_t s);

// ---- small helpers ---------------------------------------------------------
hipError_t launch_set_info(int32_t* info, int32_t value, hipStream_t s);
// X (n x n): upper triangle := NaN if *info != 0 (info must not be null).
hipError_t launch_nan_upper_if_info(double* X, int64_t ldx, int64_t n, const int32_t* info, hipStream_t s);

}  // namespace cqr2
