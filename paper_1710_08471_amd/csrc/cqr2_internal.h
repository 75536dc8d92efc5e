// Internal launch interface between the C ABI (cqr2_api.hip) and the kernels
// (cqr2_kernels.hip).  Not installed; no torch types anywhere.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace cqr2 {

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
hipError_t launch_gram_partials(const GramPlan& p, const double* A, int64_t m, int n, int64_t lda,
                                double* partials, const int32_t* info, hipStream_t s);
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

// ---- R = R2 R1 -------------------------------------------------------------
hipError_t launch_upper_product(const double* R2, const double* R1, int64_t ldin, double* R, int64_t ldr,
                                int n, const int32_t* info, int32_t* user_info, hipStream_t s);

// ---- small helpers ---------------------------------------------------------
hipError_t launch_set_info(int32_t* info, int32_t value, hipStream_t s);

}  // namespace cqr2
