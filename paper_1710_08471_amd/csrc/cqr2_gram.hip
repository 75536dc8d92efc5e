// Gram matrix W = AᵀA for n <= 128 (the Syrk of the paper's preliminaries;
// Algorithm 4 step 1), FP64, with fixed-order reductions (no FP atomics):
// bit-reproducible for a given (m, n, lda).
#include "cqr2_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#include "gram_dev.h"

namespace cqr2 {

constexpr int kGramSplits = 256;  // workgroups along m for large m (one per MI355X CU)

// reset_info: this is the first kernel of a factorization -- no earlier
// phase can have failed, and workgroup 0 clears the info word for the kernels
// after it (no workgroup of this kernel reads it).
template <int NG, int NW>
__global__ __launch_bounds__(NW * 64) void k_gram_partials(const double* __restrict__ A, int64_t m, int n,
                                                           int64_t lda, int64_t stages, int64_t spw,
                                                           double* __restrict__ partials, int32_t* info,
                                                           int reset_info) {
  __shared__ double lds[2 * GramStage<NG, NW>::kBuf];
  if (reset_info) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *info = 0;
  } else if (info != nullptr && *info != 0) {
    return;
  }
  constexpr int nblk = NG * (NG + 1) / 2;
  const int64_t st0 = (int64_t)blockIdx.x * spw;
  const int64_t st1 = st0 + spw < stages ? st0 + spw : stages;
  double* out = partials + (int64_t)blockIdx.x * nblk * 16;
  gram_block<NG, NW>(A, m, n, lda, st0, st1, lds, out);
}

// Fixed-order sum of the per-workgroup partial Grams: 8 threads per entry each
// add a contiguous range of partials in order, then the 8 results are added in
// order.  Writes the lower triangle and its mirror.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ part, int splits, int nblk, int n,
                                                     double* __restrict__ W, int64_t ldw,
                                                     const int32_t* __restrict__ info) {
  __shared__ double red[8][32];
  if (info != nullptr && *info != 0) return;
  const int lane = threadIdx.x & 31;
  const int sub = threadIdx.x >> 5;
  const int total = nblk * 16;
  const int e = blockIdx.x * 32 + lane;
  double v = 0.0;
  if (e < total) {
    const int s0 = (splits * sub) / 8, s1 = (splits * (sub + 1)) / 8;
    // in split order; the loads go out eight at a time
    int s = s0;
    for (; s + 8 <= s1; s += 8) {
      double x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) x[j] = part[(int64_t)(s + j) * total + e];
#pragma unroll
      for (int j = 0; j < 8; ++j) v += x[j];
    }
    for (; s < s1; ++s) v += part[(int64_t)s * total + e];
  }
  red[sub][lane] = v;
  __syncthreads();
  if (sub == 0 && e < total) {
    double t = red[0][lane];
#pragma unroll
    for (int k = 1; k < 8; ++k) t += red[k][lane];
    const int b = e >> 4, ij = e & 15;
    int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > b) --I;
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    const int J = b - I * (I + 1) / 2;
    const int row = 4 * I + (ij >> 2), col = 4 * J + (ij & 3);
    if (row >= col && row < n) {
      W[row + (int64_t)col * ldw] = t;
      W[col + (int64_t)row * ldw] = t;
    }
  }
}

static int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// The split count depends only on (m, n) -- never on the device -- so the
// summation order, and with it every result bit, is the same on any GPU.
GramPlan plan_gram(int64_t m, int64_t n) {
  GramPlan p{};
  const int groups = (int)((n + 3) / 4);
  p.ng = pow2_at_least(groups < 1 ? 1 : groups);
  p.nw = p.ng >= 16 ? 8 : (p.ng >= 2 ? p.ng / 2 : 1);
  p.nblk = p.ng * (p.ng + 1) / 2;
  p.stages = (m + kStageRows - 1) / kStageRows;
  if (p.stages < 1) p.stages = 1;
  const int64_t target = kGramSplits;
  // Small problems: do not spread fewer than 4 stages per workgroup.
  int64_t s = p.stages / 4;
  if (s < 1) s = 1;
  if (s > target) s = target;
  p.stages_per_wg = (p.stages + s - 1) / s;
  p.splits = (int)((p.stages + p.stages_per_wg - 1) / p.stages_per_wg);
  p.partial_bytes = (size_t)p.splits * p.nblk * 16 * sizeof(double);
  return p;
}

hipError_t launch_gram_partials(const GramPlan& p, const double* A, int64_t m, int n, int64_t lda,
                                double* partials, const int32_t* info, hipStream_t s, int32_t* reset_info) {
  dim3 grid(p.splits);
#define CQR2_GRAM_CASE(NGV, NWV)                                                                     \
  case NGV:                                                                                          \
    hipLaunchKernelGGL((k_gram_partials<NGV, NWV>), grid, dim3(NWV * 64), 0, s, A, m, n, lda,        \
                       p.stages, p.stages_per_wg, partials,                                          \
                       reset_info != nullptr ? reset_info : const_cast<int32_t*>(info),              \
                       reset_info != nullptr ? 1 : 0);                                               \
    break;
  switch (p.ng) {
    CQR2_GRAM_CASE(1, 1)
    CQR2_GRAM_CASE(2, 1)
    CQR2_GRAM_CASE(4, 2)
    CQR2_GRAM_CASE(8, 4)
    CQR2_GRAM_CASE(16, 8)
    CQR2_GRAM_CASE(32, 8)
    default: return hipErrorInvalidValue;
  }
#undef CQR2_GRAM_CASE
  return hipGetLastError();
}

hipError_t launch_gram_reduce(const GramPlan& p, const double* partials, int n, double* W, int64_t ldw,
                              const int32_t* info, hipStream_t s) {
  const int total = p.nblk * 16;
  dim3 grid((total + 31) / 32);
  hipLaunchKernelGGL(k_gram_reduce, grid, dim3(256), 0, s, partials, p.splits, p.nblk, n, W, ldw, info);
  return hipGetLastError();
}

}  // namespace cqr2
