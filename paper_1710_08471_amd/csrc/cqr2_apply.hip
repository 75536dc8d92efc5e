// Q = A R^{-1} for n <= 128 (Algorithm 4 step 3: MM with the explicit
// upper-triangular inverse), FP64, streaming A once and writing Q once.
#include "cqr2_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#include "apply_dev.h"

namespace cqr2 {

template <int NT>
__global__ __launch_bounds__(64 * ApplyLayout<NT / 4>::W, 1) void k_apply_rinv(
    const double* A, int64_t m, int n, int64_t lda, const double* __restrict__ U, int64_t urs, int64_t ucs,
    double* Q, int64_t ldq, const int32_t* __restrict__ info, int nwg) {
  // nwg == gridDim.x.  Each workgroup takes a contiguous range of stages
  // (measured slightly faster than dealing them round-robin: the workgroups'
  // concurrent accesses then spread over the whole of A and Q), walked from
  // its end: the Gram before this kernel reads the same ranges upwards, so the
  // rows it read last come first.
  __shared__ double sa[2 * NT * kApplyRows];
  if (info != nullptr && *info != 0) return;
  const int64_t stages = (m + kApplyRows - 1) / kApplyRows;
  const int64_t per = (stages + nwg - 1) / nwg;
  const int64_t s0 = (int64_t)blockIdx.x * per;
  const int64_t s1 = s0 + per < stages ? s0 + per : stages;
  apply_block<NT>(A, m, n, lda, U, urs, ucs, Q, ldq, s0, s1, true, sa);
}

hipError_t launch_apply_rinv(const double* A, int64_t m, int n, int64_t lda, const double* U, int64_t urs,
                             int64_t ucs, double* Q, int64_t ldq, const int32_t* info, int num_cus, hipStream_t s) {
  const int nt = padded_order(n);
  const int64_t stages = (m + kApplyRows - 1) / kApplyRows;
  int64_t wgs = num_cus > 0 ? num_cus : 256;
  if (wgs > stages) wgs = stages;
  if (wgs < 1) wgs = 1;
  dim3 grid((unsigned)wgs);
  switch (nt) {
    case 32:
      hipLaunchKernelGGL((k_apply_rinv<32>), grid, dim3(64 * ApplyLayout<8>::W), 0, s, A, m, n, lda, U, urs, ucs,
                         Q, ldq, info, (int)wgs);
      break;
    case 64:
      hipLaunchKernelGGL((k_apply_rinv<64>), grid, dim3(64 * ApplyLayout<16>::W), 0, s, A, m, n, lda, U, urs, ucs,
                         Q, ldq, info, (int)wgs);
      break;
    case 128:
      hipLaunchKernelGGL((k_apply_rinv<128>), grid, dim3(64 * ApplyLayout<32>::W), 0, s, A, m, n, lda, U, urs,
                         ucs, Q, ldq, info, (int)wgs);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace cqr2
