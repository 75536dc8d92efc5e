// CholInv (Algorithm 2) of an n x n SPD matrix, n <= 128, in one workgroup:
// the Cholesky factor and its triangular inverse together, FP64.
#include "cqr2_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#include "cholinv_dev.h"

namespace cqr2 {

template <int T, int G>
__global__ __launch_bounds__(G * G) void k_cholinv(const double* __restrict__ W, int64_t ldw, int n,
                                                 double* __restrict__ R, int64_t ldr, double* __restrict__ Rinv,
                                                 int64_t ldri, double* __restrict__ Upad, int np,
                                                 int32_t* __restrict__ info, int info_offset) {
  __shared__ double colbuf[2 * G * T];
  const CholInvSrc src{W, ldw, nullptr, 0, 0};
  cholinv_body<T, G>(src, n, R, ldr, Rinv, ldri, Upad, np, info, info_offset, colbuf);
}

int padded_order(int64_t n) {
  if (n <= 32) return 32;
  if (n <= 64) return 64;
  return 128;
}

// Thread grid of the one-workgroup CholInv: G x G threads, each owning a
// T x T cyclic tile of the padded order G T.  Up to n = 64 a 16 x 16 grid has
// the shorter per-column critical path; above, 32 x 32 threads share the
// larger Schur updates.
hipError_t launch_cholinv(const double* W, int64_t ldw, int n, double* R, int64_t ldr, double* Rinv,
                          int64_t ldri, double* Upad, int np, int32_t* info, int info_offset,
                          hipStream_t s) {
  const int order = padded_order(n);
#define CQR2_CI(TV, GV)                                                                                         \
  hipLaunchKernelGGL((k_cholinv<TV, GV>), dim3(1), dim3(GV * GV), 0, s, W, ldw, n, R, ldr, Rinv, ldri, Upad, np, \
                     info, info_offset)
  if (order == 32) CQR2_CI(2, 16);
  else if (order == 64) CQR2_CI(4, 16);
  else if (order == 128) CQR2_CI(4, 32);
  else return hipErrorInvalidValue;
#undef CQR2_CI
  return hipGetLastError();
}

}  // namespace cqr2
