// CholInv (Algorithm 2) of an n x n SPD matrix, n <= 128, in one workgroup:
// the Cholesky factor and its triangular inverse together, FP64.
#include "cqr2_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#include "cholinv_dev.h"

namespace cqr2 {

// Columns per barrier of the one-problem kernel: 4, or 2 at the largest
// tile (T = 8), where a wider block would not fit the register file.
template <int T>
constexpr int cholinv_block() { return T >= 8 ? 2 : 4; }

template <int T, int G>
__global__ __launch_bounds__(G * G) void k_cholinv(const double* __restrict__ W, int64_t ldw, int n,
                                                 double* __restrict__ R, int64_t ldr, double* __restrict__ Rinv,
                                                 int64_t ldri, double* __restrict__ Upad, int np,
                                                 int32_t* __restrict__ info, int info_offset) {
  constexpr int B = cholinv_block<T>();
  __shared__ double colbuf[(2 * B + 1) * G * T];
  const CholInvSrc src{W, ldw, nullptr, 0, 0};
  cholinv_body<T, G, B>(src, n, R, ldr, Rinv, ldri, Upad, np, info, info_offset, colbuf);
}

int padded_order(int64_t n) {
  if (n <= 32) return 32;
  if (n <= 64) return 64;
  return 128;
}

// Thread grid of the one-workgroup CholInv: 16 x 16 threads, each owning a
// T x T cyclic tile of the padded order 16 T (T = 2, 4, 8).
hipError_t launch_cholinv(const double* W, int64_t ldw, int n, double* R, int64_t ldr, double* Rinv,
                          int64_t ldri, double* Upad, int np, int32_t* info, int info_offset,
                          hipStream_t s) {
  const int order = padded_order(n);
#define CQR2_CI(TV)                                                                                           \
  hipLaunchKernelGGL((k_cholinv<TV, 16>), dim3(1), dim3(256), 0, s, W, ldw, n, R, ldr, Rinv, ldri, Upad, np, info, \
                     info_offset)
  if (order == 32) CQR2_CI(2);
  else if (order == 64) CQR2_CI(4);
  else if (order == 128) CQR2_CI(8);
  else return hipErrorInvalidValue;
#undef CQR2_CI
  return hipGetLastError();
}

}  // namespace cqr2
