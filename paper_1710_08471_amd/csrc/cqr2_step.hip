// Multi-problem step kernel: one launch advances every problem of a table by
// one phase of CholeskyQR2 (Algorithm 5 = two passes of Algorithm 4, then
// R = R2 R1), for problems of different m and n <= 128.  It serves the batched
// entry point (six steps in a row) and the continuous-batching server, where
// problems admitted at different times share each launch.
//
// Each workgroup looks up its task by binary search over the table and runs
// the same device code as the one-problem kernels: a Gram partial over up to
// 4096 rows, CholInv with the partial Grams summed (in split order) as it
// loads, or Q = A U over up to 4096 rows.  Phase 5 adds one workgroup that
// forms R = R2 R1 and publishes the info word.
#include "cqr2_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#include "apply_dev.h"
#include "cholinv_dev.h"
#include "gram_dev.h"

namespace cqr2 {

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

StepLayout step_layout(int64_t m, int64_t n) {
  StepLayout L;
  L.np = padded_order(n);
  L.ng = L.np / 4;
  L.nblk = L.ng * (L.ng + 1) / 2;
  const int64_t stages = m > 0 ? (m + 63) / 64 : 1;
  L.splits = (int)((stages + kStepStages - 1) / kStepStages);
  size_t off = 0;
  L.off_info = off; off += align256(16);
  L.off_part = off; off += align256((size_t)L.splits * L.nblk * 16 * sizeof(double));
  L.off_r1 = off;   off += align256((size_t)n * n * sizeof(double));
  L.off_r2 = off;   off += align256((size_t)n * n * sizeof(double));
  L.off_u1 = off;   off += align256((size_t)L.np * L.np * sizeof(double));
  L.off_u2 = off;   off += align256((size_t)L.np * L.np * sizeof(double));
  L.total = off;
  return L;
}

int step_workgroups(int64_t m, int phase) {
  const int64_t stages = m > 0 ? (m + 63) / 64 : 1;
  const int chunks = (int)((stages + kStepStages - 1) / kStepStages);
  switch (phase) {
    case 0: case 2: case 3: return chunks;
    case 1: case 4: return 1;
    case 5: return chunks + 1;
    default: return 0;
  }
}

// R = R2 R1 (upper triangular, n x n, column-major with leading dimension n),
// each entry summed over k = i..j in ascending order; NaN after a breakdown.
__device__ void step_upper_product(const double* __restrict__ R2, const double* __restrict__ R1, int n,
                                   double* __restrict__ R, int64_t ldr, int32_t st) {
  for (int e = threadIdx.x; e < n * n; e += kStepThreads) {
    const int i = e % n, j = e / n;
    double v = 0.0;
    if (i <= j)
      for (int k = i; k <= j; ++k) v = fma(R2[i + (int64_t)k * n], R1[k + (int64_t)j * n], v);
    R[i + (int64_t)j * ldr] = st != 0 ? __builtin_nan("") : v;
  }
}

template <int NP>
__device__ __forceinline__ void step_run(const StepTask& t, int sub, double* lds) {
  constexpr int NG = NP / 4;
  constexpr int NBLK = NG * (NG + 1) / 2;
  constexpr int NT = NP < 64 ? 64 : NP;  // Q = A U runs on at least 16 column groups (8 waves)
  const int n = t.n;
  const int64_t m = t.m;
  const int64_t stages = m > 0 ? (m + 63) / 64 : 1;
  const int splits = (int)((stages + kStepStages - 1) / kStepStages);
  const int64_t s0 = (int64_t)sub * kStepStages;
  const int64_t s1 = s0 + kStepStages < stages ? s0 + kStepStages : stages;
  // workspace (same offsets as step_layout)
  const size_t part_off = 256;
  const size_t part_bytes = ((size_t)splits * NBLK * 16 * sizeof(double) + 255) / 256 * 256;
  const size_t rr = (((size_t)n * n * sizeof(double)) + 255) / 256 * 256;
  const size_t uu = (((size_t)NP * NP * sizeof(double)) + 255) / 256 * 256;
  int32_t* info = (int32_t*)t.ws;
  double* part = (double*)(t.ws + part_off);
  double* R1 = (double*)(t.ws + part_off + part_bytes);
  double* R2 = (double*)(t.ws + part_off + part_bytes + rr);
  double* U1 = (double*)(t.ws + part_off + part_bytes + 2 * rr);
  double* U2 = (double*)(t.ws + part_off + part_bytes + 2 * rr + uu);

  switch (t.phase) {
    case 0:  // Gram of A; the first workgroup resets the info word
      if (sub == 0 && threadIdx.x == 0) *info = 0;
      gram_block<NG, 8>(t.A, m, n, t.lda, s0, s1, lds, part + (int64_t)sub * NBLK * 16);
      break;
    case 3:  // Gram of Q1
      if (*info != 0) return;
      gram_block<NG, 8>(t.Q, m, n, t.ldq, s0, s1, lds, part + (int64_t)sub * NBLK * 16);
      break;
    case 1:
    case 4: {
      const CholInvSrc src{nullptr, 0, part, splits, NBLK};
      const bool p1 = t.phase == 1;
      cholinv_body<NP / 16, 16, 2>(src, n, p1 ? R1 : R2, n, nullptr, 0, p1 ? U1 : U2, NP, info, p1 ? 0 : n, lds);
      break;
    }
    case 2:
      if (*info != 0) return;
      apply_block<NT>(t.A, m, n, t.lda, U1, NP, 1, t.Q, t.ldq, s0, s1, false, lds);
      break;
    case 5: {
      const int32_t st = *info;
      if (sub == t.nwg - 1) {
        step_upper_product(R2, R1, n, t.R, t.ldr, st);
        if (threadIdx.x == 0 && t.user_info != nullptr) *t.user_info = st;
        return;
      }
      if (st != 0) return;
      apply_block<NT>(t.Q, m, n, t.ldq, U2, NP, 1, t.Q, t.ldq, s0, s1, false, lds);
      break;
    }
    default: break;
  }
}

__global__ __launch_bounds__(kStepThreads, 1) void k_step(const StepTask* __restrict__ tasks, int ntasks) {
  __shared__ double lds[2 * 128 * 64];  // the largest stage pair (Gram or Q = A U at n = 128)
  const int wg = blockIdx.x;
  int lo = 0, hi = ntasks - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (tasks[mid].wg0 <= wg) lo = mid;
    else hi = mid - 1;
  }
  const StepTask t = tasks[lo];
  const int sub = wg - t.wg0;
  if (sub < 0 || sub >= t.nwg) return;
  const int np = t.n <= 32 ? 32 : (t.n <= 64 ? 64 : 128);
  if (np == 32) step_run<32>(t, sub, lds);
  else if (np == 64) step_run<64>(t, sub, lds);
  else step_run<128>(t, sub, lds);
}

hipError_t launch_step(const StepTask* d_tasks, int ntasks, int total_wgs, hipStream_t s) {
  if (ntasks <= 0 || total_wgs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_step, dim3((unsigned)total_wgs), dim3(kStepThreads), 0, s, d_tasks, ntasks);
  return hipGetLastError();
}

}  // namespace cqr2
