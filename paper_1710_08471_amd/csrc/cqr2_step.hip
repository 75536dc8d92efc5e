// Multi-problem step kernel: one launch advances every problem of a table by
// one phase of CholeskyQR2 (Algorithm 5 = two passes of Algorithm 4, then
// R = R2 R1), for problems of different m and n <= 256.  It serves the batched
// entry point and the continuous-batching server, where problems admitted at
// different times share each launch.
//
// Each workgroup looks up its task by binary search over the table and runs
// the same device code as the one-problem kernels.  n <= 128: a Gram partial
// over a chunk of 1024-4096 rows, CholInv with the partial Grams summed (in
// split order) as it loads, or Q = A U over a chunk; the last phase adds one
// workgroup that forms R = R2 R1 and publishes the info word.  128 < n <= 256:
// the same steps with the wide Gram and Q bodies over chunks of 512-2048
// rows, a phase that
// sums the partial Grams, and a one-workgroup CholInv that splits W once at
// 128 (Algorithm 2's recursion, first level) and forms the coupling blocks
// with in-workgroup MFMA products.
#include "cqr2_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#include "apply_dev.h"
#include "cholinv_dev.h"
#include "gram_dev.h"
#include "stream16_dev.h"
#include "wide_dev.h"

namespace cqr2 {

static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// ---- 128 < n <= 256: workspace layout (host and device) -------------------
constexpr int kWideRedWGs = kWideLower * 256 / kStepThreads;  // one partial-Gram entry per thread
constexpr int kWL = 256;                                       // leading dimension of the 256 x 256 blocks
constexpr size_t kWideBlock = (size_t)kWL * kWL * sizeof(double);
enum { WB_W = 0, WB_R1, WB_R2, WB_RI, WB_U1, WB_U2, WB_T, WB_COUNT };

// 32-row stages per wide Gram / Q workgroup: about 64 workgroups per problem,
// each between 512 and 2048 rows (short workgroups pack a launch better; the
// lower bound keeps the partial Grams well below A's bytes)
__host__ __device__ inline int64_t wide_stages_per_chunk(int64_t m) {
  const int64_t stages = m > 0 ? (m + kWideRows - 1) / kWideRows : 1;
  int64_t spc = (stages + 63) / 64;
  if (spc < kStepWideMinStages) spc = kStepWideMinStages;
  if (spc > kStepWideStages) spc = kStepWideStages;
  return spc;
}
__host__ __device__ inline int wide_chunks(int64_t m) {
  const int64_t stages = m > 0 ? (m + kWideRows - 1) / kWideRows : 1;
  const int64_t spc = wide_stages_per_chunk(m);
  return (int)((stages + spc - 1) / spc);
}
// workgroups of the sum phase: about one per split (every entry reads one
// value per split), at most one entry per thread
__host__ __device__ inline int wide_reduce_wgs(int64_t m) {
  const int s = wide_chunks(m) + 3;
  return s < kWideRedWGs ? s : kWideRedWGs;
}
// n <= 128: 64-row stages per Gram / Q workgroup, about 32 workgroups per
// problem, each between 1024 and 4096 rows (the CholInv phase sums the
// partials in one workgroup, so their number stays small)
__host__ __device__ inline int64_t narrow_stages_per_chunk(int64_t m) {
  const int64_t stages = m > 0 ? (m + 63) / 64 : 1;
  int64_t spc = (stages + 31) / 32;
  if (spc < kStepMinStages) spc = kStepMinStages;
  if (spc > kStepStages) spc = kStepStages;
  return spc;
}
__host__ __device__ inline int narrow_chunks(int64_t m) {
  const int64_t stages = m > 0 ? (m + 63) / 64 : 1;
  const int64_t spc = narrow_stages_per_chunk(m);
  return (int)((stages + spc - 1) / spc);
}

// info word (256 bytes), the partial Grams, then the 256 x 256 blocks
__host__ __device__ inline size_t wide_off(int64_t m, int block) {
  return 256 + (size_t)wide_chunks(m) * kWideLower * 256 * sizeof(double) + (size_t)block * kWideBlock;
}

StepLayout step_layout(int64_t m, int64_t n) {
  StepLayout L;
  if (n > 128) {
    L.np = kWL;
    L.splits = wide_chunks(m);
    L.off_info = 0;
    L.off_part = 256;
    L.off_w = wide_off(m, WB_W);
    L.off_r1 = wide_off(m, WB_R1);
    L.off_r2 = wide_off(m, WB_R2);
    L.off_ri = wide_off(m, WB_RI);
    L.off_u1 = wide_off(m, WB_U1);
    L.off_u2 = wide_off(m, WB_U2);
    L.off_t = wide_off(m, WB_T);
    L.total = wide_off(m, WB_COUNT);
    return L;
  }
  L.np = padded_order(n);
  L.ng = L.np / 4;
  L.nblk = L.ng * (L.ng + 1) / 2;
  const int64_t stages = m > 0 ? (m + 63) / 64 : 1;
  L.splits = narrow_chunks(m);
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

double step_wg_cost(int64_t m, int64_t n, int phase) {
  if (n > 128) {
    const double rows = (double)(m < wide_stages_per_chunk(m) * kWideRows ? m : wide_stages_per_chunk(m) * kWideRows);
    switch (phase) {
      case 0: case 4: return 0.33 * rows;   // Gram: 680 us per 2048 rows
      case 3: case 7: return 0.40 * rows;   // Q = A U: 820 us per 2048 rows
      case 2: case 6: return 350.0;         // CholInv
      default: return 20.0;                 // sum of the partials
    }
  }
  const int64_t crow = narrow_stages_per_chunk(m) * 64;
  const double f = (double)(m < crow ? (m > 0 ? m : 1) : crow) / 4096.0;  // rows of a chunk / 4096
  const double x = (double)(n < 16 ? 16 : n) - 16.0;
  switch (phase) {
    case 0: case 3: return (60.0 + 2.8 * x) * f;    // Gram over 4096 rows
    case 2: case 5: return (140.0 + 3.6 * x) * f;   // Q = A U over 4096 rows
    default: return 12.0 + 1.2 * x;                 // CholInv
  }
}

int step_phases(int64_t n) { return n > 128 ? kStepWidePhases : kStepPhases; }

int step_workgroups(int64_t m, int64_t n, int phase) {
  if (n > 128) {
    const int chunks = wide_chunks(m);
    switch (phase) {
      case 0: case 3: case 4: return chunks;
      case 1: case 5: return wide_reduce_wgs(m);
      case 2: case 6: return 1;
      case 7: return chunks + 1;
      default: return 0;
    }
  }
  const int64_t stages = m > 0 ? (m + 63) / 64 : 1;
  const int chunks = narrow_chunks(m);
  switch (phase) {
    case 0: case 2: case 3: return chunks;
    case 1: case 4: return 1;
    case 5: return chunks + 1;
    default: return 0;
  }
}

// ---- 128 < n <= 256 ----------------------------------------------------------
// Small products inside one workgroup: C(i, j) = alpha sum_k opA(i, k) opB(k, j)
// [+ Cin(i, j)] for i < M, j < N, k < K (each at most 256), with
// opA(i, k) = A[i rs + k cs] and opB(k, j) = B[k rs + j cs].  Output panels of
// 128 x 128; wave w owns tile row w of a panel (eight 16 x 16 tiles, MFMA
// 16x16x4 f64); K runs in chunks of 32 staged through LDS k-major (As[k][i],
// Bs[k][j]).  The flags name zeros of the operands, so whole k-steps (and
// chunks) are skipped, and select the output.
enum : int {
  WG_A_UPPER = 1,    // opA(i, k) = 0 for k < i
  WG_A_LOWER = 2,    // opA(i, k) = 0 for k > i
  WG_B_UPPER = 4,    // opB(k, j) = 0 for k > j
  WG_LOWER_OUT = 8,  // only the tiles on or below the diagonal are formed and written
  WG_UPPER_OUT = 16  // entries below the diagonal are written as 0
};
struct WgOp {
  const double* p;
  int64_t rs, cs;
};
constexpr int kWgPanel = 128, kWgKC = 32, kWgLd = kWgPanel + 4;  // LDS: 2 x 32 x 132 doubles

__device__ __forceinline__ void wg_stage(const WgOp& o, bool rows_are_i, int lim_i, int K, int i0, int k0,
                                         double* dst) {
  // dst[kk * kWgLd + ii] = opA(i0 + ii, k0 + kk) (rows_are_i) or
  // opB(k0 + kk, i0 + ii), 0 outside; the index with unit stride in memory
  // runs fastest across threads, and every load is in flight before the
  // first store
  constexpr int kPer = kWgKC * kWgPanel / kStepThreads;
  const bool k_fast = rows_are_i ? o.cs == 1 : o.rs == 1;
  const int64_t si = rows_are_i ? o.rs : o.cs, sk = rows_are_i ? o.cs : o.rs;
  double v[kPer];
  int slot[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int e = threadIdx.x + u * kStepThreads;
    const int kk = k_fast ? e % kWgKC : e / kWgPanel;
    const int ii = k_fast ? e / kWgKC : e % kWgPanel;
    const int i = i0 + ii, k = k0 + kk;
    v[u] = (i < lim_i && k < K) ? o.p[i * si + k * sk] : 0.0;
    slot[u] = kk * kWgLd + ii;
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) dst[slot[u]] = v[u];
}

__device__ __forceinline__ void wg_gemm(int M, int N, int K, WgOp a, WgOp b, double alpha, const double* cin, int64_t ldcin,
                        double* c, int64_t ldc, int flags, double* lds) {
  double* As = lds;
  double* Bs = lds + kWgKC * kWgLd;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int pi = 0; pi * kWgPanel < M; ++pi)
    for (int pj = 0; pj * kWgPanel < N; ++pj) {
      if ((flags & WG_LOWER_OUT) && pj > pi) continue;
      const int I = pi * 8 + w;  // global tile row of this wave
      int kmin = 0, kmax = K;
      if (flags & WG_A_UPPER) kmin = pi * kWgPanel;
      if ((flags & WG_A_LOWER) && (pi + 1) * kWgPanel < kmax) kmax = (pi + 1) * kWgPanel;
      if ((flags & WG_B_UPPER) && (pj + 1) * kWgPanel < kmax) kmax = (pj + 1) * kWgPanel;
      d4 acc[8];
#pragma unroll
      for (int t = 0; t < 8; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
      for (int k0 = kmin; k0 < kmax; k0 += kWgKC) {
        wg_stage(a, true, M, K, pi * kWgPanel, k0, As);
        wg_stage(b, false, N, K, pj * kWgPanel, k0, Bs);
        __syncthreads();
        if (16 * I < M) {
#pragma unroll
          for (int kk = 0; kk < kWgKC; kk += 4) {
            const int k = k0 + kk;
            if ((flags & WG_A_UPPER) && k < 16 * I) continue;
            if ((flags & WG_A_LOWER) && k >= 16 * (I + 1)) continue;
            const double af = As[(kk + (lane >> 4)) * kWgLd + 16 * w + (lane & 15)];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
              const int J = pj * 8 + t;
              if (16 * J >= N) continue;
              if ((flags & WG_LOWER_OUT) && J > I) continue;
              if ((flags & WG_B_UPPER) && k >= 16 * (J + 1)) continue;
              const double bf = Bs[(kk + (lane >> 4)) * kWgLd + 16 * t + (lane & 15)];
              acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(af, bf, acc[t], 0, 0, 0);
            }
          }
        }
        __syncthreads();
      }
      if (16 * I >= M) continue;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int J = pj * 8 + t;
        if (16 * J >= N) continue;
        if ((flags & WG_LOWER_OUT) && J > I) continue;
        // entry r of lane l: D(4r + l/16, l%16)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = 16 * I + 4 * r + (lane >> 4), j = 16 * J + (lane & 15);
          if (i < M && j < N) {
            double v = alpha * acc[t][r];
            if (cin != nullptr) v += cin[i + (int64_t)j * ldcin];
            if ((flags & WG_UPPER_OUT) && i > j) v = 0.0;
            c[i + (int64_t)j * ldc] = v;
          }
        }
      }
    }
}

// R = R2 R1 (upper triangular, n x n; R1, R2 column-major with leading
// dimension ld, zero below the diagonal), written to R (ldr) with zeros below
// the diagonal; NaN everywhere after a breakdown (st != 0).
__device__ __forceinline__ void step_upper_product(const double* R2, const double* R1, int64_t ld, int n, double* R,
                                                   int64_t ldr, int32_t st, double* lds) {
  if (st == 0) {
    wg_gemm(n, n, n, WgOp{R2, 1, ld}, WgOp{R1, 1, ld}, 1.0, nullptr, 0, R, ldr, WG_A_UPPER | WG_B_UPPER | WG_UPPER_OUT,
            lds);
    return;
  }
  for (int e = threadIdx.x; e < n * n; e += kStepThreads) R[e % n + (int64_t)(e / n) * ldr] = __builtin_nan("");
}

// W = the sum of the partial Grams in split order, both triangles (256 x 256,
// column-major); the nwg workgroups of the phase share the entries.
__device__ __forceinline__ void wide_reduce(const double* __restrict__ part, int splits, int n,
                                            double* __restrict__ W, int sub, int nwg) {
  constexpr int total = kWideLower * 256;
  for (int e = sub * kStepThreads + threadIdx.x; e < total; e += nwg * kStepThreads) {
    double v = 0.0;
    int s = 0;
    for (; s + 8 <= splits; s += 8) {
      double x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) x[j] = part[(int64_t)(s + j) * total + e];
#pragma unroll
      for (int j = 0; j < 8; ++j) v += x[j];
    }
    for (; s < splits; ++s) v += part[(int64_t)s * total + e];
    // partial layout: tile (I, J) at I (I+1)/2 + J, entry r of lane l at r 64 + l
    const int tile = e >> 8, r = (e >> 6) & 3, l = e & 63;
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= tile) ++I;
    const int J = tile - I * (I + 1) / 2;
    const int row = 16 * I + 4 * r + (l >> 4), col = 16 * J + (l & 15);
    if (row >= col && row < n) {
      W[row + (int64_t)col * kWL] = v;
      W[col + (int64_t)row * kWL] = v;
    }
  }
}

// CholInv (Algorithm 2) for 128 < n <= 256 in one workgroup: one level of the
// recursion at h = 128, the diagonal blocks by the register-resident body,
// the coupling blocks by wg_gemm:
//   R11, R11^-1 = CholInv(W11);  R12 = R11^-T W12;  S = W22 - R12ᵀ R12;
//   R22, R22^-1 = CholInv(S);    (R^-1)12 = -R11^-1 R12 R22^-1.
// W, R, Ri (R^-1) and T (scratch) are 256 x 256 column-major; U receives the
// zero-padded row-major image of R^-1 read by the Q = A U body.  A breakdown
// sets *info = info_offset + column (1-based) and leaves U NaN.
__device__ __forceinline__ void wide_cholinv(const double* W, int n, double* R, double* Ri, double* T, double* U, int32_t* info,
                             int info_offset, double* lds) {
  int h = 128;  // opaque to the optimizer: both blocks run the body compiled for a run-time order
  asm volatile("" : "+s"(h));
  const int n2 = n - h;
  for (int e = threadIdx.x; e < h * h; e += kStepThreads) {
    const int i = h + e % h, j = e / h;  // the lower-left blocks are zero
    R[i + (int64_t)j * kWL] = 0.0;
    Ri[i + (int64_t)j * kWL] = 0.0;
  }
  cholinv_body<8, 16, 2>(CholInvSrc{W, kWL, nullptr, 0, 0}, h, R, kWL, Ri, kWL, nullptr, 0, info, info_offset, lds);
  __syncthreads();
  if (*info == 0) {
    wg_gemm(h, n2, h, WgOp{Ri, kWL, 1}, WgOp{W + h, kWL, 1}, 1.0, nullptr, 0, R + (int64_t)h * kWL, kWL,
            WG_A_LOWER, lds);  // R12(i, j) = sum_k R11^-1(k, i) W(h + j, k)
    __syncthreads();
    wg_gemm(n2, n2, h, WgOp{R + (int64_t)h * kWL, kWL, 1}, WgOp{R + (int64_t)h * kWL, 1, kWL}, -1.0,
            W + h + (int64_t)h * kWL, kWL, T, kWL, WG_LOWER_OUT, lds);  // S = W22 - R12ᵀ R12
    __syncthreads();
  }
  cholinv_body<8, 16, 2>(CholInvSrc{T, kWL, nullptr, 0, 0}, n2, R + h + (int64_t)h * kWL, kWL,
                         Ri + h + (int64_t)h * kWL, kWL, nullptr, 0, info, info_offset + h, lds);
  __syncthreads();
  const bool ok = *info == 0;
  if (ok) {
    wg_gemm(h, n2, n2, WgOp{R + (int64_t)h * kWL, 1, kWL}, WgOp{Ri + h + (int64_t)h * kWL, 1, kWL}, 1.0, nullptr,
            0, T, kWL, WG_B_UPPER, lds);  // T = R12 R22^-1
    __syncthreads();
    wg_gemm(h, n2, h, WgOp{Ri, 1, kWL}, WgOp{T, 1, kWL}, -1.0, nullptr, 0, Ri + (int64_t)h * kWL, kWL, WG_A_UPPER,
            lds);  // (R^-1)12 = -R11^-1 T
    __syncthreads();
  }
  // U[p 256 + q] = R^-1(p, q) for p <= q < n, else 0: 64 x 64 blocks through LDS
  const double nan = __builtin_nan("");
  for (int bp = 0; bp < 4; ++bp)
    for (int bq = 0; bq < 4; ++bq) {
      for (int e = threadIdx.x; e < 64 * 64; e += kStepThreads) {
        const int pp = e % 64, qq = e / 64, p = 64 * bp + pp, q = 64 * bq + qq;
        double v = 0.0;
        if (p <= q && q < n) v = ok ? Ri[p + (int64_t)q * kWL] : nan;
        lds[qq * 65 + pp] = v;
      }
      __syncthreads();
      for (int e = threadIdx.x; e < 64 * 64; e += kStepThreads) {
        const int qq = e % 64, pp = e / 64;
        U[(int64_t)(64 * bp + pp) * kWL + 64 * bq + qq] = lds[qq * 65 + pp];
      }
      __syncthreads();
    }
}

__device__ __forceinline__ void wide_gram(const double* A, int64_t m, int n, int64_t lda, int64_t st0, int64_t st1,
                                          double* lds, double* out) {
  const bool direct_ok = (((uintptr_t)A & 15u) == 0) && (((lda * (int64_t)sizeof(double)) & 15) == 0);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  switch (wave) {
    case 0: gram_wide_wave<double, 0>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 1: gram_wide_wave<double, 1>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 2: gram_wide_wave<double, 2>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 3: gram_wide_wave<double, 3>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 4: gram_wide_wave<double, 4>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 5: gram_wide_wave<double, 5>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 6: gram_wide_wave<double, 6>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 7: gram_wide_wave<double, 7>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    default: break;
  }
}

// Q = A U over 32-row stages [s0, s1); Q may equal A.
__device__ __forceinline__ void wide_apply(const double* A, int64_t m, int n, int64_t lda, const double* U,
                                           double* Q, int64_t ldq, int64_t s0, int64_t s1, double* lds) {
  constexpr int SR = 32, NBUF = 2;
  for (int e = threadIdx.x; e < NBUF * kWCols * SR; e += kStepThreads)
    if ((e % (kWCols * SR)) / SR >= n) lds[e] = 0.0;
  const bool direct_ok = (((uintptr_t)A & 15u) == 0) && (((lda * (int64_t)sizeof(double)) & 15) == 0) &&
                         lda <= ((int64_t)1 << 26);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#define CQR2_WA(WV) apply256_body<double, false, SR, NBUF, WV>(A, m, n, lda, U, Q, ldq, s0, s1, direct_ok, lds)
  switch (wave) {
    case 0: CQR2_WA(0); break;
    case 1: CQR2_WA(1); break;
    case 2: CQR2_WA(2); break;
    case 3: CQR2_WA(3); break;
    case 4: CQR2_WA(4); break;
    case 5: CQR2_WA(5); break;
    case 6: CQR2_WA(6); break;
    case 7: CQR2_WA(7); break;
    default: break;
  }
#undef CQR2_WA
}

__device__ __forceinline__ void step_run_wide(const StepTask& t, int sub, double* lds) {
  const int n = t.n;
  const int64_t m = t.m;
  int32_t* info = (int32_t*)t.ws;
  double* part = (double*)(t.ws + 256);
  double* W = (double*)(t.ws + wide_off(m, WB_W));
  double* R1 = (double*)(t.ws + wide_off(m, WB_R1));
  double* R2 = (double*)(t.ws + wide_off(m, WB_R2));
  double* Ri = (double*)(t.ws + wide_off(m, WB_RI));
  double* U1 = (double*)(t.ws + wide_off(m, WB_U1));
  double* U2 = (double*)(t.ws + wide_off(m, WB_U2));
  double* T = (double*)(t.ws + wide_off(m, WB_T));
  const int splits = wide_chunks(m);
  const int64_t nst = m > 0 ? (m + kWideRows - 1) / kWideRows : 0;
  const int64_t spc = wide_stages_per_chunk(m);
  const int64_t s0 = (int64_t)sub * spc;
  const int64_t s1 = s0 + spc < nst ? s0 + spc : nst;
  double* out = part + (int64_t)sub * kWideLower * 256;
  switch (t.phase) {
    case 0:  // Gram of A; the first workgroup resets the info word
      if (sub == 0 && threadIdx.x == 0) *info = 0;
      wide_gram(t.A, m, n, t.lda, s0, s1, lds, out);
      break;
    case 4:  // Gram of Q1
      if (*info != 0) return;
      wide_gram(t.Q, m, n, t.ldq, s0, s1, lds, out);
      break;
    case 1:
    case 5:
      if (*info != 0) return;
      wide_reduce(part, splits, n, W, sub, t.nwg);
      break;
    case 2: wide_cholinv(W, n, R1, Ri, T, U1, info, 0, lds); break;
    case 6: wide_cholinv(W, n, R2, Ri, T, U2, info, n, lds); break;
    case 3:
      if (*info != 0) return;
      wide_apply(t.A, m, n, t.lda, U1, t.Q, t.ldq, s0, s1, lds);
      break;
    case 7: {
      const int32_t st = *info;
      if (sub == t.nwg - 1) {  // R = R2 R1 (NaN after a breakdown) and the info word
        step_upper_product(R2, R1, kWL, n, t.R, t.ldr, st, lds);
        if (threadIdx.x == 0 && t.user_info != nullptr) *t.user_info = st;
        return;
      }
      if (st != 0) return;
      wide_apply(t.Q, m, n, t.ldq, U2, t.Q, t.ldq, s0, s1, lds);
      break;
    }
    default: break;
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
  const int splits = narrow_chunks(m);
  const int64_t spc = narrow_stages_per_chunk(m);
  const int64_t s0 = (int64_t)sub * spc;
  const int64_t s1 = s0 + spc < stages ? s0 + spc : stages;
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
        step_upper_product(R2, R1, n, n, t.R, t.ldr, st, lds);
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
  // the largest stage pair: Gram or Q = A U at n = 128, or a 32-row pair at n = 256
  __shared__ __attribute__((aligned(16))) double lds[2 * 128 * 64];
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
  if (t.n > 128) {
    step_run_wide(t, sub, lds);
    return;
  }
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
