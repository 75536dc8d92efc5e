// General FP64 GEMM for gfx950 with MFMA 4x4x4 (4 blocks):
//   C = alpha * op(A) op(B) + beta * C      (column-major, op = N or T)
// used where CholeskyQR2 works on large blocks: the recursive CholInv of
// Algorithm 2 (L21 = A21 Y11ᵀ, A22 - L21 L21ᵀ, Y21 = -Y22 L21 Y11), Gram and
// Q = A R^{-1} for wide matrices, and R = R2 R1.
//
// Triangular structure is exploited by limiting each tile's reduction range
// and by skipping output tiles: flags say that op(A) is lower/upper
// triangular, op(B) is lower/upper triangular, or that only the lower/upper
// triangle of C is needed.  Optional split of the reduction dimension: each
// split writes a partial product to a workspace and a second kernel adds the
// partials in a fixed order (deterministic; no floating-point atomics).
#include "cqr2_internal.h"

#include <hip/hip_runtime.h>
#include <cstdint>

namespace cqr2 {

// Tile sizes: a workgroup computes a 64 x 64 block of C with 4 waves in a
// 2 x 2 arrangement of 32 x 32 wave tiles; the reduction dimension is staged
// through LDS in chunks of kGK.
#ifndef CQR2_GEMM_KC
#define CQR2_GEMM_KC 16
#endif
constexpr int kGM = 64, kGN = 64, kGK = CQR2_GEMM_KC;
constexpr int kGStage = kGK * kGM / 256;  // entries of each operand chunk per thread

// One MFMA 4x4x4 (4 blocks) with the blocks as four groups of 4 rows:
// lane l supplies op(A)(r0 + (l&15), k0 + (l>>4)) and op(B)(k0 + (l>>4), c0 + (l&3))
// and receives C(r0 + 4((l>>2)&3) + (l>>4), c0 + (l&3)).
//
// LDS images: As[k][row] (64 rows per k, rows of odd k XOR 16: the 4 k x 16
// rows of a fragment spread over both bank halves), Bs[k][col].
__device__ __forceinline__ int as_pos(int k, int r) { return k * kGM + (r ^ ((k & 1) << 4)); }
__device__ __forceinline__ int bs_pos(int k, int c) { return k * kGN + c; }

struct GemmArgs {
  int64_t M, N, K;
  const void* A;     // element type per kernel instance (double or float)
  int64_t lda;
  const void* B;
  int64_t ldb;
  void* C;           // double, or float for the FP32-arithmetic instance
  int64_t ldc;
  double alpha, beta;
  int transA, transB;
  int flags;
  int splits;          // reduction splits (grid.z)
  int64_t kchunk;      // reduction length per split (multiple of kGK)
  double* partial;     // splits > 1: workspace of splits * ldp * N doubles
  int64_t ldp;         // leading dimension of a partial (>= M)
  const int32_t* info; // optional: skip when *info != 0
};

template <typename TA>
__device__ __forceinline__ double load_opA(const GemmArgs& g, int64_t i, int64_t k) {
  const TA* A = (const TA*)g.A;
  return (double)(g.transA ? A[k + i * g.lda] : A[i + k * g.lda]);
}
template <typename TB>
__device__ __forceinline__ double load_opB(const GemmArgs& g, int64_t k, int64_t j) {
  const TB* B = (const TB*)g.B;
  return (double)(g.transB ? B[j + k * g.ldb] : B[k + j * g.ldb]);
}

// Entries outside a declared triangle are never read (they may hold anything).
__device__ __forceinline__ bool a_in_triangle(const GemmArgs& g, int64_t i, int64_t k) {
  return !((g.flags & GEMM_A_LOWER) && k > i) && !((g.flags & GEMM_A_UPPER) && k < i);
}
__device__ __forceinline__ bool b_in_triangle(const GemmArgs& g, int64_t k, int64_t j) {
  return !((g.flags & GEMM_B_UPPER) && k > j) && !((g.flags & GEMM_B_LOWER) && k < j);
}

// Reduction range of output tile (i0, j0) for split `split` (triangular operands).
__device__ __forceinline__ void gemm_krange(const GemmArgs& g, int64_t i0, int64_t j0, int split, int64_t& kb,
                                            int64_t& ke) {
  kb = 0;
  ke = g.K;
  if (g.flags & GEMM_A_LOWER) ke = ke < i0 + 64 ? ke : i0 + 64;   // op(A)(i,k) = 0 for k > i
  if (g.flags & GEMM_A_UPPER) kb = kb > i0 ? kb : i0;             // op(A)(i,k) = 0 for k < i
  if (g.flags & GEMM_B_UPPER) ke = ke < j0 + 64 ? ke : j0 + 64;   // op(B)(k,j) = 0 for k > j
  if (g.flags & GEMM_B_LOWER) kb = kb > j0 ? kb : j0;             // op(B)(k,j) = 0 for k < j
  const int64_t sb = (int64_t)split * g.kchunk, se = sb + g.kchunk;
  kb = kb > sb ? kb : sb;
  ke = ke < se ? ke : se;
  kb = (kb / kGK) * kGK;  // chunk-aligned start (entries below kb are zero by structure)
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256, 2) void k_gemm(GemmArgs g) {
  __shared__ double As[2][kGK * kGM];
  __shared__ double Bs[2][kGK * kGN];
  if (g.info != nullptr && *g.info != 0) return;
  const int64_t i0 = (int64_t)blockIdx.x * kGM, j0 = (int64_t)blockIdx.y * kGN;
  const int split = blockIdx.z;
  // Output tiles entirely outside the requested triangle of C.
  if ((g.flags & GEMM_C_LOWER) && i0 + kGM <= j0) return;
  if ((g.flags & GEMM_C_UPPER) && j0 + kGN <= i0) return;
  int64_t kb, ke;
  gemm_krange(g, i0, j0, split, kb, ke);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;  // wave tile origin within the block

  // Staging: each thread moves kGStage entries of the A chunk and of the B chunk.
  double ra[kGStage], rb[kGStage];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int t = 0; t < kGStage; ++t) {
      const int e = tid + 256 * t;
      // A chunk 64 x kGK: for op N walk rows fastest (coalesced), for op T walk k fastest.
      int r, k;
      if (g.transA) { k = e % kGK; r = e / kGK; } else { r = e & 63; k = e >> 6; }
      const int64_t gi = i0 + r, gk = k0 + k;
      ra[t] = (gi < g.M && gk < ke && a_in_triangle(g, gi, gk)) ? load_opA<TA>(g, gi, gk) : 0.0;
      int kk, c;
      if (g.transB) { c = e & 63; kk = e >> 6; } else { kk = e % kGK; c = e / kGK; }
      const int64_t bk = k0 + kk, gj = j0 + c;
      rb[t] = (gj < g.N && bk < ke && b_in_triangle(g, bk, gj)) ? load_opB<TB>(g, bk, gj) : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int t = 0; t < kGStage; ++t) {
      const int e = tid + 256 * t;
      int r, k;
      if (g.transA) { k = e % kGK; r = e / kGK; } else { r = e & 63; k = e >> 6; }
      As[buf][as_pos(k, r)] = ra[t];
      int kk, c;
      if (g.transB) { c = e & 63; kk = e >> 6; } else { kk = e % kGK; c = e / kGK; }
      Bs[buf][bs_pos(kk, c)] = rb[t];
    }
  };

  double acc[2][8];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int cg = 0; cg < 8; ++cg) acc[rt][cg] = 0.0;

  const int nchunks = ke > kb ? (int)((ke - kb + kGK - 1) / kGK) : 0;
  if (nchunks > 0) {
    gload(kb);
    sstore(0);
  }
  __syncthreads();
  const int ar = lane & 15, ak = lane >> 4, bc = lane & 3;
  for (int ch = 0; ch < nchunks; ++ch) {
    const int cur = ch & 1;
    if (ch + 1 < nchunks) gload(kb + (int64_t)(ch + 1) * kGK);
#pragma unroll
    for (int ks = 0; ks < kGK; ks += 4) {
      double a[2], b[8];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) a[rt] = As[cur][as_pos(ks + ak, wr + 16 * rt + ar)];
#pragma unroll
      for (int cg = 0; cg < 8; ++cg) b[cg] = Bs[cur][bs_pos(ks + ak, wc + 4 * cg + bc)];
#pragma unroll
      for (int rt = 0; rt < 2; ++rt)
#pragma unroll
        for (int cg = 0; cg < 8; ++cg) acc[rt][cg] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[rt], b[cg], acc[rt][cg], 0, 0, 0);
    }
    if (ch + 1 < nchunks) sstore(cur ^ 1);
    __syncthreads();
  }

  const int orow = 4 * ((lane >> 2) & 3) + (lane >> 4), ocol = lane & 3;
  auto out_ok = [&](int rt, int cg) {
    const int64_t i = i0 + wr + 16 * rt + orow, j = j0 + wc + 4 * cg + ocol;
    if (i >= g.M || j >= g.N) return false;
    if ((g.flags & GEMM_C_LOWER) && i < j) return false;
    if ((g.flags & GEMM_C_UPPER) && i > j) return false;
    return true;
  };
  if (g.splits > 1) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt)
#pragma unroll
      for (int cg = 0; cg < 8; ++cg) {
        const int64_t i = i0 + wr + 16 * rt + orow, j = j0 + wc + 4 * cg + ocol;
        if (out_ok(rt, cg)) g.partial[(int64_t)split * g.ldp * g.N + i + j * g.ldp] = acc[rt][cg];
      }
    return;
  }
  // with beta != 0 every old value of C is loaded before the first store (a
  // store could alias a later load as far as the compiler knows)
  double old[2][8];
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int cg = 0; cg < 8; ++cg) {
      const int64_t i = i0 + wr + 16 * rt + orow, j = j0 + wc + 4 * cg + ocol;
      old[rt][cg] = (g.beta != 0.0 && out_ok(rt, cg)) ? ((const double*)g.C)[i + j * g.ldc] : 0.0;
    }
#pragma unroll
  for (int rt = 0; rt < 2; ++rt)
#pragma unroll
    for (int cg = 0; cg < 8; ++cg) {
      const int64_t i = i0 + wr + 16 * rt + orow, j = j0 + wc + 4 * cg + ocol;
      if (!out_ok(rt, cg)) continue;
      const double v = g.alpha * acc[rt][cg];
      ((double*)g.C)[i + j * g.ldc] = (g.beta == 0.0) ? v : v + g.beta * old[rt][cg];
    }
}

// C = alpha * sum_s partial_s + beta * C, partials added in split order.
__global__ __launch_bounds__(256) void k_gemm_reduce(GemmArgs g) {
  if (g.info != nullptr && *g.info != 0) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.M * g.N) return;
  const int64_t i = e % g.M, j = e / g.M;
  if ((g.flags & GEMM_C_LOWER) && i < j) return;
  if ((g.flags & GEMM_C_UPPER) && i > j) return;
  // every split writes its partial (zero when its reduction range is empty)
  double s = 0.0;
  for (int t = 0; t < g.splits; ++t) s += g.partial[(int64_t)t * g.ldp * g.N + i + j * g.ldp];
  const double v = g.alpha * s;
  double* cp = (double*)g.C + i + j * g.ldc;
  *cp = (g.beta == 0.0) ? v : v + g.beta * *cp;
}

// ---- FP32 arithmetic: C(float) = op(A) op(B) with A, B rounded to FP32 ------
// v_mfma_f32_16x16x4_f32, per lane l: A operand (row l%16, k l/16), B operand
// (k l/16, column l%16), result entry r: (row 4(l/16) + r, column l%16).  A
// workgroup computes a 64 x 64 tile (waves 2 x 2, each 2 x 2 MFMA tiles);
// products and sums are FP32 (no split of the reduction).
__global__ __launch_bounds__(256, 2) void k_gemm_f32(GemmArgs g) {
  __shared__ float As[2][kGK * kGM];
  __shared__ float Bs[2][kGK * kGN];
  typedef float f4 __attribute__((ext_vector_type(4)));
  if (g.info != nullptr && *g.info != 0) return;
  const int64_t i0 = (int64_t)blockIdx.x * kGM, j0 = (int64_t)blockIdx.y * kGN;
  int64_t kb, ke;
  gemm_krange(g, i0, j0, 0, kb, ke);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave & 1) * 32, wc = (wave >> 1) * 32;
  float ra[kGStage], rb[kGStage];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int t = 0; t < kGStage; ++t) {
      const int e = tid + 256 * t;
      int r, k;
      if (g.transA) { k = e % kGK; r = e / kGK; } else { r = e & 63; k = e >> 6; }
      const int64_t gi = i0 + r, gk = k0 + k;
      ra[t] = (gi < g.M && gk < ke && a_in_triangle(g, gi, gk)) ? (float)load_opA<double>(g, gi, gk) : 0.0f;
      int kk, c;
      if (g.transB) { c = e & 63; kk = e >> 6; } else { kk = e % kGK; c = e / kGK; }
      const int64_t bk = k0 + kk, gj = j0 + c;
      rb[t] = (gj < g.N && bk < ke && b_in_triangle(g, bk, gj)) ? (float)load_opB<double>(g, bk, gj) : 0.0f;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int t = 0; t < kGStage; ++t) {
      const int e = tid + 256 * t;
      int r, k;
      if (g.transA) { k = e % kGK; r = e / kGK; } else { r = e & 63; k = e >> 6; }
      As[buf][as_pos(k, r)] = ra[t];
      int kk, c;
      if (g.transB) { c = e & 63; kk = e >> 6; } else { kk = e % kGK; c = e / kGK; }
      Bs[buf][bs_pos(kk, c)] = rb[t];
    }
  };
  f4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
  const int nchunks = ke > kb ? (int)((ke - kb + kGK - 1) / kGK) : 0;
  if (nchunks > 0) {
    gload(kb);
    sstore(0);
  }
  __syncthreads();
  const int r16 = lane & 15, k4 = lane >> 4;
  for (int ch = 0; ch < nchunks; ++ch) {
    const int cur = ch & 1;
    if (ch + 1 < nchunks) gload(kb + (int64_t)(ch + 1) * kGK);
#pragma unroll
    for (int ks = 0; ks < kGK; ks += 4) {
      float a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) a[t] = As[cur][as_pos(ks + k4, wr + 16 * t + r16)];
#pragma unroll
      for (int t = 0; t < 2; ++t) b[t] = Bs[cur][bs_pos(ks + k4, wc + 16 * t + r16)];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[x], b[y], acc[x][y], 0, 0, 0);
    }
    if (ch + 1 < nchunks) sstore(cur ^ 1);
    __syncthreads();
  }
  float* C = (float*)g.C;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wr + 16 * x + 4 * k4 + r, j = j0 + wc + 16 * y + r16;
        if (i < g.M && j < g.N) C[i + j * g.ldc] = (float)g.alpha * acc[x][y][r];
      }
}

size_t gemm_workspace_bytes(int64_t M, int64_t N, int splits) {
  if (splits <= 1) return 0;
  return (size_t)splits * (size_t)M * (size_t)N * sizeof(double);
}

int gemm_pick_splits(int64_t M, int64_t N, int64_t K, int num_cus) {
  const int64_t tiles = ((M + kGM - 1) / kGM) * ((N + kGN - 1) / kGN);
  const int64_t target = (int64_t)(num_cus > 0 ? num_cus : 256) * 2;
  if (tiles >= target / 2 || K < 4 * kGK) return 1;
  int64_t s = target / (tiles > 0 ? tiles : 1);
  const int64_t maxs = K / (2 * kGK);
  if (s > maxs) s = maxs;
  if (s > 256) s = 256;
  return s < 1 ? 1 : (int)s;
}

static hipError_t launch_gemm_impl(int ta_f32, int tb_f32, int transA, int transB, int64_t M, int64_t N, int64_t K,
                                   double alpha, const void* A, int64_t lda, const void* B, int64_t ldb, double beta,
                                   double* C, int64_t ldc, int flags, int splits, double* work, const int32_t* info,
                                   hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.alpha = alpha; g.beta = beta;
  g.transA = transA; g.transB = transB; g.flags = flags;
  g.info = info;
  if (splits < 1) splits = 1;
  int64_t kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + kGK - 1) / kGK * kGK;
  if (kchunk < kGK) kchunk = kGK;
  splits = K > 0 ? (int)((K + kchunk - 1) / kchunk) : 1;
  g.splits = splits;
  g.kchunk = kchunk;
  g.partial = work;
  g.ldp = M;
  if (splits > 1 && work == nullptr) return hipErrorInvalidValue;
  dim3 grid((unsigned)((M + kGM - 1) / kGM), (unsigned)((N + kGN - 1) / kGN), (unsigned)splits);
  if (!ta_f32 && !tb_f32) hipLaunchKernelGGL((k_gemm<double, double>), grid, dim3(256), 0, s, g);
  else if (ta_f32 && tb_f32) hipLaunchKernelGGL((k_gemm<float, float>), grid, dim3(256), 0, s, g);
  else if (ta_f32) hipLaunchKernelGGL((k_gemm<float, double>), grid, dim3(256), 0, s, g);
  else hipLaunchKernelGGL((k_gemm<double, float>), grid, dim3(256), 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  const int64_t total = M * N;
  hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_gemm(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                       int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int flags,
                       int splits, double* work, const int32_t* info, hipStream_t s) {
  return launch_gemm_impl(0, 0, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, flags, splits, work,
                          info, s);
}

hipError_t launch_gemm_in32(int a_f32, int b_f32, int transA, int transB, int64_t M, int64_t N, int64_t K,
                            double alpha, const void* A, int64_t lda, const void* B, int64_t ldb, double beta,
                            double* C, int64_t ldc, int flags, int splits, double* work, const int32_t* info,
                            hipStream_t s) {
  return launch_gemm_impl(a_f32, b_f32, transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, flags, splits,
                          work, info, s);
}

hipError_t launch_gemm_f32(int transA, int transB, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                           const double* B, int64_t ldb, float* C, int64_t ldc, int flags, const int32_t* info,
                           hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.alpha = 1.0; g.beta = 0.0;
  g.transA = transA; g.transB = transB; g.flags = flags & (GEMM_A_LOWER | GEMM_A_UPPER | GEMM_B_LOWER | GEMM_B_UPPER);
  g.info = info;
  g.splits = 1;
  g.kchunk = (K + kGK - 1) / kGK * kGK;
  if (g.kchunk < kGK) g.kchunk = kGK;
  dim3 grid((unsigned)((M + kGM - 1) / kGM), (unsigned)((N + kGN - 1) / kGN), 1);
  hipLaunchKernelGGL(k_gemm_f32, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace cqr2
