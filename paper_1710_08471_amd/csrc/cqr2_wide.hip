// Tall-skinny kernels for 128 < n <= 256 (the same steps as the n <= 128
// kernels, at twice the width):
//   k_gram_wide     partial Grams W = AᵀA over row blocks (Syrk; Algorithm 4
//                   step 1), all lower 16 x 16 tiles of one workgroup's rows
//                   held in registers, A read once;
//   k_gram_wide_reduce  fixed-order sum of the partials into W (lower);
//   k_tall          Q = A U for upper-triangular U (Algorithm 4 step 3), one
//                   128 x 256 output tile per workgroup, A read once; FP64
//                   arithmetic, or FP32 products and sums into an FP32 Q
//                   (pass 1 of the mixed-precision form).
// and, for any n > 256, the Gram by 128 x 256 tiles of its lower triangle:
//   k_syrk_tile     partial tiles over row splits, MFMA 4x4x4 fed the way
//                   k_tall is fed;
//   k_syrk_reduce   fixed-order sum of the partial tiles into W (lower);
//   k_syrk_update   the same tiles with the whole (short) reduction in one
//                   workgroup, added into W (the blocked CholInv's trailing
//                   update);
// and R = R2 R1 for n > 256:
//   k_upper_seg     k_tall's tiles on R2 and R1's upper image, each tile's
//                   reduction cut into segments;
//   k_upper_seg_reduce  fixed-order sum of a tile's segments.
#include "cqr2_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

#include "sync_dev.h"
#include "wide_dev.h"

namespace cqr2 {

template <typename TA>
__global__ __launch_bounds__(64 * kWideWaves, 1) void k_gram_wide(const TA* __restrict__ A, int64_t m, int n,
                                                                  int64_t lda, int64_t stages, int64_t spw,
                                                                  double* __restrict__ partials,
                                                                  const int32_t* __restrict__ info) {
  __shared__ __attribute__((aligned(16))) TA lds[2 * kWideBuf];
  if (info != nullptr && *info != 0) return;
  const int64_t st0 = (int64_t)blockIdx.x * spw;
  const int64_t st1 = st0 + spw < stages ? st0 + spw : stages;
  // 16-byte copies: A aligned and every column start aligned
  const bool direct_ok = (((uintptr_t)A & 15u) == 0) && (((lda * (int64_t)sizeof(TA)) & 15) == 0);
  double* out = partials + (int64_t)blockIdx.x * kWideLower * 256;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  switch (wave) {
    case 0: gram_wide_wave<TA, 0>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 1: gram_wide_wave<TA, 1>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 2: gram_wide_wave<TA, 2>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 3: gram_wide_wave<TA, 3>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 4: gram_wide_wave<TA, 4>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 5: gram_wide_wave<TA, 5>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 6: gram_wide_wave<TA, 6>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 7: gram_wide_wave<TA, 7>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    default: break;
  }
}

// n <= 128: the same body over 128 columns (36 lower tiles, four waves; two
// workgroups per CU).  The mixed form's Grams at n <= 128.
template <typename TA>
__global__ __launch_bounds__(256, 2) void k_gram128(const TA* __restrict__ A, int64_t m, int n, int64_t lda,
                                                   int64_t stages, int64_t spw, double* __restrict__ partials,
                                                   const int32_t* __restrict__ info) {
  __shared__ __attribute__((aligned(16))) TA lds[2 * 128 * kWideRows];
  if (info != nullptr && *info != 0) return;
  const int64_t st0 = (int64_t)blockIdx.x * spw;
  const int64_t st1 = st0 + spw < stages ? st0 + spw : stages;
  const bool direct_ok = (((uintptr_t)A & 15u) == 0) && (((lda * (int64_t)sizeof(TA)) & 15) == 0);
  double* out = partials + (int64_t)blockIdx.x * kLower128 * 256;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  switch (wave) {
    case 0: gram_cols_wave<TA, 128, 0>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 1: gram_cols_wave<TA, 128, 1>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 2: gram_cols_wave<TA, 128, 2>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 3: gram_cols_wave<TA, 128, 3>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    default: break;
  }
}

// Sum of the partials in split order (8 contiguous sub-ranges added in
// order), written to the lower triangle of W (n x n, ldw); ntiles lower
// tiles per split (136, or 36 for the 128-column Gram).
__global__ __launch_bounds__(256) void k_gram_wide_reduce(const double* __restrict__ part, int splits, int ntiles,
                                                          int n, double* __restrict__ W, int64_t ldw,
                                                          const int32_t* __restrict__ info) {
  __shared__ double red[8][32];
  if (info != nullptr && *info != 0) return;
  const int lanei = threadIdx.x & 31, sub = threadIdx.x >> 5;
  const int total = ntiles * 256;
  const int e = blockIdx.x * 32 + lanei;
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
  red[sub][lanei] = v;
  __syncthreads();
  if (sub != 0 || e >= total) return;
  double t = red[0][lanei];
#pragma unroll
  for (int k = 1; k < 8; ++k) t += red[k][lanei];
  const int tile = e >> 8, r = (e >> 6) & 3, l = e & 63;
  int I = 0;
  while ((I + 1) * (I + 2) / 2 <= tile) ++I;
  const int J = tile - I * (I + 1) / 2;
  const int row = 16 * I + 4 * r + (l >> 4), col = 16 * J + (l & 15);
  if (row >= col && row < n) W[row + (int64_t)col * ldw] = t;
}

WideGramPlan plan_gram_wide(int64_t m, int64_t n) {
  WideGramPlan p{};
  const bool narrow = n <= 128;  // the 128-column kernel: smaller workgroups, twice as many
  p.ntiles = narrow ? kLower128 : kWideLower;
  p.stages = m > 0 ? (m + kWideRows - 1) / kWideRows : 1;
  int64_t s = p.stages / 4;  // at least 4 stages per workgroup
  if (s < 1) s = 1;
  const int64_t cap = narrow ? 2 * kWideSplits : kWideSplits;
  if (s > cap) s = cap;
  p.stages_per_wg = (p.stages + s - 1) / s;
  p.splits = (int)((p.stages + p.stages_per_wg - 1) / p.stages_per_wg);
  p.partial_bytes = (size_t)p.splits * p.ntiles * 256 * sizeof(double);
  return p;
}

hipError_t launch_gram_wide(const WideGramPlan& p, int a_f32, const void* A, int64_t m, int n, int64_t lda,
                            double* partials, double* W, int64_t ldw, const int32_t* info, hipStream_t s) {
  if (n > kWideCols) return hipErrorInvalidValue;
  if (p.ntiles == kLower128 && n > 128) return hipErrorInvalidValue;
  if (p.ntiles == kLower128) {
    if (a_f32)
      hipLaunchKernelGGL(k_gram128<float>, dim3(p.splits), dim3(256), 0, s, (const float*)A, m, n, lda, p.stages,
                         p.stages_per_wg, partials, info);
    else
      hipLaunchKernelGGL(k_gram128<double>, dim3(p.splits), dim3(256), 0, s, (const double*)A, m, n, lda, p.stages,
                         p.stages_per_wg, partials, info);
  } else if (a_f32) {
    hipLaunchKernelGGL(k_gram_wide<float>, dim3(p.splits), dim3(64 * kWideWaves), 0, s, (const float*)A, m, n, lda,
                       p.stages, p.stages_per_wg, partials, info);
  } else {
    hipLaunchKernelGGL(k_gram_wide<double>, dim3(p.splits), dim3(64 * kWideWaves), 0, s, (const double*)A, m, n,
                       lda, p.stages, p.stages_per_wg, partials, info);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int total = p.ntiles * 256;
  hipLaunchKernelGGL(k_gram_wide_reduce, dim3((total + 31) / 32), dim3(256), 0, s, partials, p.splits, p.ntiles, n,
                     W, ldw, info);
  return hipGetLastError();
}

// ============================================================================
// Gram for n > 256 (Syrk; Algorithm 4 step 1), by 128 x 256 tiles of its
// lower triangle, on MFMA 4x4x4 in the manner of the tall kernel below.
//
// Workgroup (tile t, row split s) owns W(128 ti .., 256 tj ..) for the lower
// tiles (256 tj <= 128 ti + 127, ordered by ti then tj) and the 16-row chunks
// of its split.  Each chunk of the two column panels A(rows, 128 ti ..) and
// A(rows, 256 tj ..) is copied straight from global memory into a ring of
// three LDS buffers (16 KB + 32 KB; two chunks in flight while one is
// multiplied); each wave waits for its own copies by count, then a barrier
// publishes them.  In LDS a panel is column-major, 16 values per column, the
// k index of column c stored XOR 2 ((c >> 1) & 7) (the copies gather their
// source rows to match), so a fragment's 16 columns spread over the banks.
// Wave w owns the 64 x 64 block (64 (w / 4), 64 (w % 4)) of the tile: MFMA
// 4x4x4 with lane l holding A(k + l / 16, i + l % 16) and A(k + l / 16,
// j + l % 4), output lane l is W(i + 4 ((l >> 2) & 3) + l / 16, j + l % 4).
// Blocks and column groups wholly above the diagonal are skipped.  Columns
// past n are read from column n - 1 (finite data in outputs never written);
// rows past m are zero.  Partial tiles are summed over the splits in a fixed
// order by k_syrk_reduce.  An FP32 input (mixed precision's Q1) is staged as
// FP32 (16 columns per copy, the k slots XOR 4 ((c >> 2) & 3), which keeps
// the 4-value pieces of the copies whole) and widened exactly when read.
// ============================================================================
constexpr int kSyI = 128, kSyJ = 256, kSyK = 16, kSyBufs = 3;
constexpr int kSyWave = 64 * 64;       // doubles of one wave's partial block
constexpr int kSyTile = 8 * kSyWave;   // doubles of one workgroup's partial tile

// XOR on the k slots of column c in LDS (it keeps the values of one 16-byte copy together)
template <typename TA>
__device__ __forceinline__ int syrk_swz(int c) {
  if constexpr (sizeof(TA) == 8) return 2 * ((c >> 1) & 7);
  else return 4 * ((c >> 2) & 3);
}

// lower tile t -> (ti, tj): block row ti holds ti / 2 + 1 tiles, so the
// tiles of block rows 2a and 2a + 1 start at a (a + 1) and (a + 1)^2
__device__ __forceinline__ void syrk_tile(int t, int& ti, int& tj) {
  int a = (int)((sqrt(4.0 * t + 1.0) - 1.0) * 0.5);
  while (a * (a + 1) > t) --a;
  while ((a + 1) * (a + 2) <= t) ++a;
  if (t < (a + 1) * (a + 1)) {
    ti = 2 * a;
    tj = t - a * (a + 1);
  } else {
    ti = 2 * a + 1;
    tj = t - (a + 1) * (a + 1);
  }
}

static int syrk_ntiles(int64_t n) {
  const int64_t TI = (n + kSyI - 1) / kSyI;
  int64_t c = 0;
  for (int64_t ti = 0; ti < TI; ++ti) c += (ti >> 1) + 1;
  return (int)c;
}

// UPDATE: one split over all of m, and the tile goes straight into W:
// W(i, j) += alpha (AᵀA)(i, j) for j <= i < n; tiles from tile_base on (tile
// 0 is the leading 128 x 128 diagonal block).
template <typename TA, bool UPDATE>
__device__ __forceinline__ void syrk_tile_body(const TA* __restrict__ A, int64_t m, int n, int64_t lda,
                                               int64_t chunks_per_split, double* __restrict__ partials, int ntiles,
                                               int tile_base, double alpha, double* __restrict__ W, int64_t ldw) {
  constexpr int kES = (int)sizeof(TA);
  constexpr int kIBytes = kSyK * kSyI * kES, kJBytes = kSyK * kSyJ * kES, kBufBytes = kIBytes + kJBytes;
  // one copy moves 16 bytes per lane: 8 columns of FP64 or 16 of FP32
  constexpr int kColsPerCopy = 64 * 16 / (kSyK * kES);
  constexpr int kICopies = kSyI / kColsPerCopy / 8, kJCopies = kSyJ / kColsPerCopy / 8;  // per wave
  constexpr int kPerChunk = kICopies + kJCopies;
  __shared__ __attribute__((aligned(16))) char smem[kSyBufs * kBufBytes];
  int ti, tj;
  syrk_tile((int)blockIdx.x + tile_base, ti, tj);
  const int I0 = kSyI * ti, J0 = kSyJ * tj;
  const int64_t total_chunks = (m + kSyK - 1) / kSyK;
  const int64_t cb = (int64_t)blockIdx.y * chunks_per_split;
  const int64_t ce = cb + chunks_per_split < total_chunks ? cb + chunks_per_split : total_chunks;
  const int nch = ce > cb ? (int)(ce - cb) : 0;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = 64 * (wave >> 2), wc = 64 * (wave & 3);
  const bool aligned = (((uintptr_t)A & 15u) == 0) && (((lda * kES) & 15) == 0);
  auto ibuf = [&](int b) { return (TA*)(smem + b * kBufBytes); };
  auto jbuf = [&](int b) { return (TA*)(smem + b * kBufBytes + kIBytes); };
  auto direct_chunk = [&](int p) { return aligned && (cb + p + 1) * kSyK <= m; };
  auto issue = [&](int p) {
    const int b = p % kSyBufs;
    const int64_t row0 = (cb + p) * kSyK;
    TA* Ib = ibuf(b);
    TA* Jb = jbuf(b);
    if (direct_chunk(p)) {
      // one copy: kColsPerCopy columns x 16 rows; lane i -> column it kColsPerCopy + i / (64 / kColsPerCopy),
      // k slots kv (i % (64 / kColsPerCopy)) .. + kv - 1, kv = 16 / kES values
      constexpr int kLanesPerCol = 64 / kColsPerCopy, kV = 16 / kES;
      const int sub = lane / kLanesPerCol, kp = kV * (lane % kLanesPerCol);
#pragma unroll
      for (int t = 0; t < kICopies; ++t) {
        const int it = kICopies * wave + t, c = kColsPerCopy * it + sub;
        const int col = I0 + c < n ? I0 + c : n - 1;
        __builtin_amdgcn_global_load_lds((const void*)(A + row0 + (kp ^ syrk_swz<TA>(c)) + (int64_t)col * lda),
                                         (__attribute__((address_space(3))) void*)(Ib + kColsPerCopy * it * kSyK), 16,
                                         0, 0);
      }
#pragma unroll
      for (int t = 0; t < kJCopies; ++t) {
        const int it = kJCopies * wave + t, c = kColsPerCopy * it + sub;
        const int col = J0 + c < n ? J0 + c : n - 1;
        __builtin_amdgcn_global_load_lds((const void*)(A + row0 + (kp ^ syrk_swz<TA>(c)) + (int64_t)col * lda),
                                         (__attribute__((address_space(3))) void*)(Jb + kColsPerCopy * it * kSyK), 16,
                                         0, 0);
      }
    } else {
      for (int e = tid; e < kSyK * (kSyI + kSyJ); e += 512) {
        const int c = e / kSyK, k = e % kSyK;
        const bool in_i = c < kSyI;
        const int cc = in_i ? c : c - kSyI;
        int col = (in_i ? I0 : J0) + cc;
        col = col < n ? col : n - 1;
        const int64_t r = row0 + k;
        (in_i ? Ib : Jb)[cc * kSyK + (k ^ syrk_swz<TA>(cc))] = r < m ? A[r + (int64_t)col * lda] : (TA)0;
      }
    }
  };

  double acc[4][16];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 16; ++b) acc[a][b] = 0.0;
  // this wave's 64 x 64 block: nothing to do above the diagonal or past n
  const bool live = (J0 + wc <= I0 + wr + 63) && (I0 + wr < n) && (J0 + wc < n);
  if (nch > 0) issue(0);
  if (nch > 1) issue(1);
  const int ar = lane & 15, ak = lane >> 4, bc = lane & 3;
  for (int p = 0; p < nch; ++p) {
    if (p + 1 < nch && direct_chunk(p + 1)) wait_vmcnt<kPerChunk>();
    else wait_vmcnt<0>();
    lds_barrier();
    if (p + 2 < nch) issue(p + 2);
    const TA* Ib = ibuf(p % kSyBufs);
    const TA* Jb = jbuf(p % kSyBufs);
    if (live) {
#pragma unroll
      for (int ks = 0; ks < kSyK; ks += 4) {
        const int kk = ks + ak;
        double a[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) {
          const int c = wr + 16 * rt + ar;
          a[rt] = (double)Ib[c * kSyK + (kk ^ syrk_swz<TA>(c))];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (J0 + wc + 16 * q <= I0 + wr + 63) {  // uniform: the column group reaches the lower triangle
            double b[4];
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4) {
              const int c = wc + 16 * q + 4 * c4 + bc;
              b[c4] = (double)Jb[c * kSyK + (kk ^ syrk_swz<TA>(c))];
            }
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4)
#pragma unroll
              for (int rt = 0; rt < 4; ++rt)
                acc[rt][4 * q + c4] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[rt], b[c4], acc[rt][4 * q + c4], 0, 0, 0);
          }
        }
      }
    }
  }
  if constexpr (UPDATE) {
    if (!live) return;
    // a row tile's 16 values of W are all loaded before any is stored (the
    // stores could alias later loads as far as the compiler knows)
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int i = I0 + wr + 16 * rt + 4 * ((lane >> 2) & 3) + (lane >> 4);
      double w[16];
#pragma unroll
      for (int cg = 0; cg < 16; ++cg) {
        const int j = J0 + wc + 4 * cg + (lane & 3);
        w[cg] = (i < n && j <= i) ? W[i + (int64_t)j * ldw] : 0.0;
      }
#pragma unroll
      for (int cg = 0; cg < 16; ++cg) {
        const int j = J0 + wc + 4 * cg + (lane & 3);
        if (i < n && j <= i) W[i + (int64_t)j * ldw] = fma(alpha, acc[rt][cg], w[cg]);
      }
    }
  } else {
    // lane-major partial block: entry (rt, cg) of lane l at (rt 16 + cg) 64 + l
    double* out = partials + ((int64_t)blockIdx.y * ntiles + blockIdx.x) * kSyTile + wave * kSyWave;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int cg = 0; cg < 16; ++cg) out[(rt * 16 + cg) * 64 + lane] = acc[rt][cg];
  }
}

template <typename TA>
__global__ __launch_bounds__(512, 1) void k_syrk_tile(const TA* __restrict__ A, int64_t m, int n, int64_t lda,
                                                      int64_t chunks_per_split, double* __restrict__ partials,
                                                      int ntiles, const int32_t* __restrict__ info) {
  if (info != nullptr && *info != 0) return;
  syrk_tile_body<TA, false>(A, m, n, lda, chunks_per_split, partials, ntiles, 0, 0.0, nullptr, 0);
}

__global__ __launch_bounds__(512, 1) void k_syrk_update(const double* __restrict__ A, int64_t m, int n, int64_t lda,
                                                        int tile_base, double alpha, double* __restrict__ W,
                                                        int64_t ldw, const int32_t* __restrict__ info) {
  if (info != nullptr && *info != 0) return;
  syrk_tile_body<double, true>(A, m, n, lda, (m + kSyK - 1) / kSyK, nullptr, 0, tile_base, alpha, W, ldw);
}

// W(i, j), i >= j: the partial tiles summed in split order.
__global__ __launch_bounds__(256) void k_syrk_reduce(const double* __restrict__ part, int splits, int ntiles, int n,
                                                     double* __restrict__ W, int64_t ldw,
                                                     const int32_t* __restrict__ info) {
  if (info != nullptr && *info != 0) return;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)ntiles * kSyTile) return;
  const int tile = (int)(e / kSyTile), rem = (int)(e % kSyTile);
  int ti, tj;
  syrk_tile(tile, ti, tj);
  const int wave = rem / kSyWave, x = rem % kSyWave;
  const int lane = x & 63, cg = (x >> 6) & 15, rt = x >> 10;
  const int i = kSyI * ti + 64 * (wave >> 2) + 16 * rt + 4 * ((lane >> 2) & 3) + (lane >> 4);
  const int j = kSyJ * tj + 64 * (wave & 3) + 4 * cg + (lane & 3);
  if (i >= n || j > i) return;
  double v = 0.0;
  for (int s = 0; s < splits; ++s) v += part[(int64_t)s * ntiles * kSyTile + e];
  W[i + (int64_t)j * ldw] = v;
}

hipError_t launch_syrk_update(const double* A, int64_t m, int n, int64_t lda, double alpha, double* W, int64_t ldw,
                              int skip_first_block_row, const int32_t* info, hipStream_t s) {
  if (n <= 0 || m < 0) return hipSuccess;
  const int base = skip_first_block_row ? 1 : 0;
  const int tiles = syrk_ntiles(n) - base;
  if (tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_syrk_update, dim3(tiles), dim3(512), 0, s, A, m, n, lda, base, alpha, W, ldw, info);
  return hipGetLastError();
}

// Splits fill the device several times over (about 4096 workgroups, one per
// CU at a time), with at least 32 chunks (512 rows) each and at most 1 GiB of
// partial tiles.
SyrkPlan plan_syrk(int64_t m, int64_t n) {
  SyrkPlan p{};
  p.npairs = syrk_ntiles(n);
  p.stages = m > 0 ? (m + kSyK - 1) / kSyK : 0;
  const int64_t tile_bytes = (int64_t)kSyTile * sizeof(double);
  int64_t s = (4096 + p.npairs - 1) / p.npairs;
  const int64_t by_rows = p.stages / 32 > 0 ? p.stages / 32 : 1;
  const int64_t by_bytes = ((int64_t)1 << 30) / (tile_bytes * p.npairs) > 0 ? ((int64_t)1 << 30) / (tile_bytes * p.npairs) : 1;
  if (s > by_rows) s = by_rows;
  if (s > by_bytes) s = by_bytes;
  if (s < 1) s = 1;
  p.stages_per_wg = p.stages > 0 ? (p.stages + s - 1) / s : 1;
  p.splits = p.stages > 0 ? (int)((p.stages + p.stages_per_wg - 1) / p.stages_per_wg) : 1;
  p.partial_bytes = (size_t)p.splits * p.npairs * tile_bytes;
  return p;
}

hipError_t launch_syrk(const SyrkPlan& p, int a_f32, const void* A, int64_t m, int n, int64_t lda, double* partials,
                       double* W, int64_t ldw, const int32_t* info, hipStream_t s) {
  if (a_f32)
    hipLaunchKernelGGL((k_syrk_tile<float>), dim3(p.npairs, p.splits), dim3(512), 0, s, (const float*)A, m, n, lda,
                       p.stages_per_wg, partials, p.npairs, info);
  else
    hipLaunchKernelGGL((k_syrk_tile<double>), dim3(p.npairs, p.splits), dim3(512), 0, s, (const double*)A, m, n, lda,
                       p.stages_per_wg, partials, p.npairs, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = (int64_t)p.npairs * kSyTile;
  hipLaunchKernelGGL(k_syrk_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, partials, p.splits,
                     p.npairs, n, W, ldw, info);
  return hipGetLastError();
}

// ============================================================================
// Q = A U for upper-triangular U (Algorithm 4 step 3).
//
// U comes as a zero-padded row-major image (U(k, j) at U[ld k + j], ld = n
// rounded up to 256, zero outside the n x n upper triangle), so a chunk of 16
// rows of U for 256 columns is 32 KB of contiguous memory.  A workgroup owns
// 128 rows of A and 256 output columns (grid.y walks the column tiles; the
// reduction stops at the tile's last column, U(k, j) = 0 for k > j): 8 waves, wave w covers rows 64 (w / 4) .. +64 and a 64-column
// group; the two waves sharing a SIMD (w, w + 4) get the lightest and the
// heaviest share of the triangle.  The reduction walks 16-column chunks of A
// and 16-row chunks of U, both copied straight from global memory into a
// ring of three LDS buffers (two chunks in flight while one is multiplied);
// each wave waits for its own copies by count, then a barrier publishes them.
// A wave skips the column groups a chunk cannot reach (U(k, j) = 0, k > j).
//
// FP64 arithmetic: MFMA 4x4x4 with lane l holding A(r0 + (l&15), k + (l>>4))
// and U(k + (l>>4), c0 + (l&3)); output lane l is Q(r0 + 4((l>>2)&3) + (l>>4),
// c0 + (l&3)).  FP32 arithmetic (F32MATH): MFMA 16x16x4 f32 on Qᵀ = Uᵀ Aᵀ,
// first operand U(k, j0 + l%16), second A(i0 + l%16, k), result entry r of
// lane l is Q(i0 + l%16, j0 + 4(l/16) + r).
// A is FP64 or FP32 (TA), kept in LDS as TA and converted when read.
// ============================================================================
constexpr int kTallRows = 128;
constexpr int kTallK = 16;
constexpr int kTallUld = 256;
constexpr int kTallBufs = 3;

__device__ __forceinline__ int tall_wave_col0(int w) {
  const int g = w & 3;
  return 64 * ((w < 4) ? g : 3 - g);
}

template <typename TA, bool F32MATH>
__global__ __launch_bounds__(512, 1) void k_tall(const TA* __restrict__ A, int64_t m, int n, int64_t lda,
                                                 const double* __restrict__ U, int64_t ldu, void* __restrict__ Qv,
                                                 int64_t ldq, const int32_t* __restrict__ info) {
  constexpr int kABytes = kTallK * kTallRows * (int)sizeof(TA);
  constexpr int kUBytes = kTallK * kTallUld * 8;
  constexpr int kBufBytes = kABytes + kUBytes;
  // per wave and chunk: A columns of 1 KB (2 per wave) or 2 FP32 columns per KB (1 per wave); U rows 2 KB (4 per wave)
  constexpr int kAInstr = sizeof(TA) == 8 ? 2 : 1;
  constexpr int kUInstr = 4;
  constexpr int kPerChunk = kAInstr + kUInstr;
  __shared__ __attribute__((aligned(16))) char smem[kTallBufs * kBufBytes];
  if (info != nullptr && *info != 0) return;
  const int64_t i0 = (int64_t)blockIdx.x * kTallRows;
  const int j0 = (int)blockIdx.y * kTallUld;  // this workgroup's 256 output columns
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = 64 * (wave >> 2), wc = j0 + tall_wave_col0(wave);  // wc: global column of the wave's group
  const int kend = n < j0 + kTallUld ? n : j0 + kTallUld;           // U(k, j) = 0 for k > j
  const int nchunks = (kend + kTallK - 1) / kTallK;
  const bool direct = (i0 + kTallRows <= m) && (((uintptr_t)A & 15u) == 0) &&
                      (((lda * (int64_t)sizeof(TA)) & 15) == 0);

  auto abuf = [&](int b) { return (TA*)(smem + b * kBufBytes); };
  auto ubuf = [&](int b) { return (double*)(smem + b * kBufBytes + kABytes); };

  // Columns of a chunk past n are read from column n - 1 (finite data times
  // the zero rows of U), which keeps every wave's copy count per chunk fixed.
  auto issue = [&](int ch) {
    const int b = ch % kTallBufs;
    const int k0 = ch * kTallK;
    TA* As = abuf(b);
    if (direct) {
      if constexpr (sizeof(TA) == 8) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int kc = 2 * wave + t;  // one column: 128 rows, lane i -> rows 2i, 2i+1
          const int col = k0 + kc < n ? k0 + kc : n - 1;
          __builtin_amdgcn_global_load_lds((const void*)(A + i0 + 2 * lane + (int64_t)col * lda),
                                           (__attribute__((address_space(3))) void*)(As + kc * kTallRows), 16, 0,
                                           0);
        }
      } else {
        const int kc = 2 * wave + (lane >> 5);  // two columns: lane i -> rows 4(i&31) .. +3
        const int col = k0 + kc < n ? k0 + kc : n - 1;
        __builtin_amdgcn_global_load_lds((const void*)(A + i0 + 4 * (lane & 31) + (int64_t)col * lda),
                                         (__attribute__((address_space(3))) void*)(As + 2 * wave * kTallRows), 16,
                                         0, 0);
      }
    } else {
      for (int e = tid; e < kTallK * kTallRows; e += 512) {
        const int r = e % kTallRows, kc = e / kTallRows;
        const int64_t gi = i0 + r;
        const int col = k0 + kc < n ? k0 + kc : n - 1;
        As[kc * kTallRows + r] = gi < m ? A[gi + (int64_t)col * lda] : (TA)0;
      }
    }
    double* Us = ubuf(b);
#pragma unroll
    for (int t = 0; t < kUInstr; ++t) {
      const int h = 4 * wave + t;  // half-row h/2 of the chunk, 128 doubles
      const int kr = h >> 1, c0 = 128 * (h & 1);
      __builtin_amdgcn_global_load_lds((const void*)(U + (int64_t)(k0 + kr) * ldu + j0 + c0 + 2 * lane),
                                       (__attribute__((address_space(3))) void*)(Us + kr * kTallUld + c0), 16, 0, 0);
    }
  };

  // zero the buffers once (a ragged tile's rows past m are then never garbage)
  for (int e = tid; e < kTallBufs * kBufBytes / 8; e += 512) ((double*)smem)[e] = 0.0;
  lds_barrier();

  if constexpr (!F32MATH) {
    double acc[4][16];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 16; ++b) acc[a][b] = 0.0;
    issue(0);
    if (nchunks > 1) issue(1);
    const int ar = lane & 15, ak = lane >> 4, bc = lane & 3;
    for (int ch = 0; ch < nchunks; ++ch) {
      if (direct && ch + 1 < nchunks) wait_vmcnt<kPerChunk>();
      else wait_vmcnt<0>();
      lds_barrier();
      if (ch + 2 < nchunks) issue(ch + 2);
      const TA* As = abuf(ch % kTallBufs);
      const double* Us = ubuf(ch % kTallBufs);
      const int k0 = ch * kTallK;
      if (wc + 63 >= k0 && wc < n) {
#pragma unroll
        for (int ks = 0; ks < kTallK; ks += 4) {
          const int kk = ks + ak;
          double a[4];
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) a[rt] = (double)As[kk * kTallRows + wr + 16 * rt + ar];
#pragma unroll
          for (int q = 0; q < 4; ++q) {  // 16 columns at a time: U(k, j) = 0 for every k > j
            if (wc + 16 * q + 15 >= k0 + ks) {
              double b[4];
#pragma unroll
              for (int c = 0; c < 4; ++c) b[c] = Us[kk * kTallUld + (wc - j0) + 16 * q + 4 * c + bc];
#pragma unroll
              for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int rt = 0; rt < 4; ++rt)
                  acc[rt][4 * q + c] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[rt], b[c], acc[rt][4 * q + c], 0, 0, 0);
            }
          }
        }
      }
    }
    double* Q = (double*)Qv;
    const int orow = 4 * ((lane >> 2) & 3) + (lane >> 4), ocol = lane & 3;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int64_t i = i0 + wr + 16 * rt + orow;
      if (i >= m) continue;
#pragma unroll
      for (int cg = 0; cg < 16; ++cg) {
        const int j = wc + 4 * cg + ocol;
        if (j < n) Q[i + (int64_t)j * ldq] = acc[rt][cg];
      }
    }
  } else {
    typedef float f4 __attribute__((ext_vector_type(4)));
    f4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = f4{0.f, 0.f, 0.f, 0.f};
    issue(0);
    if (nchunks > 1) issue(1);
    const int l16 = lane & 15, k4 = lane >> 4;
    for (int ch = 0; ch < nchunks; ++ch) {
      if (direct && ch + 1 < nchunks) wait_vmcnt<kPerChunk>();
      else wait_vmcnt<0>();
      lds_barrier();
      if (ch + 2 < nchunks) issue(ch + 2);
      const TA* As = abuf(ch % kTallBufs);
      const double* Us = ubuf(ch % kTallBufs);
      const int k0 = ch * kTallK;
      if (wc + 63 >= k0 && wc < n) {
#pragma unroll
        for (int ks = 0; ks < kTallK; ks += 4) {
          const int kk = ks + k4;
          float a[4], u[4];
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) a[rt] = (float)As[kk * kTallRows + wr + 16 * rt + l16];
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) u[ct] = (float)Us[kk * kTallUld + (wc - j0) + 16 * ct + l16];
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) {
            if (wc + 16 * ct + 15 >= k0 + ks) {
#pragma unroll
              for (int rt = 0; rt < 4; ++rt)
                acc[rt][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(u[ct], a[rt], acc[rt][ct], 0, 0, 0);
            }
          }
        }
      }
    }
    float* Q = (float*)Qv;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      const int64_t i = i0 + wr + 16 * rt + l16;
      if (i >= m) continue;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = wc + 16 * ct + 4 * k4 + r;
          if (j < n) Q[i + (int64_t)j * ldq] = acc[rt][ct][r];
        }
    }
  }
}

// ============================================================================
// R = X Y for upper-triangular X, Y (n x n): the tall kernel's 128 x 256 tiles
// and chunk pipeline, with X column-major (ldx, zero below its diagonal) as A
// and Y as its zero-padded row-major image.  A tile (I, J) reduces over
// k in [128 I, min(n, 256 (J + 1))) only; that range is cut into segments of
// at most kSegChunks 16-wide chunks so that the far-corner tiles (whole-n
// reductions) spread over several workgroups.  Work items run over the tiles
// in row-major order, each tile's segments in turn; a tile with one segment
// writes R directly, the others write partial tiles that k_upper_seg_reduce
// adds in segment order.  Tiles wholly below the diagonal are skipped (R's
// lower triangle is left to the caller).
// ============================================================================
constexpr int kSegChunks = 64;  // 1024 of the reduction (measured: 16 to 256 chunks, 64 fastest at n = 4096)

struct SegItem {
  int I, J, cb, ce;  // tile and chunk range
  int slot;          // partial slot, or -1 for a one-segment tile
};

// the work item `item` of the order above (or I = -1 past the last)
__device__ __host__ inline SegItem seg_item(int n, int item) {
  const int TI = (n + kTallRows - 1) / kTallRows, TJ = (n + kTallUld - 1) / kTallUld;
  int slot = 0;
  for (int I = 0; I < TI; ++I)
    for (int J = 0; J < TJ; ++J) {
      const int kend = n < kTallUld * (J + 1) ? n : kTallUld * (J + 1);
      const int cb = (kTallRows * I) / kTallK, ce = (kend + kTallK - 1) / kTallK;
      if (ce <= cb) continue;
      const int nseg = (ce - cb + kSegChunks - 1) / kSegChunks;
      if (item < nseg) {
        const int b = cb + item * kSegChunks, e = b + kSegChunks < ce ? b + kSegChunks : ce;
        return SegItem{I, J, b, e, nseg > 1 ? slot + item : -1};
      }
      item -= nseg;
      if (nseg > 1) slot += nseg;
    }
  return SegItem{-1, -1, 0, 0, -1};
}

__global__ __launch_bounds__(512, 1) void k_upper_seg(const double* __restrict__ X, int n, int64_t ldx,
                                                      const double* __restrict__ Y, int64_t ldy,
                                                      double* __restrict__ R, int64_t ldr,
                                                      double* __restrict__ part, const int32_t* __restrict__ info) {
  constexpr int kABytes = kTallK * kTallRows * 8;
  constexpr int kUBytes = kTallK * kTallUld * 8;
  constexpr int kBufBytes = kABytes + kUBytes;
  constexpr int kPerChunk = 2 + 4;  // per wave and chunk: two 1 KB X columns, four 1 KB halves of Y rows
  __shared__ __attribute__((aligned(16))) char smem[kTallBufs * kBufBytes];
  if (info != nullptr && *info != 0) return;
  const SegItem it = seg_item(n, (int)blockIdx.x);
  if (it.I < 0) return;
  const int64_t i0 = (int64_t)it.I * kTallRows;
  const int j0 = it.J * kTallUld;
  const int count = it.ce - it.cb;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = 64 * (wave >> 2), wc = j0 + tall_wave_col0(wave);
  const bool direct = (i0 + kTallRows <= n) && (((uintptr_t)X & 15u) == 0) && (((ldx * 8) & 15) == 0);
  auto abuf = [&](int b) { return (double*)(smem + b * kBufBytes); };
  auto ubuf = [&](int b) { return (double*)(smem + b * kBufBytes + kABytes); };
  // chunk c of this item (absolute chunk it.cb + c) into buffer c % kTallBufs;
  // columns of X past n are read from column n - 1 (times zero rows of Y)
  auto issue = [&](int c) {
    const int b = c % kTallBufs;
    const int k0 = (it.cb + c) * kTallK;
    double* As = abuf(b);
    if (direct) {
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int kc = 2 * wave + t;
        const int col = k0 + kc < n ? k0 + kc : n - 1;
        __builtin_amdgcn_global_load_lds((const void*)(X + i0 + 2 * lane + (int64_t)col * ldx),
                                         (__attribute__((address_space(3))) void*)(As + kc * kTallRows), 16, 0, 0);
      }
    } else {
      for (int e = tid; e < kTallK * kTallRows; e += 512) {
        const int r = e % kTallRows, kc = e / kTallRows;
        const int64_t gi = i0 + r;
        const int col = k0 + kc < n ? k0 + kc : n - 1;
        As[kc * kTallRows + r] = gi < n ? X[gi + (int64_t)col * ldx] : 0.0;
      }
    }
    double* Us = ubuf(b);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int h = 4 * wave + t;
      const int kr = h >> 1, c0 = 128 * (h & 1);
      __builtin_amdgcn_global_load_lds((const void*)(Y + (int64_t)(k0 + kr) * ldy + j0 + c0 + 2 * lane),
                                       (__attribute__((address_space(3))) void*)(Us + kr * kTallUld + c0), 16, 0, 0);
    }
  };
  for (int e = tid; e < kTallBufs * kBufBytes / 8; e += 512) ((double*)smem)[e] = 0.0;
  lds_barrier();

  double acc[4][16];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 16; ++b) acc[a][b] = 0.0;
  issue(0);
  if (count > 1) issue(1);
  const int ar = lane & 15, ak = lane >> 4, bc = lane & 3;
  for (int c = 0; c < count; ++c) {
    if (direct && c + 1 < count) wait_vmcnt<kPerChunk>();
    else wait_vmcnt<0>();
    lds_barrier();
    if (c + 2 < count) issue(c + 2);
    const double* As = abuf(c % kTallBufs);
    const double* Us = ubuf(c % kTallBufs);
    const int k0 = (it.cb + c) * kTallK;
    if (wc + 63 >= k0 && wc < n) {
#pragma unroll
      for (int ks = 0; ks < kTallK; ks += 4) {
        const int kk = ks + ak;
        double a[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) a[rt] = As[kk * kTallRows + wr + 16 * rt + ar];
#pragma unroll
        for (int q = 0; q < 4; ++q) {  // Y(k, j) = 0 for every k > j
          if (wc + 16 * q + 15 >= k0 + ks) {
            double b[4];
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4) b[c4] = Us[kk * kTallUld + (wc - j0) + 16 * q + 4 * c4 + bc];
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4)
#pragma unroll
              for (int rt = 0; rt < 4; ++rt)
                acc[rt][4 * q + c4] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[rt], b[c4], acc[rt][4 * q + c4], 0, 0, 0);
          }
        }
      }
    }
  }
  // output lane l: (r0 + 4 ((l >> 2) & 3) + (l >> 4), c0 + (l & 3)); a partial tile is
  // 128 x 256 column-major (ld 128)
  double* out = it.slot < 0 ? R + i0 + (int64_t)j0 * ldr : part + (int64_t)it.slot * kTallRows * kTallUld;
  const int64_t ldo = it.slot < 0 ? ldr : kTallRows;
  const int orow = 4 * ((lane >> 2) & 3) + (lane >> 4), ocol = lane & 3;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
    const int ri = wr + 16 * rt + orow;
    if (i0 + ri >= n) continue;
#pragma unroll
    for (int cg = 0; cg < 16; ++cg) {
      const int cj = wc - j0 + 4 * cg + ocol;
      if (j0 + cj < n) out[ri + (int64_t)cj * ldo] = acc[rt][cg];
    }
  }
}

// The t-th tile with several segments (row-major order): its tile, first
// partial slot and segment count (I = -1 past the last).
__device__ inline void seg_multi_tile(int n, int t, int& I_, int& J_, int& slot_, int& nseg_) {
  const int TI = (n + kTallRows - 1) / kTallRows, TJ = (n + kTallUld - 1) / kTallUld;
  int slot = 0;
  I_ = -1;
  for (int I = 0; I < TI; ++I)
    for (int J = 0; J < TJ; ++J) {
      const int kend = n < kTallUld * (J + 1) ? n : kTallUld * (J + 1);
      const int cb = (kTallRows * I) / kTallK, ce = (kend + kTallK - 1) / kTallK;
      if (ce <= cb) continue;
      const int nseg = (ce - cb + kSegChunks - 1) / kSegChunks;
      if (nseg <= 1) continue;
      if (t == 0) {
        I_ = I, J_ = J, slot_ = slot, nseg_ = nseg;
        return;
      }
      --t;
      slot += nseg;
    }
}

// R tiles with several segments: their partial tiles added in segment order,
// kSegReduceWGs workgroups per tile (blockIdx.y: the piece), the loads of all
// segments of an entry issued before the sum.
constexpr int kSegReduceWGs = 4;
constexpr int kSegMaxParts = (4096 / kTallK + kSegChunks - 1) / kSegChunks;  // segments of a 4096-long reduction

__global__ __launch_bounds__(256) void k_upper_seg_reduce(int n, double* __restrict__ R, int64_t ldr,
                                                          const double* __restrict__ part,
                                                          const int32_t* __restrict__ info) {
  if (info != nullptr && *info != 0) return;
  int I, J, slot, nseg;
  seg_multi_tile(n, (int)blockIdx.x, I, J, slot, nseg);
  if (I < 0) return;
  const double* p0 = part + (int64_t)slot * kTallRows * kTallUld;
  constexpr int kPiece = kTallRows * kTallUld / kSegReduceWGs;
  for (int e = (int)blockIdx.y * kPiece + (int)threadIdx.x; e < ((int)blockIdx.y + 1) * kPiece; e += 256) {
    const int ri = e % kTallRows, cj = e / kTallRows;
    const int64_t i = (int64_t)I * kTallRows + ri, j = (int64_t)J * kTallUld + cj;
    if (i >= n || j >= n) continue;
    double v = 0.0;
    for (int s0 = 0; s0 < nseg; s0 += kSegMaxParts) {
      double x[kSegMaxParts];
#pragma unroll
      for (int q = 0; q < kSegMaxParts; ++q)
        x[q] = s0 + q < nseg ? p0[(int64_t)(s0 + q) * kTallRows * kTallUld + e] : 0.0;
#pragma unroll
      for (int q = 0; q < kSegMaxParts; ++q)
        if (s0 + q < nseg) v += x[q];
    }
    R[i + j * ldr] = v;
  }
}

// Items, partial slots and multi-segment tiles of the segmented product (the
// host side of seg_item).
static void upper_seg_plan(int n, int* items, int* slots, int* multi) {
  const int TI = (n + kTallRows - 1) / kTallRows, TJ = (n + kTallUld - 1) / kTallUld;
  int it = 0, sl = 0, mt = 0;
  for (int I = 0; I < TI; ++I)
    for (int J = 0; J < TJ; ++J) {
      const int kend = n < kTallUld * (J + 1) ? n : kTallUld * (J + 1);
      const int cb = (kTallRows * I) / kTallK, ce = (kend + kTallK - 1) / kTallK;
      if (ce <= cb) continue;
      const int nseg = (ce - cb + kSegChunks - 1) / kSegChunks;
      it += nseg;
      if (nseg > 1) sl += nseg, ++mt;
    }
  *items = it;
  *slots = sl;
  *multi = mt;
}

size_t upper_seg_partial_bytes(int64_t n) {
  int items = 0, slots = 0, multi = 0;
  upper_seg_plan((int)n, &items, &slots, &multi);
  return (size_t)slots * kTallRows * kTallUld * sizeof(double);
}

hipError_t launch_upper_seg(const double* X, int n, int64_t ldx, const double* Yimg, double* R, int64_t ldr,
                            double* part, const int32_t* info, hipStream_t s) {
  int items = 0, slots = 0, multi = 0;
  upper_seg_plan(n, &items, &slots, &multi);
  if (items <= 0) return hipSuccess;
  if (slots > 0 && part == nullptr) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_upper_seg, dim3((unsigned)items), dim3(512), 0, s, X, n, ldx, Yimg, upper_image_ld(n), R, ldr,
                     part, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || multi == 0) return e;
  hipLaunchKernelGGL(k_upper_seg_reduce, dim3((unsigned)multi, kSegReduceWGs), dim3(256), 0, s, n, R, ldr, part,
                     info);
  return hipGetLastError();
}

// Row-major, zero-padded image of the upper triangle of an n x n column-major
// X (ldx): T[ldt k + j] = X(k, j) for k <= j < n, else 0, for k, j < ldt
// (ldt = n rounded up to 256).
__global__ __launch_bounds__(256) void k_upper_image(const double* __restrict__ X, int64_t ldx, int n,
                                                     double* __restrict__ T, int64_t ldt) {
  __shared__ double tile[32][33];
  const int bk = blockIdx.y * 32, bj = blockIdx.x * 32;  // T rows k, columns j
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int q = ty; q < 32; q += 8) {  // read X(k = bk + tx, j = bj + q): coalesced along k
    const int k = bk + tx, j = bj + q;
    tile[q][tx] = (k <= j && j < n) ? X[k + (int64_t)j * ldx] : 0.0;
  }
  __syncthreads();
  for (int q = ty; q < 32; q += 8) {  // write T[k = bk + q][j = bj + tx]: coalesced along j
    T[(int64_t)(bk + q) * ldt + bj + tx] = tile[tx][q];
  }
}

int64_t upper_image_ld(int64_t n) { return (n + kTallUld - 1) / kTallUld * kTallUld; }

hipError_t launch_upper_image(const double* X, int64_t ldx, int n, double* T, hipStream_t s) {
  const int64_t ld = upper_image_ld(n);
  hipLaunchKernelGGL(k_upper_image, dim3((unsigned)(ld / 32), (unsigned)(ld / 32)), dim3(256), 0, s, X, ldx, n, T,
                     ld);
  return hipGetLastError();
}

hipError_t launch_tall_gemm(int a_f32, const void* A, int64_t m, int n, int64_t lda, const double* Uimg, double* Q,
                            int64_t ldq, const int32_t* info, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  // n <= 256: the MFMA 16x16x4 streaming kernels (128 or 256 columns)
  if (n <= 128) return launch_apply128(a_f32, 0, A, m, n, lda, Uimg, Q, ldq, info, s);
  if (n <= kTallUld) return launch_apply256(a_f32, 0, A, m, n, lda, Uimg, Q, ldq, info, s);
  const int64_t ld = upper_image_ld(n);
  dim3 grid((unsigned)((m + kTallRows - 1) / kTallRows), (unsigned)(ld / kTallUld));
  if (a_f32)
    hipLaunchKernelGGL((k_tall<float, false>), grid, dim3(512), 0, s, (const float*)A, m, n, lda, Uimg, ld,
                       (void*)Q, ldq, info);
  else
    hipLaunchKernelGGL((k_tall<double, false>), grid, dim3(512), 0, s, (const double*)A, m, n, lda, Uimg, ld,
                       (void*)Q, ldq, info);
  return hipGetLastError();
}

hipError_t launch_tall_gemm_f32(const double* A, int64_t m, int n, int64_t lda, const double* Uimg, float* Q,
                                int64_t ldq, const int32_t* info, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (n <= 128) return launch_apply128(0, 1, A, m, n, lda, Uimg, Q, ldq, info, s);
  if (n <= kTallUld) return launch_apply256(0, 1, A, m, n, lda, Uimg, Q, ldq, info, s);
  const int64_t ld = upper_image_ld(n);
  dim3 grid((unsigned)((m + kTallRows - 1) / kTallRows), (unsigned)(ld / kTallUld));
  hipLaunchKernelGGL((k_tall<double, true>), grid, dim3(512), 0, s, A, m, n, lda, Uimg, ld, (void*)Q, ldq, info);
  return hipGetLastError();
}

}  // namespace cqr2
