// Device code of the wide Gram (128 < n <= 256), shared by the one-problem
// kernel k_gram_wide and the multi-problem step kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace cqr2 {

// ============================================================================
// Gram, 128 < n <= 256: v_mfma_f64_16x16x4f64.
//
// Operands per lane l: A-operand (row l%16, k l/16), B-operand (k l/16,
// column l%16); result entry r of lane l is D(4r + l/16, l%16).  With the
// "fragment" f_c(l) = A(k0 + l/16, 16c + l%16) of a 4-row step, the tile
// (I, J) of W accumulates mfma(f_I, f_J).  The 16 x 17 / 2 = 136 lower tiles
// are dealt to 8 waves by tile rows in snake order (rows w and 15 - w, 17
// tiles each); a wave keeps its 17 accumulators (4 doubles per lane each)
// for its whole row range.
//
// A streams through LDS in 32-row stages (column-major, 32 doubles per
// column, rows of column c stored XOR 2 (c & 15), so the 16 lanes of a
// fragment row hit 16 distinct bank pairs; the XOR is even, so the row pairs
// of the 16-byte direct loads stay adjacent).  Double-buffered: 2 x 64 KB.
// An FP32 input (mixed precision's Q1) is staged as FP32 and widened exactly
// when a fragment is read.
// ============================================================================
constexpr int kWideRows = 32;
constexpr int kWideCols = 256;
constexpr int kWideTiles = kWideCols / 16;                        // 16
constexpr int kWideLower = kWideTiles * (kWideTiles + 1) / 2;     // 136
constexpr int kLower128 = 8 * 9 / 2;                                // 36: the 128-column Gram
constexpr int kWideWaves = 8;
constexpr int kWideBuf = kWideCols * kWideRows;                   // doubles per stage
constexpr int kWideSplits = 256;

__device__ __forceinline__ int wide_pos(int c, int r) { return c * kWideRows + (r ^ ((c & 15) << 1)); }
// FP32 stages (Q1 of the mixed-precision form): 32 floats per column, rows
// XOR 4 ((c >> 1) & 7), which keeps the 4-row groups of the 16-byte copies
// together and spreads a fragment row's 16 columns over 16 distinct banks.
__device__ __forceinline__ int wide_pos_f(int c, int r) { return c * kWideRows + (r ^ (((c >> 1) & 7) << 2)); }
template <typename TA>
__device__ __forceinline__ int wide_slot(int c, int r) {
  if constexpr (sizeof(TA) == 8) return wide_pos(c, r);
  else return wide_pos_f(c, r);
}

typedef double wd4 __attribute__((ext_vector_type(4)));

// COLS = 256 (eight waves) or 128 (four waves, tile rows w and 7 - w).
template <int COLS, int W>
struct WideWave {
  static constexpr int I0 = W, I1 = COLS / 16 - 1 - W;
  static constexpr int NT = (I0 + 1) + (I1 + 1);   // tiles of this wave
  static constexpr int NF = I1 + 1;                 // fragments needed (columns tiles 0..I1)
  static constexpr int tile_i(int t) { return t <= I0 ? I0 : I1; }
  static constexpr int tile_j(int t) { return t <= I0 ? t : t - (I0 + 1); }
};

template <typename TA, int COLS, int W>
__device__ __forceinline__ void gram_cols_wave(const TA* __restrict__ A, int64_t m, int n, int64_t lda,
                                               int64_t st0, int64_t st1, bool direct_ok, TA* lds,
                                               double* __restrict__ out) {
  static_assert(COLS == 128 || COLS == 256, "128 or 256 columns");
  constexpr int kWaves = COLS / 32;
  constexpr int kBuf = COLS * kWideRows;  // elements per stage
  using WW = WideWave<COLS, W>;
  const int tid = threadIdx.x, lane = tid & 63;
  wd4 acc[WW::NT];
#pragma unroll
  for (int t = 0; t < WW::NT; ++t) acc[t] = wd4{0.0, 0.0, 0.0, 0.0};

  for (int e = tid; e < 2 * kBuf; e += 64 * kWaves)
    if ((e % kBuf) / kWideRows >= n) lds[e] = (TA)0;
  auto fill = [&](int64_t st, TA* buf) {
    const int64_t row0 = st * kWideRows;
    if (direct_ok && row0 + kWideRows <= m) {
      if constexpr (sizeof(TA) == 8) {
        // one instruction: 4 columns x 32 rows; lane i -> column 4p + (i>>4), LDS rows 2(i&15), +1
        const int sub = lane >> 4, lrow = 2 * (lane & 15);
        for (int p = W; p < COLS / 4; p += kWaves) {
          const int col = 4 * p + sub;
          if (col < n) {
            const int grow = lrow ^ ((col & 15) << 1);
            __builtin_amdgcn_global_load_lds((const void*)(A + row0 + grow + (int64_t)col * lda),
                                             (__attribute__((address_space(3))) void*)(buf + 4 * p * kWideRows),
                                             16, 0, 0);
          }
        }
      } else {
        // one instruction: 8 columns x 32 rows; lane i -> column 8p + (i>>3), LDS rows 4(i&7) .. +3
        const int sub = lane >> 3, lrow = 4 * (lane & 7);
        for (int p = W; p < COLS / 8; p += kWaves) {
          const int col = 8 * p + sub;
          if (col < n) {
            const int grow = lrow ^ (((col >> 1) & 7) << 2);
            __builtin_amdgcn_global_load_lds((const void*)(A + row0 + grow + (int64_t)col * lda),
                                             (__attribute__((address_space(3))) void*)(buf + 8 * p * kWideRows),
                                             16, 0, 0);
          }
        }
      }
    } else {
      for (int e = tid; e < kBuf; e += 64 * kWaves) {
        const int c = e / kWideRows, r = e % kWideRows;
        const int64_t row = row0 + r;
        buf[wide_slot<TA>(c, r)] = (row < m && c < n) ? A[row + (int64_t)c * lda] : (TA)0;
      }
    }
  };
  if (st0 < st1) fill(st0, lds);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int64_t st = st0; st < st1; ++st) {
    const int cur = (int)((st - st0) & 1);
    TA* bcur = lds + cur * kBuf;
    if (st + 1 < st1) fill(st + 1, lds + (cur ^ 1) * kBuf);
    // lane index behind an opaque copy, so the fragment addresses are formed
    // here and not hoisted out of the stage loop into registers
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int fc = ln & 15, fk = ln >> 4;
    // the fragments of k-step ks + 1 are read while the products of k-step ks run
    double f[2][WW::NF];
#pragma unroll
    for (int c = 0; c < WW::NF; ++c) f[0][c] = (double)bcur[wide_slot<TA>(16 * c + fc, fk)];
#pragma unroll
    for (int ks = 0; ks < kWideRows / 4; ++ks) {
      if (ks + 1 < kWideRows / 4) {
#pragma unroll
        for (int c = 0; c < WW::NF; ++c)
          f[(ks + 1) & 1][c] = (double)bcur[wide_slot<TA>(16 * c + fc, 4 * (ks + 1) + fk)];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int t = 0; t < WW::NT; ++t)
        if (16 * WW::tile_i(t) < n)  // uniform: tiles past column n stay zero
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[ks & 1][WW::tile_i(t)], f[ks & 1][WW::tile_j(t)], acc[t], 0,
                                                        0, 0);
      __builtin_amdgcn_sched_barrier(0);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  // tile (I, J) -> lower-order index I (I+1)/2 + J; 4 x 64 doubles, lane-major
#pragma unroll
  for (int t = 0; t < WW::NT; ++t) {
    const int I = WW::tile_i(t), J = WW::tile_j(t);
    double* o = out + (int64_t)(I * (I + 1) / 2 + J) * 256;
#pragma unroll
    for (int r = 0; r < 4; ++r) o[r * 64 + lane] = acc[t][r];
  }
}

template <typename TA, int W>
__device__ __forceinline__ void gram_wide_wave(const TA* __restrict__ A, int64_t m, int n, int64_t lda,
                                               int64_t st0, int64_t st1, bool direct_ok, TA* lds,
                                               double* __restrict__ out) {
  gram_cols_wave<TA, 256, W>(A, m, n, lda, st0, st1, direct_ok, lds, out);
}

}  // namespace cqr2
