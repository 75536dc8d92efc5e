// Device code of the Gram kernel (W = AᵀA, n <= 128), shared by the
// one-problem kernel and the multi-problem step kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

namespace cqr2 {
// ============================================================================
// Gram matrix: split-K over 64-row stages, FP64 MFMA 4x4x4 (4 blocks).
//
// v_mfma_f64_4x4x4_4b_f64, per lane l: block = (l>>2)&3; A operand row i = l&3,
// B operand column j = l&3, both with reduction index k = l>>4; result row
// i = l>>4, column j = l&3.  If lane l holds A[row0 + (l>>2)][4c + (l&3)] for a
// 4-column group c (a "fragment"), then mfma(frag(I), frag(J)) adds to block b
// the partial Gram of columns 4I..4I+3 x 4J..4J+3 over the 4 rows
// row0 + 4k + b: the four hardware blocks act as a 4-way split of the 16 rows.
// The four partial sums are added (lanes l, l^4, l^8, l^12) once at the end.
//
// Work split inside a workgroup: see GramLayout.
// ============================================================================
constexpr int kStageRows = 64;  // rows of A per LDS stage (one 512-byte segment per column)

// LDS layout of a stage: column-major, 64 doubles per column, with the rows of
// column c stored XOR s(c & 3), s = {0, 12, 20, 24}.  A fragment read touches
// 4 columns x 16 consecutive rows; with this swizzle any 16 consecutive lanes
// (4 columns x 4 rows) hit 16 distinct 8-byte bank slots mod 128 bytes and
// any 32 consecutive lanes hit 32 distinct slots mod 256 bytes, so the read is
// conflict-free whether the LDS serves 16 or 32 lanes per cycle.  XOR keeps
// bit 0, so row pairs stay together for the 16-byte direct loads.
__device__ __forceinline__ int stage_swz(int c) { return (0x18140C00u >> (8 * (c & 3))) & 0xff; }
__device__ __forceinline__ int stage_pos(int c, int r) { return c * kStageRows + (r ^ stage_swz(c)); }

// Which wave computes block (I, J), J <= I, of the lower block triangle.
// Eight waves and NG >= 16: square patches of a 4 x 4 grid of super-blocks
// (S = NG / 4 block rows each); the six off-diagonal patches go to waves 0..5,
// the diagonal patches (0,0) + (3,3) to wave 6 and (1,1) + (2,2) to wave 7, so
// a wave multiplies 2 S fragments per k-step (the two waves of a SIMD, w and
// w + 4, carry 128 or 136 blocks together).  Otherwise: block rows dealt in
// snake order, which balances the MFMAs when NG is a multiple of 2 NW.
template <int NG, int NW>
struct GramLayout {
  static constexpr bool patches = NW == 8 && NG >= 16;
  static constexpr int S = NG / 4;
  static constexpr int wave_of_row(int I) {
    const int P = 2 * NW;
    const int rr = I % P;
    return rr < NW ? rr : P - 1 - rr;
  }
  static constexpr int patch_wave(int R, int C) {
    if (R == C) return (R == 0 || R == 3) ? 6 : 7;
    return R * (R - 1) / 2 + C;  // (1,0) 0, (2,0) 1, (2,1) 2, (3,0) 3, (3,1) 4, (3,2) 5
  }
  static constexpr int wave_of_block(int I, int J) { return patches ? patch_wave(I / S, J / S) : wave_of_row(I); }
};

template <int NG, int NW, int W>
struct WaveBlocks {
  using L = GramLayout<NG, NW>;
  static constexpr int count_blocks() {
    int c = 0;
    for (int I = 0; I < NG; ++I)
      for (int J = 0; J <= I; ++J)
        if (L::wave_of_block(I, J) == W) ++c;
    return c;
  }
  static constexpr int count = count_blocks();
  static constexpr int cap = count > 0 ? count : 1;
  // fragments (4-column groups) the wave reads per k-step
  static constexpr int count_frags() {
    int c = 0;
    for (int g = 0; g < NG; ++g) {
      bool used = false;
      for (int I = 0; I < NG; ++I)
        for (int J = 0; J <= I; ++J)
          if (L::wave_of_block(I, J) == W && (I == g || J == g)) used = true;
      c += used ? 1 : 0;
    }
    return c;
  }
  static constexpr int NFW = count_frags() > 0 ? count_frags() : 1;
  struct List {
    int I[cap];
    int J[cap];
    int fi[cap];   // position of group I in FC
    int fj[cap];   // position of group J in FC
    int FC[NFW];   // the 4-column groups read, ascending
  };
  static constexpr List make() {
    List l{};
    int pos[NG] = {};
    int nf = 0;
    for (int g = 0; g < NG; ++g) {
      bool used = false;
      for (int I = 0; I < NG; ++I)
        for (int J = 0; J <= I; ++J)
          if (L::wave_of_block(I, J) == W && (I == g || J == g)) used = true;
      if (used) {
        l.FC[nf] = g;
        pos[g] = nf++;
      }
    }
    int k = 0;
    for (int I = 0; I < NG; ++I)
      for (int J = 0; J <= I; ++J)
        if (L::wave_of_block(I, J) == W) {
          l.I[k] = I;
          l.J[k] = J;
          l.fi[k] = pos[I];
          l.fj[k] = pos[J];
          ++k;
        }
    return l;
  }
  static constexpr List list = make();
};

template <int NG, int NW>
struct GramStage {
  static constexpr int kCols = 4 * NG;
  static constexpr int kThreads = NW * 64;
  static constexpr int kBuf = kCols * kStageRows;  // doubles per stage buffer

  // Asynchronous global -> LDS copy of a full stage (all 64 rows < m).  One
  // instruction moves 1 KB = two columns x 64 rows; lane i fills LDS rows
  // 2(i&31), +1 of column 2p + (i >= 32) from the global rows that stage_pos
  // maps there.
  // Needs A 16-byte aligned and lda even.  Columns >= n are never loaded.
  __device__ static inline void load_direct(const double* A, int n, int64_t lda, int64_t row0, double* buf,
                                            int wave, int lane) {
    const int hi = lane >> 5;
    const int lrow = 2 * (lane & 31);
    for (int p = wave; p < kCols / 2; p += NW) {
      const int col = 2 * p + hi;
      const int grow = lrow ^ stage_swz(col);
      if (col < n) {
        const double* src = A + row0 + grow + (int64_t)col * lda;
        __builtin_amdgcn_global_load_lds((const void*)src,
                                         (__attribute__((address_space(3))) void*)(buf + 2 * p * kStageRows),
                                         16, 0, 0);
      }
    }
  }
  // Register path (ragged last stage, or unaligned A): masked loads, zero fill.
  __device__ static inline void load_regs(const double* A, int64_t m, int n, int64_t lda, int64_t row0, double* buf,
                                          int tid) {
    for (int e = tid; e < kCols * kStageRows; e += kThreads) {
      const int c = e / kStageRows, r = e % kStageRows;
      const int64_t row = row0 + r;
      buf[stage_pos(c, r)] = (row < m && c < n) ? A[row + (int64_t)c * lda] : 0.0;
    }
  }
};

template <int NG, int NW, int W>
__device__ __forceinline__ void gram_wave_body(const double* __restrict__ A, int64_t m, int n, int64_t lda,
                                               int64_t st0, int64_t st1, bool direct_ok, double* lds,
                                               double* __restrict__ out) {
  using WB = WaveBlocks<NG, NW, W>;
  using ST = GramStage<NG, NW>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;

  double acc[WB::cap];
#pragma unroll
  for (int b = 0; b < WB::cap; ++b) acc[b] = 0.0;

  // Columns >= n are never loaded by the direct path: zero them once.
  for (int e = tid; e < 2 * ST::kBuf; e += ST::kThreads) {
    const int c = (e % ST::kBuf) / kStageRows;
    if (c >= n) lds[e] = 0.0;
  }
  auto fill = [&](int64_t st, double* buf) {
    const int64_t row0 = st * kStageRows;
    if (direct_ok && row0 + kStageRows <= m)
      ST::load_direct(A, n, lda, row0, buf, W, lane);
    else
      ST::load_regs(A, m, n, lda, row0, buf, tid);
  };
  if (st0 < st1) fill(st0, lds);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  // Fragment c of k-step t: lane l reads row 16t + (l>>2) of column 4c + (l&3).
  const int fcol = lane & 3;
  const int frow = lane >> 2;
  for (int64_t st = st0; st < st1; ++st) {
    const int cur = (int)((st - st0) & 1);
    double* bcur = lds + cur * ST::kBuf;
    double* bnext = lds + (cur ^ 1) * ST::kBuf;
    if (st + 1 < st1) fill(st + 1, bnext);
    if constexpr (WB::count > 0) {
#pragma unroll 1
      for (int t = 0; t < kStageRows / 16; ++t) {
        const int r = 16 * t + frow;
        double f[WB::NFW];
#pragma unroll
        for (int c = 0; c < WB::NFW; ++c) f[c] = bcur[stage_pos(4 * WB::list.FC[c] + fcol, r)];
#pragma unroll
        for (int b = 0; b < WB::count; ++b)
          acc[b] = __builtin_amdgcn_mfma_f64_4x4x4f64(f[WB::list.fi[b]], f[WB::list.fj[b]], acc[b], 0, 0, 0);
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  // Add the four k-split partial sums held by lanes l, l^4, l^8, l^12.
  if constexpr (WB::count > 0) {
#pragma unroll
    for (int b = 0; b < WB::count; ++b) {
      double v = acc[b];
      v += __shfl_xor(v, 4);
      v += __shfl_xor(v, 8);
      if (((lane >> 2) & 3) == 0) {
        const int I = WB::list.I[b], J = WB::list.J[b];
        const int bidx = I * (I + 1) / 2 + J;
        out[bidx * 16 + (lane >> 4) * 4 + (lane & 3)] = v;
      }
    }
  }
}

// All NW waves of a workgroup: partial Gram of stages [st0, st1) of A into
// out (nblk x 16 doubles).  Every wave reaches the same barriers.
template <int NG, int NW>
__device__ __forceinline__ void gram_block(const double* __restrict__ A, int64_t m, int n, int64_t lda, int64_t st0,
                                           int64_t st1, double* lds, double* __restrict__ out) {
  const bool direct_ok = (((uintptr_t)A & 15u) == 0) && ((lda & 1) == 0);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  switch (wave) {
    case 0: gram_wave_body<NG, NW, 0>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 1: if constexpr (NW > 1) gram_wave_body<NG, NW, 1>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 2: if constexpr (NW > 2) gram_wave_body<NG, NW, 2>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 3: if constexpr (NW > 3) gram_wave_body<NG, NW, 3>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 4: if constexpr (NW > 4) gram_wave_body<NG, NW, 4>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 5: if constexpr (NW > 5) gram_wave_body<NG, NW, 5>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 6: if constexpr (NW > 6) gram_wave_body<NG, NW, 6>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    case 7: if constexpr (NW > 7) gram_wave_body<NG, NW, 7>(A, m, n, lda, st0, st1, direct_ok, lds, out); break;
    default: break;
  }
}

}  // namespace cqr2
