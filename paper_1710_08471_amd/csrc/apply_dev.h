// Device code of the Q = A U kernel (n <= 128), shared by the one-problem
// kernel and the multi-problem step kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

namespace cqr2 {
// ============================================================================
// Q = A U with U upper triangular (NT x NT padded, NT = 32, 64 or 128), FP64
// MFMA 4x4x4 (4 blocks).
//
// The four hardware blocks are four groups of 4 rows of A sharing one 4x4
// fragment of U: with lane l holding A(row0 + (l&15), 4I + (l>>4)) and
// U(4I + (l>>4), 4J + (l&3)), mfma adds to output lane l the product for
// row row0 + 4((l>>2)&3) + (l>>4), column 4J + (l&3).
//
// Each wave owns a balanced set of output column groups {J, NG-1-J, ...} and
// keeps the U fragments of those columns (I <= J) in registers for the whole
// kernel: U is the same for every row.  A streams through LDS in 64-row
// stages (asynchronous global -> LDS copies, double-buffered, 512 contiguous
// bytes per column), so only A fragments are read from LDS and the bytes in
// flight cost no registers.  Stores of a stage are issued at the start of the
// next iteration and target rows no later load touches (the stages run in one
// direction), so Q == A (in place) is safe.
// ============================================================================
constexpr int kApplyRows = 64;  // rows per stage (4 tiles of 16)
constexpr int kApplyTiles = kApplyRows / 16;

// LDS image of a 64-row column: rows of odd columns stored XOR 16, so the
// 4 columns x 16 rows of an A fragment fall on both bank halves.
__device__ __forceinline__ int apply_pos(int c, int r) { return c * kApplyRows + (r ^ ((c & 1) << 4)); }

template <int NG>
struct ApplyLayout {
  static constexpr int W = NG >= 16 ? 8 : NG / 2;  // waves
  static constexpr int JPW = NG / W;               // column groups per wave (pairs)
  static_assert(NG % (2 * W) == 0, "column groups must split evenly over the waves");
  // j-th column group of wave w
  static constexpr int group(int w, int j) {
    const int pair = w + W * (j / 2);
    return (j & 1) ? NG - 1 - pair : pair;
  }
  static constexpr int frags_of(int w) {
    int c = 0;
    for (int j = 0; j < JPW; ++j) c += group(w, j) + 1;
    return c;
  }
  static constexpr int max_group(int w) {
    int g = 0;
    for (int j = 0; j < JPW; ++j) g = group(w, j) > g ? group(w, j) : g;
    return g;
  }
  // k-th fragment of wave w in consumption order: rows I ascending, slots
  // ascending within a row (only slots with group >= I).
  struct Ops {
    int I[NG * NG];
    int j[NG * NG];
    int n;
  };
  static constexpr Ops ops(int w) {
    Ops o{};
    int k = 0;
    for (int I = 0; I < NG; ++I)
      for (int t = 0; t < JPW; ++t)
        if (group(w, t) >= I) {
          o.I[k] = I;
          o.j[k] = t;
          ++k;
        }
    o.n = k;
    return o;
  }
  static constexpr bool check() {
    int owner[NG] = {};
    for (int w = 0; w < W; ++w)
      for (int j = 0; j < JPW; ++j) owner[group(w, j)] += 1;
    for (int g = 0; g < NG; ++g)
      if (owner[g] != 1) return false;
    for (int w = 0; w < W; ++w)
      if (frags_of(w) != frags_of(0) || ops(w).n != frags_of(w)) return false;
    return true;
  }
};
static_assert(ApplyLayout<8>::check() && ApplyLayout<16>::check() && ApplyLayout<32>::check(),
              "Q = A U column-group split is not balanced");

template <int NT, int W>
struct ApplyWave {
  static constexpr int NG = NT / 4;
  using L = ApplyLayout<NG>;
  static constexpr int JPW = L::JPW;
  static constexpr int NF = L::frags_of(W);
  static constexpr typename L::Ops OPS = L::ops(W);
  static constexpr int ROWS = L::max_group(W) + 1;  // rows I of U with work for this wave

  // The wave's U fragments, entry (l>>4, l&3) of fragment (I, J) per lane.
  __device__ static inline void load_u(const double* __restrict__ U, int64_t urs, int64_t ucs, int n, int lane,
                                       double (&u)[NF]) {
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int I = OPS.I[k], J = L::group(W, OPS.j[k]);
      const int r = 4 * I + (lane >> 4), c = 4 * J + (lane & 3);
      u[k] = (r <= c && c < n) ? U[(int64_t)r * urs + (int64_t)c * ucs] : 0.0;
    }
  }

  // acc(rt, j) += A(tile rt) U over one stage; A fragments of row I + 1 are
  // read from LDS while row I is multiplied.
  __device__ static inline void stage(const double* __restrict__ sa, int lane, const double (&u)[NF],
                                      double (&acc)[kApplyTiles][JPW]) {
    const int ar = lane & 15, ac = lane >> 4;
    double a[2][kApplyTiles];
#pragma unroll
    for (int rt = 0; rt < kApplyTiles; ++rt) a[0][rt] = sa[apply_pos(ac, 16 * rt + ar)];
    int k = 0;
#pragma unroll
    for (int I = 0; I < ROWS; ++I) {
      if (I + 1 < ROWS) {
#pragma unroll
        for (int rt = 0; rt < kApplyTiles; ++rt) a[(I + 1) & 1][rt] = sa[apply_pos(4 * (I + 1) + ac, 16 * rt + ar)];
      }
#pragma unroll
      for (int t = 0; t < JPW; ++t) {
        if (L::group(W, t) >= I) {
#pragma unroll
          for (int rt = 0; rt < kApplyTiles; ++rt)
            acc[rt][t] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[I & 1][rt], u[k], acc[rt][t], 0, 0, 0);
          ++k;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
};

template <int NT, int W>
__device__ __forceinline__ void apply_wave_run(const double* A, int64_t m, int n, int64_t lda,
                                               const double* __restrict__ U, int64_t urs, int64_t ucs, double* Q,
                                               int64_t ldq, int64_t s_begin, int64_t s_end, bool descending,
                                               double* sa, bool direct_ok) {
  using AW = ApplyWave<NT, W>;
  using L = typename AW::L;
  constexpr int JPW = AW::JPW;
  constexpr int kThreads = 64 * L::W;
  constexpr int kBuf = NT * kApplyRows;
  const int tid = threadIdx.x;
  const int lane = tid & 63;

  double u[AW::NF];
  AW::load_u(U, urs, ucs, n, lane, u);

  auto fill = [&](int64_t st, double* buf) {
    const int64_t row0 = st * kApplyRows;
    if (direct_ok && row0 + kApplyRows <= m) {
      // one instruction: 2 columns x 64 rows; lane i -> column 2p + (i>>5),
      // LDS rows 2(i&31), +1
      const int hi = lane >> 5;
      const int lrow = 2 * (lane & 31);
      for (int p = W; p < NT / 2; p += L::W) {
        const int col = 2 * p + hi;
        if (col < n) {
          const int grow = lrow ^ ((col & 1) << 4);
          __builtin_amdgcn_global_load_lds((const void*)(A + row0 + grow + (int64_t)col * lda),
                                           (__attribute__((address_space(3))) void*)(buf + 2 * p * kApplyRows),
                                           16, 0, 0);
        }
      }
    } else {
      for (int e = tid; e < kBuf; e += kThreads) {
        const int c = e / kApplyRows, r = e % kApplyRows;
        const int64_t row = row0 + r;
        buf[apply_pos(c, r)] = (row < m && c < n) ? A[row + (int64_t)c * lda] : 0.0;
      }
    }
  };
  // Columns >= n are never loaded: zero them in both stage buffers once.
  for (int e = tid; e < 2 * kBuf; e += kThreads)
    if ((e % kBuf) / kApplyRows >= n) sa[e] = 0.0;

  // stages s_begin .. s_end - 1, in ascending or descending order
  const int64_t count = s_end - s_begin;
  auto stage_at = [&](int64_t i) { return descending ? s_end - 1 - i : s_begin + i; };
  if (count > 0) fill(stage_at(0), sa);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  const int orow = 4 * ((lane >> 2) & 3) + (lane >> 4);
  const int ocol = lane & 3;
  double acc[kApplyTiles][JPW];
  auto store = [&](int64_t sidx) {
#pragma unroll
    for (int rt = 0; rt < kApplyTiles; ++rt) {
      const int64_t r = sidx * kApplyRows + 16 * rt + orow;
      if (r < m) {
#pragma unroll
        for (int t = 0; t < JPW; ++t) {
          const int col = 4 * L::group(W, t) + ocol;
          if (col < n) Q[r + (int64_t)col * ldq] = acc[rt][t];
        }
      }
    }
  };
  int cur = 0;
  int64_t prev = -1;
  for (int64_t i = 0; i < count; ++i) {
    const int64_t st = stage_at(i);
    if (prev >= 0) store(prev);
    if (i + 1 < count) fill(stage_at(i + 1), sa + (cur ^ 1) * kBuf);
#pragma unroll
    for (int rt = 0; rt < kApplyTiles; ++rt)
#pragma unroll
      for (int t = 0; t < JPW; ++t) acc[rt][t] = 0.0;
    AW::stage(sa + cur * kBuf, lane, u, acc);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    cur ^= 1;
    prev = st;
  }
  if (prev >= 0) store(prev);
}

// All waves of a workgroup: Q = A U over the 64-row stages s_begin ..
// s_end - 1, taken in descending order if `descending`.
template <int NT>
__device__ __forceinline__ void apply_block(const double* A, int64_t m, int n, int64_t lda,
                                            const double* __restrict__ U, int64_t urs, int64_t ucs, double* Q,
                                            int64_t ldq, int64_t s_begin, int64_t s_end, bool descending,
                                            double* sa) {
  const bool direct_ok = (((uintptr_t)A & 15u) == 0) && ((lda & 1) == 0);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int W = ApplyLayout<NT / 4>::W;
#define CQR2_AW(WV) apply_wave_run<NT, WV>(A, m, n, lda, U, urs, ucs, Q, ldq, s_begin, s_end, descending, sa, direct_ok)
  switch (wave) {
    case 0: CQR2_AW(0); break;
    case 1: if constexpr (W > 1) CQR2_AW(1); break;
    case 2: if constexpr (W > 2) CQR2_AW(2); break;
    case 3: if constexpr (W > 3) CQR2_AW(3); break;
    case 4: if constexpr (W > 4) CQR2_AW(4); break;
    case 5: if constexpr (W > 5) CQR2_AW(5); break;
    case 6: if constexpr (W > 6) CQR2_AW(6); break;
    case 7: if constexpr (W > 7) CQR2_AW(7); break;
    default: break;
  }
#undef CQR2_AW
}

}  // namespace cqr2
