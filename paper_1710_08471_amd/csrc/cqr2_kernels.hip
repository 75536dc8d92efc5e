// HIP kernels (gfx950) for one CholeskyQR pass and the CholeskyQR2 driver:
//   Gram  W = AᵀA              (paper: Syrk, Section "Preliminaries"; Algorithm 4 step 1)
//   CholInv(W) -> R, R^{-1}    (Algorithm 2)
//   Q = A R^{-1}               (Algorithm 4 step 3, MM with an upper-triangular right factor)
// All arithmetic is IEEE FP64.  Reductions use fixed orders (no FP atomics),
// so results are bit-reproducible for a given (m, n, lda, device).
#include "cqr2_internal.h"

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
// Work split inside a workgroup: the block-lower-triangle rows I = 0..NG-1
// (row I has I+1 blocks) are dealt to waves in snake order, which gives every
// wave the same number of MFMAs when NG is a multiple of 2*NW.
// ============================================================================
constexpr int kGramSplits = 256;  // workgroups along m for large m (one per MI355X CU)
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

template <int NG, int NW>
struct GramLayout {
  static constexpr int wave_of_row(int I) {
    const int P = 2 * NW;
    const int rr = I % P;
    return rr < NW ? rr : P - 1 - rr;
  }
  static constexpr int blocks_of(int w) {
    int c = 0;
    for (int I = 0; I < NG; ++I)
      if (wave_of_row(I) == w) c += I + 1;
    return c;
  }
  static constexpr int max_row(int w) {
    int mx = -1;
    for (int I = 0; I < NG; ++I)
      if (wave_of_row(I) == w) mx = I;
    return mx;
  }
};

template <int NG, int NW, int W>
struct WaveBlocks {
  using L = GramLayout<NG, NW>;
  static constexpr int count = L::blocks_of(W);
  static constexpr int cap = count > 0 ? count : 1;
  struct List {
    int I[cap];
    int J[cap];
  };
  static constexpr List make() {
    List l{};
    int k = 0;
    for (int I = 0; I < NG; ++I)
      if (L::wave_of_row(I) == W)
        for (int J = 0; J <= I; ++J) {
          l.I[k] = I;
          l.J[k] = J;
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
  constexpr int MR = GramLayout<NG, NW>::max_row(W);
  constexpr int NF = MR >= 0 ? MR + 1 : 1;
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
        double f[NF];
#pragma unroll
        for (int c = 0; c < NF; ++c) f[c] = bcur[stage_pos(4 * c + fcol, r)];
#pragma unroll
        for (int b = 0; b < WB::count; ++b)
          acc[b] = __builtin_amdgcn_mfma_f64_4x4x4f64(f[WB::list.I[b]], f[WB::list.J[b]], acc[b], 0, 0, 0);
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

template <int NG, int NW>
__global__ __launch_bounds__(NW * 64) void k_gram_partials(const double* __restrict__ A, int64_t m, int n,
                                                           int64_t lda, int64_t stages, int64_t spw,
                                                           double* __restrict__ partials,
                                                           const int32_t* __restrict__ info) {
  __shared__ double lds[2 * GramStage<NG, NW>::kBuf];
  if (info != nullptr && *info != 0) return;
  constexpr int nblk = NG * (NG + 1) / 2;
  const int64_t st0 = (int64_t)blockIdx.x * spw;
  const int64_t st1 = st0 + spw < stages ? st0 + spw : stages;
  const bool direct_ok = (((uintptr_t)A & 15u) == 0) && ((lda & 1) == 0);
  double* out = partials + (int64_t)blockIdx.x * nblk * 16;
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

// Fixed-order sum of the per-workgroup partial Grams: 8 threads per entry each
// add a contiguous range of partials in order, then the 8 results are added in
// order.  Writes the lower triangle and its mirror.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* __restrict__ part, int splits, int nblk, int n,
                                                     double* __restrict__ W, int64_t ldw,
                                                     const int32_t* __restrict__ info) {
  __shared__ double red[8][32];
  if (info != nullptr && *info != 0) return;
  const int lane = threadIdx.x & 31;
  const int sub = threadIdx.x >> 5;
  const int total = nblk * 16;
  const int e = blockIdx.x * 32 + lane;
  double v = 0.0;
  if (e < total) {
    const int s0 = (splits * sub) / 8, s1 = (splits * (sub + 1)) / 8;
    for (int s = s0; s < s1; ++s) v += part[(int64_t)s * total + e];
  }
  red[sub][lane] = v;
  __syncthreads();
  if (sub == 0 && e < total) {
    double t = red[0][lane];
#pragma unroll
    for (int k = 1; k < 8; ++k) t += red[k][lane];
    const int b = e >> 4, ij = e & 15;
    int I = (int)((sqrt(8.0 * b + 1.0) - 1.0) * 0.5);
    while (I * (I + 1) / 2 > b) --I;
    while ((I + 1) * (I + 2) / 2 <= b) ++I;
    const int J = b - I * (I + 1) / 2;
    const int row = 4 * I + (ij >> 2), col = 4 * J + (ij & 3);
    if (row >= col && row < n) {
      W[row + (int64_t)col * ldw] = t;
      W[col + (int64_t)row * ldw] = t;
    }
  }
}

static int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// The split count depends only on (m, n) -- never on the device -- so the
// summation order, and with it every result bit, is the same on any GPU.
GramPlan plan_gram(int64_t m, int64_t n) {
  GramPlan p{};
  const int groups = (int)((n + 3) / 4);
  p.ng = pow2_at_least(groups < 1 ? 1 : groups);
  p.nw = p.ng >= 16 ? 8 : (p.ng >= 2 ? p.ng / 2 : 1);
  p.nblk = p.ng * (p.ng + 1) / 2;
  p.stages = (m + kStageRows - 1) / kStageRows;
  if (p.stages < 1) p.stages = 1;
  const int64_t target = kGramSplits;
  // Small problems: do not spread fewer than 4 stages per workgroup.
  int64_t s = p.stages / 4;
  if (s < 1) s = 1;
  if (s > target) s = target;
  p.stages_per_wg = (p.stages + s - 1) / s;
  p.splits = (int)((p.stages + p.stages_per_wg - 1) / p.stages_per_wg);
  p.partial_bytes = (size_t)p.splits * p.nblk * 16 * sizeof(double);
  return p;
}

hipError_t launch_gram_partials(const GramPlan& p, const double* A, int64_t m, int n, int64_t lda,
                                double* partials, const int32_t* info, hipStream_t s) {
  dim3 grid(p.splits);
#define CQR2_GRAM_CASE(NGV, NWV)                                                                     \
  case NGV:                                                                                          \
    hipLaunchKernelGGL((k_gram_partials<NGV, NWV>), grid, dim3(NWV * 64), 0, s, A, m, n, lda,        \
                       p.stages, p.stages_per_wg, partials, info);                                   \
    break;
  switch (p.ng) {
    CQR2_GRAM_CASE(1, 1)
    CQR2_GRAM_CASE(2, 1)
    CQR2_GRAM_CASE(4, 2)
    CQR2_GRAM_CASE(8, 4)
    CQR2_GRAM_CASE(16, 8)
    CQR2_GRAM_CASE(32, 8)
    default: return hipErrorInvalidValue;
  }
#undef CQR2_GRAM_CASE
  return hipGetLastError();
}

hipError_t launch_gram_reduce(const GramPlan& p, const double* partials, int n, double* W, int64_t ldw,
                              const int32_t* info, hipStream_t s) {
  const int total = p.nblk * 16;
  dim3 grid((total + 31) / 32);
  hipLaunchKernelGGL(k_gram_reduce, grid, dim3(256), 0, s, partials, p.splits, p.nblk, n, W, ldw, info);
  return hipGetLastError();
}

// ============================================================================
// CholInv (Algorithm 2) for n <= 128 in one workgroup.
//
// The recursion's net effect, column by column: pivot d = W'(j,j), L(j,j) =
// sqrt(d), Y(j,j) = 1/L(j,j); L(i,j) = W'(i,j) * Y(j,j) (Algorithm 2's
// L21 = A21 Y11ᵀ at its 1x1 base); Schur update W' -= L(:,j) L(:,j)ᵀ; and the
// inverse's update Z(i,k) -= L(i,j) Y(j,k) (Y21 = -Y22 L21 Y11 unrolled).
// The n x n register-resident matrix M holds W' / L in its lower triangle and
// Zᵀ / Yᵀ (= R^{-1}) in its strict upper triangle; thread (r, c) of a 16 x 16
// grid owns M(r + 16a, c + 16b) (a cyclic distribution, so the shrinking
// trailing matrix stays spread over all threads).  One barrier per column:
// the owners of column j publish it to a double-buffered LDS vector, every
// thread forms L(:,j) and Y(j,:) from it and applies the rank-1 updates.
// ============================================================================
template <int T, int G>
__global__ __launch_bounds__(G * G) void k_cholinv(const double* __restrict__ W, int64_t ldw, int n,
                                                 double* __restrict__ R, int64_t ldr, double* __restrict__ Rinv,
                                                 int64_t ldri, double* __restrict__ Upad, int np,
                                                 int32_t* __restrict__ info, int info_offset) {
  constexpr int NP = G * T;
  __shared__ double colbuf[2][NP];
  const int tid = threadIdx.x;
  const int r = tid / G, c = tid % G;
  int fail = 0;
  if (info != nullptr && *info != 0) fail = -1;  // an earlier phase failed: skip, NaN outputs

  double M[T][T];
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = 0; b < T; ++b) {
      const int p = r + G * a, q = c + G * b;
      double v = 0.0;
      if (p >= q) v = (p < n) ? W[p + (int64_t)q * ldw] : (p == q ? 1.0 : 0.0);
      M[a][b] = v;
    }

  if (fail == 0) {
#pragma unroll
    for (int jb = 0; jb < T; ++jb) {
      if (G * jb >= n || fail != 0) break;
      for (int jc = 0; jc < G; ++jc) {
        const int j = G * jb + jc;
        if (j >= n) break;
        double* buf = colbuf[j & 1];
        if (c == jc) {
#pragma unroll
          for (int a = 0; a < T; ++a) buf[r * T + a] = M[a][jb];
        }
        __syncthreads();
        const double d = buf[jc * T + jb];
        if (!(d > 0.0)) {  // non-positive or NaN pivot (uniform across the workgroup)
          fail = j + 1;
          break;
        }
        const double sd = sqrt(d);
        const double y = 1.0 / sd;
        double lvp[T], yvp[T], lvq[T];
#pragma unroll
        for (int a = 0; a < T; ++a) {
          const int p = r + G * a;
          const double v = buf[r * T + a];
          lvp[a] = (p > j) ? v * y : 0.0;
          yvp[a] = (p < j) ? v * y : (p == j ? y : 0.0);
        }
#pragma unroll
        for (int b = 0; b < T; ++b) {
          const int q = c + G * b;
          lvq[b] = (q > j) ? buf[c * T + b] * y : 0.0;
        }
        if (c == jc) {
#pragma unroll
          for (int a = 0; a < T; ++a) {
            const int p = r + G * a;
            M[a][jb] = (p > j) ? lvp[a] : (p == j ? sd : yvp[a]);
          }
        }
        const bool low_diag = r >= c;  // element (a,a) of this thread is in the lower triangle
#pragma unroll
        for (int b = jb; b < T; ++b) {
#pragma unroll
          for (int a = 0; a < T; ++a) {
            if (a > b) {
              M[a][b] = fma(-lvp[a], lvq[b], M[a][b]);
            } else if (a < b) {
              if (a <= jb) M[a][b] = fma(-yvp[a], lvq[b], M[a][b]);
            } else {
              const double f = low_diag ? lvp[a] : yvp[a];
              M[a][b] = fma(-f, lvq[b], M[a][b]);
            }
          }
        }
      }
    }
  }

  const double nan = __builtin_nan("");
  if (fail > 0 && tid == 0 && info != nullptr) *info = info_offset + fail;
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = 0; b < T; ++b) {
      const int p = r + G * a, q = c + G * b;
      const double v = M[a][b];
      if (p < n && q < n) {
        if (p >= q) {
          R[q + (int64_t)p * ldr] = fail ? nan : v;  // R(q,p) = L(p,q)
          if (p > q) R[p + (int64_t)q * ldr] = 0.0;
        }
        if (Rinv != nullptr) {
          if (p < q) {
            Rinv[p + (int64_t)q * ldri] = fail ? nan : v;
            Rinv[q + (int64_t)p * ldri] = 0.0;
          } else if (p == q) {
            Rinv[p + (int64_t)p * ldri] = fail ? nan : 1.0 / v;
          }
        }
      }
      if (Upad != nullptr && p < np && q < np) {
        double u = 0.0;
        if (p < q) u = v;
        else if (p == q) u = 1.0 / v;
        Upad[(int64_t)p * np + q] = fail ? nan : u;
      }
    }
}

int padded_order(int64_t n) {
  if (n <= 32) return 32;
  if (n <= 64) return 64;
  return 128;
}

// Thread grid of the one-workgroup CholInv: G x G threads, each owning a
// (n/G) x (n/G) cyclic tile.
#ifndef CQR2_CHOLINV_G
#define CQR2_CHOLINV_G 32
#endif

hipError_t launch_cholinv(const double* W, int64_t ldw, int n, double* R, int64_t ldr, double* Rinv,
                          int64_t ldri, double* Upad, int np, int32_t* info, int info_offset,
                          hipStream_t s) {
  constexpr int G = CQR2_CHOLINV_G;
  const int t = padded_order(n) / G;
  switch (t) {
#define CQR2_CI(TV)                                                                                           \
  case TV:                                                                                                    \
    hipLaunchKernelGGL((k_cholinv<TV, G>), dim3(1), dim3(G * G), 0, s, W, ldw, n, R, ldr, Rinv, ldri, Upad, np, \
                       info, info_offset);                                                                    \
    break;
    CQR2_CI(1)
    CQR2_CI(2)
    CQR2_CI(4)
#if CQR2_CHOLINV_G == 16
    CQR2_CI(8)
#endif
#undef CQR2_CI
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

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
// next iteration and target rows no later load touches, so Q == A (in place)
// is safe.
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
                                               int64_t ldq, int nwg, double* sa, bool direct_ok) {
  using AW = ApplyWave<NT, W>;
  using L = typename AW::L;
  constexpr int JPW = AW::JPW;
  constexpr int kThreads = 64 * L::W;
  constexpr int kBuf = NT * kApplyRows;
  const int tid = threadIdx.x;
  const int lane = tid & 63;

  double u[AW::NF];
  AW::load_u(U, urs, ucs, n, lane, u);

  const int64_t stages = (m + kApplyRows - 1) / kApplyRows;
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

  int64_t st = blockIdx.x;
  if (st < stages) fill(st, sa);
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
  for (; st < stages; st += nwg) {
    if (prev >= 0) store(prev);
    const int64_t nxt = st + nwg;
    if (nxt < stages) fill(nxt, sa + (cur ^ 1) * kBuf);
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

template <int NT>
__global__ __launch_bounds__(64 * ApplyLayout<NT / 4>::W, 1) void k_apply_rinv(
    const double* A, int64_t m, int n, int64_t lda, const double* __restrict__ U, int64_t urs, int64_t ucs,
    double* Q, int64_t ldq, const int32_t* __restrict__ info, int nwg) {
  // nwg == gridDim.x, passed in so the stage loop keeps it in a register.
  __shared__ double sa[2 * NT * kApplyRows];
  if (info != nullptr && *info != 0) return;
  const bool direct_ok = (((uintptr_t)A & 15u) == 0) && ((lda & 1) == 0);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  constexpr int W = ApplyLayout<NT / 4>::W;
  switch (wave) {
    case 0: apply_wave_run<NT, 0>(A, m, n, lda, U, urs, ucs, Q, ldq, nwg, sa, direct_ok); break;
    case 1: if constexpr (W > 1) apply_wave_run<NT, 1>(A, m, n, lda, U, urs, ucs, Q, ldq, nwg, sa, direct_ok); break;
    case 2: if constexpr (W > 2) apply_wave_run<NT, 2>(A, m, n, lda, U, urs, ucs, Q, ldq, nwg, sa, direct_ok); break;
    case 3: if constexpr (W > 3) apply_wave_run<NT, 3>(A, m, n, lda, U, urs, ucs, Q, ldq, nwg, sa, direct_ok); break;
    case 4: if constexpr (W > 4) apply_wave_run<NT, 4>(A, m, n, lda, U, urs, ucs, Q, ldq, nwg, sa, direct_ok); break;
    case 5: if constexpr (W > 5) apply_wave_run<NT, 5>(A, m, n, lda, U, urs, ucs, Q, ldq, nwg, sa, direct_ok); break;
    case 6: if constexpr (W > 6) apply_wave_run<NT, 6>(A, m, n, lda, U, urs, ucs, Q, ldq, nwg, sa, direct_ok); break;
    case 7: if constexpr (W > 7) apply_wave_run<NT, 7>(A, m, n, lda, U, urs, ucs, Q, ldq, nwg, sa, direct_ok); break;
    default: break;
  }
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

__global__ void k_set_info(int32_t* info, int32_t value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *info = value;
}

hipError_t launch_set_info(int32_t* info, int32_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_info, dim3(1), dim3(64), 0, s, info, value);
  return hipGetLastError();
}

}  // namespace cqr2
