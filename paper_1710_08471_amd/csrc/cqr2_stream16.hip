// Streaming kernels for 64 < n <= 128 on FP64 MFMA 16x16x4, one workgroup of
// eight waves per CU walking a contiguous range of row stages:
//   GRAM        partial Grams W = AᵀA of the workgroup's rows (Syrk; Algorithm
//               4 step 1), 36 lower 16 x 16 tiles;
//   APPLY       Q = A U for upper-triangular U (Algorithm 4 step 3), in place
//               allowed (Q == A);
//   APPLY_GRAM  Q1 = A U and, from the stored values of Q1, its partial Grams
//               (Algorithm 5: the second CholeskyQR starts with the Gram of
//               Q1), so pass 1 reads A once and Q1 is never re-read for
//               pass 2's Gram.
// and the fixed-order sum of the partial Grams into W.
//
// MFMA 16x16x4 f64, per lane l: first operand (row l%16, k l/16), second
// operand (k l/16, column l%16), result entry r = D(4r + l/16, l%16).
//
// A stage of SR rows x 128 columns sits in LDS column-major, SR doubles per
// column, the rows of column c stored XOR 2 (c & 15): the 16 lanes of a
// Gram fragment (16 columns, one row) hit 16 distinct 8-byte slots, and the
// XOR is even, so the row pairs of the 16-byte direct copies stay together.
// Stages are copied straight from global memory into a ring of NBUF LDS
// buffers (global_load_lds, 16 bytes per lane); each wave waits for its own
// copies by count, with its later stores still in flight, and a barrier then
// publishes the stage.
//
// Work split (8 waves; waves w and w + 4 share a SIMD):
//   apply: wave w owns output column tiles P = w & 3 and 7 - P (36 k-steps of
//          4 per 16-row tile in all, so every SIMD has the same work) and half
//          of the stage's 16-row tiles; its U fragments stay in registers.
//   Gram:  SIMD s owns the lower tile rows 7 - s and s (nine tiles), five
//          for wave s and four for wave s + 4.
#include "cqr2_internal.h"

#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

#include "stream16_dev.h"
#include "sync_dev.h"

namespace cqr2 {

namespace {

constexpr int kCols = 128;
constexpr int kTiles = kCols / 16;              // 8 column tiles
constexpr int kLower = kTiles * (kTiles + 1) / 2;  // 36 lower tiles
constexpr int kWaves = 8;
constexpr int kThreads = 64 * kWaves;
constexpr int kSplits = 256;                    // workgroups along m for large m

// stage rows and ring depth per kernel (measured at 1M x 128)
constexpr int kGramSR = 64, kGramNBUF = 2;
constexpr int kApplySR = 32, kApplyNBUF = 4;
constexpr int kFusedSR = 32, kFusedNBUF = 3;
// The workgroups' stage ranges are planned in 64-row units, so every kernel
// covers the same rows per workgroup whatever its stage size.
constexpr int kPlanRows = 64;

enum { MODE_GRAM = 0, MODE_APPLY = 1, MODE_APPLY_GRAM = 2 };


// Gram tiles of wave W: SIMD s = W & 3 owns the tile rows 7 - s and s (nine
// tiles, row 7 - s first); wave s takes the first five, wave s + 4 the last
// four.  Each wave reads the fragments of the column tiles its tiles touch.
template <int W>
struct GramTiles {
  static constexpr int S = W & 3;
  static constexpr int FIRST = W < 4 ? 0 : 5;
  static constexpr int N = W < 4 ? 5 : 4;
  static constexpr int tile_i(int k) { return k < kTiles - S ? kTiles - 1 - S : S; }
  static constexpr int tile_j(int k) { return k < kTiles - S ? k : k - (kTiles - S); }
  struct List {
    int I[5], J[5], fi[5], fj[5];
    int F[6];  // column tiles read, in first-use order
    int nf;
  };
  static constexpr List make() {
    List l{};
    int pos[kTiles] = {-1, -1, -1, -1, -1, -1, -1, -1};
    for (int k = 0; k < N; ++k) {
      const int I = tile_i(FIRST + k), J = tile_j(FIRST + k);
      l.I[k] = I;
      l.J[k] = J;
      if (pos[I] < 0) { pos[I] = l.nf; l.F[l.nf++] = I; }
      if (pos[J] < 0) { pos[J] = l.nf; l.F[l.nf++] = J; }
      l.fi[k] = pos[I];
      l.fj[k] = pos[J];
    }
    return l;
  }
  static constexpr List list = make();
  static constexpr int NF = list.nf;
  static constexpr bool check() {
    // every lower tile belongs to exactly one wave
    int seen[kTiles][kTiles] = {};
    for (int w = 0; w < kWaves; ++w) {
      const int s = w & 3, first = w < 4 ? 0 : 5, cnt = w < 4 ? 5 : 4;
      for (int k = first; k < first + cnt; ++k) {
        const int I = k < kTiles - s ? kTiles - 1 - s : s, J = k < kTiles - s ? k : k - (kTiles - s);
        if (J > I) return false;
        seen[I][J] += 1;
      }
    }
    for (int I = 0; I < kTiles; ++I)
      for (int J = 0; J <= I; ++J)
        if (seen[I][J] != 1) return false;
    return true;
  }
};
static_assert(GramTiles<0>::check(), "Gram tiles must cover the lower triangle once");

template <int W>
struct WaveRole {
  static constexpr int P = W & 3;
  static constexpr int J0 = P, J1 = kTiles - 1 - P;       // apply column tiles
  static constexpr int K0 = 4 * (J0 + 1), K1 = 4 * (J1 + 1);  // k-steps of each (U(k, j) = 0 for k > j)
  static constexpr int HALF = W >> 2;                     // which half of the stage's row tiles
};

template <int MODE, int SR, int NBUF, int W>
__device__ __forceinline__ void wave_body(const double* A, int64_t m, int n, int64_t lda,
                                          const double* __restrict__ U, double* Q, int64_t ldq,
                                          double* __restrict__ out, int64_t s_begin, int64_t s_end, bool desc,
                                          bool direct_ok, bool qvec_ok, double* smem) {
  using R = WaveRole<W>;
  constexpr int kBuf = kCols * SR;          // doubles per stage buffer
  constexpr int kRT = SR / 16;              // 16-row tiles per stage
  constexpr int kRTW = kRT / 2;             // row tiles per wave (apply)
  constexpr int kLPC = SR / 2;              // lanes per column of a direct copy
  constexpr int kCPI = 64 / kLPC;           // columns per copy instruction
  constexpr int kInstr = kCols / kCPI;      // copy instructions per stage
  static_assert(kRT % 2 == 0 && kInstr % kWaves == 0, "stage shape");
  constexpr bool kApply = MODE != MODE_GRAM;
  constexpr bool kGram = MODE != MODE_APPLY;

  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t count = s_end - s_begin;
  auto stage_at = [&](int64_t i) { return desc ? s_end - 1 - i : s_begin + i; };

  // ---- U fragments (apply): u0[t] = U(4t + l/16, 16 J0 + l%16), likewise u1 ----
  double u0[R::K0], u1[R::K1];
  if constexpr (kApply) {
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int t = 0; t < R::K0; ++t) u0[t] = U[(4 * t + lk) * kCols + 16 * R::J0 + lr];
#pragma unroll
    for (int t = 0; t < R::K1; ++t) u1[t] = U[(4 * t + lk) * kCols + 16 * R::J1 + lr];
  }

  // copies per wave and stage (an instruction whose first column is < n is issued)
  int fcount = 0;
#pragma unroll
  for (int p = W; p < kInstr; p += kWaves) fcount += (kCPI * p < n) ? 1 : 0;

  auto fill = [&](int64_t st, double* buf) {
    const int64_t row0 = st * SR;
    if (direct_ok && row0 + SR <= m) {
      const int sub = lane / kLPC, lrow = 2 * (lane % kLPC);
#pragma unroll
      for (int p = W; p < kInstr; p += kWaves) {
        if (kCPI * p < n) {
          // buffer form of the LDS copy (the compiler keeps its LDS-read waits
          // counted past it); resource base at this instruction's first column
          const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
              (void*)(A + row0 + (int64_t)(kCPI * p) * lda), 0, 0x7fffffff, kBufferRsrcWord3);
          const int col = kCPI * p + sub;
          if (col < n) {
            const int grow = lrow ^ ((col & 15) << 1);
            const int voff = (int)(((int64_t)sub * lda + grow) * (int64_t)sizeof(double));
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(buf + kCPI * p * SR),
                                                     16, voff, 0, 0, 0);
          }
        }
      }
    } else {
      // ragged last stage or unaligned A: plain loads (waited for here), zeros past m
      for (int e = tid; e < kBuf; e += kThreads) {
        const int c = e / SR, r = e % SR;
        const int64_t row = row0 + r;
        if (c < n) buf[spos<SR>(c, r)] = row < m ? A[row + (int64_t)c * lda] : 0.0;
      }
    }
  };

  // ---- Gram accumulators ----
  using G = GramTiles<W>;
  d4 gacc[G::N];
#pragma unroll
  for (int t = 0; t < G::N; ++t) gacc[t] = d4{0.0, 0.0, 0.0, 0.0};

  // stores issued per iteration (the count the next waits allow in flight)
  int shist[NBUF > 1 ? NBUF - 1 : 1] = {};

  for (int64_t i = 0; i < NBUF - 1 && i < count; ++i) fill(stage_at(i), smem + (int)(i % NBUF) * kBuf);

  for (int64_t i = 0; i < count; ++i) {
    // wait for stage i's copies: allowed in flight are the copies of later
    // stages already issued and the stores of the last NBUF - 1 iterations
    int later = 0;
    for (int64_t s = i + 1; s <= i + NBUF - 2 && s < count; ++s) later += fcount;
    for (int h = 0; h < NBUF - 1; ++h) later += shist[h];
    wait_vmcnt_fenced(later > 32 ? 32 : later);
    lds_barrier();
    if (i + NBUF - 1 < count) fill(stage_at(i + NBUF - 1), smem + (int)((i + NBUF - 1) % NBUF) * kBuf);
    double* buf = smem + (int)(i % NBUF) * kBuf;
    const int64_t st = stage_at(i);
    const int64_t row0 = st * SR;
    int issued = 0;
    // The LDS addresses below are cheap to form from the lane index; an opaque
    // copy of it keeps the compiler from hoisting all of them out of the stage
    // loop into registers.
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int lr = ln & 15, lk = ln >> 4;

    if constexpr (kApply) {
      d4 acc[kRTW][2];
#pragma unroll
      for (int a = 0; a < kRTW; ++a) acc[a][0] = acc[a][1] = d4{0.0, 0.0, 0.0, 0.0};
      // A fragment of row tile rt, k-step t: lane l holds A(16 rt + l%16, 4t + l/16);
      // the next k-step's fragments are read while this one multiplies
      auto afrag = [&](int t, int q) { return buf[spos<SR>(4 * t + lk, 16 * (R::HALF * kRTW + q) + lr)]; };
      double a[2][kRTW];
#pragma unroll
      for (int q = 0; q < kRTW; ++q) a[0][q] = afrag(0, q);
#pragma unroll
      for (int t = 0; t < R::K1; ++t) {
        if (t + 1 < R::K1) {
#pragma unroll
          for (int q = 0; q < kRTW; ++q) a[(t + 1) & 1][q] = afrag(t + 1, q);
        }
        // the reads above go out before this step's products
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < kRTW; ++q) {
          d4& c1 = acc[q][1];
          d4& c0 = acc[q][0];
          if constexpr (MODE == MODE_APPLY) {
            // Qᵀ = Uᵀ Aᵀ: entry r of lane l is Q(16 rt + l%16, 16 J + 4r + l/16)
            c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(u1[t], a[t & 1][q], c1, 0, 0, 0);
            if (t < R::K0) c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(u0[t], a[t & 1][q], c0, 0, 0, 0);
          } else {
            // Q = A U: entry r of lane l is Q(16 rt + 4r + l/16, 16 J + l%16)
            c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t & 1][q], u1[t], c1, 0, 0, 0);
            if (t < R::K0) c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t & 1][q], u0[t], c0, 0, 0, 0);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if constexpr (MODE == MODE_APPLY) {
        // coalesced stores: per entry r, 4 columns x 16 consecutive rows
#pragma unroll
        for (int q = 0; q < kRTW; ++q) {
          const int64_t rbase = row0 + 16 * (R::HALF * kRTW + q);
          if (rbase < m) {
            const int64_t row = rbase + lr;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const int J = h ? R::J1 : R::J0;
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                if (16 * J + 4 * r < n) {
                  const int col = 16 * J + 4 * r + lk;
                  if (row < m && col < n) Q[row + (int64_t)col * ldq] = acc[q][h][r];
                  ++issued;
                }
              }
            }
          }
        }
      } else {
        // Q1 tile -> LDS (over the consumed A stage), columns >= n as zero
        lds_barrier();
#pragma unroll
        for (int q = 0; q < kRTW; ++q) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int col = 16 * (h ? R::J1 : R::J0) + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int row = 16 * (R::HALF * kRTW + q) + 4 * r + lk;
              buf[spos<SR>(col, row)] = col < n ? acc[q][h][r] : 0.0;
            }
          }
        }
        lds_barrier();
      }
    }

    if constexpr (kGram) {
      // one 16-byte read per column tile C and row block t of 8 rows: lane l
      // holds X(8t + 2 (l/16), 16 C + l%16) and the row below it, the fragments
      // of two k-steps (the even and the odd rows of the block).  Tile (I, J)
      // += X_Iᵀ X_J over both.  The next block's fragments are read while this
      // one multiplies.
      auto gfrag = [&](int t, int c) {
        return *reinterpret_cast<const double2*>(buf + spos<SR>(16 * G::list.F[c] + lr, 8 * t + 2 * lk));
      };
      double2 f[2][G::NF];
#pragma unroll
      for (int c = 0; c < G::NF; ++c) f[0][c] = gfrag(0, c);
#pragma unroll
      for (int t = 0; t < SR / 8; ++t) {
        if (t + 1 < SR / 8) {
#pragma unroll
          for (int c = 0; c < G::NF; ++c) f[(t + 1) & 1][c] = gfrag(t + 1, c);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < G::N; ++k)
          gacc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[t & 1][G::list.fi[k]].x, f[t & 1][G::list.fj[k]].x, gacc[k],
                                                         0, 0, 0);
#pragma unroll
        for (int k = 0; k < G::N; ++k)
          gacc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[t & 1][G::list.fi[k]].y, f[t & 1][G::list.fj[k]].y, gacc[k],
                                                         0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
    }

    if constexpr (MODE == MODE_APPLY_GRAM) {
      // Q1 stage -> global: 16 bytes per lane, whole 16-byte row pairs
      const int sub = lane / kLPC, lrow = 2 * (lane % kLPC);
#pragma unroll
      for (int p = W; p < kInstr; p += kWaves) {
        if (kCPI * p < n) {
          const int col = kCPI * p + sub;
          const int grow = lrow ^ ((col & 15) << 1);
          const double2 v = *reinterpret_cast<const double2*>(buf + kCPI * p * SR + 2 * lane);
          const int64_t row = row0 + grow;
          if (col < n && row < m) {
            double* q = Q + row + (int64_t)col * ldq;
            if (qvec_ok && row + 1 < m) {
              *reinterpret_cast<double2*>(q) = v;
            } else {
              q[0] = v.x;
              if (row + 1 < m) q[1] = v.y;
            }
          }
          ++issued;
        }
      }
    }
    if constexpr (NBUF > 1) {
#pragma unroll
      for (int h = NBUF - 2; h > 0; --h) shist[h] = shist[h - 1];
      shist[0] = issued;
    }
  }

  if constexpr (kGram) {
    // tile (I, J) -> lower-order index I (I + 1) / 2 + J; 4 x 64 doubles, lane-major
#pragma unroll
    for (int k = 0; k < G::N; ++k) {
      double* o = out + (int64_t)(G::list.I[k] * (G::list.I[k] + 1) / 2 + G::list.J[k]) * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) o[r * 64 + lane] = gacc[k][r];
    }
  }
}

// ---- Q1 = A U with the Gram of the stored Q1, producer / consumer -----------
// Waves 0..3 (one per SIMD) form Q1 stage i from A stage i (column tiles P and
// 7 - P, both 16-row tiles of an SR = 32 stage, taken as its even and odd
// rows) and write it to an LDS tile; the other waves accumulate the Gram of Q1
// stage i - 1 from the other LDS tile and store that stage to global memory.
// One barrier per stage.  With NWF = 8 waves, Gram wave 4 + s owns the nine
// lower tiles of rows 7 - s and s (SIMD s); with NWF = 12, those nine tiles go
// to two waves of SIMD s, five and four (GramTiles).  Every SIMD gets 72
// products of each kind per stage.
template <int NWF, int W>
struct FusedTiles {
  struct List {
    int I[9], J[9], fi[9], fj[9];
    int F[8];
    int n, nf;
  };
  static constexpr List make() {
    List l{};
    int pos[kTiles] = {-1, -1, -1, -1, -1, -1, -1, -1};
    auto add = [&](int I, int J) {
      if (pos[I] < 0) { pos[I] = l.nf; l.F[l.nf++] = I; }
      if (pos[J] < 0) { pos[J] = l.nf; l.F[l.nf++] = J; }
      l.I[l.n] = I; l.J[l.n] = J; l.fi[l.n] = pos[I]; l.fj[l.n] = pos[J];
      ++l.n;
    };
    if (W < 4) return l;
    if (NWF == 8) {
      const int S = W - 4, GA = kTiles - 1 - S, GB = S;
      for (int j = 0; j <= GA; ++j) add(GA, j);
      for (int j = 0; j <= GB; ++j) add(GB, j);
    } else {
      const int g = W - 4, S = g & 3, first = g < 4 ? 0 : 5, cnt = g < 4 ? 5 : 4;
      for (int k = first; k < first + cnt; ++k) {
        const int I = k < kTiles - S ? kTiles - 1 - S : S, J = k < kTiles - S ? k : k - (kTiles - S);
        add(I, J);
      }
    }
    return l;
  }
  static constexpr List list = make();
  static constexpr int N = list.n > 0 ? list.n : 1;
  static constexpr int NF = list.nf > 0 ? list.nf : 1;
};

template <int SR, int NBUF, int NWF, int W>
__device__ __forceinline__ void fused_body(const double* A, int64_t m, int n, int64_t lda,
                                           const double* __restrict__ U, double* Q, int64_t ldq,
                                           double* __restrict__ out, int64_t s_begin, int64_t s_end, bool desc,
                                           bool direct_ok, bool qvec_ok, double* smem) {
  constexpr int kBuf = kCols * SR;
  constexpr int kLPC = SR / 2;
  constexpr int kCPI = 64 / kLPC;
  constexpr int kInstr = kCols / kCPI;
  constexpr int kThr = 64 * NWF;
  constexpr int kGW = NWF - 4;              // Gram waves
  constexpr bool kApplyWave = W < 4;
  static_assert(SR == 32, "the apply waves take a 32-row stage as two interleaved row tiles");
  double* qbuf = smem + NBUF * kBuf;        // two Q1 tiles

  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t count = s_end - s_begin;
  auto stage_at = [&](int64_t i) { return desc ? s_end - 1 - i : s_begin + i; };

  constexpr int P = W & 3;
  constexpr int J0 = P, J1 = kTiles - 1 - P;
  constexpr int K0 = 4 * (J0 + 1), K1 = 4 * (J1 + 1);
  double u0[kApplyWave ? K0 : 1], u1[kApplyWave ? K1 : 1];
  if constexpr (kApplyWave) {
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int t = 0; t < K0; ++t) u0[t] = U[(4 * t + lk) * kCols + 16 * J0 + lr];
#pragma unroll
    for (int t = 0; t < K1; ++t) u1[t] = U[(4 * t + lk) * kCols + 16 * J1 + lr];
  }
  using G = FusedTiles<NWF, W>;
  d4 gacc[G::N];
#pragma unroll
  for (int k = 0; k < G::N; ++k) gacc[k] = d4{0.0, 0.0, 0.0, 0.0};

  int fcount = 0;
  for (int p = W; p < kInstr; p += NWF) fcount += (kCPI * p < n) ? 1 : 0;
  auto fill = [&](int64_t st, double* buf) {
    const int64_t row0 = st * SR;
    if (direct_ok && row0 + SR <= m) {
      const int sub = lane / kLPC, lrow = 2 * (lane % kLPC);
#pragma unroll
      for (int p = W; p < kInstr; p += NWF) {
        if (kCPI * p < n) {
          const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
              (void*)(A + row0 + (int64_t)(kCPI * p) * lda), 0, 0x7fffffff, kBufferRsrcWord3);
          const int col = kCPI * p + sub;
          if (col < n) {
            const int grow = lrow ^ ((col & 15) << 1);
            const int voff = (int)(((int64_t)sub * lda + grow) * (int64_t)sizeof(double));
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(buf + kCPI * p * SR),
                                                     16, voff, 0, 0, 0);
          }
        }
      }
    } else {
      for (int e = tid; e < kBuf; e += kThr) {
        const int c = e / SR, r = e % SR;
        const int64_t row = row0 + r;
        if (c < n) buf[spos<SR>(c, r)] = row < m ? A[row + (int64_t)c * lda] : 0.0;
      }
    }
  };

  int shist[NBUF - 1] = {};
  for (int64_t i = 0; i < NBUF - 1 && i < count; ++i) fill(stage_at(i), smem + (int)(i % NBUF) * kBuf);

  for (int64_t i = 0; i <= count; ++i) {
    int later = 0;
    for (int64_t s2 = i + 1; s2 <= i + NBUF - 2 && s2 < count; ++s2) later += fcount;
    for (int h = 0; h < NBUF - 1; ++h) later += shist[h];
    wait_vmcnt_fenced(later > 32 ? 32 : later);
    lds_barrier();
    if (i + NBUF - 1 < count) fill(stage_at(i + NBUF - 1), smem + (int)((i + NBUF - 1) % NBUF) * kBuf);
    int issued = 0;
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int lr = ln & 15, lk = ln >> 4;

    if constexpr (kApplyWave) {
      if (i < count) {
        const double* buf = smem + (int)(i % NBUF) * kBuf;
        double* qb = qbuf + (int)(i & 1) * kBuf;
        // row tile q = 0 holds the stage's even rows, q = 1 its odd rows: one
        // 16-byte read gives lane l A(2 (l%16), 4t + l/16) and the row below;
        // the reads run two k-steps ahead of the products
        d4 acc[2][2];
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[q][0] = acc[q][1] = d4{0.0, 0.0, 0.0, 0.0};
        auto afrag = [&](int t) { return *reinterpret_cast<const double2*>(buf + spos<SR>(4 * t + lk, 2 * lr)); };
        double2 a[3];
        a[0] = afrag(0);
        a[1] = afrag(1);
#pragma unroll
        for (int t = 0; t < K1; ++t) {
          if (t + 2 < K1) a[(t + 2) % 3] = afrag(t + 2);
          __builtin_amdgcn_sched_barrier(0);
          // Q = A U: entry r of lane l is Q(row 4r + l/16 of the tile, 16 J + l%16)
          acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t % 3].x, u1[t], acc[0][1], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t % 3].y, u1[t], acc[1][1], 0, 0, 0);
          if (t < K0) {
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t % 3].x, u0[t], acc[0][0], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t % 3].y, u0[t], acc[1][0], 0, 0, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        // Q1 tile -> LDS (tile row i of tile q is stage row 2 i + q), columns >= n as zero
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int col = 16 * (h ? J1 : J0) + lr;
#pragma unroll
            for (int r = 0; r < 4; ++r) qb[spos<SR>(col, 2 * (4 * r + lk) + q)] = col < n ? acc[q][h][r] : 0.0;
          }
      }
    } else {
      if (i >= 1) {
        const double* qb = qbuf + (int)((i - 1) & 1) * kBuf;
        // Gram of Q1 stage i - 1: one 16-byte read per column tile and row
        // block t of 8 rows gives lane l Q1(8t + 2 (l/16), 16 c + l%16) and the
        // row below (two k-steps); tile (I, J) += Q1_Iᵀ Q1_J
        auto gfrag = [&](int t, int c) {
          return *reinterpret_cast<const double2*>(qb + spos<SR>(16 * G::list.F[c] + lr, 8 * t + 2 * lk));
        };
        double2 f[2][G::NF];
#pragma unroll
        for (int c = 0; c < G::NF; ++c) f[0][c] = gfrag(0, c);
#pragma unroll
        for (int t = 0; t < SR / 8; ++t) {
          if (t + 1 < SR / 8) {
#pragma unroll
            for (int c = 0; c < G::NF; ++c) f[(t + 1) & 1][c] = gfrag(t + 1, c);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int k = 0; k < G::N; ++k)
            gacc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[t & 1][G::list.fi[k]].x, f[t & 1][G::list.fj[k]].x,
                                                           gacc[k], 0, 0, 0);
#pragma unroll
          for (int k = 0; k < G::N; ++k)
            gacc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[t & 1][G::list.fi[k]].y, f[t & 1][G::list.fj[k]].y,
                                                           gacc[k], 0, 0, 0);
          __builtin_amdgcn_sched_barrier(0);
        }
        // Q1 stage i - 1 -> global: 16 bytes per lane, whole row pairs
        const int64_t row0 = stage_at(i - 1) * SR;
        const int sub = lane / kLPC, lrow = 2 * (lane % kLPC);
#pragma unroll
        for (int p = W - 4; p < kInstr; p += kGW) {
          if (kCPI * p < n) {
            const int col = kCPI * p + sub;
            const int grow = lrow ^ ((col & 15) << 1);
            const double2 v = *reinterpret_cast<const double2*>(qb + kCPI * p * SR + 2 * lane);
            const int64_t row = row0 + grow;
            if (col < n && row < m) {
              double* q = Q + row + (int64_t)col * ldq;
              if (qvec_ok && row + 1 < m) {
                *reinterpret_cast<double2*>(q) = v;
              } else {
                q[0] = v.x;
                if (row + 1 < m) q[1] = v.y;
              }
            }
            ++issued;
          }
        }
      }
    }
#pragma unroll
    for (int h = NBUF - 2; h > 0; --h) shist[h] = shist[h - 1];
    shist[0] = issued;
  }

  if constexpr (!kApplyWave) {
#pragma unroll
    for (int k = 0; k < G::N; ++k) {
      const int I = G::list.I[k], J = G::list.J[k];
      double* o = out + (int64_t)(I * (I + 1) / 2 + J) * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) o[r * 64 + lane] = gacc[k][r];
    }
  }
}

constexpr int kFusedWaves = 12;  // four Q1 waves, eight Gram waves (three per SIMD)

// The fused kernel (see fused_body); partial Grams as k_stream16.
template <int SR, int NBUF, int NWF>
__device__ __forceinline__ void fused16_kernel(const double* A, int64_t m, int n, int64_t lda,
                                               const double* __restrict__ U, double* Q, int64_t ldq,
                                               double* __restrict__ partials, int64_t stages, int64_t spw, int desc,
                                               const int32_t* info) {
  __shared__ __attribute__((aligned(16))) double smem[(NBUF + 2) * kCols * SR];
  if (info != nullptr && *info != 0) return;
  constexpr int kF = kPlanRows / SR;
  const int64_t nst = (m + SR - 1) / SR;
  const int64_t u0 = (int64_t)blockIdx.x * spw;
  const int64_t u1 = u0 + spw < stages ? u0 + spw : stages;
  const int64_t s0 = u0 * kF;
  const int64_t s1 = u1 * kF < nst ? u1 * kF : nst;
  for (int e = threadIdx.x; e < (NBUF + 2) * kCols * SR; e += 64 * NWF)
    if ((e % (kCols * SR)) / SR >= n) smem[e] = 0.0;
  const bool direct_ok = (((uintptr_t)A & 15u) == 0) && ((lda & 1) == 0) && lda <= ((int64_t)1 << 26);
  const bool qvec_ok = (((uintptr_t)Q & 15u) == 0) && ((ldq & 1) == 0);
  double* out = partials + (int64_t)blockIdx.x * kLower * 256;
  const bool d = desc != 0;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#define CQR2_F16(WV) fused_body<SR, NBUF, NWF, WV>(A, m, n, lda, U, Q, ldq, out, s0, s1, d, direct_ok, qvec_ok, smem)
  switch (wave) {
    case 0: CQR2_F16(0); break;
    case 1: CQR2_F16(1); break;
    case 2: CQR2_F16(2); break;
    case 3: CQR2_F16(3); break;
    case 4: CQR2_F16(4); break;
    case 5: CQR2_F16(5); break;
    case 6: CQR2_F16(6); break;
    case 7: CQR2_F16(7); break;
    case 8: if constexpr (NWF > 8) CQR2_F16(8); break;
    case 9: if constexpr (NWF > 9) CQR2_F16(9); break;
    case 10: if constexpr (NWF > 10) CQR2_F16(10); break;
    case 11: if constexpr (NWF > 11) CQR2_F16(11); break;
    default: break;
  }
#undef CQR2_F16
}

// Each workgroup walks its range of SR-row stages (descending if desc);
// partial Grams of the workgroup at partials + blockIdx.x * 36 * 256.  reset_info: the first kernel
// of a factorization clears the info word (workgroup 0) and reads none.
template <int MODE, int SR, int NBUF>
__device__ __forceinline__ void stream16_kernel(const double* A, int64_t m, int n, int64_t lda,
                                                const double* __restrict__ U, double* Q, int64_t ldq,
                                                double* __restrict__ partials, int64_t stages, int64_t spw, int desc,
                                                int32_t* info, int reset_info) {
  __shared__ __attribute__((aligned(16))) double smem[NBUF * kCols * SR];
  if (reset_info) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *info = 0;
  } else if (info != nullptr && *info != 0) {
    return;
  }
  // the plan's units are 64-row blocks; this kernel's stages are SR rows
  constexpr int kF = kPlanRows / SR;
  const int64_t nst = (m + SR - 1) / SR;
  const int64_t u0 = (int64_t)blockIdx.x * spw;
  const int64_t u1 = u0 + spw < stages ? u0 + spw : stages;
  const int64_t s0 = u0 * kF;
  const int64_t s1 = u1 * kF < nst ? u1 * kF : nst;
  // columns >= n are never copied: zero them in every buffer once
  for (int e = threadIdx.x; e < NBUF * kCols * SR; e += kThreads)
    if ((e % (kCols * SR)) / SR >= n) smem[e] = 0.0;
  // direct copies: 16-byte row pairs, and a column pair's byte offset within
  // the 32-bit buffer offset
  const bool direct_ok = (((uintptr_t)A & 15u) == 0) && ((lda & 1) == 0) && lda <= ((int64_t)1 << 26);
  const bool qvec_ok = (((uintptr_t)Q & 15u) == 0) && ((ldq & 1) == 0);
  double* out = partials != nullptr ? partials + (int64_t)blockIdx.x * kLower * 256 : nullptr;
  const bool d = desc != 0;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#define CQR2_S16(WV) wave_body<MODE, SR, NBUF, WV>(A, m, n, lda, U, Q, ldq, out, s0, s1, d, direct_ok, qvec_ok, smem)
  switch (wave) {
    case 0: CQR2_S16(0); break;
    case 1: CQR2_S16(1); break;
    case 2: CQR2_S16(2); break;
    case 3: CQR2_S16(3); break;
    case 4: CQR2_S16(4); break;
    case 5: CQR2_S16(5); break;
    case 6: CQR2_S16(6); break;
    case 7: CQR2_S16(7); break;
    default: break;
  }
#undef CQR2_S16
}

// Sum of the partials in split order (8 contiguous sub-ranges added in
// order, then the 8 sums in order); writes the lower triangle of W and its
// mirror.
__device__ __forceinline__ void stream16_reduce(const double* __restrict__ part, int splits, int n,
                                                         double* __restrict__ W, int64_t ldw,
                                                         const int32_t* __restrict__ info) {
  __shared__ double red[8][32];
  if (info != nullptr && *info != 0) return;
  const int li = threadIdx.x & 31, sub = threadIdx.x >> 5;
  constexpr int total = kLower * 256;
  const int e = blockIdx.x * 32 + li;
  double v = 0.0;
  if (e < total) {
    const int s0 = (splits * sub) / 8, s1 = (splits * (sub + 1)) / 8;
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
  red[sub][li] = v;
  __syncthreads();
  if (sub != 0 || e >= total) return;
  double t = red[0][li];
#pragma unroll
  for (int k = 1; k < 8; ++k) t += red[k][li];
  const int tile = e >> 8, r = (e >> 6) & 3, l = e & 63;
  int I = 0;
  while ((I + 1) * (I + 2) / 2 <= tile) ++I;
  const int J = tile - I * (I + 1) / 2;
  const int row = 16 * I + 4 * r + (l >> 4), col = 16 * J + (l & 15);
  if (row >= col && row < n) {
    W[row + (int64_t)col * ldw] = t;
    W[col + (int64_t)row * ldw] = t;
  }
}


}  // namespace

// The named kernels (one name per role, for traces and counters).
template <int SR, int NBUF>
__global__ __launch_bounds__(kThreads, 1) void k_gram16(const double* A, int64_t m, int n, int64_t lda,
                                                       double* __restrict__ partials, int64_t stages, int64_t spw,
                                                       int32_t* info, int reset_info) {
  stream16_kernel<MODE_GRAM, SR, NBUF>(A, m, n, lda, nullptr, nullptr, 0, partials, stages, spw, 0, info, reset_info);
}

template <int SR, int NBUF>
__global__ __launch_bounds__(kThreads, 1) void k_apply16(const double* A, int64_t m, int n, int64_t lda,
                                                        const double* __restrict__ U, double* Q, int64_t ldq,
                                                        int64_t stages, int64_t spw, int32_t* info) {
  stream16_kernel<MODE_APPLY, SR, NBUF>(A, m, n, lda, U, Q, ldq, nullptr, stages, spw, 0, info, 0);
}

template <int SR, int NBUF, int NWF>
__global__ __launch_bounds__(64 * NWF, 1) void k_fused16(const double* A, int64_t m, int n, int64_t lda,
                                                        const double* __restrict__ U, double* Q, int64_t ldq,
                                                        double* __restrict__ partials, int64_t stages, int64_t spw,
                                                        const int32_t* info) {
  fused16_kernel<SR, NBUF, NWF>(A, m, n, lda, U, Q, ldq, partials, stages, spw, 1, info);
}

template <typename TA, bool F32, int SR, int NBUF>
__global__ __launch_bounds__(kThreads, 1) void k_apply256(const TA* A, int64_t m, int n, int64_t lda,
                                                         const double* __restrict__ U, void* Q, int64_t ldq,
                                                         int64_t stages, int64_t spw, const int32_t* info) {
  __shared__ __attribute__((aligned(16))) TA smem[NBUF * kWCols * SR];
  if (info != nullptr && *info != 0) return;
  constexpr int kF = kPlanRows / SR;
  const int64_t nst = (m + SR - 1) / SR;
  const int64_t u0 = (int64_t)blockIdx.x * spw;
  const int64_t u1 = u0 + spw < stages ? u0 + spw : stages;
  const int64_t s0 = u0 * kF;
  const int64_t s1 = u1 * kF < nst ? u1 * kF : nst;
  for (int e = threadIdx.x; e < NBUF * kWCols * SR; e += kThreads)
    if ((e % (kWCols * SR)) / SR >= n) smem[e] = (TA)0;
  const bool direct_ok = (((uintptr_t)A & 15u) == 0) && (((lda * (int64_t)sizeof(TA)) & 15) == 0) &&
                         lda <= ((int64_t)1 << 26);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#define CQR2_A256(WV) apply256_body<TA, F32, SR, NBUF, WV>(A, m, n, lda, U, Q, ldq, s0, s1, direct_ok, smem)
  switch (wave) {
    case 0: CQR2_A256(0); break;
    case 1: CQR2_A256(1); break;
    case 2: CQR2_A256(2); break;
    case 3: CQR2_A256(3); break;
    case 4: CQR2_A256(4); break;
    case 5: CQR2_A256(5); break;
    case 6: CQR2_A256(6); break;
    case 7: CQR2_A256(7); break;
    default: break;
  }
#undef CQR2_A256
}

// Q = A U for n <= 128 with the 128-column form of the same body: four waves,
// several workgroups per CU.  The mixed form's kernels at n <= 128 (FP32
// arithmetic into an FP32 Q1; FP32 Q1 widened exactly), and FP64 column
// blocks of the partial inverse.
template <typename TA, bool F32, int SR, int NBUF>
__global__ __launch_bounds__(256, 2) void k_apply128(const TA* A, int64_t m, int n, int64_t lda,
                                                    const double* __restrict__ U, void* Q, int64_t ldq,
                                                    int64_t stages, int64_t spw, const int32_t* info) {
  __shared__ __attribute__((aligned(16))) TA smem[NBUF * 128 * SR];
  if (info != nullptr && *info != 0) return;
  constexpr int kF = kPlanRows / SR;
  const int64_t nst = (m + SR - 1) / SR;
  const int64_t u0 = (int64_t)blockIdx.x * spw;
  const int64_t u1 = u0 + spw < stages ? u0 + spw : stages;
  const int64_t s0 = u0 * kF;
  const int64_t s1 = u1 * kF < nst ? u1 * kF : nst;
  for (int e = threadIdx.x; e < NBUF * 128 * SR; e += 256)
    if ((e % (128 * SR)) / SR >= n) smem[e] = (TA)0;
  const bool direct_ok = (((uintptr_t)A & 15u) == 0) && (((lda * (int64_t)sizeof(TA)) & 15) == 0) &&
                         lda <= ((int64_t)1 << 26);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#define CQR2_A128(WV) applyw_body<TA, F32, 128, SR, NBUF, WV>(A, m, n, lda, U, Q, ldq, s0, s1, direct_ok, smem)
  switch (wave) {
    case 0: CQR2_A128(0); break;
    case 1: CQR2_A128(1); break;
    case 2: CQR2_A128(2); break;
    case 3: CQR2_A128(3); break;
    default: break;
  }
#undef CQR2_A128
}

__global__ __launch_bounds__(256) void k_gram16_reduce(const double* __restrict__ part, int splits, int n,
                                                       double* __restrict__ W, int64_t ldw,
                                                       const int32_t* __restrict__ info) {
  stream16_reduce(part, splits, n, W, ldw, info);
}

Stream16Plan plan_stream16(int64_t m) {
  Stream16Plan p{};
  p.stages = m > 0 ? (m + kPlanRows - 1) / kPlanRows : 1;
  int64_t s = p.stages / 4;  // at least 4 stages per workgroup
  if (s < 1) s = 1;
  if (s > kSplits) s = kSplits;
  p.stages_per_wg = (p.stages + s - 1) / s;
  p.splits = (int)((p.stages + p.stages_per_wg - 1) / p.stages_per_wg);
  p.partial_bytes = (size_t)p.splits * kLower * 256 * sizeof(double);
  return p;
}

hipError_t launch_stream16_gram(const Stream16Plan& p, const double* A, int64_t m, int n, int64_t lda,
                                double* partials, const int32_t* info, hipStream_t s, int32_t* reset_info) {
  hipLaunchKernelGGL((k_gram16<kGramSR, kGramNBUF>), dim3(p.splits), dim3(kThreads), 0, s, A, m, n, lda, partials,
                     p.stages, p.stages_per_wg, reset_info != nullptr ? reset_info : const_cast<int32_t*>(info),
                     reset_info != nullptr ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_stream16_apply(const Stream16Plan& p, const double* A, int64_t m, int n, int64_t lda,
                                 const double* Upad, double* Q, int64_t ldq, const int32_t* info, hipStream_t s) {
  hipLaunchKernelGGL((k_apply16<kApplySR, kApplyNBUF>), dim3(p.splits), dim3(kThreads), 0, s, A, m, n, lda, Upad, Q,
                     ldq, p.stages, p.stages_per_wg, const_cast<int32_t*>(info));
  return hipGetLastError();
}

hipError_t launch_stream16_apply_gram(const Stream16Plan& p, const double* A, int64_t m, int n, int64_t lda,
                                      const double* Upad, double* Q, int64_t ldq, double* partials,
                                      const int32_t* info, hipStream_t s) {
  hipLaunchKernelGGL((k_fused16<kFusedSR, kFusedNBUF, kFusedWaves>), dim3(p.splits), dim3(64 * kFusedWaves), 0, s, A,
                     m, n, lda, Upad, Q, ldq, partials, p.stages, p.stages_per_wg, info);
  return hipGetLastError();
}

hipError_t launch_apply256(int a_f32, int f32_math, const void* A, int64_t m, int n, int64_t lda,
                           const double* Uimg, void* Q, int64_t ldq, const int32_t* info, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  const Stream16Plan p = plan_stream16(m);
  const dim3 g(p.splits), b(kThreads);
  if (f32_math)
    hipLaunchKernelGGL((k_apply256<double, true, 32, 2>), g, b, 0, s, (const double*)A, m, n, lda, Uimg, Q, ldq,
                       p.stages, p.stages_per_wg, info);
  else if (a_f32)
    hipLaunchKernelGGL((k_apply256<float, false, 32, 4>), g, b, 0, s, (const float*)A, m, n, lda, Uimg, Q, ldq,
                       p.stages, p.stages_per_wg, info);
  else
    hipLaunchKernelGGL((k_apply256<double, false, 32, 2>), g, b, 0, s, (const double*)A, m, n, lda, Uimg, Q, ldq,
                       p.stages, p.stages_per_wg, info);
  return hipGetLastError();
}

hipError_t launch_apply128(int a_f32, int f32_math, const void* A, int64_t m, int n, int64_t lda,
                           const double* Uimg, void* Q, int64_t ldq, const int32_t* info, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  // 64-row plan units, at least two per workgroup, at most 1024 workgroups
  const int64_t stages = (m + kPlanRows - 1) / kPlanRows;
  int64_t wgs = stages / 2;
  if (wgs < 1) wgs = 1;
  if (wgs > 1024) wgs = 1024;
  const int64_t spw = (stages + wgs - 1) / wgs;
  const dim3 g((unsigned)((stages + spw - 1) / spw)), b(256);
  if (f32_math)
    hipLaunchKernelGGL((k_apply128<double, true, 32, 2>), g, b, 0, s, (const double*)A, m, n, lda, Uimg, Q, ldq,
                       stages, spw, info);
  else if (a_f32)
    hipLaunchKernelGGL((k_apply128<float, false, 32, 4>), g, b, 0, s, (const float*)A, m, n, lda, Uimg, Q, ldq,
                       stages, spw, info);
  else
    hipLaunchKernelGGL((k_apply128<double, false, 32, 2>), g, b, 0, s, (const double*)A, m, n, lda, Uimg, Q, ldq,
                       stages, spw, info);
  return hipGetLastError();
}

hipError_t launch_stream16_reduce(const Stream16Plan& p, const double* partials, int n, double* W, int64_t ldw,
                                  const int32_t* info, hipStream_t s) {
  constexpr int total = kLower * 256;
  hipLaunchKernelGGL(k_gram16_reduce, dim3((total + 31) / 32), dim3(256), 0, s, partials, p.splits, n, W, ldw, info);
  return hipGetLastError();
}

}  // namespace cqr2
