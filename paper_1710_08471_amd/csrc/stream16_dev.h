// Device code shared by the MFMA 16x16x4 streaming kernels and the
// multi-problem step kernel: the LDS stage layout, the buffer resource word,
// and the body of Q = A U for 128 < n <= 256.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <type_traits>

#include "sync_dev.h"

namespace cqr2 {

// dword 3 of a raw buffer resource on gfx9-family parts (32-bit data format,
// no swizzle): loads within num_records bytes of the base
constexpr int kBufferRsrcWord3 = 0x00020000;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Stage of SR rows in LDS, column-major, the rows of column c stored XOR
// 2 (c & 15)
template <int SR>
__device__ __forceinline__ int spos(int c, int r) {
  return c * SR + (r ^ ((c & 15) << 1));
}

// ---- Q = A U for 64 < n <= 256 -----------------------------------------------
// U as its zero-padded row-major image (ld 256).  COLS = 256 (eight waves) or
// 128 (four waves); wave w owns the output column tiles w and COLS/16 - 1 - w
// (at COLS = 256, 68 k-steps of 4 per 16-row tile in all, the same for every
// wave) with their U fragments in registers, and both
// 16-row tiles of each 32-row stage: one read gives lane l A(2 (l%16),
// 4t + l/16) and the row below, the even-row and the odd-row tile.  Products
// on Qᵀ = Uᵀ Aᵀ, so a store covers 4 columns x 16 alternate rows (the other
// tile's store fills the rows between).  Stages run through a ring of NBUF
// LDS buffers with counted waits; Q may equal A.
//   TA = float: A (the mixed form's Q1) is staged as FP32 and widened exactly.
//   F32: FP32 MFMA with FP32 running sums, k ascending in steps of 4, on
//        fl32(A) and fl32(U), into an FP32 Q (the mixed form's pass 1).
// Result layouts: FP64 16x16x4 entry r of lane l is D(4r + l/16, l%16);
// FP32 16x16x4 entry r is D(4 (l/16) + r, l%16).
constexpr int kWCols = 256;  // leading dimension of the U image; the widest stage

template <typename TA, int SR>
__device__ __forceinline__ int wpos(int c, int r) {
  if constexpr (sizeof(TA) == 8) return spos<SR>(c, r);
  else return c * SR + r;  // a fragment read takes 16 lanes x 8 contiguous bytes of one column
}

template <typename TA, bool F32, int COLS, int SR, int NBUF, int W>
__device__ __forceinline__ void applyw_body(const TA* A, int64_t m, int n, int64_t lda,
                                            const double* __restrict__ U, void* Qv, int64_t ldq, int64_t s_begin,
                                            int64_t s_end, bool direct_ok, TA* smem) {
  static_assert(SR == 32, "two interleaved 16-row tiles per stage");
  static_assert(!F32 || sizeof(TA) == 8, "FP32 arithmetic takes the FP64 A");
  static_assert(COLS == 128 || COLS == 256, "128 or 256 columns");
  using UT = typename std::conditional<F32, float, double>::type;
  constexpr int kWaves = COLS / 32;
  constexpr int kThreads = 64 * kWaves;
  constexpr int kBuf = COLS * SR;              // elements of TA per stage
  constexpr int kRowsPerLane = 16 / (int)sizeof(TA);  // rows per 16-byte copy
  constexpr int kLPC = SR / kRowsPerLane;
  constexpr int kCPI = 64 / kLPC;
  constexpr int kInstr = COLS / kCPI;
  constexpr int J0 = W, J1 = COLS / 16 - 1 - W;
  constexpr int K0 = 4 * (J0 + 1), K1 = 4 * (J1 + 1);
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t count = s_end - s_begin;

  UT u0[K0], u1[K1];
  {
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int t = 0; t < K0; ++t) u0[t] = (UT)U[(4 * t + lk) * kWCols + 16 * J0 + lr];
#pragma unroll
    for (int t = 0; t < K1; ++t) u1[t] = (UT)U[(4 * t + lk) * kWCols + 16 * J1 + lr];
  }
  int fcount = 0;
#pragma unroll
  for (int p = W; p < kInstr; p += kWaves) fcount += (kCPI * p < n) ? 1 : 0;
  auto fill = [&](int64_t st, TA* buf) {
    const int64_t row0 = st * SR;
    if (direct_ok && row0 + SR <= m) {
      const int sub = lane / kLPC, lrow = kRowsPerLane * (lane % kLPC);
#pragma unroll
      for (int p = W; p < kInstr; p += kWaves) {
        if (kCPI * p < n) {
          const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
              (void*)(A + row0 + (int64_t)(kCPI * p) * lda), 0, 0x7fffffff, kBufferRsrcWord3);
          const int col = kCPI * p + sub;
          if (col < n) {
            const int grow = sizeof(TA) == 8 ? (lrow ^ ((col & 15) << 1)) : lrow;
            const int voff = (int)(((int64_t)sub * lda + grow) * (int64_t)sizeof(TA));
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void*)(buf + kCPI * p * SR),
                                                     16, voff, 0, 0, 0);
          }
        }
      }
    } else {
      for (int e = tid; e < kBuf; e += kThreads) {
        const int c = e / SR, r = e % SR;
        const int64_t row = row0 + r;
        if (c < n) buf[wpos<TA, SR>(c, r)] = row < m ? A[row + (int64_t)c * lda] : (TA)0;
      }
    }
  };

  int shist[NBUF - 1] = {};
  for (int64_t i = 0; i < NBUF - 1 && i < count; ++i) fill(s_begin + i, smem + (int)(i % NBUF) * kBuf);
  for (int64_t i = 0; i < count; ++i) {
    int later = 0;
    for (int64_t s2 = i + 1; s2 <= i + NBUF - 2 && s2 < count; ++s2) later += fcount;
    for (int h = 0; h < NBUF - 1; ++h) later += shist[h];
    wait_vmcnt_fenced(later > 32 ? 32 : later);
    lds_barrier();
    if (i + NBUF - 1 < count) fill(s_begin + i + NBUF - 1, smem + (int)((i + NBUF - 1) % NBUF) * kBuf);
    const TA* buf = smem + (int)(i % NBUF) * kBuf;
    const int64_t row0 = (s_begin + i) * SR;
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int lr = ln & 15, lk = ln >> 4;
    // A fragment pair of k-step t: rows 2 (l%16) and 2 (l%16) + 1 of column 4t + l/16
    auto afrag = [&](int t) -> double2 {
      if constexpr (sizeof(TA) == 8) {
        return *reinterpret_cast<const double2*>(buf + wpos<TA, SR>(4 * t + lk, 2 * lr));
      } else {
        const float2 v = *reinterpret_cast<const float2*>(buf + wpos<TA, SR>(4 * t + lk, 2 * lr));
        return double2{(double)v.x, (double)v.y};
      }
    };
    using AccT = typename std::conditional<F32, f4, d4>::type;
    AccT acc[2][2];
#pragma unroll
    for (int q = 0; q < 2; ++q) acc[q][0] = acc[q][1] = AccT{0, 0, 0, 0};
    double2 a[3];
    a[0] = afrag(0);
    a[1] = afrag(1);
    // at COLS = 128 the k-steps past n (zero columns of A) and a tile past n
    // are skipped (uniform branches); at COLS = 256 both tests fold away
    const bool on1 = COLS == 256 || 16 * J1 < n;
#pragma unroll
    for (int t = 0; t < K1; ++t) {
      if (t + 2 < K1) a[(t + 2) % 3] = afrag(t + 2);
      __builtin_amdgcn_sched_barrier(0);
      const bool kon = COLS == 256 || 4 * t < n;
      if (!kon) {
      } else if constexpr (F32) {
        const float ax = (float)a[t % 3].x, ay = (float)a[t % 3].y;
        if (on1) {
          acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(u1[t], ax, acc[0][1], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(u1[t], ay, acc[1][1], 0, 0, 0);
        }
        if (t < K0) {
          acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(u0[t], ax, acc[0][0], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(u0[t], ay, acc[1][0], 0, 0, 0);
        }
      } else {
        if (on1) {
          acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(u1[t], a[t % 3].x, acc[0][1], 0, 0, 0);
          acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(u1[t], a[t % 3].y, acc[1][1], 0, 0, 0);
        }
        if (t < K0) {
          acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(u0[t], a[t % 3].x, acc[0][0], 0, 0, 0);
          acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(u0[t], a[t % 3].y, acc[1][0], 0, 0, 0);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    int issued = 0;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int J = h ? J1 : J0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // column of entry r: 16 J + 4r + l/16 (FP64) or 16 J + 4 (l/16) + r (FP32)
        if (F32 ? 16 * J + r < n : 16 * J + 4 * r < n) {
          const int col = F32 ? 16 * J + 4 * lk + r : 16 * J + 4 * r + lk;
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int64_t row = row0 + 2 * lr + q;
            if (row < m && col < n) {
              if constexpr (F32) ((float*)Qv)[row + (int64_t)col * ldq] = acc[q][h][r];
              else ((double*)Qv)[row + (int64_t)col * ldq] = acc[q][h][r];
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
}


template <typename TA, bool F32, int SR, int NBUF, int W>
__device__ __forceinline__ void apply256_body(const TA* A, int64_t m, int n, int64_t lda,
                                              const double* __restrict__ U, void* Qv, int64_t ldq, int64_t s_begin,
                                              int64_t s_end, bool direct_ok, TA* smem) {
  applyw_body<TA, F32, 256, SR, NBUF, W>(A, m, n, lda, U, Qv, ldq, s_begin, s_end, direct_ok, smem);
}

}  // namespace cqr2
