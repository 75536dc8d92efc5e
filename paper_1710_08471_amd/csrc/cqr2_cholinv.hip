// CholInv (Algorithm 2) of an n x n SPD matrix, n <= 128, in one workgroup:
// the Cholesky factor and its triangular inverse together, FP64.
#include "cqr2_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>

namespace cqr2 {

// ============================================================================
// CholInv (Algorithm 2) for n <= 128 in one workgroup.
//
// The recursion's net effect, column by column: pivot d = W'(j,j), L(j,j) =
// sqrt(d), Y(j,j) = 1/L(j,j); L(i,j) = W'(i,j) * Y(j,j) (Algorithm 2's
// L21 = A21 Y11ᵀ at its 1x1 base); Schur update W' -= L(:,j) L(:,j)ᵀ; and the
// inverse's update Z(i,k) -= L(i,j) Y(j,k) (Y21 = -Y22 L21 Y11 unrolled).
// The n x n register-resident matrix M holds W' / L in its lower triangle and
// Zᵀ / Yᵀ (= R^{-1}) in its strict upper triangle; thread (r, c) of a G x G
// grid owns M(r + G a, c + G b) (a cyclic distribution, so the shrinking
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
// T x T cyclic tile of the padded order G T.  Up to n = 64 a 16 x 16 grid has
// the shorter per-column critical path; above, 32 x 32 threads share the
// larger Schur updates.
hipError_t launch_cholinv(const double* W, int64_t ldw, int n, double* R, int64_t ldr, double* Rinv,
                          int64_t ldri, double* Upad, int np, int32_t* info, int info_offset,
                          hipStream_t s) {
  const int order = padded_order(n);
#define CQR2_CI(TV, GV)                                                                                         \
  hipLaunchKernelGGL((k_cholinv<TV, GV>), dim3(1), dim3(GV * GV), 0, s, W, ldw, n, R, ldr, Rinv, ldri, Upad, np, \
                     info, info_offset)
  if (order == 32) CQR2_CI(2, 16);
  else if (order == 64) CQR2_CI(4, 16);
  else if (order == 128) CQR2_CI(4, 32);
  else return hipErrorInvalidValue;
#undef CQR2_CI
  return hipGetLastError();
}

}  // namespace cqr2
