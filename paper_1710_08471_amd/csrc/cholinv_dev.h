// Device code of the one-workgroup CholInv (Algorithm 2, n <= 128), shared
// by the one-problem kernel and the multi-problem step kernel.
#pragma once
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
// Input of the factorization: the lower triangle of W (n x n, ldw), or -- when
// `part` is set -- the sum, in split order, of `splits` partial Grams laid
// out as the Gram kernel writes them (per split: lower 4x4 blocks (I, J),
// block index I (I+1)/2 + J, 16 doubles row-major inside a block).
struct CholInvSrc {
  const double* W;
  int64_t ldw;
  const double* part;
  int splits;
  int nblk;
};

__device__ __forceinline__ double cholinv_src(const CholInvSrc& s, int p, int q) {
  if (s.part == nullptr) return s.W[p + (int64_t)q * s.ldw];
  const int I = p >> 2, J = q >> 2;
  const int64_t e = (int64_t)(I * (I + 1) / 2 + J) * 16 + (p & 3) * 4 + (q & 3);
  const int64_t stride = (int64_t)s.nblk * 16;
  double v = 0.0;
  for (int k = 0; k < s.splits; ++k) v += s.part[e + k * stride];
  return v;
}

// Threads tid < G*G do the work; any further threads of the workgroup run
// the same loop as shadows (same barriers, no stores) so the body can sit in
// a workgroup larger than the grid.  colbuf: 2 * G * T doubles of LDS.
template <int T, int G>
__device__ __forceinline__ void cholinv_body(const CholInvSrc& src, int n, double* __restrict__ R, int64_t ldr,
                                             double* __restrict__ Rinv, int64_t ldri, double* __restrict__ Upad,
                                             int np, int32_t* __restrict__ info, int info_offset, double* colbuf_) {
  constexpr int NP = G * T;
  double (*colbuf)[NP] = reinterpret_cast<double (*)[NP]>(colbuf_);
  const int tid = threadIdx.x;
  const bool worker = tid < G * G;
  const int r = (tid % (G * G)) / G, c = tid % G;
  int fail = 0;
  if (info != nullptr && *info != 0) fail = -1;  // an earlier phase failed: skip, NaN outputs

  double M[T][T];
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = 0; b < T; ++b) {
      const int p = r + G * a, q = c + G * b;
      double v = 0.0;
      if (worker && p >= q) v = (p < n) ? cholinv_src(src, p, q) : (p == q ? 1.0 : 0.0);
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
        if (worker && c == jc) {
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

  if (!worker) return;
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

}  // namespace cqr2
