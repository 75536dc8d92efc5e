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
// trailing matrix stays spread over all threads).  The owners of a block of
// columns publish them to a double-buffered LDS panel, every thread forms the
// L and Y entries it needs from it and applies the rank-B updates.
// ============================================================================
// s = sqrt(d) and y = 1/sqrt(d) for d > 0, each within a few ulp: the
// hardware reciprocal square root as a seed, two steps of the coupled
// (Goldschmidt) iteration for sqrt(d) and 1/(2 sqrt(d)), then one Newton
// correction of the square root.  Inputs below 2^-960 are scaled by an exact
// power of two first.  A much shorter dependency chain than sqrt() followed
// by a correctly rounded division.
__device__ __forceinline__ void sqrt_rsqrt(double d, double& s, double& y) {
  const bool tiny = d < 0x1p-960;
  const double ds = tiny ? d * 0x1p+960 : d;
  const double y0 = __builtin_amdgcn_rsq(ds);
  double g = ds * y0, h = 0.5 * y0;
  double e = fma(-g, h, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  e = fma(-g, h, 0.5);
  g = fma(g, e, g);
  h = fma(h, e, h);
  const double rr = fma(-g, g, ds);
  g = fma(rr, h, g);
  s = tiny ? g * 0x1p-480 : g;
  y = tiny ? (2.0 * h) * 0x1p+480 : 2.0 * h;
}

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
  // split order; the loads go out eight at a time
  double v = 0.0;
  int k = 0;
  for (; k + 8 <= s.splits; k += 8) {
    double x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = s.part[e + (k + j) * stride];
#pragma unroll
    for (int j = 0; j < 8; ++j) v += x[j];
  }
  for (; k < s.splits; ++k) v += s.part[e + k * stride];
  return v;
}

// Blocked form: B columns per barrier.  The owners of columns j0 .. j0+B-1
// publish them; every thread factors the B x B diagonal block itself (the
// same operations in the same order, so every thread gets the same bits),
// forms for each of its rows p the vector v(p) of L(p, j) (p below the block)
// or Y(j, p) (p above or inside it), and for each of its columns q the vector
// L(q, j), j in the block, and applies one rank-B update: the Schur update
// M(p, q) -= sum_j L(p, j) L(q, j) below the diagonal and the inverse's update
// Z(q, p) -= sum_j L(q, j) Y(j, p) above it (Y(j, p) = 0 for rows p below
// the block).
// B = 1 is the column-by-column form.
//
// Threads tid < G*G do the work; any further threads of the workgroup run
// the same loop as shadows (the same barriers and pivot tests, no element
// updates, no stores) so the body can sit in a workgroup larger than the
// grid.  colbuf: (2 B + 1) G T doubles of LDS.
template <int T, int G, int B>
__device__ __forceinline__ void cholinv_body(const CholInvSrc& src, int n, double* __restrict__ R, int64_t ldr,
                                             double* __restrict__ Rinv, int64_t ldri, double* __restrict__ Upad,
                                             int np, int32_t* __restrict__ info, int info_offset, double* colbuf_) {
  constexpr int NP = G * T;
  static_assert(G % B == 0, "a block of columns must not straddle two column blocks of the grid");
  // colbuf[buffer][k][idx]: column j0 + k of the block, row p stored at idx (p % G) T + p / G
  double (*colbuf)[B][NP] = reinterpret_cast<double (*)[B][NP]>(colbuf_);
  const int tid = threadIdx.x;
  const bool worker = tid < G * G;
  const int r = (tid % (G * G)) / G, c = tid % G;
  int fail = 0;
  if (info != nullptr && *info != 0) fail = -1;  // an earlier phase failed: skip, NaN outputs

  double M[T][T];
  // Y(j, j) for j < n, after the colbuf panels: the same reciprocal square
  // root the off-diagonal recurrences used, written and later read by the
  // owner of the diagonal entry
  double* ydiag = colbuf_ + 2 * B * NP;
  if (src.part == nullptr) {
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
      for (int b = 0; b < T; ++b) {
        const int p = r + G * a, q = c + G * b;
        double v = 0.0;
        if (worker && p >= q) v = (p < n) ? cholinv_src(src, p, q) : (p == q ? 1.0 : 0.0);
        M[a][b] = v;
      }
  } else {
    // the sum of the partial Grams, split by split (the same order per entry
    // as cholinv_src: from 0, splits ascending), with the loads of a quarter
    // of the tile (two rows) of one split in flight together
    const int64_t stride = (int64_t)src.nblk * 16;
#pragma unroll
    for (int a = 0; a < T; ++a)
#pragma unroll
      for (int b = 0; b < T; ++b) {
        const int p = r + G * a, q = c + G * b;
        M[a][b] = (worker && p >= q && p >= n && p == q) ? 1.0 : 0.0;
      }
    for (int k = 0; k < src.splits; ++k) {
      const double* base = src.part + k * stride;

      constexpr int RH = T >= 4 ? T / 4 : 1;  // rows per batch
#pragma unroll
      for (int h = 0; h < T / RH; ++h) {
        double x[RH][T];
#pragma unroll
        for (int a = 0; a < RH; ++a)
#pragma unroll
          for (int b = 0; b < T; ++b) {
            const int p = r + G * (h * RH + a), q = c + G * b;
            const int I = p >> 2, J = q >> 2;
            const int off = (I * (I + 1) / 2 + J) * 16 + (p & 3) * 4 + (q & 3);  // < 16 nblk
            x[a][b] = (worker && p >= q && p < n) ? base[off] : 0.0;
          }
#pragma unroll
        for (int a = 0; a < RH; ++a)
#pragma unroll
          for (int b = 0; b < T; ++b) M[h * RH + a][b] += x[a][b];
      }
    }
  }

  if (fail == 0) {
    int step = 0;
#pragma unroll
    for (int jb = 0; jb < T; ++jb) {
      if (G * jb >= n || fail != 0) break;
      for (int jc0 = 0; jc0 < G; jc0 += B) {
        const int j0 = G * jb + jc0;
        if (j0 >= n) break;
        double (*buf)[NP] = colbuf[step & 1];
        ++step;
        if (worker && c >= jc0 && c < jc0 + B) {
#pragma unroll
          for (int a = 0; a < T; ++a) buf[c - jc0][r * T + a] = M[a][jb];
        }
        __syncthreads();
        // the diagonal block, factored by every thread: Lb lower with L(j,j) on
        // the diagonal, Yb(k, i) = Y(j0 + k, j0 + i) for i <= k
        double D[B][B], Lb[B][B], Yb[B][B], sd[B], y[B];
#pragma unroll
        for (int i = 0; i < B; ++i)
#pragma unroll
          for (int k = 0; k < B; ++k) {
            const int p = j0 + i;
            D[i][k] = buf[k][(p % G) * T + p / G];
          }
        int bad = 0;
#pragma unroll
        for (int jj = 0; jj < B; ++jj) {
          double d = D[jj][jj];
#pragma unroll
          for (int ii = 0; ii < jj; ++ii) d = fma(-Lb[jj][ii], Lb[jj][ii], d);
          if (!(d > 0.0) && bad == 0) bad = j0 + jj + 1;  // non-positive or NaN pivot (uniform)
          sqrt_rsqrt(d, sd[jj], y[jj]);
          Lb[jj][jj] = sd[jj];
#pragma unroll
          for (int kk = jj + 1; kk < B; ++kk) {
            double t = D[kk][jj];
#pragma unroll
            for (int ii = 0; ii < jj; ++ii) t = fma(-Lb[kk][ii], Lb[jj][ii], t);
            Lb[kk][jj] = t * y[jj];
          }
          Yb[jj][jj] = y[jj];
#pragma unroll
          for (int pp = 0; pp < jj; ++pp) {
            double t = D[pp][jj];  // upper entry: Z(j0 + jj, j0 + pp)
#pragma unroll
            for (int ii = pp; ii < jj; ++ii) t = fma(-Lb[jj][ii], Yb[ii][pp], t);
            Yb[jj][pp] = t * y[jj];
          }
        }
        if (bad != 0) {
          fail = bad;
          break;
        }
        // shadow threads (beyond the G x G grid) skip the per-element work;
        // they keep only the barriers and the pivot test above
        if (worker) {
          // rows: v(p); the same recurrence gives L(p, j) below the block and
          // Y(j, p) above it; rows inside the block take Yb
          double v[T][B];
#pragma unroll
          for (int a = 0; a < T; ++a) {
            const int p = r + G * a;
#pragma unroll
            for (int jj = 0; jj < B; ++jj) {
              double t = buf[jj][r * T + a];
#pragma unroll
              for (int ii = 0; ii < jj; ++ii) t = fma(-Lb[jj][ii], v[a][ii], t);
              v[a][jj] = t * y[jj];
            }
            // p - j0 = G (a - jb) + (r - jc0) with r, jc0 in [0, G) and jc0 <= G - B:
            // negative for a < jb, at least B for a > jb, so only the register
            // row a == jb (both compile-time here) can hold rows of the block
            if (a == jb) {
              const int pp = p - j0;  // register arrays take compile-time indices only
#pragma unroll
              for (int i = 0; i < B; ++i)
                if (pp == i) {
#pragma unroll
                  for (int jj = 0; jj < B; ++jj) v[a][jj] = jj >= i ? Yb[jj][i] : 0.0;
                }
            }
          }
          // columns right of the block: L(q, j)
          double lq[T][B];
#pragma unroll
          for (int b = jb; b < T; ++b) {
#pragma unroll
            for (int jj = 0; jj < B; ++jj) {
              double t = buf[jj][c * T + b];
#pragma unroll
              for (int ii = 0; ii < jj; ++ii) t = fma(-Lb[jj][ii], lq[b][ii], t);
              lq[b][jj] = t * y[jj];
            }
          }
          // owners finalize the block's columns
#pragma unroll
          for (int kk = 0; kk < B; ++kk) {
            if (c != jc0 + kk) continue;
#pragma unroll
            for (int a = 0; a < T; ++a) {
              double val = v[a][kk];  // L(p, j) below the block, Y(j, p) above it
              if (a == jb) {  // the only register row that can hold rows of the block (see above)
                const int pp = r + G * a - j0;
#pragma unroll
                for (int i = 0; i < B; ++i)
                  if (pp == i) val = i > kk ? Lb[i][kk] : (i == kk ? sd[kk] : Yb[kk][i]);
                if (pp == kk) ydiag[j0 + kk] = y[kk];  // Y(j, j): the reciprocal the recurrences used
              }
              M[a][jb] = val;
            }
          }
          // rank-B update of every element right of the block: below the
          // diagonal with v(p) = L(p, .), above it with Y(., p), which is v(p)
          // for rows above or inside the block and zero for rows below it
          const bool right_of_block = c >= jc0 + B;  // column c + G jb lies right of the block
          const bool low_diag = r >= c;              // element (a, a) of this thread lies on or below the diagonal
#pragma unroll
          for (int a = 0; a < T; ++a) {
            // rows above or inside the block: all of a < jb, none of a > jb (see above)
            const bool row_up = a < jb ? true : (a > jb ? false : r + G * a < j0 + B);
            double vu[B];
#pragma unroll
            for (int jj = 0; jj < B; ++jj) vu[jj] = row_up ? v[a][jj] : 0.0;
#pragma unroll
            for (int b = jb; b < T; ++b) {
              if (b == jb && !right_of_block) continue;
              // rows below the block (a > jb) above the diagonal (b > a): Y(., p) = 0, no update
              if (a > jb && b > a) continue;
              double t = M[a][b];
#pragma unroll
              for (int jj = 0; jj < B; ++jj) {
                const double f = a > b ? v[a][jj] : (a < b ? vu[jj] : (low_diag ? v[a][jj] : vu[jj]));
                t = fma(-f, lq[b][jj], t);
              }
              M[a][b] = t;
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
            Rinv[p + (int64_t)p * ldri] = fail ? nan : ydiag[p];
          }
        }
      }
      if (Upad != nullptr && p < np && q < np) {
        double u = 0.0;
        if (p < q) u = v;
        else if (p == q) u = p < n ? ydiag[p] : 1.0;
        Upad[(int64_t)p * np + q] = fail ? nan : u;
      }
    }
}

}  // namespace cqr2
