// Device-side drivers built from the kernels: the recursive CholInv of
// Algorithm 2 for any n (base case: the single-workgroup kernel for n <= 128;
// from n = 512 the recursion split at 128 columns, run block by block with
// look-ahead), CholeskyQR2 (Algorithms 4 and 5) for n > 128 on the tiled
// kernels, and the least-squares solve on a finished factorization.
// Everything is enqueued on the caller's stream, except the blocked CholInv's
// bulk products, which fan out to two streams of the library and join back
// through events; nothing synchronizes with the host.
#include "cqr2_internal.h"

#include <hip/hip_runtime.h>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

namespace cqr2 {

constexpr int kBaseN = 128;  // largest CholInv handled by one workgroup

int64_t cholinv_split(int64_t n) {
  // h = largest multiple of the base size not above n/2 (at least one base block)
  int64_t h = (n / 2) / kBaseN * kBaseN;
  return h < kBaseN ? kBaseN : h;
}

int inverse_blocks(int64_t n, int depth, Block* out, int cap) {
  if (cap < 1) return 0;
  if (depth <= 0 || n <= kBaseN) {
    out[0] = {0, n};
    return 1;
  }
  const int64_t h = cholinv_split(n);
  const int a = inverse_blocks(h, depth - 1, out, cap);
  const int b = inverse_blocks(n - h, depth - 1, out + a, cap - a);
  for (int i = a; i < a + b; ++i) {
    out[i].c0 += h;
    out[i].c1 += h;
  }
  return a + b;
}

// Reduction splits used by every GEMM of the recursion, fixed by the shape only.
static int rec_splits(int64_t M, int64_t N, int64_t K) { return gemm_pick_splits(M, N, K, kPlanCUs); }

// ---- The recursion unrolled into 128-column blocks, with look-ahead --------
// Algorithm 2 splits W at any h; taking h = 128 at every level turns the
// recursion into a loop over the 128-column blocks k of W (a right-looking
// Cholesky that carries the inverse along):
//   base(k)   R_kk and R_kk^-1 from the updated diagonal block (one workgroup);
//   panel(k)  R_{k,>k} = R_kk^-T W_{>k,k}^T;
//   update(k) W_{>k,>k} -= R_{k,>k}^T R_{k,>k}  (lower triangle);
// and the off-diagonal blocks of the inverse come from the block form of the
// same equations on the leading (k+1) blocks, split before block k:
//   inv(k)    R^-1_{<k,k} = -R^-1_{<k,<k} (R_{<k,k} R_kk^-1).
// The only serial chain is the diagonal blocks.  The caller's stream runs
// base(k), panel(k) and the update of the diagonal block k + 1 by steps k - 1
// and k together (one product over block rows k - 1 and k of R), then
// base(k + 1).  Stream B runs the rest of update(k): first block column
// k + 1 below its diagonal block (the next panel's input), then the trailing
// lower triangle below block row k + 2 (one launch of the tiled SYRK in
// update mode).  Stream C runs inv(k).  Each block of W takes every step's
// update exactly once.  Events order every pair of steps that touch the same
// block:
//   B and C wait for panel(k) (recorded after base(k) and panel(k));
//   the caller's stream waits for B's first part of step k - 1 before
//   panel(k); B's second part of step k - 2, which wrote the diagonal block
//   k + 1 and block column k, comes before it on B;
//   the caller's stream joins B and C at the end.
// Used for n >= kLookaheadMinN at full inverse depth.
constexpr int64_t kLookaheadMinN = 512;

struct LookaheadLayout {
  size_t b_ws, c_x, c_ws, total;  // offsets of the helper streams' scratch, and the total
};

static size_t la_align(size_t x) { return (x + 255) / 256 * 256; }


// Reduction splits of inv(k)'s long product R^-1_{<k,<k} X (c0 x bk x c0): at
// most 256 of the reduction per workgroup, since the chain does not wait for
// it and its last steps would otherwise run past the chain.
static int la_inv_splits(int64_t c0, int64_t bk) {
  const int s = rec_splits(c0, bk, c0);
  int64_t by_len = (c0 + 255) / 256;
  if (by_len > 16) by_len = 16;
  return by_len > s ? (int)by_len : s;
}

static LookaheadLayout lookahead_layout(int64_t n) {
  size_t b = 0, cx = 0, cw = 0;
  auto mx = [](size_t& v, size_t x) { v = x > v ? x : v; };
  for (int64_t c0 = 0; c0 < n; c0 += kBaseN) {
    const int64_t bk = n - c0 < kBaseN ? n - c0 : kBaseN, c1 = c0 + bk, r1 = n - c1;
    if (r1 > 0) {
      const int64_t b1 = r1 < kBaseN ? r1 : kBaseN, r2 = r1 - b1;
      if (r2 > 0) mx(b, gemm_workspace_bytes(r2, b1, rec_splits(r2, b1, bk)));
    }
    if (c0 > 0) {
      mx(cx, (size_t)c0 * bk * sizeof(double));
      mx(cw, gemm_workspace_bytes(c0, bk, rec_splits(c0, bk, bk)));
      mx(cw, gemm_workspace_bytes(c0, bk, la_inv_splits(c0, bk)));
    }
  }
  LookaheadLayout L{};
  L.b_ws = 0;
  L.c_x = L.b_ws + la_align(b);
  L.c_ws = L.c_x + la_align(cx);
  L.total = L.c_ws + la_align(cw);
  return L;
}

size_t cholinv_rec_workspace(int64_t n) {
  // scratch T (h x n2 <= n*n/4) + the largest GEMM split workspace of the recursion
  if (n <= kBaseN) return 0;
  const size_t la = n >= kLookaheadMinN ? lookahead_layout(n).total : 0;
  const int64_t h = cholinv_split(n), n2 = n - h;
  size_t ws = 0;
  auto upd = [&](int64_t M, int64_t N, int64_t K) {
    const size_t b = gemm_workspace_bytes(M, N, rec_splits(M, N, K));
    ws = b > ws ? b : ws;
  };
  upd(h, n2, h);
  upd(n2, n2, h);
  upd(h, n2, n2);
  const size_t inner = cholinv_rec_workspace(h) > cholinv_rec_workspace(n2) ? cholinv_rec_workspace(h)
                                                                            : cholinv_rec_workspace(n2);
  const size_t mine = (size_t)h * n2 * sizeof(double) + ws;
  const size_t rec = mine > inner ? mine : inner;
  return rec > la ? rec : la;
}

__global__ void k_zero_block(double* X, int64_t ldx, int64_t rows, int64_t cols) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  X[(e % rows) + (e / rows) * ldx] = 0.0;
}

static hipError_t zero_block(double* X, int64_t ldx, int64_t rows, int64_t cols, hipStream_t s) {
  const int64_t total = rows * cols;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_block, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, X, ldx, rows, cols);
  return hipGetLastError();
}

#define CQR2_HIP(expr)              \
  do {                              \
    hipError_t _e = (expr);         \
    if (_e != hipSuccess) return _e; \
  } while (0)

// W: n x n (ldw), lower triangle read; its trailing blocks are overwritten by
// Schur complements.  R, Rinv: n x n upper (ldr, ldri), strictly lower parts 0.
// work: >= cholinv_rec_workspace(n) bytes.
// Zeros below the diagonal of R and Rinv (n x n), in one launch.
__global__ void k_zero_lower2(double* R, int64_t ldr, double* Rinv, int64_t ldri, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int64_t i = e % n, j = e / n;
  if (i <= j) return;
  R[i + j * ldr] = 0.0;
  Rinv[i + j * ldri] = 0.0;
}

// Helper streams and events of the look-ahead form, one set per device,
// created on first use and kept until the process ends: B and C carry the
// bulk products next to the chain on the caller's stream.  They run at the
// default priority and do not synchronize with the null stream.  The mutex
// keeps one factorization's records and waits together when several host
// threads enqueue.
struct LookaheadStreams {
  std::mutex mu;
  hipStream_t b = nullptr, c = nullptr;
  std::vector<hipEvent_t> ev;
};
constexpr int kMaxDevices = 64;
static LookaheadStreams g_la[kMaxDevices];

static hipError_t lookahead_events(LookaheadStreams& L, size_t count) {
  if (L.b == nullptr) CQR2_HIP(hipStreamCreateWithFlags(&L.b, hipStreamNonBlocking));
  if (L.c == nullptr) CQR2_HIP(hipStreamCreateWithFlags(&L.c, hipStreamNonBlocking));
  while (L.ev.size() < count) {
    hipEvent_t e;
    CQR2_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    L.ev.push_back(e);
  }
  return hipSuccess;
}

// ---- The chain's two small products ------------------------------------------
// MFMA 16x16x4 (FP64) with both operands read straight from global memory (a
// few hundred KB, just written): no LDS staging, the whole reduction in one
// launch.  Operand lane l holds A(row l%16, k + l/16) and B(k + l/16, column
// l%16); result entry r of lane l is D(4r + l/16, l%16).  The operands of up
// to kChainBatch k-steps are loaded before their products.
typedef double chain_d4 __attribute__((ext_vector_type(4)));
constexpr int kChainBatch = 32;

// The 16 x 16 tile's sum over k in [kb, ke) of opA(i, k) opB(k, j), in the
// result layout above; lda_(k) and ldb_(k) return this lane's opA(i, k) and
// opB(k, j) (0 outside the matrices).
template <typename LA, typename LB>
__device__ __forceinline__ chain_d4 chain_mfma(int kb, int ke, int k4, LA lda_, LB ldb_) {
  chain_d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = kb; k0 < ke; k0 += 4 * kChainBatch) {
    double a[kChainBatch], b[kChainBatch];
#pragma unroll
    for (int q = 0; q < kChainBatch; ++q) {
      const int k = k0 + 4 * q + k4;
      a[q] = k < ke ? lda_(k) : 0.0;
      b[q] = k < ke ? ldb_(k) : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kChainBatch; ++q)
      if (k0 + 4 * q < ke) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q], acc, 0, 0, 0);
  }
  return acc;
}

// D = alpha A B for A (M x K, lda) and B (K x N, ldb), both column-major:
// A upper (A(i, k) = 0 for k < i) if AUP, B upper (B(k, j) = 0 for k > j) if
// BUP -- the reduction of a tile then skips those k, and the entries it still
// reads inside a 16 x 16 diagonal block must be stored zeros -- and D stored
// transposed (D(i, j) at C[j + i ldc]) if TOUT, else at C[i + j ldc].  One
// wave per 16 x 16 tile, four per workgroup.
template <bool AUP, bool BUP, bool TOUT>
__global__ __launch_bounds__(256) void k_chain_nn(const double* __restrict__ A, int64_t lda,
                                                  const double* __restrict__ B, int64_t ldb, int M, int N, int K,
                                                  double alpha, double* __restrict__ C, int64_t ldc,
                                                  const int32_t* __restrict__ info) {
  if (info != nullptr && *info != 0) return;
  const int lane = threadIdx.x & 63;
  const int t = (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  const int tn = (N + 15) / 16, I = t / tn, J = t % tn;
  if (16 * I >= M) return;  // past the last tile (wave-uniform; no barrier follows)
  const int r16 = lane & 15, k4 = lane >> 4;
  const int i = 16 * I + r16, j = 16 * J + r16;
  const int kb = AUP ? 16 * I : 0;
  const int ke = BUP ? (K < 16 * J + 16 ? K : 16 * J + 16) : K;
  const chain_d4 acc = chain_mfma(
      kb, ke, k4, [&](int k) { return i < M ? A[i + (int64_t)k * lda] : 0.0; },
      [&](int k) { return j < N ? B[k + (int64_t)j * ldb] : 0.0; });
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ii = 16 * I + 4 * r + k4, jj = 16 * J + r16;
    if (ii < M && jj < N) C[TOUT ? jj + (int64_t)ii * ldc : ii + (int64_t)jj * ldc] = alpha * acc[r];
  }
}

template <bool AUP, bool BUP, bool TOUT>
static hipError_t launch_chain_nn(const double* A, int64_t lda, const double* B, int64_t ldb, int64_t M, int64_t N,
                                  int64_t K, double alpha, double* C, int64_t ldc, const int32_t* info,
                                  hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t tiles = ((M + 15) / 16) * ((N + 15) / 16);
  hipLaunchKernelGGL((k_chain_nn<AUP, BUP, TOUT>), dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, A, lda, B,
                     ldb, (int)M, (int)N, (int)K, alpha, C, ldc, info);
  return hipGetLastError();
}

// C(i, j) -= sum_{k < K} A(k, i) A(k, j) for j <= i < M (A: K x M, lda; C: the
// lower triangle of M x M).  A workgroup per lower 16 x 16 tile; its four
// waves take a quarter of the reduction each, and wave 0 adds the four in
// wave order.
__global__ __launch_bounds__(256) void k_chain_diag(const double* __restrict__ A, int64_t lda, int M, int K,
                                                    double* __restrict__ C, int64_t ldc,
                                                    const int32_t* __restrict__ info) {
  __shared__ double part[4][4][64];
  if (info != nullptr && *info != 0) return;
  const int t = (int)blockIdx.x;
  int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while (I * (I + 1) / 2 > t) --I;
  while ((I + 1) * (I + 2) / 2 <= t) ++I;
  const int J = t - I * (I + 1) / 2;
  const int w = (int)(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int r16 = lane & 15, k4 = lane >> 4;
  const int i = 16 * I + r16, j = 16 * J + r16;
  const int kq = (K + 15) / 16 * 4;  // each wave's share, a multiple of 4
  const int kb = w * kq, ke = K < kb + kq ? K : kb + kq;
  const chain_d4 acc = chain_mfma(
      kb, ke, k4, [&](int k) { return i < M ? A[k + (int64_t)i * lda] : 0.0; },
      [&](int k) { return j < M ? A[k + (int64_t)j * lda] : 0.0; });
#pragma unroll
  for (int r = 0; r < 4; ++r) part[w][r][lane] = acc[r];
  __syncthreads();
  if (w != 0) return;
  double old[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ii = 16 * I + 4 * r + k4, jj = 16 * J + r16;
    old[r] = (ii < M && jj <= ii) ? C[ii + (int64_t)jj * ldc] : 0.0;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int ii = 16 * I + 4 * r + k4, jj = 16 * J + r16;
    const double sum = ((part[0][r][lane] + part[1][r][lane]) + part[2][r][lane]) + part[3][r][lane];
    if (ii < M && jj <= ii) C[ii + (int64_t)jj * ldc] = old[r] - sum;
  }
}

// R_{k,>k} = R_kk^-T W_{>k,k}^T, computed as (W_{>k,k} R_kk^-1)ᵀ: Wb is the
// r1 x bk block W_{>k,k} (ldw), Rikk the bk x bk upper R_kk^-1 (ldri, zero
// below its diagonal), Rk1 the bk x r1 block of R (ldr).
static hipError_t launch_chain_panel(const double* Wb, int64_t ldw, const double* Rikk, int64_t ldri, int64_t r1,
                                     int64_t bk, double* Rk1, int64_t ldr, const int32_t* info, hipStream_t s) {
  return launch_chain_nn<false, true, true>(Wb, ldw, Rikk, ldri, r1, bk, bk, 1.0, Rk1, ldr, info, s);
}

// W_d (n1 x n1, lower) -= Rdᵀ Rd for the kr x n1 block Rd of R (ldr).
static hipError_t launch_chain_diag(const double* Rd, int64_t ldr, int64_t kr, int64_t n1, double* Wd, int64_t ldw,
                                    const int32_t* info, hipStream_t s) {
  const int64_t t = (n1 + 15) / 16, tiles = t * (t + 1) / 2;
  hipLaunchKernelGGL(k_chain_diag, dim3((unsigned)tiles), dim3(256), 0, s, Rd, ldr, (int)n1, (int)kr, Wd, ldw, info);
  return hipGetLastError();
}

static hipError_t cholinv_lookahead(double* W, int64_t ldw, int64_t n, double* R, int64_t ldr, double* Rinv,
                                    int64_t ldri, char* work, int32_t* info, int info_offset, hipStream_t s) {
  int dev = 0;
  CQR2_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  LookaheadStreams& L = g_la[dev];
  std::lock_guard<std::mutex> lock(L.mu);
  const int64_t nb = (n + kBaseN - 1) / kBaseN;
  // events: P_k (base(k), and panel(k) when there is one, done), T1_k (B's
  // first part of update k done), and the joins of B and C.  Every event the
  // caller's stream records or waits for costs the chain about 6 us, even when
  // already complete, so the chain records one and waits for one per block.
  CQR2_HIP(lookahead_events(L, (size_t)(2 * nb + 2)));
  hipEvent_t* evP = L.ev.data();
  hipEvent_t* evT1 = evP + nb;
  hipEvent_t joinB = evT1[nb], joinC = evT1[nb + 1];
  const LookaheadLayout lay = lookahead_layout(n);
  double* wsB = (double*)(work + lay.b_ws);
  double* X = (double*)(work + lay.c_x);
  double* wsC = (double*)(work + lay.c_ws);
  bool b_used = false, c_used = false;
  std::vector<char> has_b((size_t)nb, 0);  // step k ran work on B
  for (int64_t k = 0; k < nb; ++k) {
    const int64_t c0 = k * kBaseN, bk = n - c0 < kBaseN ? n - c0 : kBaseN;
    const int64_t c1 = c0 + bk, r1 = n - c1;
    double* Rkk = R + c0 + c0 * ldr;
    double* Rikk = Rinv + c0 + c0 * ldri;
    CQR2_HIP(launch_cholinv(W + c0 + c0 * ldw, ldw, (int)bk, Rkk, ldr, Rikk, ldri, nullptr, 0, info,
                            info_offset + (int)c0, s));
    const int64_t b1 = r1 < kBaseN ? r1 : kBaseN, c2 = c1 + b1, r2 = n - c2;
    double* Rk1 = R + c0 + c1 * ldr;  // R_{k,>k}: bk x r1
    double* Rk2 = R + c0 + c2 * ldr;  // R_{k,>k+1}: bk x r2
    if (r1 > 0) {
      // panel(k) reads block column k below the diagonal, which B's first
      // part of step k - 1 wrote last; B's second part of step k - 2, which
      // wrote the diagonal block k + 1, precedes it on B
      if (k >= 1 && has_b[k - 1]) CQR2_HIP(hipStreamWaitEvent(s, evT1[k - 1], 0));
      // panel(k): R_{k,>k} = R_kk^-T W_{>k,k}^T
      CQR2_HIP(launch_chain_panel(W + c1 + c0 * ldw, ldw, Rikk, ldri, r1, bk, Rk1, ldr, info, s));
    }
    CQR2_HIP(hipEventRecord(evP[k], s));
    if (k >= 1) {
      // inv(k) on stream C: X = R_{<k,k} R_kk^-1, then R^-1_{<k,k} = -R^-1_{<k,<k} X
      CQR2_HIP(hipStreamWaitEvent(L.c, evP[k], 0));
      CQR2_HIP(launch_gemm(0, 0, c0, bk, bk, 1.0, R + c0 * ldr, ldr, Rikk, ldri, 0.0, X, c0, GEMM_B_UPPER,
                           rec_splits(c0, bk, bk), wsC, info, L.c));
      CQR2_HIP(launch_gemm(0, 0, c0, bk, c0, -1.0, Rinv, ldri, X, c0, 0.0, Rinv + c0 * ldri, ldri, GEMM_A_UPPER,
                           la_inv_splits(c0, bk), wsC, info, L.c));
      c_used = true;
    }
    if (r1 <= 0) break;
    if (r2 > 0) {
      // on stream B, update(k) below block row k + 1: first block column
      // k + 1 (the next panel's input), then the trailing lower triangle
      // below block row k + 2 in one launch of the tiled SYRK in update mode
      // (the diagonal block k + 2 takes update(k) on the caller's stream,
      // together with update(k + 1))
      CQR2_HIP(hipStreamWaitEvent(L.b, evP[k], 0));
      CQR2_HIP(launch_gemm(1, 0, r2, b1, bk, -1.0, Rk2, ldr, Rk1, ldr, 1.0, W + c2 + c1 * ldw, ldw, 0,
                           rec_splits(r2, b1, bk), wsB, info, L.b));
      CQR2_HIP(hipEventRecord(evT1[k], L.b));
      CQR2_HIP(launch_syrk_update(Rk2, bk, (int)r2, ldr, -1.0, W + c2 + c2 * ldw, ldw, 1, info, L.b));
      has_b[k] = 1;
      b_used = true;
    }
    // the diagonal block k + 1, the next link of the chain, takes update(k)
    // and update(k - 1) in one product (block rows k - 1 and k of R are
    // adjacent)
    const int64_t kr = k >= 1 ? 2 * kBaseN : bk;
    CQR2_HIP(launch_chain_diag(R + (c1 - kr) + c1 * ldr, ldr, kr, b1, W + c1 + c1 * ldw, ldw, info, s));
  }
  if (b_used) {
    CQR2_HIP(hipEventRecord(joinB, L.b));
    CQR2_HIP(hipStreamWaitEvent(s, joinB, 0));
  }
  if (c_used) {
    CQR2_HIP(hipEventRecord(joinC, L.c));
    CQR2_HIP(hipStreamWaitEvent(s, joinC, 0));
  }
  return hipSuccess;
}

// The recursion proper: the strictly lower blocks off the diagonal are left
// for the caller (cholinv_recursive zeroes them all in one launch).
static hipError_t cholinv_rec(double* W, int64_t ldw, int64_t n, double* R, int64_t ldr, double* Rinv, int64_t ldri,
                              char* work, int32_t* info, int info_offset, hipStream_t s, int depth) {
  if (n <= kBaseN) return launch_cholinv(W, ldw, (int)n, R, ldr, Rinv, ldri, nullptr, 0, info, info_offset, s);
  if (depth == 0 && n >= kLookaheadMinN)
    return cholinv_lookahead(W, ldw, n, R, ldr, Rinv, ldri, work, info, info_offset, s);
  const int64_t h = cholinv_split(n), n2 = n - h;
  double* W22 = W + h + h * ldw;
  double* R12 = R + h * ldr;
  double* R22 = R + h + h * ldr;
  double* Ri12 = Rinv + h * ldri;
  double* Ri22 = Rinv + h + h * ldri;
  double* T = (double*)work;
  double* gws = (double*)(work + (size_t)h * n2 * sizeof(double));
  const int sub = depth > 0 ? depth - 1 : 0;
  // leading diagonal block: its factor and inverse, recursively
  CQR2_HIP(cholinv_rec(W, ldw, h, R, ldr, Rinv, ldri, work, info, info_offset, s, sub));
  // h = 128: the leading inverse is a base case (zero below its diagonal), and
  // the products are small enough for the one-launch kernels
  const bool small = h == kBaseN && n2 <= 3 * kBaseN;
  if (depth == 0 && small) {
    CQR2_HIP(launch_chain_panel(W + h, ldw, Rinv, ldri, n2, h, R12, ldr, info, s));
  } else if (depth == 0) {
    // off-diagonal block of the factor from the leading inverse, kept transposed
    // in R's upper part: R12 = Rinv11ᵀ A21ᵀ
    CQR2_HIP(launch_gemm(1, 1, h, n2, h, 1.0, Rinv, ldri, W + h, ldw, 0.0, R12, ldr, GEMM_A_LOWER,
                         rec_splits(h, n2, h), gws, info, s));
  } else {
    // partial inverse: the same off-diagonal block by block substitution
    // over the leading block's inverted diagonal blocks; for block b the
    // columns of A21 minus the contribution of the blocks before it, times
    // that block's inverse.  T (n2 x width) lives in the scratch block.
    Block blk[256];
    const int nb = inverse_blocks(h, sub, blk, 256);
    for (int i = 0; i < nb; ++i) {
      const int64_t c0 = blk[i].c0, b = blk[i].c1 - blk[i].c0;
      CQR2_HIP(hipMemcpy2DAsync(T, n2 * sizeof(double), W + h + c0 * ldw, ldw * sizeof(double), n2 * sizeof(double),
                                b, hipMemcpyDeviceToDevice, s));
      if (c0 > 0)
        CQR2_HIP(launch_gemm(1, 0, n2, b, c0, -1.0, R12, ldr, R + c0 * ldr, ldr, 1.0, T, n2, 0, 1, nullptr, info,
                             s));
      CQR2_HIP(launch_gemm(1, 1, b, n2, b, 1.0, Rinv + c0 + c0 * ldri, ldri, T, n2, 0.0, R12 + c0, ldr,
                           GEMM_A_LOWER, 1, nullptr, info, s));
    }
  }
  // trailing Schur complement (lower triangle): A22 - R12ᵀ R12
  if (small)
    CQR2_HIP(launch_chain_diag(R12, ldr, h, n2, W22, ldw, info, s));
  else
    CQR2_HIP(launch_gemm(1, 0, n2, n2, h, -1.0, R12, ldr, R12, ldr, 1.0, W22, ldw, GEMM_C_LOWER,
                         rec_splits(n2, n2, h), gws, info, s));
  // trailing diagonal block: factor and inverse of the Schur complement
  CQR2_HIP(cholinv_rec(W22, ldw, n2, R22, ldr, Ri22, ldri, work, info, info_offset + (int)h, s, sub));
  if (depth == 0 && small) {
    // Rinv12 = -(Rinv11 R12) Rinv22; Rinv22's 16 x 16 diagonal blocks lie in
    // its base cases' diagonal blocks (zero below the diagonal)
    CQR2_HIP((launch_chain_nn<true, false, false>(Rinv, ldri, R12, ldr, h, n2, h, 1.0, T, h, info, s)));
    CQR2_HIP((launch_chain_nn<false, true, false>(T, h, Ri22, ldri, h, n2, n2, -1.0, Ri12, ldri, info, s)));
  } else if (depth == 0) {
    // off-diagonal block of the inverse from the two diagonal inverses and
    // R12: Rinv12 = -(Rinv11 R12) Rinv22
    CQR2_HIP(launch_gemm(0, 0, h, n2, h, 1.0, Rinv, ldri, R12, ldr, 0.0, T, h, GEMM_A_UPPER, rec_splits(h, n2, h),
                         gws, info, s));
    CQR2_HIP(launch_gemm(0, 0, h, n2, n2, -1.0, T, h, Ri22, ldri, 0.0, Ri12, ldri, GEMM_B_UPPER,
                         rec_splits(h, n2, n2), gws, info, s));
  } else {
    CQR2_HIP(zero_block(Ri12, ldri, h, n2, s));  // the inverse's off-diagonal block is not formed at this level
  }
  return hipSuccess;
}

hipError_t cholinv_recursive(double* W, int64_t ldw, int64_t n, double* R, int64_t ldr, double* Rinv, int64_t ldri,
                             char* work, int32_t* info, int info_offset, hipStream_t s, int depth) {
  CQR2_HIP(cholinv_rec(W, ldw, n, R, ldr, Rinv, ldri, work, info, info_offset, s, depth));
  if (n <= kBaseN) return hipSuccess;  // the one-workgroup kernel zeroes its own lower part
  const int64_t total = n * n;
  hipLaunchKernelGGL(k_zero_lower2, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, R, ldr, Rinv, ldri, n);
  return hipGetLastError();
}

// After a breakdown (*info != 0): the upper triangle of X (n x n) := NaN.
__global__ void k_nan_upper_if_info(double* X, int64_t ldx, int64_t n, const int32_t* info) {
  if (*info == 0) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int64_t i = e % n, j = e / n;
  if (i <= j) X[i + j * ldx] = __builtin_nan("");
}

hipError_t launch_nan_upper_if_info(double* X, int64_t ldx, int64_t n, const int32_t* info, hipStream_t s) {
  const int64_t total = n * n;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nan_upper_if_info, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, X, ldx, n, info);
  return hipGetLastError();
}

__global__ void k_set_info(int32_t* info, int32_t value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *info = value;
}

hipError_t launch_set_info(int32_t* info, int32_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_info, dim3(1), dim3(64), 0, s, info, value);
  return hipGetLastError();
}

// Shifted CholeskyQR's first pass factors W + s I with
// s = 11 (m n + n (n + 1)) u trace(W), u = 2^-53 (trace W = ||A||_F^2).  One
// workgroup: strided partial sums of the diagonal, then a fixed-order tree,
// so the shift is the same bits on every run.
__global__ __launch_bounds__(256) void k_shift_diag(double* W, int64_t ldw, int64_t n, int64_t m,
                                                    const int32_t* info) {
  __shared__ double part[256];
  if (info != nullptr && *info != 0) return;
  double t = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) t += W[i + i * ldw];
  part[threadIdx.x] = t;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
    __syncthreads();
  }
  const double trace = part[0];
  const double s = 11.0 * ((double)m * (double)n + (double)n * (double)(n + 1)) * 0x1p-53 * trace;
  for (int64_t i = threadIdx.x; i < n; i += 256) W[i + i * ldw] += s;
}

hipError_t launch_shift_diag(double* W, int64_t ldw, int64_t n, int64_t m, const int32_t* info, hipStream_t s) {
  hipLaunchKernelGGL(k_shift_diag, dim3(1), dim3(256), 0, s, W, ldw, n, m, info);
  return hipGetLastError();
}

// W(j, i) = W(i, j) for i > j (complete a lower-triangle result).
__global__ void k_mirror_lower(double* W, int64_t ldw, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int64_t i = e % n, j = e / n;
  if (i > j) W[j + i * ldw] = W[i + j * ldw];
}

hipError_t launch_mirror_lower(double* W, int64_t ldw, int64_t n, hipStream_t s) {
  const int64_t total = n * n;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mirror_lower, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, W, ldw, n);
  return hipGetLastError();
}

// R = upper triangle of P (n x n) with zeros below; NaN everywhere after a
// breakdown; publish the info word.
// P may equal R (in place: each thread reads and writes one element).
__global__ __launch_bounds__(256) void k_finalize_r(const double* P, int64_t ldp, double* R, int64_t ldr, int64_t n,
                                                    const int32_t* info, int32_t* user_info) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t st = info != nullptr ? *info : 0;
  if (e == 0 && user_info != nullptr) *user_info = st;
  if (e >= n * n) return;
  const int64_t i = e % n, j = e / n;
  R[i + j * ldr] = st != 0 ? __builtin_nan("") : (i <= j ? P[i + j * ldp] : 0.0);
}

hipError_t launch_finalize_r(const double* P, int64_t ldp, double* R, int64_t ldr, int64_t n, const int32_t* info,
                             int32_t* user_info, hipStream_t s) {
  const int64_t total = n * n;
  hipLaunchKernelGGL(k_finalize_r, dim3((unsigned)((total + 255) / 256 > 0 ? (total + 255) / 256 : 1)), dim3(256),
                     0, s, P, ldp, R, ldr, n, info, user_info);
  return hipGetLastError();
}

// R = triu(X Y) for upper-triangular X, Y (n x n, column-major, ld n); NaN
// after a breakdown; the info word copied to user_info.  A workgroup per 16 x 16
// tile of R: the tile's rows of X and columns of Y (k from 16 I to the tile's
// last column) go through LDS, then each thread sums its entry over k = i..j in
// ascending order.
constexpr int kUpT = 16;
constexpr int kUpMaxN = 128;

__global__ __launch_bounds__(kUpT * kUpT) void k_upper_product_final(const double* __restrict__ X,
                                                                     const double* __restrict__ Y, int n, double* R,
                                                                     int64_t ldr, const int32_t* info,
                                                                     int32_t* user_info) {
  __shared__ double xs[kUpT][kUpMaxN];
  __shared__ double ys[kUpMaxN][kUpT];
  const int I = blockIdx.x, J = blockIdx.y;
  const int ti = threadIdx.x % kUpT, tj = threadIdx.x / kUpT;
  const int i = kUpT * I + ti, j = kUpT * J + tj;
  const int32_t st = *info;
  if (I == 0 && J == 0 && threadIdx.x == 0 && user_info != nullptr) *user_info = st;
  const bool work = st == 0 && J >= I;
  if (work) {
    const int k0 = kUpT * I, k1 = min(n, kUpT * J + kUpT);
    for (int e = threadIdx.x; e < kUpT * (k1 - k0); e += kUpT * kUpT) {
      const int r = e % kUpT, k = k0 + e / kUpT;
      const int row = kUpT * I + r, col = kUpT * J + r;
      xs[r][k - k0] = row < n ? X[row + (int64_t)k * n] : 0.0;
      ys[k - k0][r] = col < n ? Y[k + (int64_t)col * n] : 0.0;
    }
  }
  __syncthreads();
  if (i >= n || j >= n) return;
  double v = 0.0;
  if (work && i <= j) {
    const int k0 = kUpT * I;
    for (int k = i; k <= j; ++k) v = fma(xs[ti][k - k0], ys[k - k0][tj], v);
  }
  R[i + (int64_t)j * ldr] = st != 0 ? __builtin_nan("") : v;
}

hipError_t launch_upper_product_final(const double* X, const double* Y, int64_t n, double* R, int64_t ldr,
                                      const int32_t* info, int32_t* user_info, hipStream_t s) {
  if (n < 1 || n > kUpMaxN) return hipErrorInvalidValue;
  const unsigned t = (unsigned)((n + kUpT - 1) / kUpT);
  hipLaunchKernelGGL(k_upper_product_final, dim3(t, t), dim3(kUpT * kUpT), 0, s, X, Y, (int)n, R, ldr, info,
                     user_info);
  return hipGetLastError();
}

// ---- CholeskyQR2 for n > 128 ------------------------------------------------
GeneralPlan plan_general(int64_t m, int64_t n, bool mixed, int depth) {
  GeneralPlan p{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) / 256 * 256;
    return o;
  };
  const size_t nn = (size_t)n * n * sizeof(double);
  p.off_info = take(16);
  p.off_w = take(nn);
  p.off_r1 = take(nn);
  p.off_ri1 = take(nn);
  p.off_r2 = take(nn);
  p.off_ri2 = take(nn);
  p.off_p = take(nn);
  p.off_uimg = take(upper_image_bytes(n));
  // the Gram's partials (FP64 or FP32 input alike)
  const size_t gws = n <= kWideMaxN ? plan_gram_wide(m, n).partial_bytes : plan_syrk(m, n).partial_bytes;
  const size_t rws = cholinv_rec_workspace(n);
  const size_t uws = n <= kWideMaxN ? 0 : upper_seg_partial_bytes(n);  // R = R2 R1's partial tiles
  size_t sws = gws > rws ? gws : rws;
  sws = sws > uws ? sws : uws;
  p.off_scratch = take(sws);
  p.off_q1 = take((size_t)m * n * (mixed ? sizeof(float) : sizeof(double)));
  if (depth > 0) {
    Block blk[256];
    const int nb = inverse_blocks(n, depth, blk, 256);
    int64_t wmax = 0;
    for (int i = 0; i < nb; ++i) wmax = blk[i].c1 - blk[i].c0 > wmax ? blk[i].c1 - blk[i].c0 : wmax;
    p.off_t = take((size_t)m * wmax * sizeof(double));
  }
  p.total = off;
  return p;
}

// Y = X R^{-1} with R^{-1} kept as inverted diagonal blocks (the partial
// inverse): for each block b in order, Y(:, b) = (X(:, b) - Y(:, <b) R(<b, b))
// R^{-1}_bb -- the copy, one GEMM and one triangular multiply per block.
static hipError_t block_solve(const double* X, int64_t ldx, int64_t m, int64_t n, double* Y, int64_t ldy,
                              const double* R, const double* Rinv, int depth, double* Uimg, double* T,
                              const int32_t* info, hipStream_t s) {
  Block blk[256];
  const int nb = inverse_blocks(n, depth, blk, 256);
  for (int i = 0; i < nb; ++i) {
    const int64_t c0 = blk[i].c0, b = blk[i].c1 - blk[i].c0;
    CQR2_HIP(launch_upper_image(Rinv + c0 + c0 * n, n, (int)b, Uimg, s));
    if (c0 == 0) {
      CQR2_HIP(launch_tall_gemm(0, X, m, (int)b, ldx, Uimg, Y, ldy, info, s));
      continue;
    }
    CQR2_HIP(hipMemcpy2DAsync(T, m * sizeof(double), X + c0 * ldx, ldx * sizeof(double), m * sizeof(double), b,
                              hipMemcpyDeviceToDevice, s));
    CQR2_HIP(launch_gemm(0, 0, m, b, c0, -1.0, Y, ldy, R + c0 * n, n, 1.0, T, m, 0, 1, nullptr, info, s));
    CQR2_HIP(launch_tall_gemm(0, T, m, (int)b, m, Uimg, Y + c0 * ldy, ldy, info, s));
  }
  return hipSuccess;
}

hipError_t factor_general(const double* A, int64_t m, int64_t n, int64_t lda, double* Q, int64_t ldq, double* R,
                          int64_t ldr, char* ws, const GeneralPlan& p, bool mixed, int32_t* d_info, hipStream_t s,
                          const TimerHook& th, bool shifted, int depth) {
  int32_t* info = (int32_t*)(ws + p.off_info);
  double* W = (double*)(ws + p.off_w);
  double* R1 = (double*)(ws + p.off_r1);
  double* Ri1 = (double*)(ws + p.off_ri1);
  double* R2 = (double*)(ws + p.off_r2);
  double* Ri2 = (double*)(ws + p.off_ri2);
  double* P = (double*)(ws + p.off_p);
  double* Uimg = (double*)(ws + p.off_uimg);
  char* scratch = ws + p.off_scratch;
  void* Q1 = ws + p.off_q1;
  const int q1f = mixed ? 1 : 0;  // element type of the stored Q1
  // n <= 256: tall-skinny kernels (A read once per step); above: tiled GEMMs
  const bool wide = n <= kWideMaxN;
  const WideGramPlan wp = plan_gram_wide(m, n);
  const SyrkPlan sp = wide ? SyrkPlan{} : plan_syrk(m, n);
  CQR2_HIP(launch_set_info(info, 0, s));
  // pass 1: CQR(A) -> Q1 (workspace), R1
  th.begin(0, s);
  if (wide)
    CQR2_HIP(launch_gram_wide(wp, 0, A, m, (int)n, lda, (double*)scratch, W, n, info, s));
  else
    CQR2_HIP(launch_syrk(sp, 0, A, m, (int)n, lda, (double*)scratch, W, n, info, s));
  th.end(0, s);
  if (shifted) CQR2_HIP(launch_shift_diag(W, n, n, m, info, s));
  th.begin(2, s);
  CQR2_HIP(cholinv_recursive(W, n, n, R1, n, Ri1, n, scratch, info, 0, s, depth));
  th.end(2, s);
  th.begin(3, s);
  if (depth > 0) {
    CQR2_HIP(block_solve(A, lda, m, n, (double*)Q1, m, R1, Ri1, depth, Uimg, (double*)(ws + p.off_t), info, s));
  } else {
    // the tall kernel reads R^{-1} as its zero-padded row-major image
    CQR2_HIP(launch_upper_image(Ri1, n, (int)n, Uimg, s));
    if (mixed)
      CQR2_HIP(launch_tall_gemm_f32(A, m, (int)n, lda, Uimg, (float*)Q1, m, info, s));
    else
      CQR2_HIP(launch_tall_gemm(0, A, m, (int)n, lda, Uimg, (double*)Q1, m, info, s));
  }
  th.end(3, s);
  // pass 2: CQR(Q1) -> Q, R2, on the stored Q1 values (FP32 ones widen exactly)
  th.begin(0, s);
  if (wide)
    CQR2_HIP(launch_gram_wide(wp, q1f, Q1, m, (int)n, m, (double*)scratch, W, n, info, s));
  else
    CQR2_HIP(launch_syrk(sp, q1f, Q1, m, (int)n, m, (double*)scratch, W, n, info, s));
  th.end(0, s);
  th.begin(2, s);
  CQR2_HIP(cholinv_recursive(W, n, n, R2, n, Ri2, n, scratch, info, (int)n, s, depth));
  th.end(2, s);
  th.begin(4, s);
  if (depth > 0) {
    CQR2_HIP(block_solve((const double*)Q1, m, m, n, Q, ldq, R2, Ri2, depth, Uimg, (double*)(ws + p.off_t), info, s));
  } else {
    CQR2_HIP(launch_upper_image(Ri2, n, (int)n, Uimg, s));
    CQR2_HIP(launch_tall_gemm(q1f, Q1, m, (int)n, m, Uimg, Q, ldq, info, s));
  }
  th.end(4, s);
  // Z = X Y for n x n upper X (zero below its diagonal) and upper Y (read
  // from its upper triangle only), Z's upper triangle: n <= 256 one wave per
  // 16 x 16 tile (Z exactly upper; Y's 16 x 16 diagonal blocks read, zero
  // below), n > 256 the segmented tall kernel on Y's upper image (Z's tiles
  // wholly below the diagonal not written)
  auto upper_times_upper = [&](const double* X, const double* Y, double* Z) -> hipError_t {
    if (wide) return launch_chain_nn<true, true, false>(X, n, Y, n, n, n, n, 1.0, Z, n, info, s);
    CQR2_HIP(launch_upper_image(Y, n, (int)n, Uimg, s));
    return launch_upper_seg(X, (int)n, n, Uimg, Z, n, (double*)scratch, info, s);
  };
  if (!shifted) {
    // R = R2 R1
    th.begin(5, s);
    CQR2_HIP(upper_times_upper(R2, R1, P));
    CQR2_HIP(launch_finalize_r(P, n, R, ldr, n, info, d_info, s));
    th.end(5, s);
    return hipSuccess;
  }
  // shifted CholeskyQR3: a third pass on Q, then R = R3 (R2 R1)
  CQR2_HIP(upper_times_upper(R2, R1, P));
  th.begin(0, s);
  if (wide)
    CQR2_HIP(launch_gram_wide(wp, 0, Q, m, (int)n, ldq, (double*)scratch, W, n, info, s));
  else
    CQR2_HIP(launch_syrk(sp, 0, Q, m, (int)n, ldq, (double*)scratch, W, n, info, s));
  th.end(0, s);
  th.begin(2, s);
  CQR2_HIP(cholinv_recursive(W, n, n, R1, n, Ri1, n, scratch, info, 2 * (int)n, s));  // R3, R3^-1
  th.end(2, s);
  th.begin(4, s);
  CQR2_HIP(launch_upper_image(Ri1, n, (int)n, Uimg, s));
  if (wide) {  // in place: with one column tile each workgroup reads only the rows it writes
    CQR2_HIP(launch_tall_gemm(0, Q, m, (int)n, ldq, Uimg, Q, ldq, info, s));
  } else {     // several column tiles read a row block across tiles: multiply into Q1, copy back
    CQR2_HIP(launch_tall_gemm(0, Q, m, (int)n, ldq, Uimg, (double*)Q1, m, info, s));
    CQR2_HIP(hipMemcpy2DAsync(Q, ldq * sizeof(double), Q1, m * sizeof(double), m * sizeof(double), n,
                              hipMemcpyDeviceToDevice, s));
  }
  th.end(4, s);
  th.begin(5, s);
  CQR2_HIP(upper_times_upper(R1, P, W));
  CQR2_HIP(launch_finalize_r(W, n, R, ldr, n, info, d_info, s));
  th.end(5, s);
  return hipSuccess;
}

// ---- least squares on a finished factorization --------------------------------
// The use of QR named in the paper's introduction: X = argmin ||A X - B|| is
// R^{-1} Qᵀ B, with R^{-1} = R1^{-1} R2^{-1} from the two passes' inverses.
namespace {
size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// X = NaN after a breakdown (the products skip their work then).
__global__ void k_nan_if_info(double* X, int64_t ldx, int64_t rows, int64_t cols, const int32_t* info) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols || *info == 0) return;
  X[(e % rows) + (e / rows) * ldx] = __builtin_nan("");
}
}  // namespace

size_t lstsq_tail_bytes(int64_t m, int64_t n, int64_t nrhs) {
  const size_t cb = align256((size_t)n * nrhs * sizeof(double));
  const int splits = gemm_pick_splits(n, nrhs, m, kPlanCUs);
  return 2 * cb + align256(gemm_workspace_bytes(n, nrhs, splits));
}

hipError_t lstsq_tail(const double* Q, int64_t ldq, const double* B, int64_t ldb, int64_t m, int64_t n,
                      int64_t nrhs, const double* U1, const double* U2, int64_t ldu, int utrans, double* X,
                      int64_t ldx, char* work, const int32_t* info, hipStream_t s) {
  const size_t cb = align256((size_t)n * nrhs * sizeof(double));
  double* C = (double*)work;
  double* T = (double*)(work + cb);
  double* part = (double*)(work + 2 * cb);
  const int splits = gemm_pick_splits(n, nrhs, m, kPlanCUs);
  // C = Qᵀ B (split over the m rows, fixed-order reduction)
  hipError_t e = launch_gemm(1, 0, n, nrhs, m, 1.0, Q, ldq, B, ldb, 0.0, C, n, 0, splits, part, info, s);
  if (e != hipSuccess) return e;
  // T = R2^{-1} C, X = R1^{-1} T
  e = launch_gemm(utrans, 0, n, nrhs, n, 1.0, U2, ldu, C, n, 0.0, T, n, GEMM_A_UPPER, 1, nullptr, info, s);
  if (e != hipSuccess) return e;
  e = launch_gemm(utrans, 0, n, nrhs, n, 1.0, U1, ldu, T, n, 0.0, X, ldx, GEMM_A_UPPER, 1, nullptr, info, s);
  if (e != hipSuccess) return e;
  const int64_t total = n * nrhs;
  hipLaunchKernelGGL(k_nan_if_info, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, X, ldx, n, nrhs, info);
  return hipGetLastError();
}

}  // namespace cqr2
