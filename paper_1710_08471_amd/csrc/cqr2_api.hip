// C ABI of libcqr2.so: argument checks, workspace planning and the
// stream-ordered launch sequence of CholeskyQR2 (Algorithm 5 = two passes of
// Algorithm 4, then R = R2 R1).  All checks run on the host before any HIP
// call, so invalid arguments never launch anything.
#include "cqr2.h"
#include "cqr2_internal.h"
#include "ws_cache.h"

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

namespace {

using cqr2::GramPlan;

constexpr size_t kAlign = 256;
constexpr int64_t kSmallN = 128;  // tall-skinny kernels: Gram, CholInv and Q = A R^-1 up to this n

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Byte ranges [p, p + bytes) overlap?
bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  if (a == nullptr || b == nullptr || abytes == 0 || bbytes == 0) return false;
  const uintptr_t x0 = (uintptr_t)a, x1 = x0 + abytes;
  const uintptr_t y0 = (uintptr_t)b, y1 = y0 + bbytes;
  return x0 < y1 && y0 < x1;
}

size_t matrix_bytes(int64_t rows, int64_t cols, int64_t ld) {
  if (rows <= 0 || cols <= 0) return 0;
  return (size_t)((cols - 1) * ld + rows) * sizeof(double);
}

bool aligned8(const void* p) { return ((uintptr_t)p & 7u) == 0; }

int device_cus() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return 256;
  return cus;
}

// Workspace layout of one factorization with n <= 128.  For 64 < n <= 128
// (padded order 128) the MFMA 16x16x4 streaming kernels run (s16), with pass
// 2's Gram fused into pass 1's Q = A R1^-1.
struct SmallLayout {
  GramPlan gram;
  cqr2::Stream16Plan s16p;
  bool s16 = false;
  int np = 0;
  size_t off_info = 0, off_part = 0, off_w = 0, off_u1 = 0, off_u2 = 0, off_r1 = 0, off_r2 = 0;
  size_t total = 0;
};

SmallLayout make_small_layout(int64_t m, int64_t n) {
  SmallLayout L;
  L.gram = cqr2::plan_gram(m, n);
  L.np = cqr2::padded_order(n);
  L.s16 = L.np == 128;
  if (L.s16) L.s16p = cqr2::plan_stream16(m);
  size_t off = 0;
  L.off_info = off; off += align_up(sizeof(int32_t) * 4);
  L.off_part = off; off += align_up(L.s16 ? L.s16p.partial_bytes : L.gram.partial_bytes);
  L.off_w = off;    off += align_up((size_t)n * n * sizeof(double));
  L.off_u1 = off;   off += align_up((size_t)L.np * L.np * sizeof(double));
  L.off_u2 = off;   off += align_up((size_t)L.np * L.np * sizeof(double));
  L.off_r1 = off;   off += align_up((size_t)n * n * sizeof(double));
  L.off_r2 = off;   off += align_up((size_t)n * n * sizeof(double));
  L.total = off;
  return L;
}

// FP64 factorizations with n <= 128 run the tall-skinny kernels; everything
// else (n > 128, and the mixed-precision form at any n) runs the tiled path.
// flags: the form in the low byte, the inverse depth above it
uint32_t flag_form(uint32_t flags) { return flags & 0xffu; }
int flag_depth(uint32_t flags) { return (int)(flags >> 8); }

bool use_small(int64_t n, uint32_t flags) {
  // (the recursion behind the inverse depth has no level at n <= 128)
  return n <= kSmallN && (flag_form(flags) == CQR2_FP64 || flag_form(flags) == CQR2_SHIFTED_CQR3);
}

bool valid_flags(uint32_t flags) {
  const uint32_t f = flag_form(flags);
  const int d = flag_depth(flags);
  if (f != CQR2_FP64 && f != CQR2_MIXED_P1_FP32 && f != CQR2_SHIFTED_CQR3) return false;
  return d >= 0 && d <= CQR2_MAX_INVERSE_DEPTH && (d == 0 || f == CQR2_FP64);
}

size_t factor_workspace(int64_t m, int64_t n, uint32_t flags) {
  return use_small(n, flags) ? make_small_layout(m, n).total
                             : cqr2::plan_general(m, n, flag_form(flags) == CQR2_MIXED_P1_FP32,
                                                  flag_depth(flags)).total;
}

// ---- timing instrumentation -------------------------------------------------
struct Timer {
  bool enabled = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  struct Rec { int cls; hipEvent_t a, b; };
  std::vector<Rec> recs;
  hipEvent_t open[CQR2_NUM_TIMERS] = {};
};
Timer g_timer;
std::mutex g_timer_mu;

hipEvent_t timer_event() {
  if (g_timer.used == g_timer.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_timer.pool.push_back(e);
  }
  return g_timer.pool[g_timer.used++];
}

void timer_begin(int cls, hipStream_t s) {
  if (!g_timer.enabled || cls < 0 || cls >= CQR2_NUM_TIMERS) return;
  std::lock_guard<std::mutex> g(g_timer_mu);
  hipEvent_t a = timer_event();
  if (a && hipEventRecord(a, s) == hipSuccess) g_timer.open[cls] = a;
}

void timer_end(int cls, hipStream_t s) {
  if (!g_timer.enabled || cls < 0 || cls >= CQR2_NUM_TIMERS) return;
  std::lock_guard<std::mutex> g(g_timer_mu);
  hipEvent_t a = g_timer.open[cls];
  if (a == nullptr) return;
  g_timer.open[cls] = nullptr;
  hipEvent_t b = timer_event();
  if (b == nullptr || hipEventRecord(b, s) != hipSuccess) return;
  g_timer.recs.push_back({cls, a, b});
}

cqr2::TimerHook timer_hook() {
  cqr2::TimerHook h;
  if (g_timer.enabled) {
    h.b = timer_begin;
    h.e = timer_end;
  }
  return h;
}

// ---- library-cached workspace for the entry points without a work argument --
// One buffer per device, shared by cqr2_factor, cqr2_cholinv (n > 128),
// cqr2_apply_rinv (n > 128) and cqr2_apply_rinv_f32 (ws_cache.h: the lease
// keeps the lock until the launches are enqueued; growing waits for the
// device before the old buffer is freed).
struct HipDev {
  static bool device(int* d) { return hipGetDevice(d) == hipSuccess; }
  static bool sync() { return hipDeviceSynchronize() == hipSuccess; }
  static bool alloc(void** p, size_t bytes) { return hipMalloc(p, bytes) == hipSuccess; }
  static void release(void* p) { (void)hipFree(p); }
};
cqr2::WorkspaceCache<HipDev> g_ws_cache;

struct WsLease {
  std::unique_lock<std::mutex> lock;
  void* ptr = nullptr;
  int err = 0;
};

WsLease cached_workspace(size_t bytes) {
  auto c = g_ws_cache.acquire(bytes, kAlign);
  WsLease l;
  l.lock = std::move(c.lock);
  l.ptr = c.ptr;
  l.err = c.ok ? 0 : CQR2_ERR_HIP;
  return l;
}

int check_hip(hipError_t e) { return e == hipSuccess ? 0 : CQR2_ERR_HIP; }

#define CQR2_TRY(expr)            \
  do {                            \
    int _rc = check_hip((expr));  \
    if (_rc != 0) return _rc;     \
  } while (0)

// The enqueued CholeskyQR2 sequence for n <= 128; arguments already validated.
int run_small(const double* A, int64_t m, int64_t n, int64_t lda, double* Q, int64_t ldq, double* R, int64_t ldr,
              char* ws, const SmallLayout& L, int32_t* d_info, hipStream_t s, int cus, bool shifted,
              const cqr2::TimerHook& th) {
  int32_t* info = (int32_t*)(ws + L.off_info);
  double* part = (double*)(ws + L.off_part);
  double* W = (double*)(ws + L.off_w);
  double* U1 = (double*)(ws + L.off_u1);
  double* U2 = (double*)(ws + L.off_u2);
  double* R1 = (double*)(ws + L.off_r1);
  double* R2 = (double*)(ws + L.off_r2);
  const int ni = (int)n;
  auto reduce = [&]() -> hipError_t {
    return L.s16 ? cqr2::launch_stream16_reduce(L.s16p, part, ni, W, n, info, s)
                 : cqr2::launch_gram_reduce(L.gram, part, ni, W, n, info, s);
  };
  auto cholinv = [&](double* Rk, double* Uk, int info_offset) -> int {
    th.begin(1, s); CQR2_TRY(reduce()); th.end(1, s);
    if (shifted && info_offset == 0) CQR2_TRY(cqr2::launch_shift_diag(W, n, n, m, info, s));
    th.begin(2, s); CQR2_TRY(cqr2::launch_cholinv(W, n, ni, Rk, n, nullptr, 0, Uk, L.np, info, info_offset, s));
    th.end(2, s);
    return 0;
  };
  constexpr int kUp = cqr2::GEMM_A_UPPER | cqr2::GEMM_B_UPPER | cqr2::GEMM_C_UPPER;
  if (L.s16) {
    // ---- pass 1: Gram of A (clears the info word), CholInv; Q1 = A U1 with
    //      the Gram of the stored Q1 (pass 2's first step) in the same launch ----
    th.begin(0, s); CQR2_TRY(cqr2::launch_stream16_gram(L.s16p, A, m, ni, lda, part, nullptr, s, info)); th.end(0, s);
    if (const int rc = cholinv(R1, U1, 0)) return rc;
    th.begin(3, s);
    CQR2_TRY(cqr2::launch_stream16_apply_gram(L.s16p, A, m, ni, lda, U1, Q, ldq, part, info, s));
    th.end(3, s);
    // ---- pass 2: CholInv of Q1's Gram, Q = Q1 U2 in place ----
    if (const int rc = cholinv(R2, U2, ni)) return rc;
    if (!shifted) {
      th.begin(4, s); CQR2_TRY(cqr2::launch_stream16_apply(L.s16p, Q, m, ni, ldq, U2, Q, ldq, info, s)); th.end(4, s);
      th.begin(5, s);
      CQR2_TRY(cqr2::launch_upper_product_final(R2, R1, n, R, ldr, info, d_info, s));
      th.end(5, s);
      return 0;
    }
    // ---- shifted CholeskyQR3: pass 2's Q with the Gram of the third pass ----
    th.begin(4, s);
    CQR2_TRY(cqr2::launch_stream16_apply_gram(L.s16p, Q, m, ni, ldq, U2, Q, ldq, part, info, s));
    th.end(4, s);
    CQR2_TRY(cqr2::launch_gemm(0, 0, n, n, n, 1.0, R2, n, R1, n, 0.0, R, ldr, kUp, 1, nullptr, info, s));
    th.begin(1, s); CQR2_TRY(reduce()); th.end(1, s);
    th.begin(2, s); CQR2_TRY(cqr2::launch_cholinv(W, n, ni, R2, n, nullptr, 0, U1, L.np, info, 2 * ni, s)); th.end(2, s);
    th.begin(4, s); CQR2_TRY(cqr2::launch_stream16_apply(L.s16p, Q, m, ni, ldq, U1, Q, ldq, info, s)); th.end(4, s);
    th.begin(5, s);
    CQR2_TRY(cqr2::launch_gemm(0, 0, n, n, n, 1.0, R2, n, R, ldr, 0.0, W, n, kUp, 1, nullptr, info, s));
    CQR2_TRY(cqr2::launch_finalize_r(W, n, R, ldr, n, info, d_info, s));
    th.end(5, s);
    return 0;
  }
  // ---- pass 1: CQR(A); the first Gram clears the info word ----
  th.begin(0, s);
  CQR2_TRY(cqr2::launch_gram_partials(L.gram, A, m, ni, lda, part, nullptr, s, info));
  th.end(0, s);
  if (const int rc = cholinv(R1, U1, 0)) return rc;
  th.begin(3, s); CQR2_TRY(cqr2::launch_apply_rinv(A, m, ni, lda, U1, L.np, 1, Q, ldq, info, cus, s)); th.end(3, s);
  // ---- pass 2: CQR(Q1), in place ----
  th.begin(0, s); CQR2_TRY(cqr2::launch_gram_partials(L.gram, Q, m, ni, ldq, part, info, s)); th.end(0, s);
  if (const int rc = cholinv(R2, U2, ni)) return rc;
  th.begin(4, s); CQR2_TRY(cqr2::launch_apply_rinv(Q, m, ni, ldq, U2, L.np, 1, Q, ldq, info, cus, s)); th.end(4, s);
  if (!shifted) {
    // ---- R = R2 R1 ----
    th.begin(5, s);
    CQR2_TRY(cqr2::launch_upper_product_final(R2, R1, n, R, ldr, info, d_info, s));
    th.end(5, s);
    return 0;
  }
  // ---- shifted CholeskyQR3: R2 R1 held in the caller's R, a third pass on Q ----
  CQR2_TRY(cqr2::launch_gemm(0, 0, n, n, n, 1.0, R2, n, R1, n, 0.0, R, ldr, kUp, 1, nullptr, info, s));
  th.begin(0, s); CQR2_TRY(cqr2::launch_gram_partials(L.gram, Q, m, ni, ldq, part, info, s)); th.end(0, s);
  th.begin(1, s); CQR2_TRY(reduce()); th.end(1, s);
  th.begin(2, s); CQR2_TRY(cqr2::launch_cholinv(W, n, ni, R2, n, nullptr, 0, U1, L.np, info, 2 * ni, s)); th.end(2, s);
  th.begin(4, s); CQR2_TRY(cqr2::launch_apply_rinv(Q, m, ni, ldq, U1, L.np, 1, Q, ldq, info, cus, s)); th.end(4, s);
  th.begin(5, s);
  CQR2_TRY(cqr2::launch_gemm(0, 0, n, n, n, 1.0, R2, n, R, ldr, 0.0, W, n, kUp, 1, nullptr, info, s));
  CQR2_TRY(cqr2::launch_finalize_r(W, n, R, ldr, n, info, d_info, s));
  th.end(5, s);
  return 0;
}

int run_factor(const double* A, int64_t m, int64_t n, int64_t lda, double* Q, int64_t ldq, double* R, int64_t ldr,
               char* ws, int32_t* d_info, uint32_t flags, hipStream_t s, bool timed = true) {
  const bool shifted = flag_form(flags) == CQR2_SHIFTED_CQR3;
  const cqr2::TimerHook th = timed ? timer_hook() : cqr2::TimerHook{};
  if (use_small(n, flags))
    return run_small(A, m, n, lda, Q, ldq, R, ldr, ws, make_small_layout(m, n), d_info, s, device_cus(), shifted, th);
  const bool mixed = flag_form(flags) == CQR2_MIXED_P1_FP32;
  const int depth = flag_depth(flags);
  const cqr2::GeneralPlan p = cqr2::plan_general(m, n, mixed, depth);
  return check_hip(cqr2::factor_general(A, m, n, lda, Q, ldq, R, ldr, ws, p, mixed, d_info, s, th, shifted, depth));
}

// ---- static scratch of the no-allocation entry point -------------------------
// One array per device (each device holds its own copy of the code object's
// globals), kept until the process ends.  Host code never uses the array's
// name as an address: the device address is looked up once per device and
// kept in g_scratch_ptr.
static __device__ __align__(256) char scratch[CQR2_NOALLOC_MAX_WORKSPACE];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call made with that device current).
int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return CQR2_ERR_HIP;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) return CQR2_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

}  // namespace

// ---- least squares ------------------------------------------------------------
namespace {
struct LstsqLayout {
  size_t off_tail = 0, total = 0;
};

LstsqLayout lstsq_layout(int64_t m, int64_t n, int64_t nrhs) {
  LstsqLayout L;
  L.off_tail = align_up(factor_workspace(m, n, CQR2_FP64));
  L.total = L.off_tail + align_up(cqr2::lstsq_tail_bytes(m, n, nrhs));
  return L;
}
}  // namespace

extern "C" {

const char* cqr2_version(void) { return "cqr2-mi355x 0.2 (gfx950)"; }

const char* cqr2_status_string(int code) {
  switch (code) {
    case 0: return "success";
    case CQR2_ERR_HIP: return "HIP runtime error";
    case CQR2_ERR_UNSUPPORTED: return "unsupported problem size";
    case CQR2_ERR_TOO_LARGE: return "request can never fit the server's arena or footprint budget";
    case CQR2_ERR_NOALLOC_LIMIT: return "problem needs more workspace than the no-allocation scratch holds";
    default: break;
  }
  if (code < 0 && code > -20) return "invalid argument (see the argument index = -code)";
  return "unknown status";
}

size_t cqr2_workspace_size(int64_t m, int64_t n, uint32_t flags) {
  if (m < n || n < 1 || !valid_flags(flags) || n > CQR2_MAX_N) return 0;
  return factor_workspace(m, n, flags);
}

int cqr2_factor_ex(const double* A, int64_t m, int64_t n, int64_t lda, double* Q, int64_t ldq, double* R,
                   int64_t ldr, void* work, size_t work_bytes, int32_t* d_info, uint32_t flags,
                   void* stream) {
  // -- host argument checks (LAPACK-style negative argument index) --
  if (n < 0) return -3;
  if (m < n) return -2;
  if (lda < (m > 1 ? m : 1)) return -4;
  if (ldq < (m > 1 ? m : 1)) return -6;
  if (ldr < (n > 1 ? n : 1)) return -8;
  if (!valid_flags(flags)) return -12;
  if (n == 0) return 0;
  if (A == nullptr || !aligned8(A)) return -1;
  if (Q == nullptr || !aligned8(Q)) return -5;
  if (R == nullptr || !aligned8(R)) return -7;
  if (n > CQR2_MAX_N) return CQR2_ERR_UNSUPPORTED;
  const size_t abytes = matrix_bytes(m, n, lda), qbytes = matrix_bytes(m, n, ldq), rbytes = matrix_bytes(n, n, ldr);
  if (overlaps(A, abytes, Q, qbytes)) return -5;
  if (overlaps(A, abytes, R, rbytes)) return -7;
  if (overlaps(Q, qbytes, R, rbytes)) return -7;
  const size_t need = factor_workspace(m, n, flags);
  if (work == nullptr || ((uintptr_t)work % kAlign) != 0) return -9;
  if (work_bytes < need) return -10;
  if (overlaps(work, work_bytes, A, abytes) || overlaps(work, work_bytes, Q, qbytes) ||
      overlaps(work, work_bytes, R, rbytes))
    return -9;
  if (d_info != nullptr && ((uintptr_t)d_info & 3u) != 0) return -11;
  return run_factor(A, m, n, lda, Q, ldq, R, ldr, (char*)work, d_info, flags, (hipStream_t)stream);
}

int cqr2_problem_check(const cqr2_problem* p) {
  if (p == nullptr) return -1;
  const int64_t m = p->m, n = p->n;
  if (n < 0) return -3;
  if (m < n) return -2;
  if (p->lda < (m > 1 ? m : 1)) return -4;
  if (p->ldq < (m > 1 ? m : 1)) return -6;
  if (p->ldr < (n > 1 ? n : 1)) return -8;
  if (p->d_info != nullptr && ((uintptr_t)p->d_info & 3u) != 0) return -11;
  if (n == 0) return 0;
  if (p->A == nullptr || !aligned8(p->A)) return -1;
  if (p->Q == nullptr || !aligned8(p->Q)) return -5;
  if (p->R == nullptr || !aligned8(p->R)) return -7;
  if (n > CQR2_MAX_N) return CQR2_ERR_UNSUPPORTED;
  const size_t ab = matrix_bytes(m, n, p->lda), qb = matrix_bytes(m, n, p->ldq), rb = matrix_bytes(n, n, p->ldr);
  if (overlaps(p->A, ab, p->Q, qb)) return -5;
  if (overlaps(p->A, ab, p->R, rb) || overlaps(p->Q, qb, p->R, rb)) return -7;
  return 0;
}

int cqr2_factor(const double* A, int64_t m, int64_t n, int64_t lda, double* Q, double* R, void* stream) {
  if (n < 0) return -3;
  if (m < n) return -2;
  if (lda < (m > 1 ? m : 1)) return -4;
  if (n == 0) return 0;
  if (A == nullptr || !aligned8(A)) return -1;
  if (Q == nullptr || !aligned8(Q)) return -5;
  if (R == nullptr || !aligned8(R)) return -6;
  if (n > CQR2_MAX_N) return CQR2_ERR_UNSUPPORTED;
  const size_t abytes = matrix_bytes(m, n, lda), rbytes = matrix_bytes(n, n, n);
  if (overlaps(A, abytes, Q, abytes)) return -5;
  if (overlaps(A, abytes, R, rbytes) || overlaps(Q, abytes, R, rbytes)) return -6;
  WsLease ws = cached_workspace(factor_workspace(m, n, CQR2_FP64));
  if (ws.err) return ws.err;
  return run_factor(A, m, n, lda, Q, lda, R, n, (char*)ws.ptr, nullptr, CQR2_FP64, (hipStream_t)stream);
}

int cqr2_factor_noalloc(const double* A, int64_t m, int64_t n, int64_t lda, double* Q, double* R, void* stream) {
  if (n < 0) return -3;
  if (m < n) return -2;
  if (lda < (m > 1 ? m : 1)) return -4;
  if (n == 0) return 0;
  if (A == nullptr || !aligned8(A)) return -1;
  if (Q == nullptr || !aligned8(Q)) return -5;
  if (R == nullptr || !aligned8(R)) return -6;
  if (n > CQR2_MAX_N) return CQR2_ERR_UNSUPPORTED;
  const size_t abytes = matrix_bytes(m, n, lda), rbytes = matrix_bytes(n, n, n);
  if (overlaps(A, abytes, Q, abytes)) return -5;
  if (overlaps(A, abytes, R, rbytes) || overlaps(Q, abytes, R, rbytes)) return -6;
  if (factor_workspace(m, n, CQR2_FP64) > CQR2_NOALLOC_MAX_WORKSPACE) return CQR2_ERR_NOALLOC_LIMIT;
  void* ws = nullptr;
  if (const int rc = scratch_address(&ws)) return rc;
  // the first Gram launch clears the info word; every other workspace block
  // is written before it is read, so the previous call's contents never leak
  return run_factor(A, m, n, lda, Q, lda, R, n, (char*)ws, nullptr, CQR2_FP64, (hipStream_t)stream, false);
}

size_t cqr2_lstsq_workspace_size(int64_t m, int64_t n, int64_t nrhs) {
  if (m < n || n < 1 || nrhs < 1 || n > CQR2_MAX_N) return 0;
  return lstsq_layout(m, n, nrhs).total;
}

int cqr2_lstsq(const double* A, int64_t m, int64_t n, int64_t lda, const double* B, int64_t ldb, int64_t nrhs,
               double* X, int64_t ldx, double* Q, int64_t ldq, double* R, int64_t ldr, void* work, size_t work_bytes,
               int32_t* d_info, void* stream) {
  if (n < 0) return -3;
  if (m < n) return -2;
  if (lda < (m > 1 ? m : 1)) return -4;
  if (ldb < (m > 1 ? m : 1)) return -6;
  if (nrhs < 0) return -7;
  if (ldx < (n > 1 ? n : 1)) return -9;
  if (ldq < (m > 1 ? m : 1)) return -11;
  if (ldr < (n > 1 ? n : 1)) return -13;
  if (n == 0) return 0;
  if (A == nullptr || !aligned8(A)) return -1;
  if (nrhs > 0 && (B == nullptr || !aligned8(B))) return -5;
  if (nrhs > 0 && (X == nullptr || !aligned8(X))) return -8;
  if (Q == nullptr || !aligned8(Q)) return -10;
  if (R == nullptr || !aligned8(R)) return -12;
  if (d_info != nullptr && ((uintptr_t)d_info & 3u) != 0) return -16;
  if (n > CQR2_MAX_N) return CQR2_ERR_UNSUPPORTED;
  const size_t ab = matrix_bytes(m, n, lda), bb = matrix_bytes(m, nrhs, ldb), xb = matrix_bytes(n, nrhs, ldx);
  const size_t qb = matrix_bytes(m, n, ldq), rb = matrix_bytes(n, n, ldr);
  if (overlaps(X, xb, A, ab) || overlaps(X, xb, B, bb)) return -8;
  if (overlaps(Q, qb, A, ab) || overlaps(Q, qb, B, bb) || overlaps(Q, qb, X, xb)) return -10;
  if (overlaps(R, rb, A, ab) || overlaps(R, rb, B, bb) || overlaps(R, rb, X, xb) || overlaps(R, rb, Q, qb))
    return -12;
  const LstsqLayout L = lstsq_layout(m, n, nrhs > 0 ? nrhs : 1);
  if (work == nullptr || ((uintptr_t)work % kAlign) != 0) return -14;
  if (work_bytes < L.total) return -15;
  if (overlaps(work, work_bytes, A, ab) || overlaps(work, work_bytes, B, bb) || overlaps(work, work_bytes, X, xb) ||
      overlaps(work, work_bytes, Q, qb) || overlaps(work, work_bytes, R, rb))
    return -14;
  hipStream_t s = (hipStream_t)stream;
  char* ws = (char*)work;
  const int rc = run_factor(A, m, n, lda, Q, ldq, R, ldr, ws, d_info, CQR2_FP64, s);
  if (rc != 0 || nrhs == 0) return rc;
  const int32_t* info = (const int32_t*)ws;  // both layouts keep the info word first
  char* tail = ws + L.off_tail;
  if (use_small(n, CQR2_FP64)) {
    // row-major U images: U[i np + k] = R^{-1}(i, k), i.e. op(U) = Uᵀ of a column-major np x np view
    const SmallLayout SL = make_small_layout(m, n);
    return check_hip(cqr2::lstsq_tail(Q, ldq, B, ldb, m, n, nrhs, (const double*)(ws + SL.off_u1),
                                      (const double*)(ws + SL.off_u2), SL.np, 1, X, ldx, tail, info, s));
  }
  const cqr2::GeneralPlan p = cqr2::plan_general(m, n, false);
  return check_hip(cqr2::lstsq_tail(Q, ldq, B, ldb, m, n, nrhs, (const double*)(ws + p.off_ri1),
                                    (const double*)(ws + p.off_ri2), n, 0, X, ldx, tail, info, s));
}

size_t cqr2_gram_workspace_size(int64_t m, int64_t n) {
  if (m < 0 || n < 1 || n > CQR2_MAX_N) return 0;
  if (n <= kSmallN) return align_up(cqr2::plan_gram(m, n).partial_bytes);
  if (n <= cqr2::kWideMaxN) return align_up(cqr2::plan_gram_wide(m, n).partial_bytes);
  return align_up(cqr2::plan_syrk(m, n).partial_bytes);
}

int cqr2_gram(const double* A, int64_t m, int64_t n, int64_t lda, double* W, int64_t ldw, void* work,
              size_t work_bytes, void* stream) {
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (lda < (m > 1 ? m : 1)) return -4;
  if (ldw < (n > 1 ? n : 1)) return -6;
  if (n == 0) return 0;
  if ((m > 0 && A == nullptr) || !aligned8(A)) return -1;  // A is not read when m == 0
  if (W == nullptr || !aligned8(W)) return -5;
  if (n > CQR2_MAX_N) return CQR2_ERR_UNSUPPORTED;
  const size_t need = cqr2_gram_workspace_size(m, n);
  if (work == nullptr || ((uintptr_t)work & 7u) != 0) return -7;
  if (work_bytes < need) return -8;
  const size_t abytes = matrix_bytes(m, n, lda), wbytes = matrix_bytes(n, n, ldw);
  if (overlaps(A, abytes, W, wbytes)) return -5;
  if (overlaps(work, work_bytes, A, abytes) || overlaps(work, work_bytes, W, wbytes)) return -7;
  hipStream_t s = (hipStream_t)stream;
  if (n <= kSmallN) {
    // m == 0 runs one workgroup over a fully masked stage and yields W = 0.
    const GramPlan p = cqr2::plan_gram(m, n);
    CQR2_TRY(cqr2::launch_gram_partials(p, A, m, (int)n, lda, (double*)work, nullptr, s));
    CQR2_TRY(cqr2::launch_gram_reduce(p, (const double*)work, (int)n, W, ldw, nullptr, s));
    return 0;
  }
  if (n <= cqr2::kWideMaxN) {
    CQR2_TRY(cqr2::launch_gram_wide(cqr2::plan_gram_wide(m, n), 0, A, m, (int)n, lda, (double*)work, W, ldw, nullptr,
                                    s));
    CQR2_TRY(cqr2::launch_mirror_lower(W, ldw, n, s));
    return 0;
  }
  // n > 256: lower triangle by 128 x 128 tiles, then mirrored.
  CQR2_TRY(cqr2::launch_syrk(cqr2::plan_syrk(m, n), 0, A, m, (int)n, lda, (double*)work, W, ldw, nullptr, s));
  CQR2_TRY(cqr2::launch_mirror_lower(W, ldw, n, s));
  return 0;
}

int cqr2_cholinv(const double* W, int64_t n, int64_t ldw, double* R, double* Rinv, int64_t ldr, int32_t* d_info,
                 void* stream) {
  if (n < 0) return -2;
  if (ldw < (n > 1 ? n : 1)) return -3;
  if (ldr < (n > 1 ? n : 1)) return -6;
  if (n == 0) return 0;
  if (W == nullptr || !aligned8(W)) return -1;
  if (R == nullptr || !aligned8(R)) return -4;
  if (Rinv == nullptr || !aligned8(Rinv)) return -5;
  if (d_info != nullptr && ((uintptr_t)d_info & 3u) != 0) return -7;
  if (n > CQR2_MAX_N) return CQR2_ERR_UNSUPPORTED;
  const size_t wb = matrix_bytes(n, n, ldw), rb = matrix_bytes(n, n, ldr);
  if (overlaps(W, wb, R, rb)) return -4;
  if (overlaps(W, wb, Rinv, rb) || overlaps(R, rb, Rinv, rb)) return -5;
  hipStream_t s = (hipStream_t)stream;
  if (n <= kSmallN) {
    if (d_info != nullptr) CQR2_TRY(cqr2::launch_set_info(d_info, 0, s));
    CQR2_TRY(cqr2::launch_cholinv(W, ldw, (int)n, R, ldr, Rinv, ldr, nullptr, 0, d_info, 0, s));
    return 0;
  }
  // The recursion overwrites the trailing blocks of its input: work on a
  // copy in the library workspace (info word, W copy, recursion scratch).
  const size_t wcopy = align_up((size_t)n * n * sizeof(double));
  WsLease lease = cached_workspace(kAlign + wcopy + cqr2::cholinv_rec_workspace(n));
  if (lease.err) return lease.err;
  char* ws = (char*)lease.ptr;
  int32_t* info = d_info != nullptr ? d_info : (int32_t*)ws;
  double* Wc = (double*)(ws + kAlign);
  CQR2_TRY(cqr2::launch_set_info(info, 0, s));
  CQR2_TRY(hipMemcpy2DAsync(Wc, n * sizeof(double), W, ldw * sizeof(double), n * sizeof(double), n,
                            hipMemcpyDeviceToDevice, s));
  CQR2_TRY(cqr2::cholinv_recursive(Wc, n, n, R, ldr, Rinv, ldr, ws + kAlign + wcopy, info, 0, s));
  // after a breakdown the products that follow it skip their work: R and Rinv
  // become NaN above the diagonal (as the one-workgroup kernel writes them)
  CQR2_TRY(cqr2::launch_nan_upper_if_info(R, ldr, n, info, s));
  CQR2_TRY(cqr2::launch_nan_upper_if_info(Rinv, ldr, n, info, s));
  return 0;
}

int cqr2_apply_rinv(const double* A, int64_t m, int64_t n, int64_t lda, const double* U, int64_t ldu, double* Q,
                    int64_t ldq, void* stream) {
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (lda < (m > 1 ? m : 1)) return -4;
  if (ldu < (n > 1 ? n : 1)) return -6;
  if (ldq < (m > 1 ? m : 1)) return -8;
  if (n == 0 || m == 0) return 0;
  if (A == nullptr || !aligned8(A)) return -1;
  if (U == nullptr || !aligned8(U)) return -5;
  if (Q == nullptr || !aligned8(Q)) return -7;
  if (n > CQR2_MAX_N) return CQR2_ERR_UNSUPPORTED;
  const size_t ab = matrix_bytes(m, n, lda), qb = matrix_bytes(m, n, ldq), ub = matrix_bytes(n, n, ldu);
  const bool in_place = (A == Q);
  if (in_place && lda != ldq) return -8;
  if (!in_place && overlaps(A, ab, Q, qb)) return -7;
  if (overlaps(U, ub, Q, qb)) return -5;
  hipStream_t s = (hipStream_t)stream;
  if (n <= kSmallN) {
    CQR2_TRY(cqr2::launch_apply_rinv(A, m, (int)n, lda, U, 1, ldu, Q, ldq, nullptr, device_cus(), s));
    return 0;
  }
  // the tall kernel reads U as its zero-padded row-major image; with several
  // 256-column tiles (n > 256) a row block is read across tiles, so an
  // in-place product multiplies from a copy of A
  const bool copy_a = in_place && n > cqr2::kWideMaxN;
  const size_t img = align_up(cqr2::upper_image_bytes(n));
  WsLease lease = cached_workspace(img + (copy_a ? (size_t)m * n * sizeof(double) : 0));
  if (lease.err) return lease.err;
  char* ws = (char*)lease.ptr;
  double* ut = (double*)ws;
  CQR2_TRY(cqr2::launch_upper_image(U, ldu, (int)n, ut, s));
  const double* src = A;
  int64_t lds = lda;
  if (copy_a) {
    double* tmp = (double*)(ws + img);
    CQR2_TRY(hipMemcpy2DAsync(tmp, m * sizeof(double), A, lda * sizeof(double), m * sizeof(double), n,
                              hipMemcpyDeviceToDevice, s));
    src = tmp;
    lds = m;
  }
  CQR2_TRY(cqr2::launch_tall_gemm(0, src, m, (int)n, lds, ut, Q, ldq, nullptr, s));
  return 0;
}

int cqr2_apply_rinv_f32(const double* A, int64_t m, int64_t n, int64_t lda, const double* U, int64_t ldu,
                        float* Q, int64_t ldq, void* stream) {
  if (m < 0) return -2;
  if (n < 0) return -3;
  if (lda < (m > 1 ? m : 1)) return -4;
  if (ldu < (n > 1 ? n : 1)) return -6;
  if (ldq < (m > 1 ? m : 1)) return -8;
  if (n == 0 || m == 0) return 0;
  if (A == nullptr || !aligned8(A)) return -1;
  if (U == nullptr || !aligned8(U)) return -5;
  if (Q == nullptr || ((uintptr_t)Q & 3u) != 0) return -7;
  if (n > CQR2_MAX_N) return CQR2_ERR_UNSUPPORTED;
  const size_t ab = matrix_bytes(m, n, lda), ub = matrix_bytes(n, n, ldu);
  const size_t qb = (size_t)((n - 1) * ldq + m) * sizeof(float);
  if (overlaps(A, ab, Q, qb)) return -7;
  if (overlaps(U, ub, Q, qb)) return -7;
  hipStream_t s = (hipStream_t)stream;
  WsLease lease = cached_workspace(align_up(cqr2::upper_image_bytes(n)));
  if (lease.err) return lease.err;
  double* ut = (double*)lease.ptr;
  CQR2_TRY(cqr2::launch_upper_image(U, ldu, (int)n, ut, s));
  CQR2_TRY(cqr2::launch_tall_gemm_f32(A, m, (int)n, lda, ut, Q, ldq, nullptr, s));
  return 0;
}

int cqr2_upper_product(const double* R2, const double* R1, double* R, int64_t n, int64_t ld, void* stream) {
  if (n < 0) return -4;
  if (ld < (n > 1 ? n : 1)) return -5;
  if (n == 0) return 0;
  if (R2 == nullptr || !aligned8(R2)) return -1;
  if (R1 == nullptr || !aligned8(R1)) return -2;
  if (R == nullptr || !aligned8(R)) return -3;
  const size_t b = matrix_bytes(n, n, ld);
  if (overlaps(R, b, R2, b) || overlaps(R, b, R1, b)) return -3;
  hipStream_t s = (hipStream_t)stream;
  CQR2_TRY(cqr2::launch_gemm(0, 0, n, n, n, 1.0, R2, ld, R1, ld, 0.0, R, ld,
                             cqr2::GEMM_A_UPPER | cqr2::GEMM_B_UPPER | cqr2::GEMM_C_UPPER, 1, nullptr, nullptr, s));
  CQR2_TRY(cqr2::launch_finalize_r(R, ld, R, ld, n, nullptr, nullptr, s));
  return 0;
}

int cqr2_timing_enable(int enable) {
  std::lock_guard<std::mutex> g(g_timer_mu);
  g_timer.enabled = enable != 0;
  return 0;
}

int cqr2_timing_reset(void) {
  std::lock_guard<std::mutex> g(g_timer_mu);
  g_timer.recs.clear();
  g_timer.used = 0;
  for (auto& o : g_timer.open) o = nullptr;
  return 0;
}

int cqr2_timing_read(double* total_ms, int64_t* launches, int max_classes) {
  std::lock_guard<std::mutex> g(g_timer_mu);
  if (total_ms == nullptr || launches == nullptr || max_classes < 0) return -1;
  for (int c = 0; c < max_classes; ++c) {
    total_ms[c] = 0.0;
    launches[c] = 0;
  }
  for (const auto& r : g_timer.recs) {
    if (hipEventSynchronize(r.b) != hipSuccess) return CQR2_ERR_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return CQR2_ERR_HIP;
    if (r.cls >= 0 && r.cls < max_classes) {
      total_ms[r.cls] += ms;
      launches[r.cls] += 1;
    }
  }
  return 0;
}

}  // extern "C"
