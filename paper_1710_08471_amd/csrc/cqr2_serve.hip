// Many CholeskyQR2 problems per launch: the batched entry point and the
// continuous-batching server (host side).  Both drive the multi-problem step
// kernel (cqr2_step.hip) for n <= 256 and the tiled path for larger n.  Server
// requests are QR factorizations or least-squares solves (the factorization
// followed by X = R^{-1} Qᵀ B).
//
// Task tables travel host -> device through a ring of pinned host buffers;
// a buffer is rewritten only after the copy that last read it has completed
// (its event), which bounds how far the host runs ahead of the GPU.
#include "cqr2.h"
#include "cqr2_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <vector>

namespace {

using cqr2::kStepMaxN;
constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

size_t mat_bytes(int64_t rows, int64_t cols, int64_t ld) {
  if (rows <= 0 || cols <= 0) return 0;
  return (size_t)((cols - 1) * ld + rows) * sizeof(double);
}

size_t problem_workspace(const cqr2_problem& p) {
  if (p.n <= 0) return 0;
  if (p.n <= kStepMaxN) return align_up(cqr2::step_layout(p.m, p.n).total);
  return align_up(cqr2::plan_general(p.m, p.n, false).total);
}

size_t problem_footprint(const cqr2_problem& p) {
  return mat_bytes(p.m, p.n, p.lda) + mat_bytes(p.m, p.n, p.ldq) + mat_bytes(p.n, p.n, p.ldr) +
         problem_workspace(p);
}

cqr2::StepTask make_task(const cqr2_problem& p, char* ws, int phase, int wg0) {
  cqr2::StepTask t{};
  t.A = p.A;
  t.lda = p.lda;
  t.Q = p.Q;
  t.ldq = p.ldq;
  t.R = p.R;
  t.ldr = p.ldr;
  t.user_info = p.d_info;
  t.ws = ws;
  t.m = p.m;
  t.n = (int32_t)p.n;
  t.phase = phase;
  t.wg0 = wg0;
  t.nwg = cqr2::step_workgroups(p.m, p.n, phase);
  return t;
}

// Pinned host staging ring for task tables.
class TableRing {
 public:
  explicit TableRing(int slots) : slots_(slots) {}
  ~TableRing() { release(); }
  void release() {
    for (auto& s : ring_) {
      if (s.ev) {
        (void)hipEventSynchronize(s.ev);
        (void)hipEventDestroy(s.ev);
      }
      if (s.host) (void)hipHostFree(s.host);
    }
    ring_.clear();
  }
  // Copies `bytes` from `src` to device `dst` on `s` through the next pinned
  // buffer (waiting for that buffer's previous copy first).
  hipError_t copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (ring_.empty()) ring_.resize(slots_);
    Slot& sl = ring_[next_];
    next_ = (next_ + 1) % slots_;
    if (sl.ev) {
      hipError_t e = hipEventSynchronize(sl.ev);
      if (e != hipSuccess) return e;
    } else {
      hipError_t e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
      if (e != hipSuccess) return e;
    }
    if (sl.cap < bytes) {
      if (sl.host) (void)hipHostFree(sl.host);
      sl.host = nullptr;
      sl.cap = 0;
      const size_t cap = std::max<size_t>(bytes, 64 * 1024);
      hipError_t e = hipHostMalloc(&sl.host, cap, hipHostMallocDefault);
      if (e != hipSuccess) return e;
      sl.cap = cap;
    }
    std::memcpy(sl.host, src, bytes);
    hipError_t e = hipMemcpyAsync(dst, sl.host, bytes, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return e;
    return hipEventRecord(sl.ev, s);
  }

 private:
  struct Slot {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
  };
  int slots_;
  int next_ = 0;
  std::vector<Slot> ring_;
};

std::mutex g_batched_mu;
TableRing* g_batched_ring = nullptr;

int to_code(hipError_t e) { return e == hipSuccess ? 0 : CQR2_ERR_HIP; }

// First-fit allocator over [0, size) with coalescing frees (offsets 256-aligned).
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
    size_ = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align_up(bytes ? bytes : kAlign);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, noff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align_up(bytes ? bytes : kAlign);
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }

 private:
  std::map<size_t, size_t> free_;
  size_t size_ = 0;
};

}  // namespace

// ---- continuous-batching server ---------------------------------------------
struct cqr2_server {
  struct Req {
    cqr2_problem p;
    int64_t tag;
    size_t ws_bytes, footprint;
    bool large;
    // least-squares requests (nrhs > 0): B (m x nrhs), X (n x nrhs); the
    // solve's workspace follows the factorization's at tail_off
    int64_t nrhs = 0, ldb = 0, ldx = 0;
    const double* B = nullptr;
    double* X = nullptr;
    size_t tail_off = 0;
  };
  struct Active {
    Req r;
    size_t ws_off;
    int phase;
  };
  struct Finishing {
    hipEvent_t ev;
    std::vector<Req> reqs;
    std::vector<size_t> offs;
  };

  // Streams for n > 256 requests: one fewer than the process's hardware
  // queues (GPU_MAX_HW_QUEUES, HIP's default 4), so that with the step stream
  // every stream has a queue of its own and the steps never wait behind a
  // large request's kernels.
  static constexpr int kMaxLargeStreams = 31;
  int n_large = 3;
  hipStream_t stream = nullptr;                 // steps
  hipStream_t large[kMaxLargeStreams] = {};     // n > 256 requests, round robin
  int large_next = 0;
  char* arena_base = nullptr;
  Arena arena;
  size_t budget = 0, in_flight_bytes = 0;
  int max_active = 0;
  std::deque<Req> queue;
  std::vector<Active> active;         // n <= 256, in phase order of admission
  int n_large_running = 0;
  std::deque<Finishing> finishing;
  std::vector<std::pair<int64_t, double>> done;
  std::vector<hipEvent_t> event_pool;
  hipEvent_t t0 = nullptr;
  // Launch pacing: a step first waits until fewer than kInFlight of its
  // earlier launches are pending on the GPU, then reaps, admits and launches.
  // The host thus stays close behind the GPU, and each launch carries every
  // request admitted up to then instead of a few requests each.
  static constexpr int kInFlight = 2;
  hipEvent_t pace[kInFlight] = {};
  bool pace_live[kInFlight] = {};
  int pace_next = 0;
  // Recorded on `stream` when a large request is admitted; the large stream
  // waits on it, so the request reads A (and B) only after everything the
  // caller enqueued on `stream` before the step that admits it.
  hipEvent_t order_ev = nullptr;
  TableRing ring{8};
  std::vector<char*> dev_tables;      // one device table per ring slot
  int dev_next = 0;
  std::vector<cqr2::StepTask> table;
  std::vector<size_t> order;

  hipEvent_t get_event() {
    if (!event_pool.empty()) {
      hipEvent_t e = event_pool.back();
      event_pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }

  // Move finished work whose events have completed to `done`; free its memory.
  // Entries complete out of order (two streams), so every entry is checked.
  int reap() {
    for (auto it = finishing.begin(); it != finishing.end();) {
      const hipError_t q = hipEventQuery(it->ev);
      if (q == hipErrorNotReady) {
        ++it;
        continue;
      }
      if (q != hipSuccess) return CQR2_ERR_HIP;
      float ms = 0.f;
      if (t0 != nullptr && hipEventElapsedTime(&ms, t0, it->ev) != hipSuccess) ms = -1.f;
      for (size_t i = 0; i < it->reqs.size(); ++i) {
        done.emplace_back(it->reqs[i].tag, (double)ms);
        arena.release(it->offs[i], it->reqs[i].ws_bytes);
        in_flight_bytes -= it->reqs[i].footprint;
        if (it->reqs[i].large) --n_large_running;
      }
      event_pool.push_back(it->ev);
      it = finishing.erase(it);
    }
    return 0;
  }

  int admit() {
    while (!queue.empty() && (int)active.size() + n_large_running < max_active) {
      Req& r = queue.front();
      if (budget && in_flight_bytes + r.footprint > budget) break;
      size_t off = 0;
      if (!arena.alloc(r.ws_bytes, &off)) break;
      in_flight_bytes += r.footprint;
      if (!r.large) {
        active.push_back({r, off, 0});
      } else {
        const cqr2_problem& p = r.p;
        const cqr2::GeneralPlan plan = cqr2::plan_general(p.m, p.n, false);
        hipStream_t ls = large[large_next];
        large_next = (large_next + 1) % n_large;
        char* ws = arena_base + off;
        if (hipEventRecord(order_ev, stream) != hipSuccess || hipStreamWaitEvent(ls, order_ev, 0) != hipSuccess)
          return CQR2_ERR_HIP;
        hipError_t e = cqr2::factor_general(p.A, p.m, p.n, p.lda, p.Q, p.ldq, p.R, p.ldr, ws, plan, false,
                                            p.d_info, ls, cqr2::TimerHook{});
        if (e != hipSuccess) return CQR2_ERR_HIP;
        if (r.nrhs > 0) {
          e = cqr2::lstsq_tail(p.Q, p.ldq, r.B, r.ldb, p.m, p.n, r.nrhs, (const double*)(ws + plan.off_ri1),
                               (const double*)(ws + plan.off_ri2), p.n, 0, r.X, r.ldx, ws + r.tail_off,
                               (const int32_t*)(ws + plan.off_info), ls);
          if (e != hipSuccess) return CQR2_ERR_HIP;
        }
        hipEvent_t ev = get_event();
        if (ev == nullptr || hipEventRecord(ev, ls) != hipSuccess) return CQR2_ERR_HIP;
        ++n_large_running;
        finishing.push_back({ev, {r}, {off}});
      }
      queue.pop_front();
    }
    return 0;
  }

  int step() {
    if (pace_live[pace_next]) {
      if (hipEventSynchronize(pace[pace_next]) != hipSuccess) return CQR2_ERR_HIP;
      pace_live[pace_next] = false;
    }
    int rc = reap();
    if (rc) return rc;
    rc = admit();
    if (rc) return rc;
    if (active.empty()) return 0;
    // longest workgroups first, so that the launch ends on short ones
    order.resize(active.size());
    for (size_t i = 0; i < active.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) {
      return cqr2::step_wg_cost(active[x].r.p.m, active[x].r.p.n, active[x].phase) >
             cqr2::step_wg_cost(active[y].r.p.m, active[y].r.p.n, active[y].phase);
    });
    table.clear();
    int wg = 0;
    for (size_t i : order) {
      const Active& a = active[i];
      table.push_back(make_task(a.r.p, arena_base + a.ws_off, a.phase, wg));
      wg += table.back().nwg;
    }
    char* dtab = dev_tables[dev_next];
    dev_next = (dev_next + 1) % (int)dev_tables.size();
    const size_t tb = table.size() * sizeof(cqr2::StepTask);
    rc = to_code(ring.copy(dtab, table.data(), tb, stream));
    if (rc) return rc;
    rc = to_code(cqr2::launch_step((const cqr2::StepTask*)dtab, (int)table.size(), wg, stream));
    if (rc) return rc;
    // least-squares requests whose factorization this step completes: the solve
    for (const Active& a : active) {
      if (a.phase != cqr2::step_phases(a.r.p.n) - 1 || a.r.nrhs == 0) continue;
      const cqr2_problem& p = a.r.p;
      const cqr2::StepLayout L = cqr2::step_layout(p.m, p.n);
      char* ws = arena_base + a.ws_off;
      rc = to_code(cqr2::lstsq_tail(p.Q, p.ldq, a.r.B, a.r.ldb, p.m, p.n, a.r.nrhs, (const double*)(ws + L.off_u1),
                                    (const double*)(ws + L.off_u2), L.np, 1, a.r.X, a.r.ldx, ws + a.r.tail_off,
                                    (const int32_t*)(ws + L.off_info), stream));
      if (rc) return rc;
    }
    if (hipEventRecord(pace[pace_next], stream) != hipSuccess) return CQR2_ERR_HIP;
    pace_live[pace_next] = true;
    pace_next = (pace_next + 1) % kInFlight;
    hipEvent_t ev = get_event();
    if (ev == nullptr || hipEventRecord(ev, stream) != hipSuccess) return CQR2_ERR_HIP;
    Finishing fin{ev, {}, {}};
    std::vector<Active> still;
    still.reserve(active.size());
    for (Active& a : active) {
      if (a.phase == cqr2::step_phases(a.r.p.n) - 1) {
        fin.reqs.push_back(a.r);
        fin.offs.push_back(a.ws_off);
      } else {
        ++a.phase;
        still.push_back(a);
      }
    }
    active.swap(still);
    if (fin.reqs.empty()) {
      event_pool.push_back(ev);  // nothing waits on it; the stream order covers reuse
    } else {
      finishing.push_back(std::move(fin));
    }
    return 0;
  }
};

extern "C" {

size_t cqr2_batched_workspace_size(const cqr2_problem* probs, int32_t count, uint32_t flags) {
  if (probs == nullptr || count < 0 || flags != CQR2_FP64) return 0;
  size_t total = 0;
  int64_t ntasks = 0;
  for (int32_t i = 0; i < count; ++i) {
    if (cqr2_problem_check(&probs[i]) != 0) return 0;
    total += problem_workspace(probs[i]);
    if (probs[i].n > 0 && probs[i].n <= kStepMaxN) ntasks += cqr2::step_phases(probs[i].n);
  }
  total += align_up((size_t)ntasks * sizeof(cqr2::StepTask));
  return total ? total : kAlign;
}

int cqr2_factor_batched(const cqr2_problem* probs, int32_t count, void* work, size_t work_bytes, uint32_t flags,
                        void* stream) {
  if (count < 0) return -2;
  if (count == 0) return 0;
  if (probs == nullptr) return -1;
  if (flags != CQR2_FP64) return -5;
  for (int32_t i = 0; i < count; ++i)
    if (cqr2_problem_check(&probs[i]) != 0) return -1;
  if (work == nullptr || ((uintptr_t)work % kAlign) != 0) return -3;
  if (work_bytes < cqr2_batched_workspace_size(probs, count, flags)) return -4;
  hipStream_t s = (hipStream_t)stream;
  // layout: the task tables of every phase, then one workspace per problem
  std::vector<int32_t> small;
  int64_t ntasks = 0;
  int phases = 0;
  for (int32_t i = 0; i < count; ++i)
    if (probs[i].n > 0 && probs[i].n <= kStepMaxN) {
      small.push_back(i);
      ntasks += cqr2::step_phases(probs[i].n);
      phases = std::max(phases, cqr2::step_phases(probs[i].n));
    }
  const size_t tab_bytes = align_up((size_t)ntasks * sizeof(cqr2::StepTask));
  char* base = (char*)work;
  std::vector<size_t> off(count);
  size_t cur = tab_bytes;
  for (int32_t i = 0; i < count; ++i) {
    off[i] = cur;
    cur += problem_workspace(probs[i]);
  }
  if (!small.empty()) {
    // launch ph runs phase ph of every problem that has one
    std::vector<cqr2::StepTask> tabs;
    std::vector<int> wgs(phases, 0), first(phases, 0), count_ph(phases, 0);
    tabs.reserve(ntasks);
    for (int ph = 0; ph < phases; ++ph) {
      first[ph] = (int)tabs.size();
      for (int32_t i : small) {
        if (ph >= cqr2::step_phases(probs[i].n)) continue;
        tabs.push_back(make_task(probs[i], base + off[i], ph, wgs[ph]));
        wgs[ph] += tabs.back().nwg;
      }
      count_ph[ph] = (int)tabs.size() - first[ph];
    }
    {
      std::lock_guard<std::mutex> g(g_batched_mu);
      if (g_batched_ring == nullptr) g_batched_ring = new TableRing(4);
      const int rc = to_code(g_batched_ring->copy(base, tabs.data(), tabs.size() * sizeof(cqr2::StepTask), s));
      if (rc) return rc;
    }
    const cqr2::StepTask* dt = (const cqr2::StepTask*)base;
    for (int ph = 0; ph < phases; ++ph) {
      const int rc = to_code(cqr2::launch_step(dt + first[ph], count_ph[ph], wgs[ph], s));
      if (rc) return rc;
    }
  }
  for (int32_t i = 0; i < count; ++i) {
    const cqr2_problem& p = probs[i];
    if (p.n <= kStepMaxN) continue;
    const cqr2::GeneralPlan plan = cqr2::plan_general(p.m, p.n, false);
    const int rc = to_code(cqr2::factor_general(p.A, p.m, p.n, p.lda, p.Q, p.ldq, p.R, p.ldr, base + off[i], plan,
                                                false, p.d_info, s, cqr2::TimerHook{}));
    if (rc) return rc;
  }
  return 0;
}

int cqr2_server_create(size_t arena_bytes, size_t footprint_budget, int32_t max_active, void* stream,
                       cqr2_server** out) {
  if (out == nullptr) return -5;
  *out = nullptr;
  if (arena_bytes == 0) return -1;
  if (max_active < 1 || max_active > 4096) return -3;
  cqr2_server* sv = new cqr2_server();
  sv->stream = (hipStream_t)stream;
  sv->budget = footprint_budget;
  sv->max_active = max_active;
  arena_bytes = align_up(arena_bytes);
  auto fail = [&](int code) {
    cqr2_server_destroy(sv);
    return code;
  };
  if (hipMalloc((void**)&sv->arena_base, arena_bytes) != hipSuccess) return fail(CQR2_ERR_HIP);
  if (hipEventCreateWithFlags(&sv->order_ev, hipEventDisableTiming) != hipSuccess) return fail(CQR2_ERR_HIP);
  for (auto& e : sv->pace)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return fail(CQR2_ERR_HIP);
  sv->arena.reset(arena_bytes);
  int hw_queues = 4;  // HIP's default hardware queues per process
  if (const char* e = std::getenv("GPU_MAX_HW_QUEUES")) {
    const int v = std::atoi(e);
    if (v > 0) hw_queues = v;
  }
  sv->n_large = std::min(std::max(hw_queues - 1, 1), cqr2_server::kMaxLargeStreams);
  for (int i = 0; i < sv->n_large; ++i)
    if (hipStreamCreateWithFlags(&sv->large[i], hipStreamNonBlocking) != hipSuccess) return fail(CQR2_ERR_HIP);
  const size_t tb = align_up((size_t)max_active * sizeof(cqr2::StepTask));
  for (int i = 0; i < 8; ++i) {
    char* d = nullptr;
    if (hipMalloc((void**)&d, tb) != hipSuccess) return fail(CQR2_ERR_HIP);
    sv->dev_tables.push_back(d);
  }
  if (cqr2_server_clock(sv) != 0) return fail(CQR2_ERR_HIP);
  *out = sv;
  return 0;
}

int cqr2_server_destroy(cqr2_server* s) {
  if (s == nullptr) return -1;
  (void)hipStreamSynchronize(s->stream);
  for (auto& ls : s->large)
    if (ls) {
      (void)hipStreamSynchronize(ls);
      (void)hipStreamDestroy(ls);
    }
  s->ring.release();
  for (char* d : s->dev_tables) (void)hipFree(d);
  for (auto& f : s->finishing) (void)hipEventDestroy(f.ev);
  for (hipEvent_t e : s->event_pool) (void)hipEventDestroy(e);
  if (s->t0) (void)hipEventDestroy(s->t0);
  if (s->order_ev) (void)hipEventDestroy(s->order_ev);
  for (hipEvent_t e : s->pace)
    if (e) (void)hipEventDestroy(e);
  if (s->arena_base) (void)hipFree(s->arena_base);
  delete s;
  return 0;
}

int cqr2_server_clock(cqr2_server* s) {
  if (s == nullptr) return -1;
  if (s->t0 == nullptr && hipEventCreate(&s->t0) != hipSuccess) return CQR2_ERR_HIP;
  if (hipEventRecord(s->t0, s->stream) != hipSuccess) return CQR2_ERR_HIP;
  return hipEventSynchronize(s->t0) == hipSuccess ? 0 : CQR2_ERR_HIP;
}

int cqr2_server_submit(cqr2_server* s, const cqr2_problem* p, int64_t tag) {
  if (s == nullptr) return -1;
  if (p == nullptr || cqr2_problem_check(p) != 0) return -2;
  if (p->n == 0) return -3;
  cqr2_server::Req r{*p, tag, problem_workspace(*p), problem_footprint(*p), p->n > kStepMaxN};
  if (r.ws_bytes > s->arena.size() || (s->budget && r.footprint > s->budget)) return CQR2_ERR_TOO_LARGE;
  s->queue.push_back(r);
  return 0;
}

int cqr2_server_submit_lstsq(cqr2_server* s, const cqr2_problem* p, const double* B, int64_t ldb, int64_t nrhs,
                             double* X, int64_t ldx, int64_t tag) {
  if (s == nullptr) return -1;
  if (p == nullptr || cqr2_problem_check(p) != 0) return -2;
  if (p->n == 0) return -2;
  const int64_t m = p->m, n = p->n;
  if (nrhs < 1) return -5;
  if (ldb < (m > 1 ? m : 1)) return -4;
  if (ldx < (n > 1 ? n : 1)) return -7;
  if (B == nullptr || ((uintptr_t)B & 7u) != 0) return -3;
  if (X == nullptr || ((uintptr_t)X & 7u) != 0) return -6;
  const size_t bb = mat_bytes(m, nrhs, ldb), xb = mat_bytes(n, nrhs, ldx);
  const size_t ab = mat_bytes(m, n, p->lda), qb = mat_bytes(m, n, p->ldq), rb = mat_bytes(n, n, p->ldr);
  auto overlap = [](const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return na && nb && x < y + nb && y < x + na;
  };
  if (overlap(B, bb, p->Q, qb) || overlap(B, bb, p->R, rb)) return -3;
  if (overlap(X, xb, p->A, ab) || overlap(X, xb, p->Q, qb) || overlap(X, xb, p->R, rb) || overlap(X, xb, B, bb))
    return -6;
  const size_t fws = problem_workspace(*p);
  const size_t tail = align_up(cqr2::lstsq_tail_bytes(m, n, nrhs));
  cqr2_server::Req r{*p, tag, fws + tail, problem_footprint(*p) + bb + xb + tail, n > kStepMaxN};
  r.nrhs = nrhs;
  r.B = B;
  r.ldb = ldb;
  r.X = X;
  r.ldx = ldx;
  r.tail_off = fws;
  if (r.ws_bytes > s->arena.size() || (s->budget && r.footprint > s->budget)) return CQR2_ERR_TOO_LARGE;
  s->queue.push_back(r);
  return 0;
}

int cqr2_server_step(cqr2_server* s, int32_t* n_active, int32_t* n_queued) {
  if (s == nullptr) return -1;
  const int rc = s->step();
  if (n_active) *n_active = (int32_t)s->active.size() + s->n_large_running;
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  return rc;
}

int cqr2_server_poll(cqr2_server* s, int64_t* tags, double* done_ms, int32_t max_count, int32_t* count) {
  if (s == nullptr) return -1;
  if (max_count < 0 || (max_count > 0 && (tags == nullptr || done_ms == nullptr))) return -4;
  if (count == nullptr) return -5;
  const int rc = s->reap();
  if (rc) return rc;
  const int32_t k = std::min<int32_t>(max_count, (int32_t)s->done.size());
  for (int32_t i = 0; i < k; ++i) {
    tags[i] = s->done[i].first;
    done_ms[i] = s->done[i].second;
  }
  s->done.erase(s->done.begin(), s->done.begin() + k);
  *count = k;
  return 0;
}

}  // extern "C"
