// Host-only check of the workspace-cache policy (ws_cache.h) with a stand-in
// device: a lease keeps the buffer alive until it is dropped, growing waits
// for the device before freeing, and each device has its own buffer.
// Prints "ok" and exits 0, or names the failed check and exits 1.
#include "ws_cache.h"

#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

namespace {

std::mutex g_log_mu;
std::vector<std::string> g_log;
std::atomic<int> g_in_use{0};
std::atomic<bool> g_freed_in_use{false};
thread_local int t_dev = 0;

void record(const std::string& e) {
  std::lock_guard<std::mutex> g(g_log_mu);
  g_log.push_back(e);
}

struct StubDev {
  static bool device(int* d) {
    *d = t_dev;
    return true;
  }
  static bool sync() {
    record("sync");
    return true;
  }
  static bool alloc(void** p, size_t bytes) {
    *p = std::malloc(bytes);
    record("alloc " + std::to_string(bytes));
    return *p != nullptr;
  }
  static void release(void* p) {
    if (g_in_use.load() != 0) g_freed_in_use = true;
    record("free");
    std::free(p);
  }
};

int fail(const char* what) {
  std::printf("FAILED: %s\n", what);
  return 1;
}

}  // namespace

int main() {
  cqr2::WorkspaceCache<StubDev> cache;
  // sequential: reuse, growth order, minimum size, one buffer per device
  void* p1;
  {
    auto l = cache.acquire(100, 256);
    if (!l.ok || l.ptr == nullptr) return fail("first acquire");
    p1 = l.ptr;
  }
  {
    auto l = cache.acquire(200, 256);
    if (l.ptr != p1) return fail("a smaller request reuses the buffer");
  }
  {
    auto l = cache.acquire(4096, 256);
    if (!l.ok) return fail("growth");
  }
  const std::vector<std::string> want = {"alloc 256", "sync", "free", "alloc 4096"};
  if (g_log != want) return fail("growth waits for the device, then frees, then allocates");
  t_dev = 1;
  {
    auto l = cache.acquire(64, 256);
    if (g_log.size() != 5 || g_log[4] != "alloc 256") return fail("a second device gets its own buffer");
  }
  t_dev = 0;

  // threads: a request that grows the buffer waits until the lease that uses it is dropped
  std::atomic<bool> a_holds{false};
  std::atomic<long> a_released_at{0}, b_acquired_at{0};
  auto now_us = [] {
    return (long)std::chrono::duration_cast<std::chrono::microseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
  };
  std::thread a([&] {
    auto l = cache.acquire(4096, 256);
    g_in_use++;
    a_holds = true;
    std::this_thread::sleep_for(std::chrono::milliseconds(100));
    std::memset(l.ptr, 0x5a, 4096);  // still valid: nobody may free it now
    g_in_use--;
    a_released_at = now_us();
  });
  while (!a_holds) std::this_thread::yield();
  std::thread b([&] {
    auto l = cache.acquire(1 << 20, 256);
    b_acquired_at = now_us();
    std::memset(l.ptr, 0, 1 << 20);
  });
  a.join();
  b.join();
  if (g_freed_in_use) return fail("a buffer was freed while a lease used it");
  if (b_acquired_at.load() < a_released_at.load()) return fail("the growing request did not wait for the lease");
  std::printf("ok\n");
  return 0;
}
