// Library-cached device workspace: one buffer per device, grown on demand and
// shared by every entry point that takes no work argument.
//
// A caller holds a Lease, and with it the cache's lock, from the lookup until
// its launches are enqueued, so no other thread can replace the buffer in
// between.  Growing the buffer waits for the device (work enqueued earlier on
// any stream may still use the old buffer) before freeing it.
//
// Dev supplies the device calls, so the policy can be tested on the host with
// a stand-in:
//   static bool device(int* d);          current device
//   static bool sync();                  wait for all work on the device
//   static bool alloc(void** p, size_t);
//   static void release(void* p);
#pragma once
#include <cstddef>
#include <mutex>
#include <vector>

namespace cqr2 {

template <typename Dev>
class WorkspaceCache {
 public:
  struct Lease {
    std::unique_lock<std::mutex> lock;
    void* ptr = nullptr;
    bool ok = false;
  };

  // A buffer of at least `bytes` (at least `min_bytes`) on the current device.
  Lease acquire(size_t bytes, size_t min_bytes) {
    Lease l;
    l.lock = std::unique_lock<std::mutex>(mu_);
    int dev = 0;
    if (!Dev::device(&dev) || dev < 0) return l;
    if ((int)slots_.size() <= dev) slots_.resize(dev + 1);
    Slot& w = slots_[dev];
    if (bytes < min_bytes) bytes = min_bytes;
    if (w.bytes < bytes) {
      if (w.ptr != nullptr) {
        if (!Dev::sync()) return l;
        Dev::release(w.ptr);
        w.ptr = nullptr;
        w.bytes = 0;
      }
      void* p = nullptr;
      if (!Dev::alloc(&p, bytes)) return l;
      w.ptr = p;
      w.bytes = bytes;
    }
    l.ptr = w.ptr;
    l.ok = true;
    return l;
  }

 private:
  struct Slot {
    void* ptr = nullptr;
    size_t bytes = 0;
  };
  std::mutex mu_;
  std::vector<Slot> slots_;
};

}  // namespace cqr2
