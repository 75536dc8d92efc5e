// Wave- and workgroup-level waits shared by the streaming kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace cqr2 {

// Workgroup barrier that waits only for this wave's LDS operations -- not for
// its outstanding global memory operations, which the caller waits for by
// count -- and that the compiler does not move memory accesses across.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// s_waitcnt limiting only the vector-memory counter to N (0 <= N < 64):
// every vector memory operation of this wave except the last N issued has
// completed.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt field");
  __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

// The same with a wave-uniform count known only at run time (0 <= n <= 32).
__device__ __forceinline__ void wait_vmcnt_dyn(int n) {
  switch (n) {
#define CQR2_W(k) \
  case k: wait_vmcnt<k>(); break;
    CQR2_W(0) CQR2_W(1) CQR2_W(2) CQR2_W(3) CQR2_W(4) CQR2_W(5) CQR2_W(6) CQR2_W(7) CQR2_W(8)
    CQR2_W(9) CQR2_W(10) CQR2_W(11) CQR2_W(12) CQR2_W(13) CQR2_W(14) CQR2_W(15) CQR2_W(16)
    CQR2_W(17) CQR2_W(18) CQR2_W(19) CQR2_W(20) CQR2_W(21) CQR2_W(22) CQR2_W(23) CQR2_W(24)
    CQR2_W(25) CQR2_W(26) CQR2_W(27) CQR2_W(28) CQR2_W(29) CQR2_W(30) CQR2_W(31) CQR2_W(32)
#undef CQR2_W
    default: wait_vmcnt<0>(); break;
  }
}

// The same as a compiler fence: no memory access is moved across the wait
// (a store moved behind it would make the count wait for too little).
template <int N>
__device__ __forceinline__ void wait_vmcnt_fence() {
  static_assert(N >= 0 && N < 64, "vmcnt field");
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

__device__ __forceinline__ void wait_vmcnt_fenced(int n) {
  switch (n) {
#define CQR2_W(k) \
  case k: wait_vmcnt_fence<k>(); break;
    CQR2_W(0) CQR2_W(1) CQR2_W(2) CQR2_W(3) CQR2_W(4) CQR2_W(5) CQR2_W(6) CQR2_W(7) CQR2_W(8)
    CQR2_W(9) CQR2_W(10) CQR2_W(11) CQR2_W(12) CQR2_W(13) CQR2_W(14) CQR2_W(15) CQR2_W(16)
    CQR2_W(17) CQR2_W(18) CQR2_W(19) CQR2_W(20) CQR2_W(21) CQR2_W(22) CQR2_W(23) CQR2_W(24)
    CQR2_W(25) CQR2_W(26) CQR2_W(27) CQR2_W(28) CQR2_W(29) CQR2_W(30) CQR2_W(31) CQR2_W(32)
#undef CQR2_W
    default: wait_vmcnt_fence<0>(); break;
  }
}

}  // namespace cqr2
