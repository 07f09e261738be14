// Direct global-to-LDS loads (gfx950 global_load_lds_dwordx4) for kernels that
// stage operand tiles in a ring of LDS buffers without passing them through
// registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gls {

// LDS byte address of a __shared__ object.
__device__ __forceinline__ uint32_t lds_address(const void* p) {
  return (uint32_t)(uintptr_t)((const __attribute__((address_space(3))) char*)p);
}

// 16 bytes per lane from global memory to LDS at lds + 16 * lane (lds is
// wave-uniform).  M0 carries the LDS address; it is saved and restored around
// the load.  Issued from inline assembly so that the compiler does not drain
// these loads at every barrier: the kernel waits on vmcnt itself.
__device__ __forceinline__ void lds_load16(const void* src, uint32_t lds) {
  uint32_t keep;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %2\n\t"
      "global_load_lds_dwordx4 %1, off\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(keep)
      : "v"(src), "s"(lds)
      : "memory");
}

// The same load addressed as a wave-uniform 64-bit base (scalar registers)
// plus a 32-bit byte offset per lane, which saves two address VGPRs per load
// stream against lds_load16.
__device__ __forceinline__ void lds_load16_sv(const void* sbase, uint32_t voff, uint32_t lds) {
  uint32_t keep;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %3\n\t"
      "global_load_lds_dwordx4 %1, %2\n\t"
      "s_mov_b32 m0, %0"
      : "=&s"(keep)
      : "v"(voff), "s"(sbase), "s"(lds)
      : "memory");
}

// Wait until at most N of this wave's vector-memory loads are in flight.
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

// Wait until at most n whole stages of L loads each are in flight (n <= 3).
template <int L>
__device__ __forceinline__ void wait_stages(int n) {
  if (n <= 0) wait_vmcnt<0>();
  else if (n == 1) wait_vmcnt<L>();
  else if (n == 2) wait_vmcnt<2 * L>();
  else wait_vmcnt<3 * L>();
}

}  // namespace gls
