// Direct-to-LDS loads (global_load_lds_dwordx4) for the GEMM tiles.
//
// Each lane moves 16 bytes from global memory into LDS without passing through vector registers:
// lane i of the wave writes bytes [16 i, 16 i + 16) of a 1 KiB run whose LDS base is uniform over
// the wave (register M0), so which element a lane fetches fixes the LDS layout.  The load is issued
// from inline assembly: with the compiler's builtin every later LDS read waits for all such loads
// in flight (s_waitcnt vmcnt(0)), which serialises a prefetch pipeline.  The callers therefore
// place their own waits (s_waitcnt vmcnt(n) before a workgroup barrier) -- the compiler does not
// count these loads.
#pragma once
#include <hip/hip_runtime.h>

namespace fc {

typedef __attribute__((address_space(3))) void* lds_ptr_t;

// 16 bytes per lane from src into LDS bytes [lds + 16 lane, lds + 16 lane + 16); lds uniform.
// No register receives data, so nothing the compiler allocates is written late; M0 is restored.
__device__ __forceinline__ void lds_dma16(const void* src, const void* lds) {
  const unsigned dst = (unsigned)(unsigned long)(lds_ptr_t)(lds);
  unsigned saved;
  asm volatile(
      "s_mov_b32 %0, m0\n\t"
      "s_mov_b32 m0, %1\n\t"
      "s_nop 0\n\t"
      "global_load_lds_dwordx4 %2, off\n\t"
      "s_mov_b32 m0, %0\n\t"
      "s_nop 0"
      : "=&s"(saved)
      : "s"(__builtin_amdgcn_readfirstlane(dst)), "v"(src)
      : "memory");
}

}  // namespace fc
