// Asynchronous 16-byte copies from global memory into LDS (global_load_lds_dwordx4).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace radon {

// Lane i's 16 bytes at `src` land at the wave-uniform LDS address `wave_dst` + 16 i
// (checked on the device: one wave, every lane's chunk at that slot and nowhere else).
// The copy completes on vmcnt.  It is issued from inline asm so that the compiler adds
// no waits for it: it cannot tell which LDS buffer the copy writes and would otherwise
// wait for the copy before every later LDS read.  No memory clobber either: that would
// keep the compiler from reading read-only tables with scalar loads, whose waits would
// then cover the copies too.  Ordering is the caller's: the destination is neither
// read nor written between the issue and a wait for vmcnt(0) followed by a barrier
// (volatile asm and barriers keep their order), and the last reads of its previous
// contents precede an earlier barrier.  vmcnt counts in issue order, so the compiler's
// own waits for later loads stay correct (they may only wait longer).
__device__ __forceinline__ void lds_copy16_async(const uint4 *src, uint4 *wave_dst) {
    const uint32_t m0 = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(__attribute__((address_space(3))) uint4 *)wave_dst);
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off" : : "s"(m0), "v"(src) : "m0");
}

}  // namespace radon
