// Host emulation of the asynchronous global -> LDS copy: the 16 bytes of lane
// (threadIdx.x % 64) land at wave_dst + lane at once (the device copy completes later,
// before the caller's vmcnt wait and barrier, so the results are the same).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace radon {

__device__ __forceinline__ void lds_copy16_async(const uint4 *src, uint4 *wave_dst) {
    wave_dst[threadIdx.x % 64] = *src;
}

}  // namespace radon
