// Uneven batches in one persistent launch (TorchRadon's batch processing, Sec. 4.1,
// extended to jobs of different image sizes and angle sets).
//
// The host groups the images of all jobs that share a geometry into image groups
// (for the forward one 16-byte chunk per lane: 4 images, FP32 values or 16-bit tap
// pairs; 8, 16 or 32 for the backprojection, the narrowest that holds the images left)
// and flattens them into
// work units -- forward: (geometry, plan item, image group); backprojection:
// (geometry, pixel tile, image group) -- sorted longest first.
// A grid sized to the resident capacity of the GPU pulls units from a device
// counter (the only atomic) until the list is exhausted; each unit runs the same
// per-item device function as the per-call kernels, so results are identical to a
// per-call run of the same arithmetic (bitwise, except that the 16-bit forward takes
// tap pairs along the image's x here, while the per-call kernels take single taps or
// pairs along the item's transverse axis).
#include "radon_batched.hpp"
#include "radon_tiles.hpp"

namespace radon {

__global__ void batch_counter_reset(int *counter) {
    if (blockIdx.x == 0 && threadIdx.x == 0) counter[0] = 0;
}

// Next work unit for the whole block (thread 0 takes it from the counter).
__device__ __forceinline__ int next_unit(int *counter, int *slot) {
    __syncthreads();                     // everyone is done with the previous unit and slot
    if (threadIdx.x == 0) *slot = atomicAdd(counter, 1);
    __syncthreads();
    return *slot;
}

template <typename T, int BC>
__device__ __forceinline__ ImageSet<T, BC> group_images(const ImageGroup &grp) {
    ImageSet<T, BC> s;
#pragma unroll
    for (int e = 0; e < BC; ++e) {
        s.in[e] = (const T *)grp.in[e];
        s.out[e] = (T *)grp.out[e];
        s.scale[e] = grp.scale[e];
    }
    s.count = min(grp.count, BC);
    return s;
}

// Both persistent kernels are compiled for one more resident block per compute unit
// than their unbounded register counts allow (forward: 6 waves per SIMD, <= 80
// registers, BF16 needs 87 unbounded; backprojection: 4 waves, <= 128 registers
// against 151-164, one spilled in 16-bit storage): 6% faster on 200 uneven jobs.
template <typename T>
__global__ __launch_bounds__(kFwdThreads, 6) void fwd_batched(const BatchJob *__restrict__ jobs,
                                                   const ImageGroup *__restrict__ groups,
                                                   const WorkUnit *__restrict__ work, int n_work,
                                                   int *counter) {
    extern __shared__ uint4 lds[];
    __shared__ int slot;
    for (;;) {
        const int w = next_unit(counter, &slot);
        if (w >= n_work) break;
        const WorkUnit u = work[w];
        const BatchJob &j = jobs[u.job];
        const FwdItem it = j.items[u.unit];
        // one 16-byte chunk per lane, four images (FP32 values, or 16-bit tap pairs): one
        // LDS plane per slab keeps several blocks resident per CU even for the widest
        // job's tile (two FP32 chunks per lane for geometries with more than four images
        // measured 7% slower over the 200-job batch)
        constexpr int BC = 4;
        const ImageSet<T, BC> imgs = group_images<T, BC>(groups[u.group]);
        if constexpr (sizeof(T) == 2) {
            const PairPointerSource<T> src{imgs.in, j.g.n};
            fwd_item<T, BC>(j.g, it, j.ranges, imgs, src, j.tile_t, lds);
        } else {
            const PointerSource<T, BC> src{imgs.in, j.g.n};
            fwd_item<T, BC>(j.g, it, j.ranges, imgs, src, j.tile_t, lds);
        }
    }
}

template <typename T, int BC>
__device__ __forceinline__ void bp_unit(const BatchJob &j, const WorkUnit &u,
                                        const ImageGroup &grp, uint4 *lds) {
    const ImageSet<T, BC> imgs = group_images<T, BC>(grp);
    const SinoPointerSource<T, BC> src{imgs.in, j.g.det_count};
    if (!j.g.fan)
        bp_tile_par<T, BC, 3, 3, kBpAngles>(j.g, u.unit, imgs, src, j.window, lds);
    else if (j.bins <= 4)
        bp_tile_fan<T, BC, 4, 3, kBpAnglesFan>(j.g, u.unit, imgs, src, j.window, lds);
    else
        bp_tile_fan<T, BC, 6, 3, kBpAnglesFan>(j.g, u.unit, imgs, src, j.window, lds);
}

template <typename T>
__global__ __launch_bounds__(256, 4) void bp_batched(const BatchJob *__restrict__ jobs,
                                                  const ImageGroup *__restrict__ groups,
                                                  const WorkUnit *__restrict__ work, int n_work,
                                                  int *counter) {
    extern __shared__ uint4 lds[];
    __shared__ int slot;
    for (;;) {
        const int w = next_unit(counter, &slot);
        if (w >= n_work) break;
        const WorkUnit u = work[w];
        if (u.wide == 1)
            bp_unit<T, kBatchBpWide>(jobs[u.job], u, groups[u.group], lds);
        else if (u.wide == 2)
            bp_unit<T, kBatchBpMid>(jobs[u.job], u, groups[u.group], lds);
        else
            bp_unit<T, kBatchBpNarrow>(jobs[u.job], u, groups[u.group], lds);
    }
}

template <typename T>
static hipError_t launch_batched_t(int direction, const BatchLaunch &L, hipStream_t s) {
    hipLaunchKernelGGL(batch_counter_reset, dim3(1), dim3(64), 0, s, L.counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (direction == 0)
        hipLaunchKernelGGL((fwd_batched<T>), dim3(L.grid), dim3(kFwdThreads), L.lds, s, L.jobs, L.groups,
                           L.work, L.n_work, L.counter);
    else
        hipLaunchKernelGGL((bp_batched<T>), dim3(L.grid), dim3(256), L.lds, s, L.jobs, L.groups,
                           L.work, L.n_work, L.counter);
    return hipGetLastError();
}

hipError_t launch_batched(int direction, int dtype, const BatchLaunch &L, hipStream_t s) {
    switch (dtype) {
    case F32: return launch_batched_t<float>(direction, L, s);
    case F16: return launch_batched_t<__half>(direction, L, s);
    case BF16: return launch_batched_t<bf16_t>(direction, L, s);
    default: return hipErrorInvalidValue;
    }
}

int batched_blocks_per_cu(int direction, int dtype, size_t lds) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (dtype * 2 + direction) {
    case F32 * 2 + 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fwd_batched<float>, kFwdThreads, lds); break;
    case F32 * 2 + 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bp_batched<float>, 256, lds); break;
    case F16 * 2 + 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fwd_batched<__half>, kFwdThreads, lds); break;
    case F16 * 2 + 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bp_batched<__half>, 256, lds); break;
    case BF16 * 2 + 0: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fwd_batched<bf16_t>, kFwdThreads, lds); break;
    case BF16 * 2 + 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, bp_batched<bf16_t>, 256, lds); break;
    default: break;
    }
    return (e == hipSuccess && nb > 0) ? nb : 1;
}

}  // namespace radon
