// Tiled forward kernels of tiling 2 (kFwdTiling[2]: slab rows, angles per item).
#include "radon_fwd_tiled.hpp"

namespace radon {

hipError_t launch_forward_tiling2(const Geom &g, const FwdWork &work, int dtype, const LaunchShape &shape,
                                   const void *x, void *y, int batch, float scale_dt, void *ws,
                                   size_t ws_bytes, hipStream_t s) {
    return launch_forward_tiled<FwdCfg2>(g, work, dtype, shape, x, y, batch, scale_dt, ws, ws_bytes, s);
}

}  // namespace radon
