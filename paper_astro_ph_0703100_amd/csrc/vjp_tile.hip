// Launch of the adjoint pipeline on FP64 positions relative to per-i-tile centres (its
// own translation unit, so the two sets of kernel instantiations compile in parallel).
#include "adjoint_pipeline.h"

namespace nbody {

nbody_status launch_vjp_tile(const TileCfg &cfg, int precision, const VjpTileArgs &a,
                             bool with_mass, hipStream_t s) {
    auto fn = engine::pick_tile<AdjointTile>(cfg.ipl, cfg.jt, precision, with_mass);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no tile-centre VJP kernel for this shape");
    if (cfg.itiles <= 0 || cfg.nseg <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fn, dim3(cfg.itiles, cfg.nseg), dim3(kTPB), 0, s, a);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
