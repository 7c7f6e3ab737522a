// Launch of the force-jerk-potential pipeline on FP64 state relative to per-i-tile
// centres (its own translation unit, so the kernel sets compile in parallel).
#include "jerk_pipeline.h"

namespace nbody {

nbody_status launch_jerk_tile(const TileCfg &cfg, int precision, bool with_pot,
                              const JerkTileArgs &a, hipStream_t s) {
    auto fn = engine::pick_tile<GravityJerkTile>(cfg.ipl, cfg.jt, precision, with_pot);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no tile-centre jerk kernel for this shape");
    if (cfg.itiles <= 0 || cfg.nseg <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fn, dim3(cfg.itiles, cfg.nseg), dim3(kTPB), 0, s, a);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
