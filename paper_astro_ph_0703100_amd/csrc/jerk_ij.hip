// Launch of the force-jerk-potential pipeline with separate i- and j-sets (its own
// translation unit, so the kernel sets compile in parallel).
#include "jerk_pipeline.h"

namespace nbody {

nbody_status launch_jerk_ij(const TileCfg &cfg, int precision, bool with_pot, const JerkIJArgs &a,
                            hipStream_t s) {
    auto fn = engine::pick_tile<GravityJerkIJ>(cfg.ipl, cfg.jt, precision, with_pot);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no separate-set jerk kernel for this shape");
    if (cfg.itiles <= 0 || cfg.nseg <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fn, dim3(cfg.itiles, cfg.nseg), dim3(kTPB), 0, s, a);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
