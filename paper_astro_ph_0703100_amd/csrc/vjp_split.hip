// Adjoint of one force evaluation on the split engine: dL/dx and dL/dm of every particle
// with its j-range spread over lanes of a wavefront, summed across the lanes in FP64,
// in one launch.
#include "adjoint_pipeline.h"
#include "outputs.h"
#include "split_engine.h"

namespace nbody {

nbody_status launch_vjp_split(const TileCfg &cfg, int precision, const VjpArgs &a, bool with_mass,
                              const VjpFinalizeArgs &f, hipStream_t s) {
    auto fn = split::pick_split<Adjoint, VjpOut>(cfg.ipl, cfg.jl, cfg.jt, precision, with_mass);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no split-engine adjoint kernel for this shape");
    if (cfg.itiles <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fn, dim3(cfg.itiles), dim3(kTPB), 0, s, a, f);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
