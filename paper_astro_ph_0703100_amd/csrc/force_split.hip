// Force evaluation of one system on the split engine: the gravity pipeline with each
// i-particle's j-range spread over lanes of a wavefront, cross-lane FP64 sums and the
// outputs (accelerations, potentials, an optional fused kick) in one launch.
#include "gravity.h"
#include "outputs.h"
#include "split_engine.h"

namespace nbody {

nbody_status launch_pair_split(const TileCfg &cfg, int precision, bool with_pot,
                               const PairArgs &a, const FinalizeArgs &f, hipStream_t s) {
    auto fn = split::pick_split<Gravity, ForceOut>(cfg.ipl, cfg.jl, cfg.jt, precision, with_pot);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no split-engine force kernel for this shape");
    if (cfg.itiles <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fn, dim3(cfg.itiles), dim3(kTPB), 0, s, a, f);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
