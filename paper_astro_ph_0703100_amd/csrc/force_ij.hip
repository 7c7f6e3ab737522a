// Pair kernel with separate i- and j-sets (the paper's library interface, Sec. 3.1):
// the GravityIJ pipeline on the tile engine.  The FP64 reduction is the single-set
// finalize with the self-term removal switched off.
#include "gravity.h"
#include "nbody_internal.h"

namespace nbody {

nbody_status launch_pair_ij(const TileCfg &cfg, int precision, bool with_pot, const IJPairArgs &a,
                            hipStream_t s) {
    auto fn = engine::pick_tile<GravityIJ>(cfg.ipl, cfg.jt, precision, with_pot);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no pair kernel for this ipl/jtile/precision");
    if (cfg.itiles <= 0 || cfg.nseg <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fn, dim3(cfg.itiles, cfg.nseg), dim3(kTPB), 0, s, a);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
