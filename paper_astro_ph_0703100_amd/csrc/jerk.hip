// Launch of the force-jerk-potential pipeline on FP32 inputs and the FP64 finalize of
// its partial sums (shared by every force-jerk path).
#include "jerk_pipeline.h"

namespace nbody {
namespace {

// One thread per (particle, output): fixed-order sums as in the force finalize (the
// partials hold no j == i term; with include_self phi gets -m_i / eps in FP64).
// Grid: (ceil(n / 256), 7 outputs, or 6 without potentials).
template <int MODE, int BATCH>
__global__ __launch_bounds__(256) void jerk_finalize_kernel(JerkFinalizeArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= a.n) return;
    double r = engine::sum_partial_output<7, MODE, BATCH>(a.part, a.nseg, (size_t)a.npad, i, c);
    const size_t n = (size_t)a.n;
    if (c == 6) {
        if (a.include_self) r -= (double)a.m[i] / (double)a.eps;
        a.pot[i] = r;
    } else if (c < 3) {
        a.acc[c * n + i] = r;
    } else {
        a.jerk[(c - 3) * n + i] = r;
    }
}

}  // namespace

nbody_status launch_jerk(const TileCfg &cfg, int precision, bool with_pot, const JerkArgs &a,
                         hipStream_t s) {
    auto fn = engine::pick_tile<GravityJerk>(cfg.ipl, cfg.jt, precision, with_pot);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no jerk kernel for this ipl/jtile/precision");
    if (cfg.itiles <= 0 || cfg.nseg <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fn, dim3(cfg.itiles, cfg.nseg), dim3(kTPB), 0, s, a);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}


template <int MODE>
void launch_jerk_finalize_mode(dim3 grid, bool deep, const JerkFinalizeArgs &a, hipStream_t s) {
    if (deep)
        hipLaunchKernelGGL((jerk_finalize_kernel<MODE, 8>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((jerk_finalize_kernel<MODE, 1>), grid, dim3(256), 0, s, a);
}


nbody_status launch_jerk_finalize(int precision, const JerkFinalizeArgs &a, hipStream_t s) {
    if (a.n <= 0) return NBODY_OK;
    const int outputs = a.pot ? 7 : 6;
    const dim3 grid((a.n + 255) / 256, outputs);
    const bool deep = engine::finalize_batch(a.n, outputs) > 1;
    switch (precision) {
        case NBODY_PLAIN: launch_jerk_finalize_mode<NBODY_PLAIN>(grid, deep, a, s); break;
        case NBODY_FP64RED: launch_jerk_finalize_mode<NBODY_FP64RED>(grid, deep, a, s); break;
        case NBODY_COMP: launch_jerk_finalize_mode<NBODY_COMP>(grid, deep, a, s); break;
        default: return set_error(NBODY_EINVAL, "unknown precision mode");
    }
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
