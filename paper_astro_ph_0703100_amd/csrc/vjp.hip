// Launch of the adjoint pipeline on FP32 positions and the FP64 finalize of its
// partial sums.
#include "adjoint_pipeline.h"
#include "outputs.h"

namespace nbody {
namespace {

// One thread per (particle, store slot), as in the force finalize: fixed-order sums of
// the segment partials (which hold no j == k term), then dL/dx_k (slots 0-2, from the
// slot's own sum and the sum B_k) or dL/dm_k (slot 3, the negated mass sum).  Grid:
// (ceil(n / 256), 4 slots, or 3 without dL/dm).
template <int MODE, int BATCH>
__global__ __launch_bounds__(256) void vjp_finalize_kernel(VjpFinalizeArgs a) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (k >= a.n) return;
    VjpOut::put(a, k, c, [&](int o) {
        return engine::sum_partial_output<kVjpOutputs, MODE, BATCH>(a.part, a.nseg,
                                                                    (size_t)a.npad, k, o);
    });
}

}  // namespace

nbody_status launch_vjp(const TileCfg &cfg, int precision, const VjpArgs &a, bool with_mass,
                        hipStream_t s) {
    auto fn = engine::pick_tile<Adjoint>(cfg.ipl, cfg.jt, precision, with_mass);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no VJP kernel for this ipl/jtile/precision");
    if (cfg.itiles <= 0 || cfg.nseg <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fn, dim3(cfg.itiles, cfg.nseg), dim3(kTPB), 0, s, a);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}


template <int MODE>
void launch_vjp_finalize_mode(dim3 grid, bool deep, const VjpFinalizeArgs &a, hipStream_t s) {
    if (deep)
        hipLaunchKernelGGL((vjp_finalize_kernel<MODE, 8>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((vjp_finalize_kernel<MODE, 1>), grid, dim3(256), 0, s, a);
}

nbody_status launch_vjp_finalize(int precision, const VjpFinalizeArgs &a, hipStream_t s) {
    if (a.n <= 0) return NBODY_OK;
    const int outputs = a.grad_mass ? 4 : 3;
    const dim3 grid((a.n + 255) / 256, outputs);
    const bool deep = engine::finalize_batch(a.n, outputs) > 1;
    switch (precision) {
        case NBODY_PLAIN: launch_vjp_finalize_mode<NBODY_PLAIN>(grid, deep, a, s); break;
        case NBODY_FP64RED: launch_vjp_finalize_mode<NBODY_FP64RED>(grid, deep, a, s); break;
        case NBODY_COMP: launch_vjp_finalize_mode<NBODY_COMP>(grid, deep, a, s); break;
        default: return set_error(NBODY_EINVAL, "unknown precision mode");
    }
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
