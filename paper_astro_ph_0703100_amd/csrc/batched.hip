// Kernels of the ragged batched path: many independent systems stored back to back
// (system k owns the global indices [offsets[k], offsets[k+1])).
//
//   * pair work: the persistent work-queue launch of the gravity pipeline over the
//     plan's cost-sorted items (one i-tile x one j-range of one system each);
//   * finalize: per particle, the fixed-order FP64 sum of its system's segment
//     partials (no j == i term: the pair kernel left it out) and the optional fused
//     leapfrog kick;
//   * per-system FP64 centres (one block per system, fixed-order reduction) and the
//     conversion of FP64 positions to FP32 relative to them.
#include "gravity.h"

namespace nbody {
namespace {

__global__ void reset_counter_kernel(unsigned int *counter) { *counter = 0u; }

template <int MODE>
__global__ __launch_bounds__(256) void batched_finalize_kernel(BatchFinalizeArgs a) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= a.total) return;
    const int k = a.sys_of[p];
    const int64_t col = p - a.offsets[k];
    const int npad = a.npad[k];
    const void *base = static_cast<const float *>(a.part) + a.part_base[k];
    double r[4];
    engine::sum_partials<4, MODE, 1>(base, a.nseg[k], (size_t)npad, (int)col, r);
    const size_t n = (size_t)a.total;
    a.acc[p] = r[0];
    a.acc[n + p] = r[1];
    a.acc[2 * n + p] = r[2];
    if (a.pot) a.pot[p] = r[3];
    if (a.kick_v) {
#pragma unroll
        for (int c = 0; c < 3; ++c) a.kick_v[c * n + p] += a.kick_h * r[c];
    }
}

// Mean position of each system in FP64: block k sums its particles with a fixed
// stride pattern and tree, so the result is reproducible.
__global__ __launch_bounds__(256) void system_centre_kernel(const int64_t *offsets, int64_t total,
                                                           const double *pos, double *centre) {
    __shared__ double sh[3][256];
    const int k = blockIdx.x;
    const int64_t b = offsets[k], e = offsets[k + 1];
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t p = b + threadIdx.x; p < e; p += 256)
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += pos[c * total + p];
#pragma unroll
    for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) centre[3 * k + threadIdx.x] = e > b ? sh[threadIdx.x][0] / (double)(e - b) : 0.0;
}

__global__ __launch_bounds__(256) void batched_convert_kernel(int64_t total, const double *pos,
                                                             const int32_t *sys_of,
                                                             const double *centre, float *out) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= total) return;
    const int k = sys_of[p];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        out[c * total + p] = (float)(pos[c * total + p] - (centre ? centre[3 * k + c] : 0.0));
}

}  // namespace

nbody_status batched_pair_kernel(int ipl, int jt, int precision, bool with_pot, const void **fn) {
    *fn = reinterpret_cast<const void *>(engine::pick_persistent<Gravity>(ipl, jt, precision, with_pot));
    return *fn ? NBODY_OK : set_error(NBODY_EUNSUPPORTED, "no batched kernel for this shape");
}

nbody_status launch_batched_pair(int ipl, int jt, int precision, bool with_pot, int grid,
                                 const PairArgs &a, const BatchSched &sc, hipStream_t s) {
    auto fn = engine::pick_persistent<Gravity>(ipl, jt, precision, with_pot);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no batched kernel for this shape");
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, sc.counter);
    NBODY_HIP_CHECK(hipGetLastError());
    if (sc.nitems <= 0 || grid <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fn, dim3(grid), dim3(kTPB), 0, s, a, sc);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_batched_finalize(int precision, const BatchFinalizeArgs &a, hipStream_t s) {
    if (a.total <= 0) return NBODY_OK;
    const dim3 grid((unsigned)((a.total + 255) / 256));
    switch (precision) {
        case NBODY_PLAIN: hipLaunchKernelGGL(batched_finalize_kernel<NBODY_PLAIN>, grid, dim3(256), 0, s, a); break;
        case NBODY_FP64RED: hipLaunchKernelGGL(batched_finalize_kernel<NBODY_FP64RED>, grid, dim3(256), 0, s, a); break;
        case NBODY_COMP: hipLaunchKernelGGL(batched_finalize_kernel<NBODY_COMP>, grid, dim3(256), 0, s, a); break;
        default: return set_error(NBODY_EINVAL, "unknown precision mode");
    }
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_system_centres(int nsys, const int64_t *offsets, int64_t total,
                                   const double *pos64, double *centre, hipStream_t s) {
    if (nsys <= 0) return NBODY_OK;
    hipLaunchKernelGGL(system_centre_kernel, dim3(nsys), dim3(256), 0, s, offsets, total, pos64, centre);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_batched_convert(int64_t total, const double *pos64, const int32_t *sys_of,
                                    const double *centre, float *pos32, hipStream_t s) {
    if (total <= 0) return NBODY_OK;
    hipLaunchKernelGGL(batched_convert_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       total, pos64, sys_of, centre, pos32);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
