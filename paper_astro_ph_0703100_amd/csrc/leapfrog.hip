// FP64 element-wise kernels of the kick-drift-kick leapfrog.  The state is
// structure-of-arrays [3][n] doubles; one lane per element of the 3n-vector.
#include "nbody_internal.h"

namespace nbody {
namespace {

// First half-kick fused with the drift: v += h a; x += dt v; the new x also goes to
// `checkpoint` when that is not null (the rollout's stored trajectory).
__global__ __launch_bounds__(256) void kick_drift_kernel(int64_t count, double *__restrict__ x,
                                                        double *__restrict__ v,
                                                        const double *__restrict__ a, double h,
                                                        double dt, double *__restrict__ checkpoint) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= count) return;
    const double vv = v[q] + h * a[q];
    v[q] = vv;
    const double xx = x[q] + dt * vv;
    x[q] = xx;
    if (checkpoint) checkpoint[q] = xx;
}

// The kick and drift of kick_drift_kernel on a fixed grid of kCentreBlocks blocks that
// stride over the particles exactly as the centre's first stage does, summing each
// thread's new positions in that order and reducing them with the same tree: the
// partials are bitwise those of a separate pass over the new positions.
__global__ __launch_bounds__(256) void kick_drift_centre_kernel(
    int64_t n, double *__restrict__ x, double *__restrict__ v, const double *__restrict__ a,
    double h, double dt, double *__restrict__ checkpoint, double *__restrict__ part) {
    __shared__ double sh[3][256];
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t q = c * n + i;
            const double vv = v[q] + h * a[q];
            v[q] = vv;
            const double xx = x[q] + dt * vv;
            x[q] = xx;
            if (checkpoint) checkpoint[q] = xx;
            s[c] += xx;
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void kick_kernel(int64_t count, double *__restrict__ v,
                                                  const double *__restrict__ a, double h) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= count) return;
    v[q] = v[q] + h * a[q];
}

__global__ __launch_bounds__(256) void copy_f64_kernel(int64_t count, const double *__restrict__ src,
                                                      double *__restrict__ dst) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= count) return;
    dst[q] = src[q];
}

__global__ __launch_bounds__(256) void fill_f64_kernel(int64_t count, double *__restrict__ dst,
                                                      double value) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= count) return;
    dst[q] = value;
}

__global__ __launch_bounds__(256) void axpy_f64_kernel(int64_t count, double *__restrict__ y,
                                                      double alpha, const double *__restrict__ x) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= count) return;
    y[q] = y[q] + alpha * x[q];
}

__global__ __launch_bounds__(256) void adj_drift_kick_kernel(int64_t count, double *__restrict__ vbar,
                                                            const double *__restrict__ xbar,
                                                            double *__restrict__ abar, double dt,
                                                            double h) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= count) return;
    const double vb = vbar[q] + dt * xbar[q];
    vbar[q] = vb;
    abar[q] = h * vb;
}

// adj_drift_kick_kernel on the centre's fixed grid, fused with the centre's first stage
// over `next` (the checkpoint the following adjoint evaluation reads), in the order and
// tree of the separate pass.
__global__ __launch_bounds__(256) void adj_drift_kick_centre_kernel(
    int64_t n, double *__restrict__ vbar, const double *__restrict__ xbar,
    double *__restrict__ abar, double dt, double h, const double *__restrict__ next,
    double *__restrict__ part) {
    __shared__ double sh[3][256];
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int64_t q = c * n + i;
            const double vb = vbar[q] + dt * xbar[q];
            vbar[q] = vb;
            abar[q] = h * vb;
            s[c] += next[q];
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = sh[threadIdx.x][0];
}

dim3 grid_for(int64_t count) { return dim3((unsigned)((count + 255) / 256)); }

}  // namespace

nbody_status launch_kick_drift(int64_t n, double *x, double *v, const double *acc, double h,
                               double dt, hipStream_t s, double *checkpoint) {
    if (n <= 0) return NBODY_OK;
    hipLaunchKernelGGL(kick_drift_kernel, grid_for(3 * n), dim3(256), 0, s, 3 * n, x, v, acc, h, dt,
                       checkpoint);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_kick_drift_centre(int64_t n, double *x, double *v, const double *acc,
                                      double h, double dt, double *checkpoint,
                                      double *centre_part, hipStream_t s) {
    if (n <= 0) return NBODY_OK;
    hipLaunchKernelGGL(kick_drift_centre_kernel, dim3(kCentreBlocks), dim3(256), 0, s, n, x, v, acc,
                       h, dt, checkpoint, centre_part);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_kick(int64_t n, double *v, const double *acc, double h, hipStream_t s) {
    if (n <= 0) return NBODY_OK;
    hipLaunchKernelGGL(kick_kernel, grid_for(3 * n), dim3(256), 0, s, 3 * n, v, acc, h);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_copy_f64(int64_t count, const double *src, double *dst, hipStream_t s) {
    if (count <= 0) return NBODY_OK;
    hipLaunchKernelGGL(copy_f64_kernel, grid_for(count), dim3(256), 0, s, count, src, dst);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_fill_f64(int64_t count, double *dst, double value, hipStream_t s) {
    if (count <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fill_f64_kernel, grid_for(count), dim3(256), 0, s, count, dst, value);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_axpy_f64(int64_t count, double *y, double alpha, const double *x, hipStream_t s) {
    if (count <= 0) return NBODY_OK;
    hipLaunchKernelGGL(axpy_f64_kernel, grid_for(count), dim3(256), 0, s, count, y, alpha, x);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_adj_drift_kick(int64_t count, double *vbar, const double *xbar, double *abar,
                                   double dt, double h, hipStream_t s) {
    if (count <= 0) return NBODY_OK;
    hipLaunchKernelGGL(adj_drift_kick_kernel, grid_for(count), dim3(256), 0, s, count, vbar, xbar,
                       abar, dt, h);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_adj_drift_kick_centre(int64_t n, double *vbar, const double *xbar, double *abar,
                                          double dt, double h, const double *next,
                                          double *centre_part, hipStream_t s) {
    if (n <= 0) return NBODY_OK;
    hipLaunchKernelGGL(adj_drift_kick_centre_kernel, dim3(kCentreBlocks), dim3(256), 0, s, n, vbar,
                       xbar, abar, dt, h, next, centre_part);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
