// Element-wise pieces of the fourth-order Hermite step (predictor-evaluate-corrector,
// Makino & Aarseth 1992), on FP64 state [3][n] flattened to 3n values.
#include "nbody_internal.h"

namespace nbody {
namespace {

// x_p = x + v dt + a dt^2/2 + j dt^3/6,  v_p = v + a dt + j dt^2/2
__global__ __launch_bounds__(256) void hermite_predict_kernel(
    int64_t count, const double *__restrict__ x, const double *__restrict__ v,
    const double *__restrict__ a, const double *__restrict__ j, double dt,
    double *__restrict__ xp, double *__restrict__ vp) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= count) return;
    const double dt2 = dt * dt;
    xp[q] = x[q] + v[q] * dt + a[q] * dt2 / 2.0 + j[q] * dt2 * dt / 6.0;
    vp[q] = v[q] + a[q] * dt + j[q] * dt2 / 2.0;
}

// v' = v + (a + a1) dt/2 + (j - j1) dt^2/12,  x' = x + (v + v') dt/2 + (a - a1) dt^2/12,
// then (a, j) <- (a1, j1) for the next step.
__global__ __launch_bounds__(256) void hermite_correct_kernel(
    int64_t count, double *__restrict__ x, double *__restrict__ v, double *__restrict__ a,
    double *__restrict__ j, const double *__restrict__ a1, const double *__restrict__ j1,
    double dt) {
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= count) return;
    const double dt2 = dt * dt;
    const double a0 = a[q], an = a1[q], j0 = j[q], jn = j1[q], v0 = v[q];
    const double vn = v0 + (a0 + an) * dt / 2.0 + (j0 - jn) * dt2 / 12.0;
    x[q] = x[q] + (v0 + vn) * dt / 2.0 + (a0 - an) * dt2 / 12.0;
    v[q] = vn;
    a[q] = an;
    j[q] = jn;
}

dim3 grid_of(int64_t count) { return dim3((unsigned)((count + 255) / 256)); }

}  // namespace

nbody_status launch_hermite_predict(int64_t n, const double *x, const double *v, const double *a,
                                    const double *j, double dt, double *xp, double *vp,
                                    hipStream_t s) {
    if (n <= 0) return NBODY_OK;
    hipLaunchKernelGGL(hermite_predict_kernel, grid_of(3 * n), dim3(256), 0, s, 3 * n, x, v, a, j,
                       dt, xp, vp);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_hermite_correct(int64_t n, double *x, double *v, double *a, double *j,
                                    const double *a1, const double *j1, double dt, hipStream_t s) {
    if (n <= 0) return NBODY_OK;
    hipLaunchKernelGGL(hermite_correct_kernel, grid_of(3 * n), dim3(256), 0, s, 3 * n, x, v, a, j,
                       a1, j1, dt);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
