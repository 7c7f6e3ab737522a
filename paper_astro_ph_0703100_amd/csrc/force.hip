// Force evaluation of one system: the gravity pipeline on the tile engine (grid
// launch), the FP64 finalize, and the FP64-position pre-pass (centre, conversion).
#include "gravity.h"
#include "outputs.h"

namespace nbody {
namespace {

// Fixed-order sum of the segment partials (PLAIN in FP32, the other modes in FP64),
// one thread per (particle, output) so that few particles with many segments still
// fill the chip.  The partials hold no j == i term (the pair kernel left it out); with
// include_self the potential gets -m_i / eps, formed in FP64.
// With kick_v set, the velocity kick of a leapfrog step follows in FP64.
// Grid: (ceil(n / 256), 4 outputs, or 3 without potentials).
template <int MODE, int BATCH>
__global__ __launch_bounds__(256) void finalize_kernel(FinalizeArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= a.n) return;
    ForceOut::put(a, i, c, [&](int o) {
        return engine::sum_partial_output<kForceOutputs, MODE, BATCH>(a.part, a.nseg,
                                                                      (size_t)a.npad, i, o);
    });
}

// Two-stage fixed-order FP64 mean of the positions [3][n]: kCentreBlocks partial
// sums, then their fixed-order sum.  Deterministic for a given n.

__global__ __launch_bounds__(256) void centre_partial_kernel(int64_t n, const double *pos,
                                                            double *part) {
    __shared__ double sh[3][256];
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += pos[c * n + i];
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

// The second stage fused with the conversion to FP32: every block adds the
// kCentreBlocks partials in the same fixed tree order, so all blocks use the identical
// centre c = sum / n, then converts its 256 particles to fp32(x - c).
__global__ __launch_bounds__(256) void centred_convert_kernel(int64_t n, const double *pos,
                                                             const double *part, float *out) {
    __shared__ double sh[3][kCentreBlocks];
#pragma unroll
    for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] = part[threadIdx.x * 3 + c];
    __syncthreads();
    for (int w = kCentreBlocks / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        __syncthreads();
    }
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * n + i] = (float)(pos[c * n + i] - sh[c][0] / (double)n);
}

__global__ __launch_bounds__(256) void convert_kernel(int64_t n, const double *pos,
                                                     const double *centre, float *out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * n + i] = (float)(pos[c * n + i] - (centre ? centre[c] : 0.0));
}

// Mean position of each i-tile of `itile` consecutive particles, FP64, one block per
// tile, fixed-order tree: the reference centres of NBODY_CENTRE_TILE.
__global__ __launch_bounds__(256) void tile_centre_kernel(int64_t n, int itile, const double *pos,
                                                         double *centres) {
    __shared__ double sh[3][256];
    const int64_t b = (int64_t)blockIdx.x * itile;
    const int64_t e = b + itile < n ? b + itile : n;
    double s[3] = {0.0, 0.0, 0.0};
    for (int64_t p = b + threadIdx.x; p < e; p += 256)
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += pos[c * n + p];
#pragma unroll
    for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) centres[3 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0] / (double)(e - b);
}

}  // namespace

nbody_status launch_tile_centres(int64_t n, int itile, const double *pos64, double *centres,
                                 hipStream_t s) {
    if (n <= 0) return NBODY_OK;
    const int64_t tiles = (n + itile - 1) / itile;
    hipLaunchKernelGGL(tile_centre_kernel, dim3((unsigned)tiles), dim3(256), 0, s, n, itile, pos64,
                       centres);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_pair_tile(const TileCfg &cfg, int precision, bool with_pot,
                              const TilePairArgs &a, hipStream_t s) {
    auto fn = engine::pick_tile<GravityTile>(cfg.ipl, cfg.jt, precision, with_pot);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no tile-centre kernel for this shape");
    if (cfg.itiles <= 0 || cfg.nseg <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fn, dim3(cfg.itiles, cfg.nseg), dim3(kTPB), 0, s, a);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_pair(const TileCfg &cfg, int precision, bool with_pot, const PairArgs &a,
                         hipStream_t s) {
    auto fn = engine::pick_tile<Gravity>(cfg.ipl, cfg.jt, precision, with_pot);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no pair kernel for this ipl/jtile/precision");
    if (cfg.itiles <= 0 || cfg.nseg <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fn, dim3(cfg.itiles, cfg.nseg), dim3(kTPB), 0, s, a);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

template <int MODE>
void launch_finalize_mode(dim3 grid, bool deep, const FinalizeArgs &a, hipStream_t s) {
    if (deep)
        hipLaunchKernelGGL((finalize_kernel<MODE, 8>), grid, dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL((finalize_kernel<MODE, 1>), grid, dim3(256), 0, s, a);
}

nbody_status launch_finalize(int precision, const FinalizeArgs &a, hipStream_t s) {
    if (a.n <= 0) return NBODY_OK;
    const int outputs = a.pot ? 4 : 3;
    const dim3 grid((a.n + 255) / 256, outputs);
    const bool deep = engine::finalize_batch(a.n, outputs) > 1;
    switch (precision) {
        case NBODY_PLAIN: launch_finalize_mode<NBODY_PLAIN>(grid, deep, a, s); break;
        case NBODY_FP64RED: launch_finalize_mode<NBODY_FP64RED>(grid, deep, a, s); break;
        case NBODY_COMP: launch_finalize_mode<NBODY_COMP>(grid, deep, a, s); break;
        default: return set_error(NBODY_EINVAL, "unknown precision mode");
    }
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

size_t centre_scratch_bytes() { return sizeof(double) * 3 * kCentreBlocks; }

nbody_status launch_centred_convert(int64_t n, const double *pos64, double *scratch,
                                    float *pos32, hipStream_t s) {
    if (n <= 0) return NBODY_OK;
    hipLaunchKernelGGL(centre_partial_kernel, dim3(kCentreBlocks), dim3(256), 0, s, n, pos64, scratch);
    NBODY_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(centred_convert_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       n, pos64, (const double *)scratch, pos32);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_centred_convert_ready(int64_t n, const double *pos64, const double *scratch,
                                          float *pos32, hipStream_t s) {
    if (n <= 0) return NBODY_OK;
    hipLaunchKernelGGL(centred_convert_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       n, pos64, scratch, pos32);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_convert(int64_t n, const double *pos64, const double *centre, float *pos32,
                            hipStream_t s) {
    if (n <= 0) return NBODY_OK;
    hipLaunchKernelGGL(convert_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, pos64,
                       centre, pos32);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
