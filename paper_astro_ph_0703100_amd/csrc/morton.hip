// Morton (Z-order) permutation of FP64 positions, so that consecutive particles - and
// therefore the i-tiles of the pair kernels - are spatially compact.  That is what
// makes per-i-tile reference centres (NBODY_CENTRE_TILE) pay off.
//
// Steps: FP64 bounding box (two-stage min/max), a 64-bit word per particle holding
// the interleaved quantised coordinates in its high bits and the particle index in its
// low bits, a bitonic sort of the words (padded to a power of two with ~0), and the
// index bits of the sorted words as the permutation.  Ties in the key are broken by
// index, so the order is unique.
#include "nbody_internal.h"

namespace nbody {
namespace {

constexpr int kBoxBlocks = 256;

__global__ __launch_bounds__(256) void box_partial_kernel(int64_t n, const double *pos, double *part) {
    __shared__ double lo[3][256], hi[3][256];
    double l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double v = pos[c * n + i];
            l[c] = fmin(l[c], v);
            h[c] = fmax(h[c], v);
        }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c][threadIdx.x] = l[c];
        hi[c][threadIdx.x] = h[c];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                lo[c][threadIdx.x] = fmin(lo[c][threadIdx.x], lo[c][threadIdx.x + w]);
                hi[c][threadIdx.x] = fmax(hi[c][threadIdx.x], hi[c][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        part[6 * blockIdx.x + threadIdx.x] = lo[threadIdx.x][0];
        part[6 * blockIdx.x + 3 + threadIdx.x] = hi[threadIdx.x][0];
    }
}

__global__ __launch_bounds__(256) void box_final_kernel(const double *part, double *box) {
    __shared__ double lo[3][kBoxBlocks], hi[3][kBoxBlocks];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        lo[c][threadIdx.x] = part[6 * threadIdx.x + c];
        hi[c][threadIdx.x] = part[6 * threadIdx.x + 3 + c];
    }
    __syncthreads();
    for (int w = kBoxBlocks / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                lo[c][threadIdx.x] = fmin(lo[c][threadIdx.x], lo[c][threadIdx.x + w]);
                hi[c][threadIdx.x] = fmax(hi[c][threadIdx.x], hi[c][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 3) {
        box[threadIdx.x] = lo[threadIdx.x][0];
        box[3 + threadIdx.x] = hi[threadIdx.x][0];
    }
}

// Spreads the low `bits` bits of v so that bit b moves to bit 3b.
__device__ __forceinline__ uint64_t spread3(uint64_t v, int bits) {
    uint64_t r = 0;
    for (int b = 0; b < bits; ++b) r |= ((v >> b) & 1ull) << (3 * b);
    return r;
}

__global__ __launch_bounds__(256) void key_kernel(int64_t n, int64_t npow, const double *pos,
                                                 const double *box, int qbits, int ibits,
                                                 uint64_t *words) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= npow) return;
    if (i >= n) {
        words[i] = ~0ull;
        return;
    }
    const double top = (double)((1ull << qbits) - 1);
    uint64_t key = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double span = box[3 + c] - box[c];
        double q = span > 0.0 ? (pos[c * n + i] - box[c]) / span * top : 0.0;
        q = q < 0.0 ? 0.0 : (q > top ? top : q);
        key |= spread3((uint64_t)q, qbits) << (2 - c);
    }
    words[i] = (key << ibits) | (uint64_t)i;
}

// One compare-exchange stage of the bitonic network (block k, distance j).
__global__ __launch_bounds__(256) void bitonic_kernel(uint64_t *a, int64_t half, int64_t j, int64_t k) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= half) return;
    const int64_t i = 2 * j * (t / j) + (t % j);
    const int64_t l = i + j;
    const bool up = (i & k) == 0;
    const uint64_t x = a[i], y = a[l];
    if ((x > y) == up) {
        a[i] = y;
        a[l] = x;
    }
}

__global__ __launch_bounds__(256) void perm_kernel(int64_t n, const uint64_t *words, uint64_t mask,
                                                  int32_t *perm) {
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    perm[r] = (int32_t)(words[r] & mask);
}

int64_t pow2_at_least(int64_t n) {
    int64_t p = 1;
    while (p < n) p <<= 1;
    return p;
}

}  // namespace

size_t morton_scratch_bytes(int64_t n) {
    return sizeof(uint64_t) * (size_t)pow2_at_least(n > 1 ? n : 1) +
           sizeof(double) * (6 * kBoxBlocks + 8);
}

nbody_status launch_morton_order(int64_t n, const double *pos64, int32_t *perm, void *scratch,
                                 hipStream_t s) {
    if (n <= 0) return NBODY_OK;
    const int64_t npow = pow2_at_least(n);
    uint64_t *words = static_cast<uint64_t *>(scratch);
    double *part = reinterpret_cast<double *>(words + npow);
    double *box = part + 6 * kBoxBlocks;
    int ibits = 0;
    while ((int64_t(1) << ibits) < n) ++ibits;
    const int qbits = (64 - ibits) / 3;
    hipLaunchKernelGGL(box_partial_kernel, dim3(kBoxBlocks), dim3(256), 0, s, n, pos64, part);
    hipLaunchKernelGGL(box_final_kernel, dim3(1), dim3(kBoxBlocks), 0, s, (const double *)part, box);
    hipLaunchKernelGGL(key_kernel, dim3((unsigned)((npow + 255) / 256)), dim3(256), 0, s, n, npow,
                       pos64, (const double *)box, qbits, ibits, words);
    NBODY_HIP_CHECK(hipGetLastError());
    const int64_t half = npow / 2;
    const dim3 grid((unsigned)((half + 255) / 256 > 0 ? (half + 255) / 256 : 1));
    for (int64_t k = 2; k <= npow; k <<= 1)
        for (int64_t j = k >> 1; j > 0; j >>= 1)
            hipLaunchKernelGGL(bitonic_kernel, grid, dim3(256), 0, s, words, half, j, k);
    NBODY_HIP_CHECK(hipGetLastError());
    const uint64_t mask = ibits >= 64 ? ~0ull : ((1ull << ibits) - 1);
    hipLaunchKernelGGL(perm_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       (const uint64_t *)words, mask, perm);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
