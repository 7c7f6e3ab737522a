// Force and potential kernels for gfx950 (CDNA4).
//
// Work decomposition (the Chamomile Scheme's J-BAG x I-POT blocking, Sec. 2.1-2.2,
// re-planned for a CDNA4 compute unit):
//   * a block of 256 lanes owns an i-tile of 256 * IPL particles; each lane keeps
//     IPL i-particles in VGPRs (lane-strided so global loads and stores coalesce);
//   * blockIdx.y selects a j-segment; the block walks it in LDS tiles of JT
//     j-particles, staged from the structure-of-arrays input with coalesced loads,
//     double-buffered so there is one barrier per tile (the J-PACKING step);
//   * every lane reads each j record from LDS with one 16-byte broadcast read and
//     evaluates IPL pair terms with 13 VALU operations and one v_rsq_f32 each;
//   * partial sums per (i, segment) go to scratch; finalize_kernel adds the
//     segments in FP64 in a fixed order and removes the j == i potential term.
// Accumulation (Sec. 2.2.2, eq. (2) and Sec. 3.4):
//   PLAIN   - one FP32 accumulator per (i, segment);
//   FP64RED - FP32 partial over each block of kBlockJ j's, then added into FP64;
//   COMP    - FP32 partial over each block, then an error-free two-sum into an
//             FP32 (hi, lo) pair.
// No floating-point atomics are used: every result is a fixed-order sum, so runs
// are bitwise reproducible for a given launch shape.
#include "nbody_internal.h"

namespace nbody {
namespace {

struct alignas(16) JRec {
    float x, y, z, m;
};

// One softened pair term of eq. (1) plus the potential, accumulated into (ax, ay,
// az, ap).  The separation is x_j - x_i; r^2 + eps^2 is an FMA chain; 1/s comes from
// the hardware reciprocal square root (about 1 ulp).  13 VALU + 1 transcendental.
template <bool POT>
__device__ __forceinline__ void pair_term(const JRec &j, float xi, float yi, float zi,
                                          float eps2, float &ax, float &ay, float &az,
                                          float &ap) {
    const float dx = j.x - xi;
    const float dy = j.y - yi;
    const float dz = j.z - zi;
    float s2 = __builtin_fmaf(dx, dx, eps2);
    s2 = __builtin_fmaf(dy, dy, s2);
    s2 = __builtin_fmaf(dz, dz, s2);
    const float ri = __builtin_amdgcn_rsqf(s2);
    const float mri = j.m * ri;
    const float ri2 = ri * ri;
    const float mri3 = mri * ri2;
    ax = __builtin_fmaf(mri3, dx, ax);
    ay = __builtin_fmaf(mri3, dy, ay);
    az = __builtin_fmaf(mri3, dz, az);
    if (POT) ap = ap - mri;
}

// Knuth's error-free sum: hi + lo += b with hi = fl(hi + b) and the rounding error
// of that addition added to lo.
__device__ __forceinline__ void two_sum(float &hi, float &lo, float b) {
    const float s = hi + b;
    const float bb = s - hi;
    const float err = (hi - (s - bb)) + (b - bb);
    hi = s;
    lo = lo + err;
}

template <int IPL, int JT, int MODE, bool POT>
__global__ __launch_bounds__(kTPB) void pair_kernel(PairArgs a) {
    __shared__ JRec tile[2][JT];
    constexpr int LPT = (JT + kTPB - 1) / kTPB;  // j records staged per lane
    const int tid = threadIdx.x;
    const int n = a.n;
    const int ibase = blockIdx.x * (kTPB * IPL);
    const float eps2 = a.eps2;

    float xi[IPL], yi[IPL], zi[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        int i = ibase + k * kTPB + tid;
        i = i < n ? i : n - 1;
        xi[k] = a.x[i];
        yi[k] = a.y[i];
        zi[k] = a.z[i];
    }

    // hi (or the plain sums), lo, and FP64 accumulators; unused ones are removed.
    float hx[IPL], hy[IPL], hz[IPL], hp[IPL];
    float lx[IPL], ly[IPL], lz[IPL], lp[IPL];
    double dx64[IPL], dy64[IPL], dz64[IPL], dp64[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        hx[k] = hy[k] = hz[k] = hp[k] = 0.0f;
        lx[k] = ly[k] = lz[k] = lp[k] = 0.0f;
        dx64[k] = dy64[k] = dz64[k] = dp64[k] = 0.0;
    }

    const int j0 = blockIdx.y * a.seg_len;
    const int j1 = min(j0 + a.seg_len, n);
    const int ntiles = j1 > j0 ? (j1 - j0 + JT - 1) / JT : 0;

    JRec stage[LPT];
    auto fetch = [&](int t) {
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const int jj = q * kTPB + tid;
            const int j = j0 + t * JT + jj;
            if (jj < JT) {
                if (j < j1) {
                    stage[q].x = a.x[j];
                    stage[q].y = a.y[j];
                    stage[q].z = a.z[j];
                    stage[q].m = a.m[j];
                } else {
                    // Padding: a massless particle at the origin adds exactly zero.
                    stage[q].x = stage[q].y = stage[q].z = stage[q].m = 0.0f;
                }
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const int jj = q * kTPB + tid;
            if (jj < JT) tile[buf][jj] = stage[q];
        }
    };

    if (ntiles > 0) {
        fetch(0);
        store(0);
    }
    __syncthreads();
    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        if (t + 1 < ntiles) fetch(t + 1);
        const JRec *tl = tile[buf];
        if constexpr (MODE == NBODY_PLAIN) {
#pragma unroll 8
            for (int jj = 0; jj < JT; ++jj) {
                const JRec pj = tl[jj];
#pragma unroll
                for (int k = 0; k < IPL; ++k)
                    pair_term<POT>(pj, xi[k], yi[k], zi[k], eps2, hx[k], hy[k], hz[k], hp[k]);
            }
        } else {
            for (int jb = 0; jb < JT; jb += kBlockJ) {
                float bx[IPL], by[IPL], bz[IPL], bp[IPL];
#pragma unroll
                for (int k = 0; k < IPL; ++k) bx[k] = by[k] = bz[k] = bp[k] = -0.0f;
#pragma unroll
                for (int jj = 0; jj < kBlockJ; ++jj) {
                    const JRec pj = tl[jb + jj];
#pragma unroll
                    for (int k = 0; k < IPL; ++k)
                        pair_term<POT>(pj, xi[k], yi[k], zi[k], eps2, bx[k], by[k], bz[k], bp[k]);
                }
#pragma unroll
                for (int k = 0; k < IPL; ++k) {
                    if constexpr (MODE == NBODY_COMP) {
                        two_sum(hx[k], lx[k], bx[k]);
                        two_sum(hy[k], ly[k], by[k]);
                        two_sum(hz[k], lz[k], bz[k]);
                        if (POT) two_sum(hp[k], lp[k], bp[k]);
                    } else {
                        dx64[k] += (double)bx[k];
                        dy64[k] += (double)by[k];
                        dz64[k] += (double)bz[k];
                        if (POT) dp64[k] += (double)bp[k];
                    }
                }
            }
        }
        if (t + 1 < ntiles) store(buf ^ 1);
        __syncthreads();
    }

    // Partial sums of this (i-tile, segment): planes [seg][word][npad].
    const size_t plane = (size_t)a.npad;
    const size_t seg = blockIdx.y;
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const size_t i = (size_t)ibase + k * kTPB + tid;
        if constexpr (MODE == NBODY_FP64RED) {
            double *p = static_cast<double *>(a.part) + seg * 4 * plane + i;
            p[0] = dx64[k];
            p[plane] = dy64[k];
            p[2 * plane] = dz64[k];
            p[3 * plane] = dp64[k];
        } else {
            float *p = static_cast<float *>(a.part) + seg * (MODE == NBODY_PLAIN ? 4 : 8) * plane + i;
            p[0] = hx[k];
            p[plane] = hy[k];
            p[2 * plane] = hz[k];
            p[3 * plane] = hp[k];
            if constexpr (MODE == NBODY_COMP) {
                p[4 * plane] = lx[k];
                p[5 * plane] = ly[k];
                p[6 * plane] = lz[k];
                p[7 * plane] = lp[k];
            }
        }
    }
}

// Sum of the segment partials of one particle in a fixed order, then removal of the
// j == i potential term -m_i * rsq(eps^2), recomputed with the same FP32 operations
// the pair kernel used for it.  PLAIN adds in FP32; the other modes in FP64.  With
// kick_v set, the velocity kick of a leapfrog step follows in FP64.
template <int MODE>
__global__ __launch_bounds__(256) void finalize_kernel(FinalizeArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const size_t plane = (size_t)a.npad;
    const float self = a.m[i] * __builtin_amdgcn_rsqf(a.eps2);
    double r[4];
    if constexpr (MODE == NBODY_PLAIN) {
        float f[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        const float *p = static_cast<const float *>(a.part) + i;
        for (int s = 0; s < a.nseg; ++s)
#pragma unroll
            for (int c = 0; c < 4; ++c) f[c] = f[c] + p[((size_t)s * 4 + c) * plane];
        if (!a.self_pot) f[3] = f[3] + self;
#pragma unroll
        for (int c = 0; c < 4; ++c) r[c] = (double)f[c];
    } else if constexpr (MODE == NBODY_COMP) {
        const float *p = static_cast<const float *>(a.part) + i;
#pragma unroll
        for (int c = 0; c < 4; ++c) r[c] = 0.0;
        for (int s = 0; s < a.nseg; ++s)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                r[c] += (double)p[((size_t)s * 8 + c) * plane];
                r[c] += (double)p[((size_t)s * 8 + 4 + c) * plane];
            }
        if (!a.self_pot) r[3] += (double)self;
    } else {
        const double *p = static_cast<const double *>(a.part) + i;
#pragma unroll
        for (int c = 0; c < 4; ++c) r[c] = 0.0;
        for (int s = 0; s < a.nseg; ++s)
#pragma unroll
            for (int c = 0; c < 4; ++c) r[c] += p[((size_t)s * 4 + c) * plane];
        if (!a.self_pot) r[3] += (double)self;
    }
    a.acc[i] = r[0];
    a.acc[(size_t)a.n + i] = r[1];
    a.acc[2 * (size_t)a.n + i] = r[2];
    if (a.pot) a.pot[i] = r[3];
    if (a.kick_v) {  // second kick of a leapfrog step, fused: v += h a
#pragma unroll
        for (int c = 0; c < 3; ++c) a.kick_v[c * (size_t)a.n + i] += a.kick_h * r[c];
    }
}

// Two-stage fixed-order FP64 mean of the positions [3][n]: kCentreBlocks partial
// sums, then one block adds them.  Deterministic for a given n.
constexpr int kCentreBlocks = 256;

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

__global__ __launch_bounds__(256) void centre_final_kernel(int64_t n, const double *part,
                                                          double *centre) {
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
    if (threadIdx.x < 3) centre[threadIdx.x] = n > 0 ? sh[threadIdx.x][0] / (double)n : 0.0;
}

__global__ __launch_bounds__(256) void convert_kernel(int64_t n, const double *pos,
                                                     const double *centre, float *out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * n + i] = (float)(pos[c * n + i] - (centre ? centre[c] : 0.0));
}

using PairFn = void (*)(PairArgs);

template <int IPL, int JT, int MODE>
PairFn pick_pot(bool pot) {
    return pot ? pair_kernel<IPL, JT, MODE, true> : pair_kernel<IPL, JT, MODE, false>;
}

template <int IPL, int JT>
PairFn pick_mode(int mode, bool pot) {
    switch (mode) {
        case NBODY_PLAIN: return pick_pot<IPL, JT, NBODY_PLAIN>(pot);
        case NBODY_FP64RED: return pick_pot<IPL, JT, NBODY_FP64RED>(pot);
        case NBODY_COMP: return pick_pot<IPL, JT, NBODY_COMP>(pot);
    }
    return nullptr;
}

template <int IPL>
PairFn pick_jt(int jt, int mode, bool pot) {
    switch (jt) {
        case 64: return pick_mode<IPL, 64>(mode, pot);
        case 128: return pick_mode<IPL, 128>(mode, pot);
        case 256: return pick_mode<IPL, 256>(mode, pot);
        case 512: return pick_mode<IPL, 512>(mode, pot);
    }
    return nullptr;
}

PairFn pick_pair(int ipl, int jt, int mode, bool pot) {
    switch (ipl) {
        case 1: return pick_jt<1>(jt, mode, pot);
        case 2: return pick_jt<2>(jt, mode, pot);
        case 4: return pick_jt<4>(jt, mode, pot);
        case 8: return pick_jt<8>(jt, mode, pot);
    }
    return nullptr;
}

}  // namespace

nbody_status launch_pair(const TileCfg &cfg, int precision, bool with_pot, const PairArgs &a,
                         hipStream_t s) {
    PairFn fn = pick_pair(cfg.ipl, cfg.jt, precision, with_pot);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no pair kernel for this ipl/jtile/precision");
    if (cfg.itiles <= 0 || cfg.nseg <= 0) return NBODY_OK;
    hipLaunchKernelGGL(fn, dim3(cfg.itiles, cfg.nseg), dim3(kTPB), 0, s, a);
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

nbody_status launch_finalize(int precision, const FinalizeArgs &a, hipStream_t s) {
    if (a.n <= 0) return NBODY_OK;
    const dim3 grid((a.n + 255) / 256);
    switch (precision) {
        case NBODY_PLAIN: hipLaunchKernelGGL(finalize_kernel<NBODY_PLAIN>, grid, dim3(256), 0, s, a); break;
        case NBODY_FP64RED: hipLaunchKernelGGL(finalize_kernel<NBODY_FP64RED>, grid, dim3(256), 0, s, a); break;
        case NBODY_COMP: hipLaunchKernelGGL(finalize_kernel<NBODY_COMP>, grid, dim3(256), 0, s, a); break;
        default: return set_error(NBODY_EINVAL, "unknown precision mode");
    }
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

size_t centre_scratch_bytes() { return sizeof(double) * 3 * kCentreBlocks; }

nbody_status launch_centre(int64_t n, const double *pos64, double *centre, double *scratch,
                           hipStream_t s) {
    hipLaunchKernelGGL(centre_partial_kernel, dim3(kCentreBlocks), dim3(256), 0, s, n, pos64, scratch);
    NBODY_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(centre_final_kernel, dim3(1), dim3(kCentreBlocks), 0, s, n,
                       (const double *)scratch, centre);
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
