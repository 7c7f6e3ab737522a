// Force-jerk-potential pipelines (device code, included by the .hip files that launch
// them): force, jerk and potential in one pass, as in the pipeline of the
// paper's Appendix A (the interaction of a fourth-order Hermite integrator, Sec. 4.1)
// on the tile engine.  With d = x_j - x_i, w = v_j - v_i and s^2 = |d|^2 + eps^2:
//   a_i    +=  m_j d / s^3
//   jerk_i +=  m_j (w - 3 (d.w / s^2) d) / s^3
//   phi_i  -=  m_j / s
// j-records are 8 floats (x, y, z, m, vx, vy, vz, 0: two LDS reads per j); i-records
// hold position and velocity.  27 FP32 VALU operations and one v_rsq_f32 per pair.
// Three pipelines: FP32 inputs (GravityJerk), FP64 state relative to per-i-tile centres
// (GravityJerkTile), and separate i- and j-sets (GravityJerkIJ).
#pragma once

#include "tile_engine.h"

namespace nbody {
namespace {

// One pair term.  The engine hands the j == i pair a massless record (null_j): with d
// and w exactly zero and m = 0 it adds exactly zero to a, the jerk and phi.
template <bool POT>
__device__ __forceinline__ void jerk_pair(const float *j, float xi, float yi, float zi, float vxi,
                                          float vyi, float vzi, float eps2, float (&acc)[7]) {
    const float dx = j[0] - xi;
    const float dy = j[1] - yi;
    const float dz = j[2] - zi;
    const float wx = j[4] - vxi;
    const float wy = j[5] - vyi;
    const float wz = j[6] - vzi;
    float s2 = __builtin_fmaf(dx, dx, eps2);
    s2 = __builtin_fmaf(dy, dy, s2);
    s2 = __builtin_fmaf(dz, dz, s2);
    const float ri = __builtin_amdgcn_rsqf(s2);
    const float ri2 = ri * ri;
    const float mri = j[3] * ri;
    const float mri3 = mri * ri2;
    float dw = dx * wx;
    dw = __builtin_fmaf(dy, wy, dw);
    dw = __builtin_fmaf(dz, wz, dw);
    const float al = (dw * ri2) * 3.0f;
    const float tx = __builtin_fmaf(-al, dx, wx);
    const float ty = __builtin_fmaf(-al, dy, wy);
    const float tz = __builtin_fmaf(-al, dz, wz);
    acc[0] = __builtin_fmaf(mri3, dx, acc[0]);
    acc[1] = __builtin_fmaf(mri3, dy, acc[1]);
    acc[2] = __builtin_fmaf(mri3, dz, acc[2]);
    acc[3] = __builtin_fmaf(mri3, tx, acc[3]);
    acc[4] = __builtin_fmaf(mri3, ty, acc[4]);
    acc[5] = __builtin_fmaf(mri3, tz, acc[5]);
    if (POT) acc[6] = acc[6] - mri;
}

struct GravityJerk {
    static constexpr int kJWords = 8;
    static constexpr int kOut = 7;  // ax, ay, az, jx, jy, jz, phi
    // 14 two-sum operations per block of 128 pairs (64 before: 1.6 % slower, and at
    // 256-j tiles the four unrolled blocks took 85 VGPRs, 5 waves per SIMD).
    static constexpr int kBlockJ = nbody::kBlockJ;
    using Args = JerkArgs;
    struct IState {
        float x, y, z, vx, vy, vz;
    };
    struct Ctx {};
    static __device__ __forceinline__ int n_i(const Args &a) { return a.n; }
    static __device__ __forceinline__ int n_j(const Args &a) { return a.n; }
    static __device__ __forceinline__ Ctx make_ctx(const Args &, int) { return {}; }
    static __device__ __forceinline__ IState load_i(const Args &a, const Ctx &, int i) {
        return {a.x[i], a.y[i], a.z[i], a.vx[i], a.vy[i], a.vz[i]};
    }
    static __device__ __forceinline__ void load_j(const Args &a, const Ctx &, int j, float (&r)[8]) {
        r[0] = a.x[j];
        r[1] = a.y[j];
        r[2] = a.z[j];
        r[3] = a.m[j];
        r[4] = a.vx[j];
        r[5] = a.vy[j];
        r[6] = a.vz[j];
        r[7] = 0.0f;
    }
    // A massless particle at rest at the origin: every term carries m = 0.
    static __device__ __forceinline__ void pad_j(float (&r)[8]) {
#pragma unroll
        for (int c = 0; c < 8; ++c) r[c] = 0.0f;
    }
    // The j == i pair: same position and velocity, no mass.
    static constexpr bool kSelf = true;
    static __device__ __forceinline__ void null_j(float (&r)[8]) { r[3] = 0.0f; }
    template <bool POT>
    static __device__ __forceinline__ void pair(const float *j, const IState &i, float eps2,
                                                float (&acc)[7]) {
        jerk_pair<POT>(j, i.x, i.y, i.z, i.vx, i.vy, i.vz, eps2, acc);
    }
};

// FP64 state relative to the block's i-tile centres (mean position and mean velocity):
// the i-records and every staged j-record are converted as fp32(x - c_I), fp32(v - w_I),
// so the pair arithmetic sees the tile's own scale.  For j == i both conversions are the
// same operation and d = w = 0 exactly.
struct GravityJerkTile {
    static constexpr int kJWords = 8;
    static constexpr int kOut = 7;
    static constexpr int kBlockJ = GravityJerk::kBlockJ;
    using Args = JerkTileArgs;
    using IState = GravityJerk::IState;
    struct Ctx {
        double cx, cy, cz, wx, wy, wz;
    };
    static __device__ __forceinline__ int n_i(const Args &a) { return a.n; }
    static __device__ __forceinline__ int n_j(const Args &a) { return a.n; }
    static __device__ __forceinline__ Ctx make_ctx(const Args &a, int i0) {
        const size_t t = 3 * (size_t)(i0 / a.itile);
        return {a.cx[t], a.cx[t + 1], a.cx[t + 2], a.cv[t], a.cv[t + 1], a.cv[t + 2]};
    }
    static __device__ __forceinline__ IState load_i(const Args &a, const Ctx &c, int i) {
        return {(float)(a.x[i] - c.cx),  (float)(a.y[i] - c.cy),  (float)(a.z[i] - c.cz),
                (float)(a.vx[i] - c.wx), (float)(a.vy[i] - c.wy), (float)(a.vz[i] - c.wz)};
    }
    static __device__ __forceinline__ void load_j(const Args &a, const Ctx &c, int j, float (&r)[8]) {
        r[0] = (float)(a.x[j] - c.cx);
        r[1] = (float)(a.y[j] - c.cy);
        r[2] = (float)(a.z[j] - c.cz);
        r[3] = a.m[j];
        r[4] = (float)(a.vx[j] - c.wx);
        r[5] = (float)(a.vy[j] - c.wy);
        r[6] = (float)(a.vz[j] - c.wz);
        r[7] = 0.0f;
    }
    static __device__ __forceinline__ void pad_j(float (&r)[8]) { GravityJerk::pad_j(r); }
    static constexpr bool kSelf = true;
    static __device__ __forceinline__ void null_j(float (&r)[8]) { GravityJerk::null_j(r); }
    template <bool POT>
    static __device__ __forceinline__ void pair(const float *j, const IState &i, float eps2,
                                                float (&acc)[7]) {
        jerk_pair<POT>(j, i.x, i.y, i.z, i.vx, i.vy, i.vz, eps2, acc);
    }
};

// Separate i- and j-sets (an active subset of a system against all of it, or two
// systems): every (i, j) pair is summed, with one softening for all.  Padding
// j-records are massless and far away (1e18), so their terms are exactly zero even
// with eps = 0 (s^2 stays a finite normal float and every product with m = 0 is 0).
struct GravityJerkIJ {
    static constexpr int kJWords = 8;
    static constexpr int kOut = 7;
    static constexpr int kBlockJ = GravityJerk::kBlockJ;
    using Args = JerkIJArgs;
    using IState = GravityJerk::IState;
    struct Ctx {};
    static __device__ __forceinline__ int n_i(const Args &a) { return a.ni; }
    static __device__ __forceinline__ int n_j(const Args &a) { return a.nj; }
    static __device__ __forceinline__ Ctx make_ctx(const Args &, int) { return {}; }
    static __device__ __forceinline__ IState load_i(const Args &a, const Ctx &, int i) {
        return {a.xi[i], a.yi[i], a.zi[i], a.vxi[i], a.vyi[i], a.vzi[i]};
    }
    static __device__ __forceinline__ void load_j(const Args &a, const Ctx &, int j, float (&r)[8]) {
        r[0] = a.x[j];
        r[1] = a.y[j];
        r[2] = a.z[j];
        r[3] = a.m[j];
        r[4] = a.vx[j];
        r[5] = a.vy[j];
        r[6] = a.vz[j];
        r[7] = 0.0f;
    }
    static __device__ __forceinline__ void pad_j(float (&r)[8]) {
        r[0] = r[1] = r[2] = 1e18f;
#pragma unroll
        for (int c = 3; c < 8; ++c) r[c] = 0.0f;
    }
    static constexpr bool kSelf = false;  // separate sets: every pair is summed
    template <bool POT>
    static __device__ __forceinline__ void pair(const float *j, const IState &i, float eps2,
                                                float (&acc)[7]) {
        jerk_pair<POT>(j, i.x, i.y, i.z, i.vx, i.vy, i.vz, eps2, acc);
    }
};

}  // namespace
}  // namespace nbody
