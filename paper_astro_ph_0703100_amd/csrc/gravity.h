// Gravity pipeline for the tile engine: softened accelerations and potentials of
// eq. (1) of the paper (the potential as accumulated by the force-jerk-potential
// pipeline of Appendix A).
#pragma once

#include "tile_engine.h"

namespace nbody {

// One softened pair term: separation x_j - x_i, s^2 = |d|^2 + eps^2 as an FMA chain,
// 1/s from the hardware reciprocal square root (about 1 ulp); a += m d / s^3 and
// phi -= m / s.  13 VALU operations and one v_rsq_f32.  The engine hands the j == i
// pair a massless record (null_j), so it adds exactly zero to a and phi.
template <bool POT>
__device__ __forceinline__ void gravity_pair(const float *j, float xi, float yi, float zi,
                                             float eps2, float (&acc)[4]) {
    const float dx = j[0] - xi;
    const float dy = j[1] - yi;
    const float dz = j[2] - zi;
    float s2 = __builtin_fmaf(dx, dx, eps2);
    s2 = __builtin_fmaf(dy, dy, s2);
    s2 = __builtin_fmaf(dz, dz, s2);
    const float ri = __builtin_amdgcn_rsqf(s2);
    const float mri = j[3] * ri;
    const float ri2 = ri * ri;
    const float mri3 = mri * ri2;
    acc[0] = __builtin_fmaf(mri3, dx, acc[0]);
    acc[1] = __builtin_fmaf(mri3, dy, acc[1]);
    acc[2] = __builtin_fmaf(mri3, dz, acc[2]);
    if (POT) acc[3] = acc[3] - mri;
}

struct Gravity {
    static constexpr int kJWords = 4;  // x, y, z, m
    static constexpr int kOut = 4;     // ax, ay, az, phi
    // 128 j's per compensation step: measured on MI355X at N = 131072 the compensated
    // kernel runs 5 % faster than with 32 (the two-sums cost 0.19 instead of 0.75 VALU
    // operations per pair), and the FP32 block error stays far below the pair rounding.
    static constexpr int kBlockJ = 128;
    using Args = PairArgs;
    struct IState {
        float x, y, z;
    };
    struct Ctx {};
    static __device__ __forceinline__ int n_i(const Args &a) { return a.n; }
    static __device__ __forceinline__ int n_j(const Args &a) { return a.n; }
    static __device__ __forceinline__ Ctx make_ctx(const Args &, int) { return {}; }
    static __device__ __forceinline__ IState load_i(const Args &a, const Ctx &, int i) {
        return {a.x[i], a.y[i], a.z[i]};
    }
    static __device__ __forceinline__ void load_j(const Args &a, const Ctx &, int j, float (&r)[4]) {
        r[0] = a.x[j];
        r[1] = a.y[j];
        r[2] = a.z[j];
        r[3] = a.m[j];
    }
    // A massless particle at the origin adds exactly zero.
    static __device__ __forceinline__ void pad_j(float (&r)[4]) { r[0] = r[1] = r[2] = r[3] = 0.0f; }
    // The j == i pair: the same place with no mass (its separation is exactly zero, so
    // every term is +0 times a finite number).
    static constexpr bool kSelf = true;
    static __device__ __forceinline__ void null_j(float (&r)[4]) { r[3] = 0.0f; }

    template <bool POT>
    static __device__ __forceinline__ void pair(const float *j, const IState &i, float eps2,
                                                float (&acc)[4]) {
        gravity_pair<POT>(j, i.x, i.y, i.z, eps2, acc);
    }
};

// The same pair body on FP64 positions taken relative to a per-i-tile FP64 reference
// centre c_I (the mean of the tile's positions): the i-records and every j-record
// staged for the tile are converted as fp32(x - c_I) while they are loaded, so the
// FP32 pair arithmetic sees coordinates of the size of the tile, not of the system.
// For the j == i pair both conversions are the same operation, so the separation is
// still exactly zero and the massless null record adds nothing.
struct GravityTile {
    static constexpr int kJWords = 4;
    static constexpr int kOut = 4;
    static constexpr int kBlockJ = Gravity::kBlockJ;
    using Args = TilePairArgs;
    using IState = Gravity::IState;
    struct Ctx {
        double cx, cy, cz;
    };
    static __device__ __forceinline__ int n_i(const Args &a) { return a.n; }
    static __device__ __forceinline__ int n_j(const Args &a) { return a.n; }
    static __device__ __forceinline__ Ctx make_ctx(const Args &a, int i0) {
        const double *c = a.centres + 3 * (size_t)(i0 / a.itile);
        return {c[0], c[1], c[2]};
    }
    static __device__ __forceinline__ IState load_i(const Args &a, const Ctx &c, int i) {
        return {(float)(a.x[i] - c.cx), (float)(a.y[i] - c.cy), (float)(a.z[i] - c.cz)};
    }
    static __device__ __forceinline__ void load_j(const Args &a, const Ctx &c, int j, float (&r)[4]) {
        r[0] = (float)(a.x[j] - c.cx);
        r[1] = (float)(a.y[j] - c.cy);
        r[2] = (float)(a.z[j] - c.cz);
        r[3] = a.m[j];
    }
    static __device__ __forceinline__ void pad_j(float (&r)[4]) { Gravity::pad_j(r); }
    static constexpr bool kSelf = true;
    static __device__ __forceinline__ void null_j(float (&r)[4]) { Gravity::null_j(r); }
    template <bool POT>
    static __device__ __forceinline__ void pair(const float *j, const IState &i, float eps2,
                                                float (&acc)[4]) {
        gravity_pair<POT>(j, i.x, i.y, i.z, eps2, acc);
    }
};

// Separate i- and j-sets, the paper's library interface (Sec. 3.1): forces on ni
// i-particles from nj j-particles, with no pair treated as a self pair, and the
// softening either uniform or given per i-particle (the paper's driver stores eps^2
// per i).  Padding j-records sit at 1e30 with zero mass: their s^2 overflows to +inf,
// rsq(+inf) = 0, and every term they add is exactly zero, also when eps = 0.
struct GravityIJ {
    static constexpr int kJWords = 4;
    static constexpr int kOut = 4;
    static constexpr int kBlockJ = Gravity::kBlockJ;
    using Args = IJPairArgs;
    struct IState {
        float x, y, z, e2;
    };
    struct Ctx {};
    static __device__ __forceinline__ int n_i(const Args &a) { return a.ni; }
    static __device__ __forceinline__ int n_j(const Args &a) { return a.nj; }
    static __device__ __forceinline__ Ctx make_ctx(const Args &, int) { return {}; }
    static __device__ __forceinline__ IState load_i(const Args &a, const Ctx &, int i) {
        float e2 = a.eps2;
        if (a.ei) {
            const float e = a.ei[i];
            e2 = e * e;
        }
        return {a.xi[i], a.yi[i], a.zi[i], e2};
    }
    static __device__ __forceinline__ void load_j(const Args &a, const Ctx &, int j, float (&r)[4]) {
        r[0] = a.x[j];
        r[1] = a.y[j];
        r[2] = a.z[j];
        r[3] = a.m[j];
    }
    static __device__ __forceinline__ void pad_j(float (&r)[4]) {
        r[0] = r[1] = r[2] = 1e30f;
        r[3] = 0.0f;
    }
    static constexpr bool kSelf = false;  // separate sets: every pair is summed
    template <bool POT>
    static __device__ __forceinline__ void pair(const float *j, const IState &i, float,
                                                float (&acc)[4]) {
        gravity_pair<POT>(j, i.x, i.y, i.z, i.e2, acc);
    }
};

}  // namespace nbody
