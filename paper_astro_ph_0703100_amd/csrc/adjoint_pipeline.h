// Adjoint pipelines for the tile engine (device code, included by the .hip files that
// launch them): vector-Jacobian product of the softened accelerations and potentials
// (eq. (1) and the potential of Appendix A) with respect to positions and masses.
//
// With d = x_j - x_k, s^2 = |d|^2 + eps^2, cotangents g = dL/da and p = dL/dphi,
// and K_kj = I/s^3 - 3 d d^T / s^5, differentiating the two sums term by term gives
//   dL/dx_k =  sum_{j != k} [ K_kj w_kj - d (m_k p_j + m_j p_k) / s^3 ],
//              w_kj = m_k g_j - m_j g_k
//           =  sum_{j != k} [ w / s^3 - (q / s^3 + 3 (d . w) / s^5) d ],  q = m_k p_j + m_j p_k
//   dL/dm_k = -sum_{j != k} [ (g_j . d) / s^3 + p_j / s ].
// The term w / s^3 splits into m_k g_j / s^3, accumulated per pair (3 FMAs), and
// -g_k m_j / s^3, whose scalar sum B_k = sum_j m_j / s^3 is accumulated (1 FMA) and
// multiplied by the particle's own g_k once, in FP64, by the output stage; d . w =
// m_k (d . g_j) - m_j (d . g_k), where d . g_j is the dL/dm term's too.  Outputs:
// [0..2] sum_j (m_k g_j / s^3 - e d) with e = (q + 3 (d . w) / s^2) / s^3, [3] B_k,
// [4] the positive sum of dL/dm_k.  The engine hands the j == k pair a record with no
// mass and no cotangents (null_j), which adds exactly zero to every sum.
// 31 VALU operations and one v_rsq_f32 per pair (38 when w was formed per pair).  The
// terms of -(d . w), -q and -e are formed instead of those of d . w, q and e (the i-record
// carries -m_k and -p_k): rounding to nearest is symmetric in sign, so every value is
// the exact negation and the sums are bitwise the same, and each step is an FMA that
// accumulates into its own addend, with no negated operand (measured 0.2-0.4 % faster).
#pragma once

#include "tile_engine.h"

namespace nbody {

namespace {

struct Adjoint {
    static constexpr int kJWords = 8;  // x, y, z, m, gx, gy, gz, p
    static constexpr int kOut = 5;     // see above: three position sums, B_k, mass sum
    // 128 j's per compensation step (32 before: 1.8 % slower at N = 16384 and 131072).
    static constexpr int kBlockJ = nbody::kBlockJ;
    using Args = VjpArgs;
    struct IState {
        float x, y, z, m, nm, gx, gy, gz, np;  // nm = -m_k, np = -p_k
    };
    struct Ctx {};
    static __device__ __forceinline__ int n_i(const Args &a) { return a.n; }
    static __device__ __forceinline__ int n_j(const Args &a) { return a.n; }
    static __device__ __forceinline__ Ctx make_ctx(const Args &, int) { return {}; }
    static __device__ __forceinline__ IState load_i(const Args &a, const Ctx &, int i) {
        const float m = a.m[i];
        return {a.x[i], a.y[i], a.z[i], m, negated(m), (float)a.gx[i], (float)a.gy[i],
                (float)a.gz[i], a.gp ? -(float)a.gp[i] : -0.0f};
    }
    // -m held in a register of its own: left visible as the negation of m, the compiler
    // would fold it into the FMAs as a source modifier, which takes the 64-bit encoding.
    static __device__ __forceinline__ float negated(float m) {
        float r = -m;
        asm volatile("" : "+v"(r));
        return r;
    }
    static __device__ __forceinline__ void load_j(const Args &a, const Ctx &, int j, float (&r)[8]) {
        r[0] = a.x[j];
        r[1] = a.y[j];
        r[2] = a.z[j];
        r[3] = a.m[j];
        r[4] = (float)a.gx[j];
        r[5] = (float)a.gy[j];
        r[6] = (float)a.gz[j];
        r[7] = a.gp ? (float)a.gp[j] : 0.0f;
    }
    // Massless, cotangent-free particle at the origin: every term below is zero.
    static __device__ __forceinline__ void pad_j(float (&r)[8]) {
#pragma unroll
        for (int c = 0; c < 8; ++c) r[c] = 0.0f;
    }
    // The j == k pair: the same position, with mass and both cotangents zero.
    static constexpr bool kSelf = true;
    static __device__ __forceinline__ void null_j(float (&r)[8]) {
#pragma unroll
        for (int c = 3; c < 8; ++c) r[c] = 0.0f;
    }

    template <bool MASS>
    static __device__ __forceinline__ void pair(const float *j, const IState &k, float eps2,
                                                float (&acc)[5]) {
        const float dx = j[0] - k.x;
        const float dy = j[1] - k.y;
        const float dz = j[2] - k.z;
        float s2 = __builtin_fmaf(dx, dx, eps2);
        s2 = __builtin_fmaf(dy, dy, s2);
        s2 = __builtin_fmaf(dz, dz, s2);
        const float r = __builtin_amdgcn_rsqf(s2);
        const float r2 = r * r;
        const float r3 = r * r2;
        const float kr3 = k.m * r3;  // m_k / s^3
        float gd = j[4] * dx;        // d . g_j
        gd = __builtin_fmaf(j[5], dy, gd);
        gd = __builtin_fmaf(j[6], dz, gd);
        float gkd = k.gx * dx;       // d . g_k
        gkd = __builtin_fmaf(k.gy, dy, gkd);
        gkd = __builtin_fmaf(k.gz, dz, gkd);
        const float mgkd = j[3] * gkd;
        const float ndw = __builtin_fmaf(k.nm, gd, mgkd);  // -(d . w)
        const float nmp = j[3] * k.np;
        const float nq = __builtin_fmaf(k.nm, j[7], nmp);  // -q
        const float t3 = r2 * 3.0f;
        const float ne = r3 * __builtin_fmaf(t3, ndw, nq);  // -e
        acc[0] = __builtin_fmaf(kr3, j[4], acc[0]);
        acc[1] = __builtin_fmaf(kr3, j[5], acc[1]);
        acc[2] = __builtin_fmaf(kr3, j[6], acc[2]);
        acc[0] = __builtin_fmaf(ne, dx, acc[0]);
        acc[1] = __builtin_fmaf(ne, dy, acc[1]);
        acc[2] = __builtin_fmaf(ne, dz, acc[2]);
        acc[3] = __builtin_fmaf(j[3], r3, acc[3]);
        if (MASS) {
            acc[4] = __builtin_fmaf(gd, r3, acc[4]);
            acc[4] = __builtin_fmaf(j[7], r, acc[4]);
        }
    }
};

// The same on FP64 positions relative to the block's i-tile centre: i's and staged j's
// are converted as fp32(x - c_I) while loaded (for j == k the two conversions are the
// same operation, so d = 0 exactly and the null record adds nothing).
struct AdjointTile {
    static constexpr int kJWords = 8;
    static constexpr int kOut = 5;
    static constexpr int kBlockJ = Adjoint::kBlockJ;
    using Args = VjpTileArgs;
    using IState = Adjoint::IState;
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
        const float m = a.m[i];
        return {(float)(a.x[i] - c.cx), (float)(a.y[i] - c.cy), (float)(a.z[i] - c.cz), m,
                Adjoint::negated(m), (float)a.gx[i], (float)a.gy[i], (float)a.gz[i],
                a.gp ? -(float)a.gp[i] : -0.0f};
    }
    static __device__ __forceinline__ void load_j(const Args &a, const Ctx &c, int j, float (&r)[8]) {
        r[0] = (float)(a.x[j] - c.cx);
        r[1] = (float)(a.y[j] - c.cy);
        r[2] = (float)(a.z[j] - c.cz);
        r[3] = a.m[j];
        r[4] = (float)a.gx[j];
        r[5] = (float)a.gy[j];
        r[6] = (float)a.gz[j];
        r[7] = a.gp ? (float)a.gp[j] : 0.0f;
    }
    static __device__ __forceinline__ void pad_j(float (&r)[8]) { Adjoint::pad_j(r); }
    static constexpr bool kSelf = true;
    static __device__ __forceinline__ void null_j(float (&r)[8]) { Adjoint::null_j(r); }
    template <bool MASS>
    static __device__ __forceinline__ void pair(const float *j, const IState &k, float eps2,
                                                float (&acc)[5]) {
        Adjoint::pair<MASS>(j, k, eps2, acc);
    }
};

}  // namespace
}  // namespace nbody
