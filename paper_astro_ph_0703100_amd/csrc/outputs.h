// Output stages shared by the FP64 finalize kernels of the tile engine and by the
// single-launch split engine (device code): what is stored for store slot c of
// particle i, given `sum(o)`, the FP64 sum over all j of the pipeline's output o.
#pragma once

#include "nbody_internal.h"

namespace nbody {

// Forces and potentials: slots 0, 1, 2 are the acceleration components (optionally
// followed by the leapfrog's second kick v += h a), slot 3 the potential (optionally
// with the j == i term -m_i / eps, formed in FP64).  Slot c stores output c.
struct ForceOut {
    using Args = FinalizeArgs;
    static constexpr int kOutputs = kForceOutputs;
    // Store slots: 4, or 3 without the last output (no potential).
    static constexpr int stores(bool full) { return full ? 4 : 3; }
    template <class Sum>
    static __device__ __forceinline__ void put(const Args &a, int i, int c, Sum sum) {
        double r = sum(c);
        if (c == 3) {
            if (a.include_self) r -= (double)a.m[i] / (double)a.eps;
            a.pot[i] = r;
            return;
        }
        a.acc[c * (size_t)a.n + i] = r;
        if (a.kick_v) a.kick_v[c * (size_t)a.n + i] += a.kick_h * r;
    }
};

// Adjoint: slots 0, 1, 2 are dL/dx_i = sum(c) - g_i,c * sum(3) (g_i the particle's own
// cotangent, as the FP32 value the pair kernel sees), slot 3 dL/dm_i = -sum(4); with
// accumulate set both are added to what the arrays hold.
struct VjpOut {
    using Args = VjpFinalizeArgs;
    static constexpr int kOutputs = kVjpOutputs;
    // Store slots: 4, or 3 without the mass gradient.
    static constexpr int stores(bool full) { return full ? 4 : 3; }
    template <class Sum>
    static __device__ __forceinline__ void put(const Args &a, int i, int c, Sum sum) {
        if (c < 3) {
            const double gk = (double)(float)a.ga[(size_t)c * a.n + i];
            const double r = sum(c) - gk * sum(3);
            double *g = a.grad_pos + (size_t)c * a.n + i;
            *g = a.accumulate ? *g + r : r;
            return;
        }
        const double gm = -sum(4);
        a.grad_mass[i] = a.accumulate ? a.grad_mass[i] + gm : gm;
    }
};

}  // namespace nbody
