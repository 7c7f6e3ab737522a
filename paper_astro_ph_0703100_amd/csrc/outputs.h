// Output stages shared by the FP64 finalize kernels of the tile engine and by the
// single-launch split engine (device code): what is stored for output c of particle i
// once its FP64 sum r over all j is known.
#pragma once

#include "nbody_internal.h"

namespace nbody {

// Forces and potentials: c = 0, 1, 2 are the acceleration components (optionally
// followed by the leapfrog's second kick v += h a), c = 3 the potential (optionally
// with the j == i term -m_i / eps, formed in FP64).
struct ForceOut {
    using Args = FinalizeArgs;
    static __device__ __forceinline__ void put(const Args &a, int i, int c, double r) {
        if (c == 3) {
            if (a.include_self) r -= (double)a.m[i] / (double)a.eps;
            a.pot[i] = r;
            return;
        }
        a.acc[c * (size_t)a.n + i] = r;
        if (a.kick_v) a.kick_v[c * (size_t)a.n + i] += a.kick_h * r;
    }
};

// Adjoint: c = 0, 1, 2 are dL/dx_i, c = 3 the positive sum whose negation is dL/dm_i;
// with accumulate set both are added to what the arrays hold.
struct VjpOut {
    using Args = VjpFinalizeArgs;
    static __device__ __forceinline__ void put(const Args &a, int i, int c, double r) {
        if (c < 3) {
            double *g = a.grad_pos + (size_t)c * a.n + i;
            *g = a.accumulate ? *g + r : r;
            return;
        }
        const double gm = -r;
        a.grad_mass[i] = a.accumulate ? a.grad_mass[i] + gm : gm;
    }
};

}  // namespace nbody
