// Host side of the adjoint: the VJP of one force evaluation and the reverse pass of
// the kick-drift-kick leapfrog over stored position checkpoints.
#include <cmath>

#include "nbody_internal.h"
#include "tuning.h"

namespace nbody {
namespace {

nbody_status check_vjp(int64_t n, const void *pos, const float *mass, float eps,
                       const double *g_acc, const double *g_pot, const double *grad_pos,
                       const double *grad_mass, const nbody_opts &o) {
    nbody_status st = check_common(n, pos, mass, eps, grad_pos, o);
    if (st) return st;
    if (n > 0 && !g_acc) return set_error(NBODY_EINVAL, "g_acc must not be NULL");
    if (misaligned(mass) || misaligned(g_acc) || misaligned(g_pot) || misaligned(grad_pos) ||
        misaligned(grad_mass))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    return NBODY_OK;
}

size_t vjp_f64_bytes(int64_t n, const TileCfg &cfg, int precision) {
    return f64_scratch_bytes(n, cfg, precision, kVjpOutputs);
}

// Adjoint pair kernel + FP64 finalize on FP32 positions.
nbody_status vjp_f32_core(int64_t n, const float *pos, const float *mass, float eps,
                          const double *g_acc, const double *g_pot, double *grad_pos,
                          double *grad_mass, bool accumulate, const nbody_opts &o,
                          const TileCfg &cfg, void *part, hipStream_t s) {
    const float e2 = eps * eps;
    VjpArgs va{pos,   pos + n, pos + 2 * n, mass, g_acc, g_acc + n, g_acc + 2 * n,
               g_pot, (int)n,  cfg.seg_len, e2,   part,  cfg.npad};
    VjpFinalizeArgs fa{part,      cfg.nseg, cfg.npad,           (int)n, g_pot,
                       grad_pos,  grad_mass, accumulate ? 1 : 0, g_acc};
    if (cfg.jl > 1) return launch_vjp_split(cfg, o.precision, va, grad_mass != nullptr, fa, s);
    nbody_status st = launch_vjp(cfg, o.precision, va, grad_mass != nullptr, s);
    if (st) return st;
    return launch_vjp_finalize(o.precision, fa, s);
}

// Centre + FP32 conversion, then the adjoint on the converted positions.
// centre_ready: with NBODY_CENTRE_SYSTEM, the centre's first stage over pos64 is already
// in ws.centre_scratch.
nbody_status vjp_f64_core(int64_t n, const double *pos64, const float *mass, float eps,
                          const double *g_acc, const double *g_pot, double *grad_pos,
                          double *grad_mass, bool accumulate, const nbody_opts &o,
                          const TileCfg &cfg, const F64Scratch &ws, hipStream_t s,
                          bool centre_ready = false) {
    nbody_status st;
    if (o.centre == NBODY_CENTRE_TILE) {
        // Per-i-tile centres in the FP32-position area (unused in this mode).
        const int itile = kTPB * cfg.ipl;
        double *centres = reinterpret_cast<double *>(ws.x32);
        if ((st = launch_tile_centres(n, itile, pos64, centres, s))) return st;
        const float e2 = eps * eps;
        VjpTileArgs va{pos64, pos64 + n, pos64 + 2 * n, mass, g_acc, g_acc + n, g_acc + 2 * n,
                       g_pot, (int)n, cfg.seg_len, e2, ws.part, cfg.npad, centres, itile};
        if ((st = launch_vjp_tile(cfg, o.precision, va, grad_mass != nullptr, s))) return st;
        VjpFinalizeArgs fa{ws.part,  cfg.nseg, cfg.npad,           (int)n, g_pot,
                           grad_pos, grad_mass, accumulate ? 1 : 0, g_acc};
        return launch_vjp_finalize(o.precision, fa, s);
    }
    if (o.centre == NBODY_CENTRE_SYSTEM) {
        st = centre_ready ? launch_centred_convert_ready(n, pos64, ws.centre_scratch, ws.x32, s)
                          : launch_centred_convert(n, pos64, ws.centre_scratch, ws.x32, s);
        if (st) return st;
    } else {
        if ((st = launch_convert(n, pos64, nullptr, ws.x32, s))) return st;
    }
    return vjp_f32_core(n, ws.x32, mass, eps, g_acc, g_pot, grad_pos, grad_mass, accumulate, o,
                        cfg, ws.part, s);
}

}  // namespace
}  // namespace nbody

using namespace nbody;

extern "C" {

size_t nbody_workspace_size_vjp(int64_t n, const nbody_opts *opts) {
    nbody_opts o = resolve_opts(opts);
    if (n <= 0) return 0;
    TileCfg c;
    if (choose_cfg(KERNEL_VJP, n, o.precision, o, &c, o.centre != NBODY_CENTRE_TILE ? kEngineSplit : 0) != NBODY_OK) return 0;
    return vjp_f64_bytes(n, c, o.precision);
}

size_t nbody_workspace_size_adjoint(int64_t n, const nbody_opts *opts) {
    const size_t base = nbody_workspace_size_vjp(n, opts);
    return base ? base + sizeof(double) * 3 * (size_t)n : 0;
}

nbody_status nbody_force_vjp(int64_t n, const float *pos, const float *mass, float eps,
                             const double *g_acc, const double *g_pot, double *grad_pos,
                             double *grad_mass, const nbody_opts *opts, void *stream) {
    clear_error();
    nbody_opts o = resolve_opts(opts);
    nbody_status st = check_vjp(n, pos, mass, eps, g_acc, g_pot, grad_pos, grad_mass, o);
    if (st) return st;
    if (misaligned(pos)) return set_error(NBODY_EINVAL, "misaligned array argument");
    if (n == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_VJP, n, o.precision, o, &cfg, kEngineSplit))) return st;
    void *ws = nullptr;
    if ((st = get_workspace(o, partial_bytes(cfg, o.precision, kVjpOutputs), s, &ws))) return st;
    return vjp_f32_core(n, pos, mass, eps, g_acc, g_pot, grad_pos, grad_mass, false, o, cfg, ws, s);
}

nbody_status nbody_force_vjp_f64(int64_t n, const double *pos64, const float *mass, float eps,
                                 const double *g_acc, const double *g_pot, double *grad_pos,
                                 double *grad_mass, const nbody_opts *opts, void *stream) {
    clear_error();
    nbody_opts o = resolve_opts(opts);
    nbody_status st = check_vjp(n, pos64, mass, eps, g_acc, g_pot, grad_pos, grad_mass, o);
    if (st) return st;
    if (misaligned(pos64)) return set_error(NBODY_EINVAL, "misaligned array argument");
    if (n == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_VJP, n, o.precision, o, &cfg, o.centre != NBODY_CENTRE_TILE ? kEngineSplit : 0))) return st;
    void *ws = nullptr;
    if ((st = get_workspace(o, vjp_f64_bytes(n, cfg, o.precision), s, &ws))) return st;
    return vjp_f64_core(n, pos64, mass, eps, g_acc, g_pot, grad_pos, grad_mass, false, o, cfg,
                        f64_scratch_layout(ws, n, cfg, o.precision, kVjpOutputs), s);
}

nbody_status nbody_leapfrog_adjoint(int64_t n, const double *traj, const float *mass, float eps,
                                    double dt, int32_t nsteps, double *xbar, double *vbar,
                                    double *mbar, const nbody_opts *opts, void *stream) {
    clear_error();
    nbody_opts o = resolve_opts(opts);
    nbody_status st = check_common(n, traj, mass, eps, xbar, o);
    if (st) return st;
    if (n > 0 && !vbar) return set_error(NBODY_EINVAL, "vbar must not be NULL");
    if (nsteps < 0) return set_error(NBODY_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(dt)) return set_error(NBODY_EINVAL, "dt must be finite");
    if (misaligned(traj) || misaligned(mass) || misaligned(xbar) || misaligned(vbar) ||
        misaligned(mbar))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    // Zero steps: the rollout is the identity, so dL/dx_0 = xbar and dL/dv_0 = vbar as
    // given, and the masses get nothing.
    if (n == 0 || nsteps == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_VJP, n, o.precision, o, &cfg, o.centre != NBODY_CENTRE_TILE ? kEngineSplit : 0))) return st;
    const size_t base = vjp_f64_bytes(n, cfg, o.precision);
    const size_t n3 = 3 * (size_t)n;
    void *ws = nullptr;
    if ((st = get_workspace(o, base + sizeof(double) * n3, s, &ws))) return st;
    const F64Scratch lay = f64_scratch_layout(ws, n, cfg, o.precision, kVjpOutputs);
    double *abar = reinterpret_cast<double *>(static_cast<char *>(ws) + base);
    const double h = 0.5 * dt;

    // abar holds the cotangent of a(x_t) summed over the two kicks that use it: the
    // second kick of step t - 1 and the first kick of step t both scale a(x_t) by h and
    // see the same vbar (nothing changes v between them), so together they give
    // abar = dt vbar; the last state's a is used by one kick only.
    if ((st = launch_fill_f64((int64_t)n3, abar, 0.0, s))) return st;
    if ((st = launch_axpy_f64((int64_t)n3, abar, h, vbar, s))) return st;
    // With the system centre, each drift-kick update also runs the centre's first stage
    // over the checkpoint the next adjoint evaluation reads.
    const bool fused = o.centre == NBODY_CENTRE_SYSTEM;
    bool ready = false;
    for (int32_t t = nsteps - 1; t >= 0; --t) {
        const double *x1 = traj + (size_t)(t + 1) * n3;
        if ((st = vjp_f64_core(n, x1, mass, eps, abar, nullptr, xbar, mbar, true, o, cfg, lay, s,
                               ready)))
            return st;
        // drift of step t (vbar += dt xbar), then both kicks that use a(x_t)
        const double hk = t > 0 ? dt : h;
        st = fused ? launch_adj_drift_kick_centre(n, vbar, xbar, abar, dt, hk, traj + (size_t)t * n3,
                                                  lay.centre_scratch, s)
                   : launch_adj_drift_kick((int64_t)n3, vbar, xbar, abar, dt, hk, s);
        if (st) return st;
        ready = fused;
    }
    return vjp_f64_core(n, traj, mass, eps, abar, nullptr, xbar, mbar, true, o, cfg, lay, s, ready);
}

}  // extern "C"
