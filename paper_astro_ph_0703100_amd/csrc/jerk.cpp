// Host entry points of the force-jerk-potential path: argument checks, launch shape,
// scratch, and (for FP64 state) the reference centres of positions and velocities.
#include <cfloat>
#include <cmath>

#include "nbody_internal.h"
#include "tuning.h"

namespace nbody {
namespace {

constexpr int kJerkOut = 7;

size_t jerk_partial_bytes(const TileCfg &c, int precision) {
    const size_t words = (size_t)(precision == NBODY_PLAIN ? 1 : 2) * kJerkOut;
    return align_up((size_t)c.nseg * words * (size_t)c.npad * 4, 256);
}

// FP64-state scratch: partial sums, FP32 relative positions and velocities [3][n] each,
// the two FP64 centres (4 doubles each) and the centre-reduction partials.
struct JerkScratch {
    void *part;
    float *x32, *v32;
    double *cx, *cv, *cscratch;
};

size_t jerk_f64_bytes(int64_t n, const TileCfg &c, int precision) {
    return jerk_partial_bytes(c, precision) + 2 * align_up(sizeof(float) * 3 * (size_t)n, 256) +
           align_up(centre_scratch_bytes() + 8 * sizeof(double), 256);
}

JerkScratch jerk_f64_layout(void *ws, int64_t n, const TileCfg &c, int precision) {
    char *b = static_cast<char *>(ws);
    const size_t pb = jerk_partial_bytes(c, precision);
    const size_t xb = align_up(sizeof(float) * 3 * (size_t)n, 256);
    JerkScratch r;
    r.part = b;
    r.x32 = reinterpret_cast<float *>(b + pb);
    r.v32 = reinterpret_cast<float *>(b + pb + xb);
    r.cx = reinterpret_cast<double *>(b + pb + 2 * xb);
    r.cv = r.cx + 4;
    r.cscratch = r.cv + 4;
    return r;
}

nbody_status check_jerk(int64_t n, const void *pos, const void *vel, const void *mass, float eps,
                        const void *acc, const void *jerk, const nbody_opts &o) {
    nbody_status st = check_common(n, pos, mass, eps, acc, o);
    if (st) return st;
    if (n > 0 && (!vel || !jerk)) return set_error(NBODY_EINVAL, "vel and jerk must not be NULL");
    return NBODY_OK;
}

nbody_status jerk_core(int64_t n, const float *pos, const float *vel, const float *mass, float eps,
                       double *acc, double *jerk, double *pot, const nbody_opts &o,
                       const TileCfg &cfg, void *part, hipStream_t s) {
    const float e2 = eps * eps;
    JerkArgs a{pos, pos + n, pos + 2 * n, mass, vel, vel + n, vel + 2 * n,
               (int)n, cfg.seg_len, e2, part, cfg.npad};
    nbody_status st = launch_jerk(cfg, o.precision, pot != nullptr, a, s);
    if (st) return st;
    JerkFinalizeArgs fa{part, cfg.nseg, cfg.npad, (int)n, mass, e2, o.self_pot ? 0 : 1,
                        acc,  jerk,     pot};
    return launch_jerk_finalize(o.precision, fa, s);
}

}  // namespace
}  // namespace nbody

using namespace nbody;

extern "C" {

size_t nbody_workspace_size_jerk(int64_t n, const nbody_opts *opts) {
    nbody_opts o = resolve_opts(opts);
    if (n <= 0) return 0;
    TileCfg c;
    if (choose_cfg(KERNEL_JERK, n, o.precision, o, &c) != NBODY_OK) return 0;
    return jerk_f64_bytes(n, c, o.precision);
}

nbody_status nbody_force_jerk(int64_t n, const float *pos, const float *vel, const float *mass,
                              float eps, double *acc, double *jerk, double *pot,
                              const nbody_opts *opts, void *stream) {
    clear_error();
    nbody_opts o = resolve_opts(opts);
    nbody_status st = check_jerk(n, pos, vel, mass, eps, acc, jerk, o);
    if (st) return st;
    if (misaligned(pos) || misaligned(vel) || misaligned(mass) || misaligned(acc) ||
        misaligned(jerk) || misaligned(pot))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    if (n == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_JERK, n, o.precision, o, &cfg))) return st;
    void *ws = nullptr;
    if ((st = get_workspace(o, jerk_partial_bytes(cfg, o.precision), s, &ws))) return st;
    return jerk_core(n, pos, vel, mass, eps, acc, jerk, pot, o, cfg, ws, s);
}

nbody_status nbody_force_jerk_f64(int64_t n, const double *pos64, const double *vel64,
                                  const float *mass, float eps, double *acc, double *jerk,
                                  double *pot, const nbody_opts *opts, void *stream) {
    clear_error();
    nbody_opts o = resolve_opts(opts);
    nbody_status st = check_jerk(n, pos64, vel64, mass, eps, acc, jerk, o);
    if (st) return st;
    if (o.centre == NBODY_CENTRE_TILE)
        return set_error(NBODY_EUNSUPPORTED, "the jerk path supports NBODY_CENTRE_NONE and _SYSTEM");
    if (misaligned(pos64) || misaligned(vel64) || misaligned(mass) || misaligned(acc) ||
        misaligned(jerk) || misaligned(pot))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    if (n == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_JERK, n, o.precision, o, &cfg))) return st;
    void *ws = nullptr;
    if ((st = get_workspace(o, jerk_f64_bytes(n, cfg, o.precision), s, &ws))) return st;
    const JerkScratch w = jerk_f64_layout(ws, n, cfg, o.precision);
    if (o.centre == NBODY_CENTRE_SYSTEM) {
        // Positions relative to the FP64 mean position, velocities relative to the FP64
        // mean velocity: differences of the shifted values are what the pairs need.
        if ((st = launch_centre(n, pos64, w.cx, w.cscratch, s))) return st;
        if ((st = launch_convert(n, pos64, w.cx, w.x32, s))) return st;
        if ((st = launch_centre(n, vel64, w.cv, w.cscratch, s))) return st;
        if ((st = launch_convert(n, vel64, w.cv, w.v32, s))) return st;
    } else {
        if ((st = launch_convert(n, pos64, nullptr, w.x32, s))) return st;
        if ((st = launch_convert(n, vel64, nullptr, w.v32, s))) return st;
    }
    return jerk_core(n, w.x32, w.v32, mass, eps, acc, jerk, pot, o, cfg, w.part, s);
}

}  // extern "C"
