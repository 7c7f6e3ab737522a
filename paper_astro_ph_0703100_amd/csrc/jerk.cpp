// Host entry points of the force-jerk-potential path: argument checks, launch shape,
// scratch, and (for FP64 state) the reference centres of positions and velocities;
// and the fourth-order Hermite integrator built on it (eager and captured in a graph).
#include <cfloat>
#include <cmath>
#include <new>

#include "nbody_internal.h"
#include "tuning.h"

namespace nbody {
namespace {

constexpr int kJerkOut = 7;

size_t jerk_partial_bytes(const TileCfg &c, int precision) {
    const size_t words = (size_t)(precision == NBODY_PLAIN ? 1 : 2) * kJerkOut;
    return align_up((size_t)c.nseg * words * (size_t)c.npad * 4, 256);
}

// FP64-state scratch: partial sums, FP32 relative positions and velocities [3][n] each
// (or, with per-i-tile centres, the tile centres of each), and the partials of the
// system-mean reductions.
struct JerkScratch {
    void *part;
    float *x32, *v32;
    double *cscratch;
};

size_t jerk_f64_bytes(int64_t n, const TileCfg &c, int precision) {
    return jerk_partial_bytes(c, precision) + 2 * align_up(sizeof(float) * 3 * (size_t)n, 256) +
           align_up(centre_scratch_bytes(), 256);
}

JerkScratch jerk_f64_layout(void *ws, int64_t n, const TileCfg &c, int precision) {
    char *b = static_cast<char *>(ws);
    const size_t pb = jerk_partial_bytes(c, precision);
    const size_t xb = align_up(sizeof(float) * 3 * (size_t)n, 256);
    JerkScratch r;
    r.part = b;
    r.x32 = reinterpret_cast<float *>(b + pb);
    r.v32 = reinterpret_cast<float *>(b + pb + xb);
    r.cscratch = reinterpret_cast<double *>(b + pb + 2 * xb);
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
    JerkFinalizeArgs fa{part, cfg.nseg, cfg.npad, (int)n, mass, eps, o.self_pot,
                        acc,  jerk,     pot};
    return launch_jerk_finalize(o.precision, fa, s);
}

// One evaluation from FP64 state: centres and FP32 conversion per opts.centre, then
// the pair kernel and the FP64 finalize.
nbody_status jerk_f64_core(int64_t n, const double *pos64, const double *vel64, const float *mass,
                           float eps, double *acc, double *jerk, double *pot, const nbody_opts &o,
                           const TileCfg &cfg, const JerkScratch &w, hipStream_t s) {
    nbody_status st;
    if (o.centre == NBODY_CENTRE_TILE) {
        // Per-i-tile mean positions and velocities (3 doubles per tile each, in the FP32
        // areas this mode does not use); the pair kernel converts as it loads.
        const int itile = kTPB * cfg.ipl;
        double *cx = reinterpret_cast<double *>(w.x32);
        double *cv = reinterpret_cast<double *>(w.v32);
        if ((st = launch_tile_centres(n, itile, pos64, cx, s))) return st;
        if ((st = launch_tile_centres(n, itile, vel64, cv, s))) return st;
        const float e2 = eps * eps;
        JerkTileArgs a{pos64, pos64 + n, pos64 + 2 * n, mass, vel64, vel64 + n, vel64 + 2 * n,
                       (int)n, cfg.seg_len, e2, w.part, cfg.npad, cx, cv, itile};
        if ((st = launch_jerk_tile(cfg, o.precision, pot != nullptr, a, s))) return st;
        JerkFinalizeArgs fa{w.part, cfg.nseg, cfg.npad, (int)n, mass, eps, o.self_pot,
                            acc,    jerk,     pot};
        return launch_jerk_finalize(o.precision, fa, s);
    }
    if (o.centre == NBODY_CENTRE_SYSTEM) {
        // Positions relative to the FP64 mean position, velocities relative to the FP64
        // mean velocity: differences of the shifted values are what the pairs need.
        if ((st = launch_centred_convert(n, pos64, w.cscratch, w.x32, s))) return st;
        if ((st = launch_centred_convert(n, vel64, w.cscratch, w.v32, s))) return st;
    } else {
        if ((st = launch_convert(n, pos64, nullptr, w.x32, s))) return st;
        if ((st = launch_convert(n, vel64, nullptr, w.v32, s))) return st;
    }
    return jerk_core(n, w.x32, w.v32, mass, eps, acc, jerk, pot, o, cfg, w.part, s);
}

// Hermite scratch: the evaluation's scratch, then predicted state and new (a, j).
struct HermiteScratch {
    JerkScratch eval;
    double *xp, *vp, *a1, *j1;
};

size_t hermite_bytes(int64_t n, const TileCfg &c, int precision) {
    return jerk_f64_bytes(n, c, precision) + 4 * align_up(sizeof(double) * 3 * (size_t)n, 256);
}

HermiteScratch hermite_layout(void *ws, int64_t n, const TileCfg &c, int precision) {
    HermiteScratch h;
    h.eval = jerk_f64_layout(ws, n, c, precision);
    char *b = static_cast<char *>(ws) + jerk_f64_bytes(n, c, precision);
    const size_t vb = align_up(sizeof(double) * 3 * (size_t)n, 256);
    h.xp = reinterpret_cast<double *>(b);
    h.vp = reinterpret_cast<double *>(b + vb);
    h.a1 = reinterpret_cast<double *>(b + 2 * vb);
    h.j1 = reinterpret_cast<double *>(b + 3 * vb);
    return h;
}

nbody_status check_hermite(int64_t n, const double *x, const double *v, const float *m, float eps,
                           double dt, int32_t nsteps, const double *acc, const double *jerk,
                           const nbody_opts &o) {
    nbody_status st = check_jerk(n, x, v, m, eps, acc, jerk, o);
    if (st) return st;
    if (nsteps < 0) return set_error(NBODY_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(dt)) return set_error(NBODY_EINVAL, "dt must be finite");
    if (misaligned(x) || misaligned(v) || misaligned(m) || misaligned(acc) || misaligned(jerk))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    return NBODY_OK;
}

// Enqueues nsteps predictor-evaluate-corrector steps (after the initial evaluation if
// `init`); (acc, jerk) must hold a and j at (x, v) when a step starts.
nbody_status enqueue_hermite(int64_t n, double *x, double *v, const float *m, float eps, double dt,
                             int32_t nsteps, double *acc, double *jerk, bool init,
                             const nbody_opts &o, const TileCfg &cfg, const HermiteScratch &h,
                             hipStream_t s) {
    nbody_status st;
    if (init && (st = jerk_f64_core(n, x, v, m, eps, acc, jerk, nullptr, o, cfg, h.eval, s)))
        return st;
    for (int32_t t = 0; t < nsteps; ++t) {
        if ((st = launch_hermite_predict(n, x, v, acc, jerk, dt, h.xp, h.vp, s))) return st;
        if ((st = jerk_f64_core(n, h.xp, h.vp, m, eps, h.a1, h.j1, nullptr, o, cfg, h.eval, s)))
            return st;
        if ((st = launch_hermite_correct(n, x, v, acc, jerk, h.a1, h.j1, dt, s))) return st;
    }
    return NBODY_OK;
}

}  // namespace
}  // namespace nbody

using namespace nbody;

extern "C" {

size_t nbody_workspace_size_jerk(int64_t n, const nbody_opts *opts) {
    nbody_opts o = resolve_opts(opts);
    if (n <= 0) return 0;
    TileCfg c;
    if (choose_cfg(KERNEL_JERK, n, o.precision, o, &c, 0) != NBODY_OK) return 0;
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
    if ((st = choose_cfg(KERNEL_JERK, n, o.precision, o, &cfg, 0))) return st;
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
    if (misaligned(pos64) || misaligned(vel64) || misaligned(mass) || misaligned(acc) ||
        misaligned(jerk) || misaligned(pot))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    if (n == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_JERK, n, o.precision, o, &cfg, 0))) return st;
    void *ws = nullptr;
    if ((st = get_workspace(o, jerk_f64_bytes(n, cfg, o.precision), s, &ws))) return st;
    return jerk_f64_core(n, pos64, vel64, mass, eps, acc, jerk, pot, o, cfg,
                         jerk_f64_layout(ws, n, cfg, o.precision), s);
}

nbody_status nbody_force_jerk_ij(int64_t ni, const float *pos_i, const float *vel_i, int64_t nj,
                                 const float *pos_j, const float *vel_j, const float *mass_j,
                                 float eps, double *acc, double *jerk, double *pot,
                                 const nbody_opts *opts, void *stream) {
    clear_error();
    nbody_opts o = resolve_opts(opts);
    if (ni < 0 || ni > INT32_MAX / 2 || nj < 0 || nj > INT32_MAX / 2)
        return set_error(NBODY_EINVAL, "ni and nj must be in [0, 2^30)");
    if (ni > 0 && (!pos_i || !vel_i || !acc || !jerk))
        return set_error(NBODY_EINVAL, "pos_i, vel_i, acc and jerk must not be NULL");
    if (ni > 0 && nj > 0 && (!pos_j || !vel_j || !mass_j))
        return set_error(NBODY_EINVAL, "pos_j, vel_j and mass_j must not be NULL");
    const float e2 = eps * eps;
    if (!std::isfinite(eps) || !(eps >= 0.0f) || !std::isfinite(e2) || (eps > 0.0f && !(e2 >= FLT_MIN)))
        return set_error(NBODY_EINVAL, "eps must be finite and >= 0 with eps^2 zero or a normal float");
    if (o.precision < NBODY_PLAIN || o.precision > NBODY_COMP)
        return set_error(NBODY_EINVAL, "precision must be NBODY_PLAIN, NBODY_FP64RED or NBODY_COMP");
    if (misaligned(pos_i) || misaligned(vel_i) || misaligned(pos_j) || misaligned(vel_j) ||
        misaligned(mass_j) || misaligned(acc) || misaligned(jerk) || misaligned(pot))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    if (ni == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    nbody_status st;
    if (nj == 0) {
        if ((st = launch_fill_f64(3 * ni, acc, 0.0, s))) return st;
        if ((st = launch_fill_f64(3 * ni, jerk, 0.0, s))) return st;
        return pot ? launch_fill_f64(ni, pot, 0.0, s) : NBODY_OK;
    }
    TileCfg cfg;
    if ((st = choose_cfg_ij(KERNEL_JERK, ni, nj, o.precision, o, &cfg, 0))) return st;
    void *ws = nullptr;
    if ((st = get_workspace(o, jerk_partial_bytes(cfg, o.precision), s, &ws))) return st;
    JerkIJArgs a{pos_i, pos_i + ni, pos_i + 2 * ni, vel_i, vel_i + ni, vel_i + 2 * ni,
                 pos_j, pos_j + nj, pos_j + 2 * nj, mass_j, vel_j, vel_j + nj, vel_j + 2 * nj,
                 (int)ni, (int)nj, cfg.seg_len, e2, ws, cfg.npad};
    if ((st = launch_jerk_ij(cfg, o.precision, pot != nullptr, a, s))) return st;
    JerkFinalizeArgs fa{ws, cfg.nseg, cfg.npad, (int)ni, nullptr, eps, 0, acc, jerk, pot};
    return launch_jerk_finalize(o.precision, fa, s);
}

size_t nbody_workspace_size_jerk_ij(int64_t ni, int64_t nj, const nbody_opts *opts) {
    nbody_opts o = resolve_opts(opts);
    if (ni <= 0 || nj <= 0) return 0;
    TileCfg c;
    if (choose_cfg_ij(KERNEL_JERK, ni, nj, o.precision, o, &c, 0) != NBODY_OK) return 0;
    return jerk_partial_bytes(c, o.precision);
}

size_t nbody_workspace_size_hermite(int64_t n, const nbody_opts *opts) {
    nbody_opts o = resolve_opts(opts);
    if (n <= 0) return 0;
    TileCfg c;
    if (choose_cfg(KERNEL_JERK, n, o.precision, o, &c, 0) != NBODY_OK) return 0;
    return hermite_bytes(n, c, o.precision);
}

nbody_status nbody_hermite(int64_t n, double *pos64, double *vel64, const float *mass, float eps,
                           double dt, int32_t nsteps, double *acc, double *jerk, int32_t flags,
                           const nbody_opts *opts, void *stream) {
    clear_error();
    nbody_opts o = resolve_opts(opts);
    nbody_status st = check_hermite(n, pos64, vel64, mass, eps, dt, nsteps, acc, jerk, o);
    if (st) return st;
    if (flags & ~NBODY_LF_INIT_ACC) return set_error(NBODY_EINVAL, "unknown flags");
    if (n == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_JERK, n, o.precision, o, &cfg, 0))) return st;
    void *ws = nullptr;
    if ((st = get_workspace(o, hermite_bytes(n, cfg, o.precision), s, &ws))) return st;
    return enqueue_hermite(n, pos64, vel64, mass, eps, dt, nsteps, acc, jerk,
                           (flags & NBODY_LF_INIT_ACC) != 0, o, cfg,
                           hermite_layout(ws, n, cfg, o.precision), s);
}

nbody_status nbody_graph_create_hermite(int64_t n, double *pos64, double *vel64, const float *mass,
                                        float eps, double dt, int32_t nsteps, double *acc,
                                        double *jerk, const nbody_opts *opts, void *stream,
                                        nbody_graph **out) {
    clear_error();
    if (!out) return set_error(NBODY_EINVAL, "out must not be NULL");
    *out = nullptr;
    nbody_opts o = resolve_opts(opts);
    nbody_status st = check_hermite(n, pos64, vel64, mass, eps, dt, nsteps, acc, jerk, o);
    if (st) return st;
    if (n == 0 || nsteps == 0) return set_error(NBODY_EINVAL, "graph needs n > 0 and nsteps > 0");
    hipStream_t user = static_cast<hipStream_t>(stream);
    if (stream_capturing(user)) return set_error(NBODY_ECAPTURE, "stream is already capturing");
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_JERK, n, o.precision, o, &cfg, 0))) return st;
    nbody_graph *g = new (std::nothrow) nbody_graph;
    if (!g) return set_error(NBODY_ENOMEM, "out of host memory");
    auto fail = [&](nbody_status code) {
        if (g->exec) (void)hipGraphExecDestroy(g->exec);
        if (g->graph) (void)hipGraphDestroy(g->graph);
        if (g->workspace) (void)hipFree(g->workspace);
        delete g;
        return code;
    };
    hipError_t e = hipGetDevice(&g->device);
    if (e != hipSuccess) return fail(hip_error(e, "hipGetDevice"));
    // The graph owns its scratch: a shared cache could be reallocated under it.
    const size_t need = hermite_bytes(n, cfg, o.precision);
    if ((e = hipMalloc(&g->workspace, need)) != hipSuccess) {
        g->workspace = nullptr;
        return fail(hip_error(e, "hipMalloc(graph workspace)"));
    }
    const HermiteScratch lay = hermite_layout(g->workspace, n, cfg, o.precision);
    st = capture_graph(g, [&](hipStream_t cs) {
        return enqueue_hermite(n, pos64, vel64, mass, eps, dt, nsteps, acc, jerk, false, o, cfg,
                               lay, cs);
    });
    if (st) return fail(st);
    *out = g;
    return NBODY_OK;
}

}  // extern "C"
