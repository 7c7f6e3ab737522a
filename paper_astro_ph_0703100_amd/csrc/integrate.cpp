// Kick-drift-kick leapfrog on FP64 state and its capture into HIP graphs.
//
// One step:  v += (dt/2) a(x);  x += dt v;  a = a(x);  v += (dt/2) a
// The first kick and the drift are one element-wise kernel; the force evaluation is
// the FP64-position path (centre, FP32 conversion, pair kernel, FP64 finalize) and
// the second kick is fused into the finalize.  a(x) carries over from one step to the
// next, so each step costs one force evaluation.
#include <cmath>
#include <functional>
#include <new>

#include "nbody_internal.h"
#include "tuning.h"

namespace nbody {
namespace {

nbody_status check_leapfrog(int64_t n, const double *x, const double *v, const float *m, float eps,
                            double dt, int32_t nsteps, const double *acc, const nbody_opts &o,
                            const double *pot = nullptr, const double *traj = nullptr) {
    nbody_status st = check_common(n, x, m, eps, acc, o);
    if (st) return st;
    if (n > 0 && !v) return set_error(NBODY_EINVAL, "vel must not be NULL");
    if (nsteps < 0) return set_error(NBODY_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(dt))
        return set_error(NBODY_EINVAL, "dt must be finite");
    if (misaligned(x) || misaligned(v) || misaligned(m) || misaligned(acc) || misaligned(pot) ||
        misaligned(traj))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    return NBODY_OK;
}

// Enqueues `nsteps` KDK steps (plus the initial force evaluation if `init`).
nbody_status enqueue_steps(int64_t n, double *x, double *v, const float *m, float eps, double dt,
                           int32_t nsteps, double *acc, double *pot, double *traj, bool init,
                           const nbody_opts &o, const TileCfg &cfg, const F64Scratch &ws,
                           hipStream_t s) {
    nbody_status st;
    const size_t n3 = 3 * (size_t)n;
    if (init || (nsteps == 0 && pot)) {
        if ((st = force_f64_core(n, x, m, eps, acc, nsteps == 0 ? pot : nullptr, o, cfg, ws,
                                 nullptr, 0.0, s)))
            return st;
    }
    if (traj && (st = launch_copy_f64((int64_t)n3, x, traj, s))) return st;
    for (int32_t t = 0; t < nsteps; ++t) {
        double *checkpoint = traj ? traj + (size_t)(t + 1) * n3 : nullptr;
        // With the system centre, the kick-drift also sums the new positions for it.
        const bool fused = o.centre == NBODY_CENTRE_SYSTEM;
        st = fused ? launch_kick_drift_centre(n, x, v, acc, 0.5 * dt, dt, checkpoint,
                                              ws.centre_scratch, s)
                   : launch_kick_drift(n, x, v, acc, 0.5 * dt, dt, s, checkpoint);
        if (st) return st;
        if ((st = force_f64_core(n, x, m, eps, acc, t + 1 == nsteps ? pot : nullptr, o, cfg, ws, v,
                                 0.5 * dt, s, fused)))
            return st;
    }
    return NBODY_OK;
}

}  // namespace

nbody_status capture_graph(nbody_graph *g, const std::function<nbody_status(hipStream_t)> &body) {
    // Capture on a private stream (the null stream cannot be captured); the launches
    // are recorded, not run.
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_error(e, "hipStreamCreate");
    if ((e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        (void)hipStreamDestroy(cs);
        return hip_error(e, "hipStreamBeginCapture");
    }
    nbody_status st = body(cs);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(cs, &graph);
    (void)hipStreamDestroy(cs);
    g->graph = graph;
    if (st) return st;
    if (e != hipSuccess) return hip_error(e, "hipStreamEndCapture");
    if ((e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0)) != hipSuccess) {
        g->exec = nullptr;
        return hip_error(e, "hipGraphInstantiate");
    }
    return NBODY_OK;
}

}  // namespace nbody

using namespace nbody;

extern "C" {

nbody_status nbody_leapfrog(int64_t n, double *pos64, double *vel64, const float *mass, float eps,
                            double dt, int32_t nsteps, double *acc, double *pot, double *traj,
                            int32_t flags, const nbody_opts *opts, void *stream) {
    clear_error();
    nbody_opts o = resolve_opts(opts);
    nbody_status st = check_leapfrog(n, pos64, vel64, mass, eps, dt, nsteps, acc, o, pot, traj);
    if (st) return st;
    if (flags & ~NBODY_LF_INIT_ACC) return set_error(NBODY_EINVAL, "unknown flags");
    if (n == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_FORCE, n, o.precision, o, &cfg, force_engines(o)))) return st;
    void *ws = nullptr;
    if ((st = get_workspace(o, f64_scratch_bytes(n, cfg, o.precision), s, &ws))) return st;
    return enqueue_steps(n, pos64, vel64, mass, eps, dt, nsteps, acc, pot, traj,
                         (flags & NBODY_LF_INIT_ACC) != 0, o, cfg,
                         f64_scratch_layout(ws, n, cfg, o.precision), s);
}

nbody_status nbody_graph_create_leapfrog(int64_t n, double *pos64, double *vel64,
                                         const float *mass, float eps, double dt, int32_t nsteps,
                                         double *acc, double *pot, const nbody_opts *opts,
                                         void *stream, nbody_graph **out) {
    clear_error();
    if (!out) return set_error(NBODY_EINVAL, "out must not be NULL");
    *out = nullptr;
    nbody_opts o = resolve_opts(opts);
    nbody_status st = check_leapfrog(n, pos64, vel64, mass, eps, dt, nsteps, acc, o, pot);
    if (st) return st;
    if (n == 0 || nsteps == 0) return set_error(NBODY_EINVAL, "graph needs n > 0 and nsteps > 0");
    hipStream_t user = static_cast<hipStream_t>(stream);
    if (stream_capturing(user)) return set_error(NBODY_ECAPTURE, "stream is already capturing");
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_FORCE, n, o.precision, o, &cfg, force_engines(o)))) return st;

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
    const size_t need = f64_scratch_bytes(n, cfg, o.precision);
    if ((e = hipMalloc(&g->workspace, need)) != hipSuccess) {
        g->workspace = nullptr;
        return fail(hip_error(e, "hipMalloc(graph workspace)"));
    }
    o.workspace = g->workspace;
    o.workspace_bytes = need;

    const F64Scratch lay = f64_scratch_layout(g->workspace, n, cfg, o.precision);
    st = capture_graph(g, [&](hipStream_t cs) {
        return enqueue_steps(n, pos64, vel64, mass, eps, dt, nsteps, acc, pot, nullptr, false, o,
                             cfg, lay, cs);
    });
    if (st) return fail(st);
    *out = g;
    return NBODY_OK;
}

nbody_status nbody_graph_launch(nbody_graph *g, void *stream) {
    clear_error();
    if (!g || !g->exec) return set_error(NBODY_EINVAL, "invalid graph");
    NBODY_HIP_CHECK(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return NBODY_OK;
}

void nbody_graph_destroy(nbody_graph *g) {
    if (!g) return;
    // Let launched replays finish before their scratch is released.
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->workspace) (void)hipFree(g->workspace);
    delete g;
}

}  // extern "C"
