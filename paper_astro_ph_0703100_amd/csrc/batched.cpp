// Ragged batches of independent systems: the plan (work items, partial-sum layout,
// device tables and scratch, built once from the host offsets) and the batched force
// and leapfrog entry points.
//
// Work items: each system with N_k particles is cut into ceil(N_k / (256 IPL))
// i-tiles and S_k j-segments of about kItemJ j's; an item is one (i-tile, segment)
// pair of one system.  Items are sorted by decreasing cost (i-lanes x j's, including
// padding) and handed to the persistent kernel's blocks through an atomic ticket, so
// large systems start first and small ones fill the tail.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "nbody_internal.h"
#include "tuning.h"

struct nbody_plan {
    int device = 0;
    int nsys = 0;
    int64_t total = 0;
    nbody_opts opts{};
    int ipl = 4, jt = 256;
    int nitems = 0;
    int64_t padded_pairs = 0;
    int64_t pairs = 0;
    // device tables
    nbody::BatchItem *items = nullptr;
    int64_t *offsets = nullptr;
    int32_t *sys_of = nullptr;
    int64_t *part_base = nullptr;
    int32_t *npad = nullptr;
    int32_t *nseg = nullptr;
    unsigned int *counter = nullptr;
    // scratch
    void *part = nullptr;
    size_t part_bytes = 0;
    float *x32 = nullptr;
    double *centre = nullptr;
    int grid[2] = {0, 0};  // persistent blocks, without / with the potential
};

namespace nbody {
namespace {

constexpr int64_t kItemJ = 4096;  // target j's per work item

void free_plan(nbody_plan *p) {
    if (!p) return;
    void *ptrs[] = {p->items, p->offsets, p->sys_of, p->part_base, p->npad,
                    p->nseg,  p->counter, p->part,   p->x32,       p->centre};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete p;
}

template <typename T>
nbody_status dev_copy(T **dst, const std::vector<T> &src) {
    const size_t bytes = sizeof(T) * (src.empty() ? 1 : src.size());
    hipError_t e = hipMalloc(reinterpret_cast<void **>(dst), bytes);
    if (e != hipSuccess) {
        *dst = nullptr;
        return hip_error(e, "hipMalloc(plan)");
    }
    if (!src.empty()) {
        e = hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_error(e, "hipMemcpy(plan)");
    }
    return NBODY_OK;
}

// Persistent grid for one kernel variant: resident blocks per CU x CUs.
nbody_status persistent_grid(const nbody_plan *p, bool with_pot, int *grid) {
    const void *fn = nullptr;
    nbody_status st = batched_pair_kernel(p->ipl, p->jt, p->opts.precision, with_pot, &fn);
    if (st) return st;
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kTPB, 0);
    if (e != hipSuccess) return hip_error(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (per_cu < 1) per_cu = 1;
    *grid = per_cu * device_info().cus;
    return NBODY_OK;
}

nbody_status check_plan_call(const nbody_plan *p, const void *pos, const float *mass,
                             const float *eps, const double *acc) {
    if (!p) return set_error(NBODY_EINVAL, "plan must not be NULL");
    if (p->total > 0 && (!pos || !mass || !eps || !acc))
        return set_error(NBODY_EINVAL, "pos, mass, eps and acc must not be NULL");
    int dev = 0;
    NBODY_HIP_CHECK(hipGetDevice(&dev));
    if (dev != p->device) return set_error(NBODY_EINVAL, "plan was created on another device");
    return NBODY_OK;
}

// Persistent pair kernel + batched finalize on FP32 positions.
nbody_status batched_core(const nbody_plan *p, const float *pos, const float *mass,
                          const float *eps, double *acc, double *pot, double *kick_v,
                          double kick_h, hipStream_t s) {
    const bool with_pot = pot != nullptr;
    const int grid = p->grid[with_pot];
    const int64_t n = p->total;
    PairArgs pa{pos, pos + n, pos + 2 * n, mass, (int)n, 0, 0.0f, p->part, 0};
    BatchSched sc{p->items, p->nitems, p->counter, eps, p->part};
    nbody_status st = launch_batched_pair(p->ipl, p->jt, p->opts.precision, with_pot, grid, pa, sc, s);
    if (st) return st;
    BatchFinalizeArgs fa{p->part, n,   p->sys_of, p->offsets, p->part_base, p->npad, p->nseg,
                         acc,     pot, kick_v,    kick_h};
    return launch_batched_finalize(p->opts.precision, fa, s);
}

nbody_status batched_f64_core(const nbody_plan *p, const double *pos64, const float *mass,
                              const float *eps, double *acc, double *pot, double *kick_v,
                              double kick_h, hipStream_t s) {
    nbody_status st;
    const double *cen = nullptr;
    if (p->opts.centre == NBODY_CENTRE_SYSTEM) {
        if ((st = launch_system_centres(p->nsys, p->offsets, p->total, pos64, p->centre, s))) return st;
        cen = p->centre;
    }
    if ((st = launch_batched_convert(p->total, pos64, p->sys_of, cen, p->x32, s))) return st;
    return batched_core(p, p->x32, mass, eps, acc, pot, kick_v, kick_h, s);
}

nbody_status enqueue_batched_steps(const nbody_plan *p, double *x, double *v, const float *m,
                                   const float *eps, double dt, int32_t nsteps, double *acc,
                                   double *pot, bool init, hipStream_t s) {
    nbody_status st;
    if (init || (nsteps == 0 && pot))
        if ((st = batched_f64_core(p, x, m, eps, acc, nsteps == 0 ? pot : nullptr, nullptr, 0.0, s)))
            return st;
    for (int32_t t = 0; t < nsteps; ++t) {
        if ((st = launch_kick_drift(p->total, x, v, acc, 0.5 * dt, dt, s))) return st;
        if ((st = batched_f64_core(p, x, m, eps, acc, t + 1 == nsteps ? pot : nullptr, v, 0.5 * dt, s)))
            return st;
    }
    return NBODY_OK;
}

}  // namespace
}  // namespace nbody

using namespace nbody;

extern "C" {

nbody_status nbody_plan_create_batched(int32_t nsys, const int64_t *h_offsets,
                                       const nbody_opts *opts, nbody_plan **out) {
    clear_error();
    if (!out) return set_error(NBODY_EINVAL, "out must not be NULL");
    *out = nullptr;
    if (nsys < 0) return set_error(NBODY_EINVAL, "nsys must be >= 0");
    if (nsys > 0 && !h_offsets) return set_error(NBODY_EINVAL, "offsets must not be NULL");
    nbody_opts o = resolve_opts(opts);
    if (o.precision < NBODY_PLAIN || o.precision > NBODY_COMP)
        return set_error(NBODY_EINVAL, "precision must be NBODY_PLAIN, NBODY_FP64RED or NBODY_COMP");
    if (o.centre != NBODY_CENTRE_NONE && o.centre != NBODY_CENTRE_SYSTEM)
        return set_error(NBODY_EUNSUPPORTED, "batched plans support NBODY_CENTRE_NONE and _SYSTEM");
    if (o.self_pot != 0) return set_error(NBODY_EUNSUPPORTED, "batched plans exclude the self term");
    if (o.workspace) return set_error(NBODY_EINVAL, "a plan owns its scratch; opts->workspace must be NULL");
    if (o.jlanes > 1) return set_error(NBODY_EUNSUPPORTED, "batched plans use the grid engine (jlanes 0 or 1)");
    if (o.jlanes < 0) return set_error(NBODY_EINVAL, "jlanes must be >= 0");
    if (o.symmetric < 0 || o.symmetric > 2)
        return set_error(NBODY_EINVAL, "symmetric must be 0 (tuned), 1 (off) or 2 (on)");
    if (o.symmetric == 2)
        return set_error(NBODY_EUNSUPPORTED, "batched plans use the grid engine (symmetric 0 or 1)");
    if (nsys > 0 && h_offsets[0] != 0) return set_error(NBODY_EINVAL, "offsets[0] must be 0");
    for (int32_t k = 0; k < nsys; ++k)
        if (h_offsets[k + 1] < h_offsets[k])
            return set_error(NBODY_EINVAL, "offsets must be non-decreasing");
    const int64_t total = nsys > 0 ? h_offsets[nsys] : 0;
    if (total > INT32_MAX / 2) return set_error(NBODY_EINVAL, "total particles must be < 2^30");

    TuneEntry te = tuned_shape(KERNEL_BATCHED, o.precision, total / std::max<int64_t>(1, nsys), 0);
    const int ipl = o.ipl ? o.ipl : te.ipl;
    const int jt = o.jtile ? o.jtile : te.jt;
    if (!(ipl == 1 || ipl == 2 || ipl == 4 || ipl == 8))
        return set_error(NBODY_EINVAL, "ipl must be 1, 2, 4 or 8");
    if (!(jt == 64 || jt == 128 || jt == 256 || jt == 512))
        return set_error(NBODY_EINVAL, "jtile must be 64, 128, 256 or 512");

    nbody_plan *p = new (std::nothrow) nbody_plan;
    if (!p) return set_error(NBODY_ENOMEM, "out of host memory");
    p->nsys = nsys;
    p->total = total;
    p->opts = o;
    p->ipl = ipl;
    p->jt = jt;
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        free_plan(p);
        return hip_error(e, "hipGetDevice");
    }

    // Items and the partial-sum layout.
    const int64_t itile = (int64_t)kTPB * ipl;
    const int wo = 4 * (o.precision == NBODY_PLAIN ? 1 : 2);  // words per (i, segment)
    const int64_t tiles_per_seg = std::max<int64_t>(1, kItemJ / jt);
    std::vector<BatchItem> items;
    std::vector<int64_t> cost, base(std::max(nsys, 1)), offs(h_offsets, h_offsets + nsys + 1);
    std::vector<int32_t> npad(std::max(nsys, 1)), nseg(std::max(nsys, 1)), sys_of((size_t)total);
    int64_t words = 0;
    for (int32_t k = 0; k < nsys; ++k) {
        const int64_t off = h_offsets[k], n = h_offsets[k + 1] - off;
        for (int64_t q = 0; q < n; ++q) sys_of[(size_t)(off + q)] = k;
        base[k] = words;
        if (n == 0) {
            npad[k] = 0;
            nseg[k] = 0;
            continue;
        }
        const int64_t t = (n + itile - 1) / itile;
        const int64_t jtiles = (n + jt - 1) / jt;
        int64_t segs = (jtiles + tiles_per_seg - 1) / tiles_per_seg;
        const int64_t per = (jtiles + segs - 1) / segs;
        segs = (jtiles + per - 1) / per;
        const int64_t seg_len = per * jt;
        npad[k] = (int32_t)(t * itile);
        nseg[k] = (int32_t)segs;
        for (int64_t ti = 0; ti < t; ++ti)
            for (int64_t si = 0; si < segs; ++si) {
                BatchItem w;
                w.sys = k;
                w.i0 = (int32_t)(off + ti * itile);
                w.ni = (int32_t)std::min(itile, n - ti * itile);
                w.j0 = (int32_t)(off + si * seg_len);
                w.nj = (int32_t)std::min(seg_len, n - si * seg_len);
                w.col0 = (int32_t)(ti * itile);
                w.part = words + si * wo * (t * itile);
                w.npad = (int32_t)(t * itile);
                w.pad_ = 0;
                items.push_back(w);
                cost.push_back(itile * ((w.nj + jt - 1) / jt) * jt);
                p->padded_pairs += cost.back();
            }
        words += segs * wo * t * itile;
        p->pairs += n * n;
    }
    // Decreasing cost; ties in creation order (system, i-tile, segment).
    std::vector<int32_t> order(items.size());
    for (size_t q = 0; q < order.size(); ++q) order[q] = (int32_t)q;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost[a] > cost[b]; });
    std::vector<BatchItem> sorted(items.size());
    for (size_t q = 0; q < order.size(); ++q) sorted[q] = items[order[q]];
    p->nitems = (int)sorted.size();

    nbody_status st = NBODY_OK;
    auto bail = [&](nbody_status code) {
        free_plan(p);
        return code;
    };
    if ((st = dev_copy(&p->items, sorted))) return bail(st);
    if ((st = dev_copy(&p->offsets, offs))) return bail(st);
    if ((st = dev_copy(&p->sys_of, sys_of))) return bail(st);
    if ((st = dev_copy(&p->part_base, base))) return bail(st);
    if ((st = dev_copy(&p->npad, npad))) return bail(st);
    if ((st = dev_copy(&p->nseg, nseg))) return bail(st);
    if ((st = dev_copy(&p->counter, std::vector<unsigned int>(1, 0u)))) return bail(st);
    p->part_bytes = (size_t)std::max<int64_t>(words, 1) * 4;
    if ((e = hipMalloc(&p->part, p->part_bytes)) != hipSuccess) {
        p->part = nullptr;
        return bail(hip_error(e, "hipMalloc(plan partials)"));
    }
    if ((e = hipMalloc(reinterpret_cast<void **>(&p->x32), sizeof(float) * 3 * std::max<int64_t>(total, 1))) != hipSuccess) {
        p->x32 = nullptr;
        return bail(hip_error(e, "hipMalloc(plan positions)"));
    }
    if ((e = hipMalloc(reinterpret_cast<void **>(&p->centre), sizeof(double) * 3 * std::max(nsys, 1))) != hipSuccess) {
        p->centre = nullptr;
        return bail(hip_error(e, "hipMalloc(plan centres)"));
    }
    for (int pot = 0; pot < 2; ++pot)
        if ((st = persistent_grid(p, pot != 0, &p->grid[pot]))) return bail(st);
    *out = p;
    return NBODY_OK;
}

void nbody_plan_destroy(nbody_plan *plan) {
    if (!plan) return;
    (void)hipDeviceSynchronize();
    free_plan(plan);
}

nbody_status nbody_plan_info(const nbody_plan *plan, int64_t *info) {
    clear_error();
    if (!plan || !info) return set_error(NBODY_EINVAL, "plan and info must not be NULL");
    info[0] = plan->nsys;
    info[1] = plan->total;
    info[2] = plan->nitems;
    info[3] = plan->grid[1];
    info[4] = plan->pairs;
    info[5] = plan->padded_pairs;
    info[6] = plan->ipl;
    info[7] = plan->jt;
    return NBODY_OK;
}

nbody_status nbody_force_batched(const nbody_plan *plan, const float *pos, const float *mass,
                                 const float *eps, double *acc, double *pot, void *stream) {
    clear_error();
    nbody_status st = check_plan_call(plan, pos, mass, eps, acc);
    if (st) return st;
    if (misaligned(pos) || misaligned(mass) || misaligned(eps) || misaligned(acc) || misaligned(pot))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    if (plan->total == 0) return NBODY_OK;
    return batched_core(plan, pos, mass, eps, acc, pot, nullptr, 0.0, static_cast<hipStream_t>(stream));
}

nbody_status nbody_force_batched_f64(const nbody_plan *plan, const double *pos64, const float *mass,
                                     const float *eps, double *acc, double *pot, void *stream) {
    clear_error();
    nbody_status st = check_plan_call(plan, pos64, mass, eps, acc);
    if (st) return st;
    if (misaligned(pos64) || misaligned(mass) || misaligned(eps) || misaligned(acc) || misaligned(pot))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    if (plan->total == 0) return NBODY_OK;
    return batched_f64_core(plan, pos64, mass, eps, acc, pot, nullptr, 0.0,
                            static_cast<hipStream_t>(stream));
}

nbody_status nbody_leapfrog_batched(const nbody_plan *plan, double *pos64, double *vel64,
                                    const float *mass, const float *eps, double dt, int32_t nsteps,
                                    double *acc, double *pot, int32_t flags, void *stream) {
    clear_error();
    nbody_status st = check_plan_call(plan, pos64, mass, eps, acc);
    if (st) return st;
    if (plan->total > 0 && !vel64) return set_error(NBODY_EINVAL, "vel must not be NULL");
    if (nsteps < 0) return set_error(NBODY_EINVAL, "nsteps must be >= 0");
    if (!std::isfinite(dt)) return set_error(NBODY_EINVAL, "dt must be finite");
    if (flags & ~NBODY_LF_INIT_ACC) return set_error(NBODY_EINVAL, "unknown flags");
    if (misaligned(pos64) || misaligned(vel64) || misaligned(mass) || misaligned(eps) ||
        misaligned(acc) || misaligned(pot))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    if (plan->total == 0) return NBODY_OK;
    return enqueue_batched_steps(plan, pos64, vel64, mass, eps, dt, nsteps, acc, pot,
                                 (flags & NBODY_LF_INIT_ACC) != 0, static_cast<hipStream_t>(stream));
}

nbody_status nbody_graph_create_leapfrog_batched(const nbody_plan *plan, double *pos64,
                                                 double *vel64, const float *mass,
                                                 const float *eps, double dt, int32_t nsteps,
                                                 double *acc, double *pot, void *stream,
                                                 nbody_graph **out) {
    clear_error();
    if (!out) return set_error(NBODY_EINVAL, "out must not be NULL");
    *out = nullptr;
    nbody_status st = check_plan_call(plan, pos64, mass, eps, acc);
    if (st) return st;
    if (plan->total == 0 || nsteps <= 0)
        return set_error(NBODY_EINVAL, "graph needs particles and nsteps > 0");
    if (!vel64) return set_error(NBODY_EINVAL, "vel must not be NULL");
    if (!std::isfinite(dt)) return set_error(NBODY_EINVAL, "dt must be finite");
    if (stream_capturing(static_cast<hipStream_t>(stream)))
        return set_error(NBODY_ECAPTURE, "stream is already capturing");
    nbody_graph *g = new (std::nothrow) nbody_graph;
    if (!g) return set_error(NBODY_ENOMEM, "out of host memory");
    g->device = plan->device;
    st = capture_graph(g, [&](hipStream_t cs) {
        return enqueue_batched_steps(plan, pos64, vel64, mass, eps, dt, nsteps, acc, pot, false, cs);
    });
    if (st) {
        nbody_graph_destroy(g);
        return st;
    }
    *out = g;
    return NBODY_OK;
}

}  // extern "C"
