// nbody_force_noalloc: nbody_force_ex for callers that cannot allocate device memory.
// The grid engine's partial sums go to a file-scope device array of fixed size instead
// of a workspace; the split engine needs none.  No hipMalloc, hipFree or allocating
// library call is made on this path.
#include <mutex>
#include <string>

#include "nbody_internal.h"
#include "tuning.h"

namespace nbody {
namespace {

// Scratch for the grid engine's segment partial sums.  Every GPU the library runs on
// holds one copy for the life of the process.
constexpr size_t kStaticScratchBytes = NBODY_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch` on each device (set up once)

// Device address of this device's copy of `scratch` (the array's name is only a host
// stand-in).  Looked up once per device, with that device current.
nbody_status scratch_ptr(void **out) {
    int dev = 0;
    NBODY_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(NBODY_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        NBODY_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return set_error(NBODY_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return NBODY_OK;
}

}  // namespace
}  // namespace nbody

using namespace nbody;

extern "C" {

nbody_status nbody_force_noalloc(int64_t n, const float *pos, const float *mass, float eps,
                                 double *acc, double *pot, const nbody_opts *opts, void *stream) {
    clear_error();
    nbody_opts o = resolve_opts(opts);
    nbody_status st = check_force_f32(n, pos, mass, eps, acc, pot, o);
    if (st) return st;
    if (o.workspace) return set_error(NBODY_EINVAL, "nbody_force_noalloc takes no workspace");
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_FORCE, n, o.precision, o, &cfg, kEngineSplit | kEngineSym))) return st;
    size_t need = partial_bytes(cfg, o.precision);
    if (need > kStaticScratchBytes && cfg.sym && o.symmetric == 0) {
        // The symmetric engine's j-side sums grow as n^2: the grid engine instead.
        o.symmetric = 1;
        if ((st = choose_cfg(KERNEL_FORCE, n, o.precision, o, &cfg, kEngineSplit))) return st;
        need = partial_bytes(cfg, o.precision);
    }
    if (need > kStaticScratchBytes && cfg.jl == 1 && !cfg.sym && o.nseg == 0 && cfg.nseg > 1) {
        // Fewer j-segments (longer ones) until the partial sums fit.
        const size_t per_seg = need / cfg.nseg;  // at most 256 bytes of alignment over
        const int64_t fit = per_seg ? (int64_t)((kStaticScratchBytes - 256) / per_seg) : 0;
        if (fit >= 1) {
            nbody_opts o2 = o;
            o2.nseg = (int32_t)fit;
            o2.jlanes = 1;
            if ((st = choose_cfg(KERNEL_FORCE, n, o.precision, o2, &cfg, kEngineSplit))) return st;
            need = partial_bytes(cfg, o.precision);
        }
    }
    if (need > kStaticScratchBytes)
        return set_error(NBODY_EINVAL, "nbody_force_noalloc: this size and launch shape need " +
                                           std::to_string(need) + " bytes of partial sums; the "
                                           "static scratch holds " +
                                           std::to_string(kStaticScratchBytes));
    if (n == 0) return NBODY_OK;
    void *ws = nullptr;
    if (need > 0 && (st = scratch_ptr(&ws))) return st;
    return force_f32_core(n, pos, mass, eps, acc, pot, o, cfg, ws, nullptr, 0.0,
                          static_cast<hipStream_t>(stream));
}

}  // extern "C"
