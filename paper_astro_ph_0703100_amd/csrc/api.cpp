// Host side of the C ABI: argument validation, launch-shape choice, scratch memory
// and dispatch to the kernels.  Nothing here touches particle data on the host.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>

#include "nbody_internal.h"
#include "tuning.h"

namespace nbody {

namespace {
thread_local std::string g_error;

constexpr int kMaxDevices = 64;
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_ws_mu;
Workspace g_ws[kMaxDevices];

std::mutex g_dev_mu;
bool g_dev_ready[kMaxDevices];
DeviceInfo g_dev[kMaxDevices];

}  // namespace

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

nbody_status set_error(nbody_status code, const std::string &msg) {
    g_error = msg;
    return code;
}

nbody_status hip_error(hipError_t e, const char *what) {
    g_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? NBODY_ENOMEM : NBODY_EHIP;
}

void clear_error() { g_error.clear(); }

const DeviceInfo &device_info() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_dev_ready[dev]) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
            g_dev[dev].cus = p.multiProcessorCount > 0 ? p.multiProcessorCount : 256;
            g_dev[dev].warp = p.warpSize;
        }
        g_dev_ready[dev] = true;
    }
    return g_dev[dev];
}

bool stream_capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

// Scratch of at least `need` bytes: the caller's buffer, or the per-device cache.  A
// capturing stream must bring its own buffer: a graph that recorded the cache's address
// would read and write freed memory after a later call grew (reallocated) the cache.
nbody_status get_workspace(const nbody_opts &o, size_t need, hipStream_t s, void **out) {
    if (need == 0) {
        *out = o.workspace;
        return NBODY_OK;
    }
    if (!o.workspace && stream_capturing(s))
        return set_error(NBODY_ECAPTURE,
                         "stream is capturing: pass opts->workspace (the library's cache may be "
                         "reallocated after the capture, which would leave the graph with freed "
                         "memory)");
    if (o.workspace) {
        if (o.workspace_bytes < need)
            return set_error(NBODY_EINVAL, "workspace too small: need " + std::to_string(need) +
                                               " bytes, got " + std::to_string(o.workspace_bytes));
        if (reinterpret_cast<uintptr_t>(o.workspace) % 256)
            return set_error(NBODY_EINVAL, "workspace must be 256-byte aligned");
        *out = o.workspace;
        return NBODY_OK;
    }
    int dev = 0;
    NBODY_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return set_error(NBODY_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace &w = g_ws[dev];
    if (w.bytes >= need) {
        *out = w.ptr;
        return NBODY_OK;
    }
    if (w.ptr) {
        // hipFree waits for the device, so no kernel still uses the old buffer.
        NBODY_HIP_CHECK(hipFree(w.ptr));
        w.ptr = nullptr;
        w.bytes = 0;
    }
    const size_t bytes = align_up(need + need / 4, 1 << 20);
    hipError_t e = hipMalloc(&w.ptr, bytes);
    if (e != hipSuccess) {
        w.ptr = nullptr;
        return hip_error(e, "hipMalloc(workspace)");
    }
    w.bytes = bytes;
    *out = w.ptr;
    return NBODY_OK;
}

// Launch shape for ni i-particles against nj j-particles: explicit options first, then
// the tuning table (its j-split only when the two sets have the same size, the shape it
// was measured on), then a default that gives every compute unit several blocks.
// engines (kEngine* bits): the engines besides the grid engine that the caller has
// kernels for (split: single-set force or adjoint without per-i-tile centres;
// symmetric: single-set force on FP32 or system-centred positions).
nbody_status choose_cfg_ij(int kernel, int64_t ni, int64_t nj, int precision, const nbody_opts &o,
                           TileCfg *cfg, int engines) {
    TileCfg c;
    if (o.jlanes < 0) return set_error(NBODY_EINVAL, "jlanes must be >= 0");
    if (o.symmetric < 0 || o.symmetric > 2)
        return set_error(NBODY_EINVAL, "symmetric must be 0 (tuned), 1 (off) or 2 (on)");
    if (o.jlanes > 1 && !(engines & kEngineSplit))
        return set_error(NBODY_EUNSUPPORTED,
                         "jlanes > 1 (split engine) is available for the single-set force and "
                         "adjoint without per-i-tile centres only");
    if (o.symmetric == 2 && !(engines & kEngineSym))
        return set_error(NBODY_EUNSUPPORTED,
                         "symmetric = 2 (symmetric engine) is available for the single-set force "
                         "on FP32 or system-centred positions only");
    if (o.symmetric == 2 && o.jlanes > 1)
        return set_error(NBODY_EINVAL, "the symmetric engine takes jlanes 0 or 1");
    const bool explicit_shape = o.ipl || o.jtile || o.nseg;
    TuneEntry t = tuned_shape(kernel, precision, nj, engines);
    const bool use_sym = ni == nj && (o.symmetric == 2 ||
                                      (o.symmetric == 0 && !o.jlanes && !explicit_shape && t.sym));
    if (use_sym) {
        const TuneEntry e{o.ipl ? o.ipl : (t.sym ? t.ipl : 4), o.jtile ? o.jtile : (t.sym ? t.jt : 64),
                          o.nseg ? o.nseg : (t.sym ? t.nseg : 0), 1, 1};
        if (!valid_shape(kernel, e))
            return set_error(NBODY_EINVAL,
                             "symmetric-engine shape needs ipl in {1, 2, 4}, jtile in {64, 128} "
                             "and nseg in [0, " + std::to_string(kMaxSeg) + "]");
        const int bi = 64 * kSymWaves * e.ipl;
        const int n = (int)ni;
        c.sym = 1;
        c.ipl = e.ipl;
        c.jt = e.jt;
        c.jl = 1;
        c.nb = (int)((ni + bi - 1) / bi);
        c.npad = c.nb * bi;
        const int64_t t0 = sym::row_tiles(n, bi, c.jt, 0);
        int64_t segt;
        if (e.nseg > 0) {
            segt = (t0 + e.nseg - 1) / e.nseg;
        } else {
            // About 16 work items per compute unit (4 resident blocks of 8 waves each, so
            // 4 rounds), each a whole number of j-tiles.
            int64_t all = 0;
            for (int b = 0; b < c.nb; ++b) all += sym::row_tiles(n, bi, c.jt, b);
            segt = all / ((int64_t)device_info().cus * 16);
        }
        c.segt = (int)std::max<int64_t>(1, std::min<int64_t>(segt, t0));  // at most a whole row
        c.nseg = sym::row_segments(n, bi, c.jt, c.segt, 0);
        int64_t items = 0;
        for (int s = 0; s < c.nseg; ++s) items += sym::items_of_segment(n, bi, c.jt, c.segt, c.nb, s);
        c.nitems = (int)items;
        c.itiles = 0;
        c.seg_len = 0;
        *cfg = c;
        return NBODY_OK;
    }
    const bool split_ok = (engines & kEngineSplit) != 0;
    const int jl = o.jlanes ? o.jlanes : (explicit_shape || o.symmetric == 2 ? 1 : t.jl);
    if (jl > 1) {
        // Split engine: one launch of ceil(ni / i-per-block) blocks, no j-segments.
        const bool from_table = t.jl > 1;
        TuneEntry e{o.ipl ? o.ipl : (from_table ? t.ipl : 1),
                    o.jtile ? o.jtile : (from_table ? t.jt : 512), o.nseg, jl};
        if (!valid_shape(kernel, e))
            return set_error(NBODY_EINVAL,
                             "split-engine shape needs jlanes in {8, 16, 32, 64}, ipl in {1, 2}, "
                             "jtile in {256, 512, 1024} (adjoint: 256, 512) and nseg = 0");
        c.ipl = e.ipl;
        c.jt = e.jt;
        c.jl = jl;
        const int64_t per_block = (int64_t)4 * (64 / jl) * c.ipl;
        c.itiles = (int)((ni + per_block - 1) / per_block);
        c.nseg = 1;
        c.seg_len = 0;
        c.npad = 0;
        *cfg = c;
        return NBODY_OK;
    }
    (void)split_ok;
    if (t.jl > 1 || t.sym) t = TuneEntry{1, 256, 0, 1};  // the table's shape is another engine's
    if (t.jl > 1) t = TuneEntry{1, 256, 0, 1};  // the table's split shape does not apply
    c.ipl = o.ipl ? o.ipl : t.ipl;
    c.jt = o.jtile ? o.jtile : t.jt;
    if (!(c.ipl == 1 || c.ipl == 2 || c.ipl == 4 || c.ipl == 8))
        return set_error(NBODY_EINVAL, "ipl must be 1, 2, 4 or 8");
    if (!(c.jt == 64 || c.jt == 128 || c.jt == 256 || c.jt == 512))
        return set_error(NBODY_EINVAL, "jtile must be 64, 128, 256 or 512");
    if (o.nseg < 0 || o.nseg > kMaxSeg)
        return set_error(NBODY_EINVAL, "nseg must be in [0, " + std::to_string(kMaxSeg) + "]");
    const int64_t itile = (int64_t)kTPB * c.ipl;
    c.itiles = (int)((ni + itile - 1) / itile);
    c.npad = (int)(c.itiles * itile);
    const int64_t jtiles = (nj + c.jt - 1) / c.jt;
    int64_t nseg = o.nseg ? o.nseg : (ni == nj ? t.nseg : 0);
    if (nseg <= 0 && c.itiles > 0) {
        // Between 16 and 48 blocks per compute unit (8 resident per CU, so 2 to 6
        // rounds: the last round stays short), and within that range segments of at
        // least 8 j-tiles, so per-block start-up and the partial sums stay small when
        // there are few i-tiles (an i-range of one system against all of it).
        const int64_t cus = device_info().cus;
        const int64_t hi = (cus * 48 + c.itiles - 1) / c.itiles;
        const int64_t lo = (cus * 16 + c.itiles - 1) / c.itiles;
        nseg = std::min(hi, std::max(lo, jtiles / 8));
    }
    if (nseg > jtiles) nseg = jtiles;
    if (nseg > kMaxSeg) nseg = kMaxSeg;
    if (nseg < 1) nseg = 1;
    const int64_t per = jtiles > 0 ? (jtiles + nseg - 1) / nseg : 1;  // tiles per segment
    c.seg_len = (int)(per * c.jt);
    c.nseg = jtiles > 0 ? (int)((jtiles + per - 1) / per) : 1;
    *cfg = c;
    return NBODY_OK;
}

nbody_status choose_cfg(int kernel, int64_t n, int precision, const nbody_opts &o, TileCfg *cfg,
                        int engines) {
    return choose_cfg_ij(kernel, n, n, precision, o, cfg, engines);
}

size_t partial_bytes(const TileCfg &c, int precision, int outputs) {
    if (c.jl > 1) return 0;  // the split engine keeps its partial sums in registers
    if (c.sym) return sym_ipart_bytes(c, precision) + sym_jpart_bytes(c, precision);
    return align_up((size_t)c.nseg * partial_words(precision, outputs) * (size_t)c.npad * 4, 256);
}

nbody_opts resolve_opts(const nbody_opts *opts) {
    nbody_opts o;
    nbody_opts_default(&o);
    if (opts) o = *opts;
    return o;
}

nbody_status check_common(int64_t n, const void *pos, const void *mass, float eps,
                          const void *acc, const nbody_opts &o) {
    if (n < 0 || n > INT32_MAX / 2) return set_error(NBODY_EINVAL, "n must be in [0, 2^30)");
    if (n > 0 && (!pos || !mass || !acc))
        return set_error(NBODY_EINVAL, "pos, mass and acc must not be NULL");
    const float e2 = eps * eps;
    if (!std::isfinite(eps) || !(eps > 0.0f) || !(e2 >= FLT_MIN) || !std::isfinite(e2))
        return set_error(NBODY_EINVAL, "eps must be finite and > 0 with eps^2 a normal float");
    if (o.precision < NBODY_PLAIN || o.precision > NBODY_COMP)
        return set_error(NBODY_EINVAL, "precision must be NBODY_PLAIN, NBODY_FP64RED or NBODY_COMP");
    if (o.self_pot != 0 && o.self_pot != 1) return set_error(NBODY_EINVAL, "self_pot must be 0 or 1");
    if (o.centre < NBODY_CENTRE_NONE || o.centre > NBODY_CENTRE_TILE)
        return set_error(NBODY_EINVAL, "centre must be NBODY_CENTRE_NONE, _SYSTEM or _TILE");
    return NBODY_OK;
}

nbody_status check_force_f32(int64_t n, const float *pos, const float *mass, float eps,
                             const double *acc, const double *pot, const nbody_opts &o) {
    nbody_status st = check_common(n, pos, mass, eps, acc, o);
    if (st) return st;
    if (misaligned(pos) || misaligned(mass) || misaligned(acc) || misaligned(pot))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    return NBODY_OK;
}

size_t f64_scratch_bytes(int64_t n, const TileCfg &cfg, int precision, int outputs) {
    return partial_bytes(cfg, precision, outputs) + align_up(sizeof(float) * 3 * (size_t)n, 256) +
           align_up(centre_scratch_bytes(), 256);
}

F64Scratch f64_scratch_layout(void *ws, int64_t n, const TileCfg &cfg, int precision,
                              int outputs) {
    char *base = static_cast<char *>(ws);
    const size_t pb = partial_bytes(cfg, precision, outputs);
    const size_t xb = align_up(sizeof(float) * 3 * (size_t)n, 256);
    F64Scratch r;
    r.part = base;
    r.x32 = reinterpret_cast<float *>(base + pb);
    r.centre_scratch = reinterpret_cast<double *>(base + pb + xb);
    return r;
}

// Pair kernel + FP64 reduction on FP32 structure-of-arrays positions.
nbody_status force_f32_core(int64_t n, const float *pos, const float *mass, float eps, double *acc,
                            double *pot, const nbody_opts &o, const TileCfg &cfg, void *ws,
                            double *kick_v, double kick_h, hipStream_t s) {
    const float e2 = eps * eps;
    PairArgs pa{pos, pos + n, pos + 2 * n, mass, (int)n, cfg.seg_len, e2, ws, cfg.npad};
    FinalizeArgs fa{ws, cfg.nseg, cfg.npad, (int)n, mass, eps, o.self_pot, acc, pot, kick_v,
                    kick_h};
    if (cfg.jl > 1) return launch_pair_split(cfg, o.precision, pot != nullptr, pa, fa, s);
    if (cfg.sym) return launch_pair_sym(cfg, o.precision, pot != nullptr, pa, fa, s);
    nbody_status st = launch_pair(cfg, o.precision, pot != nullptr, pa, s);
    if (st) return st;
    return launch_finalize(o.precision, fa, s);
}

nbody_status force_f64_core(int64_t n, const double *pos64, const float *mass, float eps,
                            double *acc, double *pot, const nbody_opts &o, const TileCfg &cfg,
                            const F64Scratch &ws, double *kick_v, double kick_h, hipStream_t s,
                            bool centre_ready) {
    nbody_status st;
    if (o.centre == NBODY_CENTRE_TILE) {
        // Per-i-tile centres (3 doubles per tile fit in the FP32-position area, which this
        // mode does not use); positions are converted inside the pair kernel.
        const int itile = kTPB * cfg.ipl;
        double *centres = reinterpret_cast<double *>(ws.x32);
        if ((st = launch_tile_centres(n, itile, pos64, centres, s))) return st;
        const float e2 = eps * eps;
        TilePairArgs ta{pos64, pos64 + n, pos64 + 2 * n, mass, (int)n, cfg.seg_len, e2,
                        ws.part, cfg.npad, centres, itile};
        if ((st = launch_pair_tile(cfg, o.precision, pot != nullptr, ta, s))) return st;
        FinalizeArgs fa{ws.part, cfg.nseg, cfg.npad, (int)n, mass, eps, o.self_pot,
                        acc,     pot,      kick_v,   kick_h};
        return launch_finalize(o.precision, fa, s);
    }
    if (o.centre == NBODY_CENTRE_SYSTEM) {
        st = centre_ready ? launch_centred_convert_ready(n, pos64, ws.centre_scratch, ws.x32, s)
                          : launch_centred_convert(n, pos64, ws.centre_scratch, ws.x32, s);
        if (st) return st;
    } else {
        if ((st = launch_convert(n, pos64, nullptr, ws.x32, s))) return st;
    }
    return force_f32_core(n, ws.x32, mass, eps, acc, pot, o, cfg, ws.part, kick_v, kick_h, s);
}

}  // namespace nbody

using namespace nbody;

extern "C" {

void nbody_opts_default(nbody_opts *opts) {
    if (!opts) return;
    std::memset(opts, 0, sizeof(*opts));
    opts->precision = NBODY_COMP;
    opts->centre = NBODY_CENTRE_SYSTEM;
    opts->self_pot = 0;
}

const char *nbody_last_error(void) { return g_error.c_str(); }

const char *nbody_version(void) { return "nbody-gfx950 0.1"; }

size_t nbody_workspace_size(int64_t n, const nbody_opts *opts) {
    nbody_opts o;
    nbody_opts_default(&o);
    if (opts) o = *opts;
    if (n <= 0) return 0;
    TileCfg c;
    if (choose_cfg(KERNEL_FORCE, n, o.precision, o, &c, force_engines(o)) != NBODY_OK)
        return 0;
    return f64_scratch_bytes(n, c, o.precision);
}

nbody_status nbody_force_ex(int64_t n, const float *pos, const float *mass, float eps, double *acc,
                            double *pot, const nbody_opts *opts, void *stream) {
    clear_error();
    nbody_opts o = resolve_opts(opts);
    nbody_status st = check_force_f32(n, pos, mass, eps, acc, pot, o);
    if (st) return st;
    if (n == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_FORCE, n, o.precision, o, &cfg, kEngineSplit | kEngineSym))) return st;
    void *ws = nullptr;
    if ((st = get_workspace(o, partial_bytes(cfg, o.precision), s, &ws))) return st;
    return force_f32_core(n, pos, mass, eps, acc, pot, o, cfg, ws, nullptr, 0.0, s);
}

nbody_status nbody_force(int64_t n, const float *pos, const float *mass, float eps, double *acc,
                         double *pot, void *stream) {
    return nbody_force_ex(n, pos, mass, eps, acc, pot, nullptr, stream);
}

nbody_status nbody_force_f64(int64_t n, const double *pos64, const float *mass, float eps,
                             double *acc, double *pot, const nbody_opts *opts, void *stream) {
    clear_error();
    nbody_opts o = resolve_opts(opts);
    nbody_status st = check_common(n, pos64, mass, eps, acc, o);
    if (st) return st;
    if (misaligned(pos64) || misaligned(mass) || misaligned(acc) || misaligned(pot))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    if (n == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    TileCfg cfg;
    if ((st = choose_cfg(KERNEL_FORCE, n, o.precision, o, &cfg, force_engines(o)))) return st;
    void *ws = nullptr;
    if ((st = get_workspace(o, f64_scratch_bytes(n, cfg, o.precision), s, &ws))) return st;
    return force_f64_core(n, pos64, mass, eps, acc, pot, o, cfg,
                          f64_scratch_layout(ws, n, cfg, o.precision), nullptr, 0.0, s);
}

nbody_status nbody_force_ij(int64_t ni, const float *pos_i, const float *eps_i, int64_t nj,
                            const float *pos_j, const float *mass_j, float eps, double *acc,
                            double *pot, const nbody_opts *opts, void *stream) {
    clear_error();
    nbody_opts o = resolve_opts(opts);
    if (ni < 0 || ni > INT32_MAX / 2 || nj < 0 || nj > INT32_MAX / 2)
        return set_error(NBODY_EINVAL, "ni and nj must be in [0, 2^30)");
    if (ni > 0 && (!pos_i || !acc)) return set_error(NBODY_EINVAL, "pos_i and acc must not be NULL");
    if (ni > 0 && nj > 0 && (!pos_j || !mass_j))
        return set_error(NBODY_EINVAL, "pos_j and mass_j must not be NULL");
    const float e2 = eps * eps;
    if (!std::isfinite(eps) || !(eps >= 0.0f) || !std::isfinite(e2) || (eps > 0.0f && !(e2 >= FLT_MIN)))
        return set_error(NBODY_EINVAL, "eps must be finite and >= 0 with eps^2 zero or a normal float");
    if (o.precision < NBODY_PLAIN || o.precision > NBODY_COMP)
        return set_error(NBODY_EINVAL, "precision must be NBODY_PLAIN, NBODY_FP64RED or NBODY_COMP");
    if (misaligned(pos_i) || misaligned(eps_i) || misaligned(pos_j) || misaligned(mass_j) ||
        misaligned(acc) || misaligned(pot))
        return set_error(NBODY_EINVAL, "misaligned array argument");
    if (ni == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    nbody_status st;
    if (nj == 0) {
        if ((st = launch_fill_f64(3 * ni, acc, 0.0, s))) return st;
        return pot ? launch_fill_f64(ni, pot, 0.0, s) : NBODY_OK;
    }
    TileCfg cfg;
    if ((st = choose_cfg_ij(KERNEL_FORCE, ni, nj, o.precision, o, &cfg, 0))) return st;
    void *ws = nullptr;
    if ((st = get_workspace(o, partial_bytes(cfg, o.precision), s, &ws))) return st;
    IJPairArgs a{pos_i, pos_i + ni, pos_i + 2 * ni, eps_i, pos_j, pos_j + nj, pos_j + 2 * nj,
                 mass_j, (int)ni, (int)nj, cfg.seg_len, e2, ws, cfg.npad};
    if ((st = launch_pair_ij(cfg, o.precision, pot != nullptr, a, s))) return st;
    FinalizeArgs fa{ws, cfg.nseg, cfg.npad, (int)ni, nullptr, eps, 0, acc, pot, nullptr, 0.0};
    return launch_finalize(o.precision, fa, s);
}

size_t nbody_workspace_size_ij(int64_t ni, int64_t nj, const nbody_opts *opts) {
    nbody_opts o = resolve_opts(opts);
    if (ni <= 0 || nj <= 0) return 0;
    TileCfg c;
    if (choose_cfg_ij(KERNEL_FORCE, ni, nj, o.precision, o, &c, 0) != NBODY_OK) return 0;
    return partial_bytes(c, o.precision);
}

nbody_status nbody_morton_order(int64_t n, const double *pos64, int32_t *perm, void *stream) {
    clear_error();
    if (n < 0 || n > INT32_MAX / 2) return set_error(NBODY_EINVAL, "n must be in [0, 2^30)");
    if (n > 0 && (!pos64 || !perm)) return set_error(NBODY_EINVAL, "pos64 and perm must not be NULL");
    if (misaligned(pos64) || misaligned(perm)) return set_error(NBODY_EINVAL, "misaligned array argument");
    if (n == 0) return NBODY_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    nbody_opts o = resolve_opts(nullptr);
    void *ws = nullptr;
    nbody_status st = get_workspace(o, morton_scratch_bytes(n), s, &ws);
    if (st) return st;
    return launch_morton_order(n, pos64, perm, ws, s);
}

}  // extern "C"
