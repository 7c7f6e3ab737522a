// Launch-shape table (see tuning.h) and its JSON form.
//
// File format (written by nbody_tune_save and by tune.py):
//   {"version": 1, "arch": "gfx950", "entries": [
//     {"kernel": 0, "precision": 2, "bucket": 17, "ipl": 4, "jtile": 256, "nseg": 16,
//      "jlanes": 1, "symmetric": 0}, ...]}
// kernel: 0 force, 1 adjoint, 2 batched, 3 force-jerk; precision: 0 plain, 1 FP64-reduced,
// 2 compensated; bucket: floor(log2 n) of the particle count (batched: mean system
// size); jlanes (1 if absent) selects the grid (1) or split (8..64) engine, symmetric
// (0 if absent) the symmetric engine.  Unknown keys are ignored.
#include "tuning.h"

#include <cctype>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "nbody_internal.h"

namespace nbody {
namespace {

constexpr int kBuckets = 32;
std::mutex g_mu;
bool g_set[KERNEL_COUNT][3][kBuckets];
TuneEntry g_tab[KERNEL_COUNT][3][kBuckets];

TuneEntry builtin(int kernel, int64_t n, int engines) {
    const bool split_ok = (engines & kEngineSplit) != 0;
    // Measured on MI355X (tune.py): one i-particle per lane (37 VGPRs, 8 waves per
    // SIMD) and many j-segments beat wider i-tiles for every kernel and size tried;
    // the j-split itself is chosen from n (nseg = 0).  Below 2^13 particles the force's
    // single-launch split engine is faster (graph-replayed evaluations, N = 2048: 5.4
    // against 9.5 us; N = 4096: 10.7 against 13.0 us); from 2^13 on the grid engine is.
    // The 2048-record tile (64 KB of LDS, two blocks per CU) only while every block fits
    // in one round.
    // Up to 2048 particles the tile is the smallest that holds every j (padding records
    // cost pair work too).
    if (kernel == KERNEL_FORCE && split_ok && n < (int64_t(1) << 13)) {
        if (n <= 2048) {
            int jt = 256;
            while (jt < n) jt *= 2;
            return TuneEntry{1, jt, 0, 64};
        }
        return n < 4096 ? TuneEntry{1, 1024, 0, 64} : TuneEntry{1, 1024, 0, 32};
    }
    if (kernel == KERNEL_BATCHED) return {1, 64, 0};
    return {1, 256, 0};
}

bool valid_entry(int kernel, int precision, int bucket, const TuneEntry &e) {
    return kernel >= 0 && kernel < KERNEL_COUNT && precision >= 0 && precision <= 2 &&
           bucket >= 0 && bucket < kBuckets && valid_shape(kernel, e);
}

}  // namespace

bool valid_shape(int kernel, const TuneEntry &e) {
    if (e.sym)
        // Symmetric engine: single-set force, 512 ipl particles per block row.
        return kernel == KERNEL_FORCE && e.sym == 1 && e.jl == 1 &&
               (e.ipl == 1 || e.ipl == 2 || e.ipl == 4) && (e.jt == 64 || e.jt == 128) &&
               e.nseg >= 0 && e.nseg <= kMaxSeg;
    if (e.jl == 1)
        return (e.ipl == 1 || e.ipl == 2 || e.ipl == 4 || e.ipl == 8) &&
               (e.jt == 64 || e.jt == 128 || e.jt == 256 || e.jt == 512) && e.nseg >= 0 &&
               e.nseg <= kMaxSeg;
    // Split engine: force and adjoint only; the adjoint's 32-byte j-records cap the
    // double-buffered tile at 512 records (32 KB of LDS); the force's 2048-record tile
    // (64 KB) is built for 32 and 64 lanes per i-particle.
    if (kernel != KERNEL_FORCE && kernel != KERNEL_VJP) return false;
    const bool jt_ok = e.jt == 256 || e.jt == 512 ||
                       (kernel == KERNEL_FORCE && (e.jt == 1024 || (e.jt == 2048 && e.jl >= 32)));
    return (e.jl == 8 || e.jl == 16 || e.jl == 32 || e.jl == 64) && (e.ipl == 1 || e.ipl == 2) &&
           jt_ok && e.nseg == 0;
}

int size_bucket(int64_t n) {
    int b = 0;
    while (b + 1 < kBuckets && (int64_t(1) << (b + 1)) <= n) ++b;
    return b;
}

TuneEntry tuned_shape(int kernel, int precision, int64_t n, int engines) {
    if (kernel < 0 || kernel >= KERNEL_COUNT || precision < 0 || precision > 2)
        return builtin(0, n, 0);
    std::lock_guard<std::mutex> lk(g_mu);
    const int b = size_bucket(n);
    if (g_set[kernel][precision][b]) {
        const TuneEntry &e = g_tab[kernel][precision][b];
        const bool usable = e.sym ? (engines & kEngineSym) != 0
                                  : (e.jl == 1 || (engines & kEngineSplit) != 0);
        if (usable) return e;
    }
    return builtin(kernel, n, engines);
}

void set_tuned_shape(int kernel, int precision, int64_t n, const TuneEntry &e) {
    if (kernel < 0 || kernel >= KERNEL_COUNT || precision < 0 || precision > 2) return;
    std::lock_guard<std::mutex> lk(g_mu);
    const int b = size_bucket(n);
    g_tab[kernel][precision][b] = e;
    g_set[kernel][precision][b] = true;
}

}  // namespace nbody

using namespace nbody;

extern "C" {

nbody_status nbody_tune_set(int32_t kernel, int32_t precision, int64_t n, int32_t ipl,
                            int32_t jtile, int32_t nseg, int32_t jlanes, int32_t symmetric) {
    clear_error();
    const TuneEntry e{ipl, jtile, nseg, jlanes, symmetric};
    if (n < 1 || !valid_entry(kernel, precision, size_bucket(n), e))
        return set_error(NBODY_EINVAL, "invalid tuning entry");
    set_tuned_shape(kernel, precision, n, e);
    return NBODY_OK;
}

nbody_status nbody_tune_get(int32_t kernel, int32_t precision, int64_t n, int32_t *shape) {
    clear_error();
    if (!shape || kernel < 0 || kernel >= KERNEL_COUNT || precision < 0 || precision > 2 || n < 1)
        return set_error(NBODY_EINVAL, "invalid tuning query");
    const TuneEntry e = tuned_shape(kernel, precision, n, kEngineSplit | kEngineSym);
    shape[0] = e.ipl;
    shape[1] = e.jt;
    shape[2] = e.nseg;
    shape[3] = e.jl;
    shape[4] = e.sym;
    return NBODY_OK;
}

void nbody_tune_reset(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto &a : g_set)
        for (auto &b : a)
            for (bool &c : b) c = false;
}

nbody_status nbody_tune_save(const char *path) {
    clear_error();
    if (!path) return set_error(NBODY_EINVAL, "path must not be NULL");
    FILE *f = std::fopen(path, "w");
    if (!f) return set_error(NBODY_EINVAL, std::string("cannot write ") + path);
    std::fprintf(f, "{\"version\": 1, \"arch\": \"gfx950\", \"entries\": [");
    bool first = true;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        for (int k = 0; k < KERNEL_COUNT; ++k)
            for (int p = 0; p < 3; ++p)
                for (int b = 0; b < kBuckets; ++b)
                    if (g_set[k][p][b]) {
                        const TuneEntry &e = g_tab[k][p][b];
                        std::fprintf(f, "%s\n  {\"kernel\": %d, \"precision\": %d, \"bucket\": %d, "
                                        "\"ipl\": %d, \"jtile\": %d, \"nseg\": %d, \"jlanes\": %d, "
                                        "\"symmetric\": %d}",
                                     first ? "" : ",", k, p, b, e.ipl, e.jt, e.nseg, e.jl, e.sym);
                        first = false;
                    }
    }
    std::fprintf(f, "\n]}\n");
    const bool ok = std::fclose(f) == 0;
    return ok ? NBODY_OK : set_error(NBODY_EINVAL, std::string("error writing ") + path);
}

// Reads every {...} object inside the "entries" array; each holds integer fields.
nbody_status nbody_tune_load(const char *path) {
    clear_error();
    if (!path) return set_error(NBODY_EINVAL, "path must not be NULL");
    FILE *f = std::fopen(path, "r");
    if (!f) return set_error(NBODY_EINVAL, std::string("cannot read ") + path);
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    std::fclose(f);
    const size_t ent = text.find("\"entries\"");
    if (ent == std::string::npos) return set_error(NBODY_EINVAL, "no \"entries\" in tuning file");
    size_t pos = text.find('[', ent);
    const size_t end = text.find(']', pos == std::string::npos ? ent : pos);
    if (pos == std::string::npos || end == std::string::npos)
        return set_error(NBODY_EINVAL, "malformed tuning file");
    // Parse and validate every entry first, so a bad file changes nothing.
    struct Parsed {
        int kernel, precision, bucket;
        TuneEntry e;
    };
    std::vector<Parsed> entries;
    while (true) {
        const size_t ob = text.find('{', pos);
        if (ob == std::string::npos || ob > end) break;
        const size_t cb = text.find('}', ob);
        if (cb == std::string::npos) return set_error(NBODY_EINVAL, "malformed tuning entry");
        int v[8] = {-1, -1, -1, -1, -1, -1, 1, 0};  // jlanes, symmetric absent: grid engine
        const char *keys[8] = {"\"kernel\"", "\"precision\"", "\"bucket\"", "\"ipl\"",
                               "\"jtile\"",  "\"nseg\"",      "\"jlanes\"", "\"symmetric\""};
        for (int q = 0; q < 8; ++q) {
            const size_t kp = text.find(keys[q], ob);
            if (kp == std::string::npos || kp > cb) continue;
            const size_t colon = text.find(':', kp);
            if (colon == std::string::npos || colon > cb) continue;
            v[q] = std::atoi(text.c_str() + colon + 1);
        }
        const TuneEntry e{v[3], v[4], v[5], v[6], v[7]};
        if (!valid_entry(v[0], v[1], v[2], e))
            return set_error(NBODY_EINVAL, "invalid tuning entry in " + std::string(path));
        entries.push_back({v[0], v[1], v[2], e});
        pos = cb + 1;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (const Parsed &p : entries) {
        g_tab[p.kernel][p.precision][p.bucket] = p.e;
        g_set[p.kernel][p.precision][p.bucket] = true;
    }
    return NBODY_OK;
}

}  // extern "C"
