// Internal declarations shared by the translation units of libnbody.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <functional>
#include <string>

#include "nbody.h"
#include "tuning.h"

// A captured HIP graph and the scratch memory it owns (if any).
struct nbody_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *workspace = nullptr;
    int device = 0;
};

namespace nbody {

// Threads per block of every pair kernel: four 64-wide wavefronts, one per SIMD of
// a compute unit.
constexpr int kTPB = 256;
// Largest number of j-segments a launch may split the j range into.
constexpr int kMaxSeg = 1024;
// Blocks of the first stage of the FP64 system centre (fixed, so the sum order is too).
constexpr int kCentreBlocks = 256;
// Default number of j's summed in plain FP32 between two compensation / FP64 steps; a
// pipeline may set its own (Op::kBlockJ), and the engine caps it at the j-tile.  128
// keeps the two-sums under 0.6 VALU operations per pair for every pipeline (force:
// 4 outputs, jerk: 7, adjoint: 5).  The FP32 block sum adds at most 127 u sum |term|
// (about sqrt(128) u sum |term| in practice), of the order of the pair rounding.
constexpr int kBlockJ = 128;

// Outputs per particle of the force (a, phi) and of the adjoint pipeline (three
// position sums, the sum that multiplies the particle's own cotangent, the mass sum).
constexpr int kForceOutputs = 4;
constexpr int kVjpOutputs = 5;

// Words (4-byte) of partial sums written per i-particle and j-segment for `outputs`
// outputs (compensated: hi and lo; FP64-reduced: one double).
inline int partial_words(int precision, int outputs = kForceOutputs) {
    return precision == NBODY_PLAIN ? outputs : 2 * outputs;
}

// Shape of one force launch.
struct TileCfg {
    int ipl = 4;     // i-particles per lane
    int jt = 256;    // j-particles per LDS tile
    int nseg = 1;    // j-segments (grid y)
    int seg_len = 0; // j's per segment, a multiple of jt
    int itiles = 0;  // i-tiles (grid x)
    int npad = 0;    // itiles * kTPB * ipl
    int jl = 1;      // lanes per i-particle's j-range: 1 = grid engine, 8..64 = split engine
                     // (then itiles = blocks of 4 * (64 / jl) * ipl i's, nseg = 1)
    // Symmetric engine (sym = 1; jl = 1): block rows of 512 * ipl particles, nb rows,
    // segt j-tiles per work item, nitems work items (the grid), smax segments in row 0
    // (nseg = smax), npad = nb * 512 * ipl.
    int sym = 0;
    int segt = 0;
    int nb = 0;
    int nitems = 0;
};

// Waves per block of the symmetric engine.
constexpr int kSymWaves = 8;

namespace sym {

// Work items of segment s: every row for s = 0 (each has its diagonal), else the rows
// whose symmetric range has more than s * segt tiles.
__host__ __device__ inline int items_of_segment(int n, int bi, int jt, int segt, int nb, int s) {
    if (s == 0) return nb;
    const long long rest = (long long)n - (long long)s * segt * jt;
    if (rest <= 0) return 0;
    const long long rows = (rest + bi - 1) / bi - 1;
    return rows > 0 ? (int)rows : 0;
}

// Symmetric j-tiles of row b.
__host__ __device__ inline int row_tiles(int n, int bi, int jt, int b) {
    const long long js = (long long)(b + 1) * bi;
    return js < n ? (int)((n - js + jt - 1) / jt) : 0;
}

// Segments (i-planes) of row b.
__host__ __device__ inline int row_segments(int n, int bi, int jt, int segt, int b) {
    const int t = row_tiles(n, bi, jt, b);
    return t > 0 ? (t + segt - 1) / segt : 1;
}

// j-side sums of block row b cover j in [(b + 1) bi, nb bi): rows of decreasing length
// stored back to back as [b][output][j - (b + 1) bi].  Length of row b (per output) and
// its first element.
__host__ __device__ inline size_t jrow_len(int nb, int bi, int b) {
    return (size_t)(nb - 1 - b) * bi;
}
__host__ __device__ inline size_t jrow_base(int nb, int bi, int b) {
    // kForceOutputs x sum over b' < b of (nb - 1 - b') bi
    return (size_t)kForceOutputs * bi * ((size_t)b * (nb - 1) - (size_t)b * (b - 1) / 2);
}

}  // namespace sym

// Arguments of the pair kernel (FP32 structure-of-arrays input).
struct PairArgs {
    const float *x, *y, *z, *m;
    int n;        // particles
    int seg_len;  // j's per segment
    float eps2;   // fp32(eps^2)
    void *part;   // partial sums [nseg][words][npad]
    int npad;
};

// Arguments of the symmetric pair kernel (each unordered pair once; FP32
// structure-of-arrays input).  Block rows of bi = 64 W IPL particles; row b's
// symmetric range is split into segments of segt j-tiles.
struct SymArgs {
    const float *x, *y, *z, *m;
    int n;
    float eps2;
    int segt;     // j-tiles per segment
    int nb;       // block rows
    int smax;     // segments of row 0 (the most of any row)
    int npad;     // nb * bi
    void *ipart;  // i-side partials [smax][words][npad]
    void *jpart;  // j-side sums, rows of sym::jrow_len words per output: FP64 (PLAIN: FP32)
};

// Arguments of the pair kernel on FP64 positions with per-i-tile reference centres.
struct TilePairArgs {
    const double *x, *y, *z;  // FP64 positions [3][n]
    const float *m;
    int n;
    int seg_len;
    float eps2;
    void *part;
    int npad;
    const double *centres;  // [i-tiles][3] FP64 centres
    int itile;              // particles per i-tile (256 * IPL)
};

// Arguments of the pair kernel with separate i- and j-sets (FP32 structure of arrays).
struct IJPairArgs {
    const float *xi, *yi, *zi;    // i positions [3][ni]
    const float *ei;              // per-i softening [ni], or nullptr: eps2 for every i
    const float *x, *y, *z, *m;   // j positions [3][nj] and masses [nj]
    int ni, nj;
    int seg_len;
    float eps2;
    void *part;
    int npad;
};

// Arguments of the force-jerk-potential kernel (FP32 structure of arrays).
struct JerkArgs {
    const float *x, *y, *z, *m;   // positions [3][n] and masses [n]
    const float *vx, *vy, *vz;    // velocities [3][n]
    int n;
    int seg_len;
    float eps2;
    void *part;                   // partial sums [nseg][7 * words][npad]
    int npad;
};

// The same on FP64 state taken relative to per-i-tile FP64 centres of position and
// velocity (converted to FP32 by each block as it loads its i's and stages its j's).
struct JerkTileArgs {
    const double *x, *y, *z;     // FP64 positions [3][n]
    const float *m;
    const double *vx, *vy, *vz;  // FP64 velocities [3][n]
    int n;
    int seg_len;
    float eps2;
    void *part;
    int npad;
    const double *cx;            // [i-tiles][3] mean position of each i-tile
    const double *cv;            // [i-tiles][3] mean velocity of each i-tile
    int itile;                   // particles per i-tile (256 * IPL)
};

// Force-jerk-potential with separate i- and j-sets (FP32 inputs, uniform softening).
struct JerkIJArgs {
    const float *xi, *yi, *zi;     // i positions [3][ni]
    const float *vxi, *vyi, *vzi;  // i velocities [3][ni]
    const float *x, *y, *z, *m;    // j positions [3][nj] and masses [nj]
    const float *vx, *vy, *vz;     // j velocities [3][nj]
    int ni, nj;
    int seg_len;
    float eps2;
    void *part;
    int npad;
};

struct JerkFinalizeArgs {
    const void *part;
    int nseg, npad, n;
    const float *m;
    float eps;
    int include_self;  // 1: add the j == i potential term -m_i / eps (in FP64)
    double *acc;   // [3][n]
    double *jerk;  // [3][n]
    double *pot;   // [n] or nullptr
};

// One work item of a ragged batch: an i-tile of one system against a j-range of the
// same system.  Indices are global (into the concatenated arrays).
struct BatchItem {
    int32_t sys;    // system index
    int32_t i0;     // first i of the tile
    int32_t ni;     // i's in the tile (<= 256 * IPL)
    int32_t j0;     // first j of the range
    int32_t nj;     // j's in the range
    int32_t col0;   // column of i0 in the system's partial planes (i0 - offset)
    int64_t part;   // word offset of this (system, segment)'s partial planes
    int32_t npad;   // plane stride of the system (its i-tiles * 256 * IPL)
    int32_t pad_;
};

// Work queue of a persistent batched launch.
struct BatchSched {
    const BatchItem *items;
    int nitems;
    unsigned int *counter;  // ticket, reset to 0 before every launch
    const float *eps;       // per-system softening [nsys]
    void *part;             // partial-sum words
};

// Arguments of the batched FP64 reduction (per particle, looked up by system).
struct BatchFinalizeArgs {
    const void *part;
    int64_t total;
    const int32_t *sys_of;     // [total] system of each particle
    const int64_t *offsets;    // [nsys + 1]
    const int64_t *part_base;  // [nsys] word offset of each system's planes
    const int32_t *npad;       // [nsys]
    const int32_t *nseg;       // [nsys]
    double *acc;               // [3][total]
    double *pot;               // [total] or nullptr
    double *kick_v;            // [3][total] or nullptr
    double kick_h;
};

// Arguments of the FP64 reduction of the partial sums.
struct FinalizeArgs {
    const void *part;
    int nseg, npad, n;
    const float *m;
    float eps;
    int include_self;  // 1: add the j == i potential term -m_i / eps (in FP64)
    double *acc;       // [3][n]
    double *pot;       // [n] or nullptr
    double *kick_v;    // [3][n]: if not null, v += kick_h * a after a is written
    double kick_h;
};

struct VjpArgs {
    const float *x, *y, *z, *m;      // FP32 positions [3][n] (relative to the centre) and masses
    const double *gx, *gy, *gz;      // dL/da [3][n]
    const double *gp;                // dL/dphi [n] or nullptr
    int n;
    int seg_len;
    float eps2;
    void *part;
    int npad;
};

// The adjoint on FP64 positions relative to per-i-tile FP64 centres.
struct VjpTileArgs {
    const double *x, *y, *z;         // FP64 positions [3][n]
    const float *m;
    const double *gx, *gy, *gz;      // dL/da [3][n]
    const double *gp;                // dL/dphi [n] or nullptr
    int n;
    int seg_len;
    float eps2;
    void *part;
    int npad;
    const double *centres;           // [i-tiles][3] mean position of each i-tile
    int itile;
};

struct VjpFinalizeArgs {
    const void *part;
    int nseg, npad, n;
    const double *gp;   // dL/dphi or nullptr
    double *grad_pos;   // [3][n]
    double *grad_mass;  // [n] or nullptr
    int accumulate;     // 1: add into grad_pos / grad_mass instead of overwriting
    const double *ga;   // dL/da [3][n]: the particle's own cotangent (its FP32 value is used)
};

// Thread-local error reporting.
nbody_status set_error(nbody_status code, const std::string &msg);
nbody_status hip_error(hipError_t e, const char *what);
void clear_error();

#define NBODY_HIP_CHECK(expr)                                   \
    do {                                                        \
        hipError_t _e = (expr);                                 \
        if (_e != hipSuccess) return ::nbody::hip_error(_e, #expr); \
    } while (0)

// True if p is not aligned for T (NULL counts as aligned).
template <typename T>
inline bool misaligned(const T *p) {
    return reinterpret_cast<uintptr_t>(p) % alignof(T) != 0;
}

// Scratch of the symmetric engine: i-side partials [nseg][words][npad], then the
// j-side sums of rows 0 .. nb - 2 (sym::jrow_base; FP64, PLAIN: FP32).
inline size_t sym_ipart_bytes(const TileCfg &c, int precision) {
    const size_t b = (size_t)c.nseg * partial_words(precision) * (size_t)c.npad * 4;
    return (b + 255) / 256 * 256;
}
inline size_t sym_jpart_bytes(const TileCfg &c, int precision) {
    if (c.nb < 2) return 0;
    const size_t words = sym::jrow_base(c.nb, kSymWaves * 64 * c.ipl, c.nb - 1);
    const size_t b = words * (precision == NBODY_PLAIN ? 4 : 8);
    return (b + 255) / 256 * 256;
}

// Host helpers (api.cpp).
bool stream_capturing(hipStream_t s);
nbody_status get_workspace(const nbody_opts &o, size_t need, hipStream_t s, void **out);
// engines (kEngine* bits of tuning.h): the engines besides the grid engine that the
// caller has kernels for.
nbody_status choose_cfg(int kernel, int64_t n, int precision, const nbody_opts &o, TileCfg *cfg,
                        int engines);
// The same for ni i-particles against nj j-particles (nj >= 1).
nbody_status choose_cfg_ij(int kernel, int64_t ni, int64_t nj, int precision, const nbody_opts &o,
                           TileCfg *cfg, int engines);
// Engines of a single-set force evaluation with these options: split and symmetric,
// except with per-i-tile centres (the grid engine's i-tiles).
inline int force_engines(const nbody_opts &o) {
    return o.centre != NBODY_CENTRE_TILE ? kEngineSplit | kEngineSym : 0;
}
size_t partial_bytes(const TileCfg &c, int precision, int outputs = kForceOutputs);
size_t align_up(size_t v, size_t a);
nbody_status check_common(int64_t n, const void *pos, const void *mass, float eps,
                          const void *acc, const nbody_opts &o);
nbody_opts resolve_opts(const nbody_opts *opts);
// Argument checks of the FP32-position force entry points (before anything is enqueued).
nbody_status check_force_f32(int64_t n, const float *pos, const float *mass, float eps,
                             const double *acc, const double *pot, const nbody_opts &o);
// Pair kernel + FP64 finalize on FP32 positions [3][n] with the partial sums in `ws`
// (partial_bytes(cfg, o.precision) bytes); with kick_v set, v += kick_h * a follows.
nbody_status force_f32_core(int64_t n, const float *pos, const float *mass, float eps, double *acc,
                            double *pot, const nbody_opts &o, const TileCfg &cfg, void *ws,
                            double *kick_v, double kick_h, hipStream_t s);

// Scratch layout of one FP64-position force evaluation: partial sums, FP32 relative
// positions [3][n] (or, with per-i-tile centres, the tile centres), and the partials of
// the system-centre reduction.
struct F64Scratch {
    void *part;
    float *x32;
    double *centre_scratch;
};
size_t f64_scratch_bytes(int64_t n, const TileCfg &cfg, int precision,
                         int outputs = kForceOutputs);
F64Scratch f64_scratch_layout(void *ws, int64_t n, const TileCfg &cfg, int precision,
                              int outputs = kForceOutputs);

// One force evaluation from FP64 positions: centre + conversion (per opts.centre),
// pair kernel, FP64 finalize (optionally followed by v += kick_h * a).
// centre_ready: with NBODY_CENTRE_SYSTEM, the first stage of the centre is already in
// ws.centre_scratch (launch_kick_drift_centre wrote it for these positions).
nbody_status force_f64_core(int64_t n, const double *pos64, const float *mass, float eps,
                            double *acc, double *pot, const nbody_opts &o, const TileCfg &cfg,
                            const F64Scratch &ws, double *kick_v, double kick_h, hipStream_t s,
                            bool centre_ready = false);

// Records the launches `body` enqueues on a capture stream into g->graph and
// instantiates g->exec (integrate.cpp).
nbody_status capture_graph(nbody_graph *g, const std::function<nbody_status(hipStream_t)> &body);

// Device properties cached per device.
struct DeviceInfo {
    int cus = 256;
    int warp = 64;
};
const DeviceInfo &device_info();

// Launchers (force.hip).
nbody_status launch_pair(const TileCfg &cfg, int precision, bool with_pot, const PairArgs &a,
                         hipStream_t s);
nbody_status launch_finalize(int precision, const FinalizeArgs &a, hipStream_t s);
// Split engine (cfg.jl > 1): pair sums and outputs in one launch (force_split.hip,
// vjp_split.hip); the finalize arguments say what is stored.
nbody_status launch_pair_split(const TileCfg &cfg, int precision, bool with_pot,
                               const PairArgs &a, const FinalizeArgs &f, hipStream_t s);
nbody_status launch_vjp_split(const TileCfg &cfg, int precision, const VjpArgs &a, bool with_mass,
                              const VjpFinalizeArgs &f, hipStream_t s);
// Symmetric engine (cfg.sym): pair kernel and its finalize (force_sym.hip).
nbody_status launch_pair_sym(const TileCfg &cfg, int precision, bool with_pot,
                             const PairArgs &a, const FinalizeArgs &f, hipStream_t s);
nbody_status launch_pair_ij(const TileCfg &cfg, int precision, bool with_pot, const IJPairArgs &a,
                            hipStream_t s);
// fp32(x - c) with c the FP64 mean of all positions (two kernels: block partial sums,
// then a fused fixed-order final sum and conversion); scratch holds the partials.
nbody_status launch_centred_convert(int64_t n, const double *pos64, double *scratch,
                                    float *pos32, hipStream_t s);
// The second stage alone, for partials already in `scratch` (written by
// launch_kick_drift_centre).
nbody_status launch_centred_convert_ready(int64_t n, const double *pos64, const double *scratch,
                                          float *pos32, hipStream_t s);
nbody_status launch_convert(int64_t n, const double *pos64, const double *centre, float *pos32,
                            hipStream_t s);
// Bytes of the centre-reduction scratch (partials of the two-stage FP64 sum).
size_t centre_scratch_bytes();
// Per-i-tile FP64 centres (mean position of each tile of `itile` particles) and the pair
// kernel that converts positions relative to them (force.hip).
nbody_status launch_tile_centres(int64_t n, int itile, const double *pos64, double *centres,
                                 hipStream_t s);
nbody_status launch_pair_tile(const TileCfg &cfg, int precision, bool with_pot,
                              const TilePairArgs &a, hipStream_t s);
// Morton (Z-order) permutation of FP64 positions (morton.hip).
nbody_status launch_morton_order(int64_t n, const double *pos64, int32_t *perm, void *scratch,
                                 hipStream_t s);
size_t morton_scratch_bytes(int64_t n);
// Leapfrog pieces (leapfrog.hip).
// v += h a; x += dt v (and checkpoint = x when checkpoint is not null).
nbody_status launch_kick_drift(int64_t n, double *x, double *v, const double *acc, double h,
                               double dt, hipStream_t s, double *checkpoint = nullptr);
// The same kick and drift, fused with the first stage of the FP64 centre of the new
// positions: writes the kCentreBlocks x 3 partials launch_centred_convert computes, in
// the same order, to `centre_part`.
nbody_status launch_kick_drift_centre(int64_t n, double *x, double *v, const double *acc,
                                      double h, double dt, double *checkpoint,
                                      double *centre_part, hipStream_t s);
nbody_status launch_kick(int64_t n, double *v, const double *acc, double h, hipStream_t s);
nbody_status launch_copy_f64(int64_t count, const double *src, double *dst, hipStream_t s);
nbody_status launch_fill_f64(int64_t count, double *dst, double value, hipStream_t s);
// y += alpha * x
nbody_status launch_axpy_f64(int64_t count, double *y, double alpha, const double *x, hipStream_t s);
// Reverse of one leapfrog step's drift and first kick: vbar += dt * xbar; abar = h * vbar.
nbody_status launch_adj_drift_kick(int64_t count, double *vbar, const double *xbar, double *abar,
                                   double dt, double h, hipStream_t s);
// The same update of the 3n-vectors, fused with the centre's first stage over `next`
// (partials to `centre_part`, as launch_centred_convert computes them).
nbody_status launch_adj_drift_kick_centre(int64_t n, double *vbar, const double *xbar, double *abar,
                                          double dt, double h, const double *next,
                                          double *centre_part, hipStream_t s);
// Ragged batches (batched.hip).
nbody_status batched_pair_kernel(int ipl, int jt, int precision, bool with_pot, const void **fn);
nbody_status launch_batched_pair(int ipl, int jt, int precision, bool with_pot, int grid,
                                 const PairArgs &a, const BatchSched &sc, hipStream_t s);
nbody_status launch_batched_finalize(int precision, const BatchFinalizeArgs &a, hipStream_t s);
nbody_status launch_system_centres(int nsys, const int64_t *offsets, int64_t total,
                                   const double *pos64, double *centre, hipStream_t s);
nbody_status launch_batched_convert(int64_t total, const double *pos64, const int32_t *sys_of,
                                    const double *centre, float *pos32, hipStream_t s);
// Force-jerk-potential kernels and their FP64 finalize (jerk.hip, jerk_tile.hip, jerk_ij.hip).
nbody_status launch_jerk(const TileCfg &cfg, int precision, bool with_pot, const JerkArgs &a,
                         hipStream_t s);
nbody_status launch_jerk_finalize(int precision, const JerkFinalizeArgs &a, hipStream_t s);
nbody_status launch_jerk_tile(const TileCfg &cfg, int precision, bool with_pot,
                              const JerkTileArgs &a, hipStream_t s);
nbody_status launch_jerk_ij(const TileCfg &cfg, int precision, bool with_pot, const JerkIJArgs &a,
                            hipStream_t s);
// Fourth-order Hermite predictor and corrector (hermite.hip).
nbody_status launch_hermite_predict(int64_t n, const double *x, const double *v, const double *a,
                                    const double *j, double dt, double *xp, double *vp,
                                    hipStream_t s);
nbody_status launch_hermite_correct(int64_t n, double *x, double *v, double *a, double *j,
                                    const double *a1, const double *j1, double dt, hipStream_t s);
// Adjoint pair kernels and their FP64 finalize (vjp.hip, vjp_tile.hip).
nbody_status launch_vjp(const TileCfg &cfg, int precision, const VjpArgs &a, bool with_mass,
                        hipStream_t s);
nbody_status launch_vjp_tile(const TileCfg &cfg, int precision, const VjpTileArgs &a,
                             bool with_mass, hipStream_t s);
nbody_status launch_vjp_finalize(int precision, const VjpFinalizeArgs &a, hipStream_t s);

}  // namespace nbody
