// Internal declarations shared by the translation units of libnbody.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "nbody.h"

namespace nbody {

// Threads per block of every pair kernel: four 64-wide wavefronts, one per SIMD of
// a compute unit.
constexpr int kTPB = 256;
// Largest number of j-segments a launch may split the j range into.
constexpr int kMaxSeg = 128;
// j's summed in plain FP32 between two compensation / FP64 steps.
constexpr int kBlockJ = 32;

// Words (4-byte) of partial sums written per i-particle and j-segment.
inline int partial_words(int precision) {
    return precision == NBODY_PLAIN ? 4 : 8;  // comp: hi[4], lo[4]; fp64red: double[4]
}

// Shape of one force launch.
struct TileCfg {
    int ipl = 4;     // i-particles per lane
    int jt = 256;    // j-particles per LDS tile
    int nseg = 1;    // j-segments (grid y)
    int seg_len = 0; // j's per segment, a multiple of jt
    int itiles = 0;  // i-tiles (grid x)
    int npad = 0;    // itiles * kTPB * ipl
};

// Arguments of the pair kernel (FP32 structure-of-arrays input).
struct PairArgs {
    const float *x, *y, *z, *m;
    int n;        // particles
    int seg_len;  // j's per segment
    float eps2;   // fp32(eps^2)
    void *part;   // partial sums [nseg][words][npad]
    int npad;
};

// Arguments of the FP64 reduction of the partial sums.
struct FinalizeArgs {
    const void *part;
    int nseg, npad, n;
    const float *m;
    float eps2;
    int self_pot;      // 1: keep the j == i term of phi
    double *acc;       // [3][n]
    double *pot;       // [n] or nullptr
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
nbody_status launch_centre(int64_t n, const double *pos64, double *centre, double *scratch,
                           hipStream_t s);
nbody_status launch_convert(int64_t n, const double *pos64, const double *centre, float *pos32,
                            hipStream_t s);
// Bytes of the centre-reduction scratch (partials of the two-stage FP64 sum).
size_t centre_scratch_bytes();

}  // namespace nbody
