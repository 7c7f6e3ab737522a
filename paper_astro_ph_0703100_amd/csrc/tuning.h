// Launch-shape table: built-in defaults, optionally overridden by a JSON file
// written by the autotuner (nbody_tune_load / nbody_tune_save).
#pragma once

#include <cstdint>

namespace nbody {

enum TuneKernel { KERNEL_FORCE = 0, KERNEL_VJP = 1, KERNEL_BATCHED = 2, KERNEL_JERK = 3, KERNEL_COUNT = 4 };

struct TuneEntry {
    int ipl;      // i-particles per lane
    int jt;       // j-tile
    int nseg;     // j-segments, 0 = chosen from n (grid engine); symmetric engine: segments
                  // of the longest block row, 0 = chosen from n
    int jl = 1;   // lanes per i-particle's j-range: 1 = grid engine, 8..64 = split engine
    int sym = 0;  // 1: symmetric engine (jl = 1)
};

// Engines a caller has kernels for besides the grid engine (bit mask).
constexpr int kEngineSplit = 1;  // split engine: single-set force and adjoint
constexpr int kEngineSym = 2;    // symmetric engine: single-set force on FP32 positions

// True if (ipl, jt, nseg, jl) is a shape the library has kernels for (kernel: TuneKernel).
bool valid_shape(int kernel, const TuneEntry &e);

// floor(log2 n) (0 for n < 2): the size bucket of the table.
int size_bucket(int64_t n);

// Shape for a kernel, precision mode and problem size (size bucket = floor(log2 n)).
// A table entry for an engine the caller has no kernel for (engines: kEngine* bits) is
// passed over for the built-in shape.
TuneEntry tuned_shape(int kernel, int precision, int64_t n, int engines);

// Replace the entry for (kernel, precision, size bucket of n).
void set_tuned_shape(int kernel, int precision, int64_t n, const TuneEntry &e);

}  // namespace nbody
