// Launch-shape table (see tuning.h).
#include "tuning.h"

#include <mutex>

#include "nbody.h"

namespace nbody {
namespace {

constexpr int kBuckets = 32;
std::mutex g_mu;
bool g_set[KERNEL_COUNT][3][kBuckets];
TuneEntry g_tab[KERNEL_COUNT][3][kBuckets];

int bucket(int64_t n) {
    int b = 0;
    while (b + 1 < kBuckets && (int64_t(1) << (b + 1)) <= n) ++b;
    return b;
}

TuneEntry builtin(int kernel, int64_t n) {
    if (kernel == KERNEL_BATCHED) {
        // n is the mean system size; small systems waste lanes of wide i-tiles.
        if (n >= 2048) return {2, 128, 0};
        return {1, 128, 0};
    }
    if (kernel == KERNEL_VJP) {
        // The adjoint keeps 8 i-values and 4 accumulators (x3 when blocked) per
        // i-particle; two per lane keep it within about 100 VGPRs.
        if (n >= 8192) return {2, 128, 0};
        return {1, 128, 0};
    }
    // More i-particles per lane amortise each LDS read over more pair terms, but
    // leave fewer i-tiles to spread over the compute units for small n.
    if (n >= 32768) return {4, 256, 0};
    if (n >= 8192) return {2, 256, 0};
    return {1, 128, 0};
}

}  // namespace

TuneEntry tuned_shape(int kernel, int precision, int64_t n) {
    if (kernel < 0 || kernel >= KERNEL_COUNT || precision < 0 || precision > 2) return builtin(0, n);
    std::lock_guard<std::mutex> lk(g_mu);
    const int b = bucket(n);
    if (g_set[kernel][precision][b]) return g_tab[kernel][precision][b];
    return builtin(kernel, n);
}

void set_tuned_shape(int kernel, int precision, int64_t n, const TuneEntry &e) {
    if (kernel < 0 || kernel >= KERNEL_COUNT || precision < 0 || precision > 2) return;
    std::lock_guard<std::mutex> lk(g_mu);
    const int b = bucket(n);
    g_tab[kernel][precision][b] = e;
    g_set[kernel][precision][b] = true;
}

}  // namespace nbody
