// Force evaluation of one system on the symmetric engine: every unordered pair once,
// its term added to both particles; the FP64 finalize adds each particle's i-side
// segment partials and the j-side sums of the block rows before it.
#include "outputs.h"
#include "sym_engine.h"

namespace nbody {
namespace {

// Finalize arguments of the symmetric engine beyond the tile engine's.
struct SymFinal {
    const void *jpart;  // rows 0 .. nb - 2 (sym::jrow_base), FP64 (PLAIN: FP32)
    int bi, jt, segt, nb;
};

// Fixed order per particle i of block row q: its row's segment partials (as the tile
// engine's finalize), then the j-planes of rows 0 .. q - 1.  Grid: (ceil(n / 256),
// 4 outputs, or 3 without potentials).
template <int MODE, int BATCH>
__global__ __launch_bounds__(256) void sym_finalize_kernel(FinalizeArgs a, SymFinal f) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (i >= a.n) return;
    const int q = i / f.bi;
    const int nseg = sym::row_segments(a.n, f.bi, f.jt, f.segt, q);
    ForceOut::put(a, i, c, [&](int o) {
        const double si = engine::sum_partial_output<kForceOutputs, MODE, BATCH>(
            a.part, nseg, (size_t)a.npad, i, o);
        using T = typename std::conditional<MODE == NBODY_PLAIN, float, double>::type;
        const T *p = static_cast<const T *>(f.jpart);
        // Particle i's output o in row b's j-plane.
        auto at = [&](int b) {
            return p[sym::jrow_base(f.nb, f.bi, b) + (size_t)o * sym::jrow_len(f.nb, f.bi, b) +
                     (size_t)(i - (b + 1) * f.bi)];
        };
        T r = (T)si;
        int b = 0;
        for (; b + BATCH <= q; b += BATCH) {
            T v[BATCH];
#pragma unroll
            for (int k = 0; k < BATCH; ++k) v[k] = at(b + k);
#pragma unroll
            for (int k = 0; k < BATCH; ++k) r = r + v[k];
        }
        for (; b < q; ++b) r = r + at(b);
        return (double)r;
    });
}

template <int MODE>
void launch_sym_finalize(dim3 grid, const FinalizeArgs &a, const SymFinal &f, hipStream_t s) {
    hipLaunchKernelGGL((sym_finalize_kernel<MODE, 8>), grid, dim3(256), 0, s, a, f);
}

using SymFn = void (*)(SymArgs);

template <int IPL, int JT, int MODE>
SymFn pick_full(bool full) {
    return full ? sym::sym_kernel<kSymWaves, IPL, JT, MODE, true>
                : sym::sym_kernel<kSymWaves, IPL, JT, MODE, false>;
}

template <int IPL, int JT>
SymFn pick_mode(int mode, bool full) {
    switch (mode) {
        case NBODY_PLAIN: return pick_full<IPL, JT, NBODY_PLAIN>(full);
        case NBODY_FP64RED: return pick_full<IPL, JT, NBODY_FP64RED>(full);
        case NBODY_COMP: return pick_full<IPL, JT, NBODY_COMP>(full);
    }
    return nullptr;
}

template <int IPL>
SymFn pick_jt(int jt, int mode, bool full) {
    switch (jt) {
        case 64: return pick_mode<IPL, 64>(mode, full);
        case 128: return pick_mode<IPL, 128>(mode, full);
    }
    return nullptr;
}

SymFn pick_sym(int ipl, int jt, int mode, bool full) {
    switch (ipl) {
        case 1: return pick_jt<1>(jt, mode, full);
        case 2: return pick_jt<2>(jt, mode, full);
        case 4: return pick_jt<4>(jt, mode, full);
    }
    return nullptr;
}

}  // namespace

nbody_status launch_pair_sym(const TileCfg &cfg, int precision, bool with_pot,
                             const PairArgs &a, const FinalizeArgs &f, hipStream_t s) {
    auto fn = pick_sym(cfg.ipl, cfg.jt, precision, with_pot);
    if (!fn) return set_error(NBODY_EUNSUPPORTED, "no symmetric-engine kernel for this shape");
    if (a.n <= 0) return NBODY_OK;
    const int bi = 64 * kSymWaves * cfg.ipl;
    const size_t ibytes = sym_ipart_bytes(cfg, precision);  // the j-side sums follow
    SymArgs sa{a.x, a.y, a.z, a.m, a.n, a.eps2, cfg.segt, cfg.nb, cfg.nseg, cfg.npad,
               a.part, static_cast<char *>(a.part) + ibytes};
    hipLaunchKernelGGL(fn, dim3(cfg.nitems), dim3(64 * kSymWaves), 0, s, sa);
    NBODY_HIP_CHECK(hipGetLastError());
    const SymFinal sf{sa.jpart, bi, cfg.jt, cfg.segt, cfg.nb};
    const int outputs = f.pot ? 4 : 3;
    const dim3 grid((f.n + 255) / 256, outputs);
    switch (precision) {
        case NBODY_PLAIN: launch_sym_finalize<NBODY_PLAIN>(grid, f, sf, s); break;
        case NBODY_FP64RED: launch_sym_finalize<NBODY_FP64RED>(grid, f, sf, s); break;
        case NBODY_COMP: launch_sym_finalize<NBODY_COMP>(grid, f, sf, s); break;
        default: return set_error(NBODY_EINVAL, "unknown precision mode");
    }
    NBODY_HIP_CHECK(hipGetLastError());
    return NBODY_OK;
}

}  // namespace nbody
