// Generic i-tile x j-tile pair engine for gfx950 (device code, header-only).
//
// The paper's library evaluates arbitrary pair interactions from a user-written pipeline
// description that reads an i-record and a j-record and accumulates outputs
// (Sec. 4.5, Appendix A).  This engine is that idea on CDNA4: a pipeline type `Op`
// supplies the records and the pair body; the engine supplies the blocking.
//
//   * a block of 256 lanes owns an i-tile of 256 * IPL particles; each lane keeps IPL
//     i-records in VGPRs (lane-strided so global loads and stores coalesce);
//   * blockIdx.y selects a j-segment; the block walks it in LDS tiles of JT
//     j-records, staged with coalesced loads and double-buffered (one barrier per
//     tile), the J-BAG / J-PACKING of Sec. 2.2;
//   * every lane reads each j-record from LDS with broadcast 16-byte reads and runs
//     the pair body for its IPL i-records;
//   * the j == i pair is left out of every sum (eq. (1) sums over the other
//     particles): in the few j-tiles that hold some of the block's own i's (i- and
//     j-sets the same, Op::kSelf), each lane swaps the record of its own particle
//     for Op::null_j of it (same position, nothing that adds), by a compare and a
//     select per pair; all other tiles run the plain pass;
//   * accumulation (Sec. 2.2.2, eq. (2); Sec. 3.4):
//       PLAIN   - one FP32 accumulator per output and (i, segment);
//       FP64RED - FP32 partial over each block of min(Op::kBlockJ, JT) j's, added into FP64;
//       COMP    - FP32 partial over each block, added into an FP32 (hi, lo) pair by an
//                 error-free two-sum;
//   * partial sums go to scratch planes [segment][word][npad]; a finalize kernel adds
//     the segments in a fixed order in FP64 (PLAIN: FP32).
// No atomics: every result is a fixed-order sum, bitwise reproducible per launch shape.
//
// An Op provides:
//   static constexpr int kJWords;            // floats per j-record (multiple of 4)
//   static constexpr int kOut;               // outputs per i
//   static constexpr int kBlockJ;            // j's per FP32 block before compensation
//   struct Args;                             // kernel arguments (seg_len, eps2, part, npad, ...)
//   static int n_i(const Args&), n_j(const Args&);  // i- and j-counts of a grid launch
//   struct IState;                           // per-i registers
//   struct Ctx;                              // per-block context (e.g. a reference centre)
//   static Ctx make_ctx(const Args&, int i0);
//   static IState load_i(const Args&, const Ctx&, int i);
//   static void load_j(const Args&, const Ctx&, int j, float (&r)[kJWords]);
//   static void pad_j(float (&r)[kJWords]);  // a record that adds exactly zero
//   static constexpr bool kSelf;             // i- and j-sets are one set (j == i exists)
//   static void null_j(float (&r)[kJWords]); // (kSelf only) turns a j-record into one at
//                                            // the same place that adds nothing: the
//                                            // j == i pair then adds exactly zero
//   template <bool FULL> static void pair(const float *jr, const IState&, float eps2,
//                                         float (&acc)[kOut]);
//   (FULL = false may skip the last output.)
#pragma once

#include <type_traits>

#include "nbody_internal.h"

namespace nbody {
namespace engine {

// s_waitcnt vmcnt(0) (expcnt and lgkmcnt left at their maxima, 7 and 15, in the gfx9
// encoding): wait for every outstanding vector-memory load of the wave.  Issued once
// after the first j-tile is staged, it tells the compiler that the i-record loads have
// completed; otherwise it waits on them inside the tile loop, where the in-order load
// counter also holds back the prefetch of the next tile (its latency then shows at
// every tile).
constexpr int kWaitVmem = 0x0F70;

// Knuth's error-free sum: hi + lo += b with hi = fl(hi + b) and the rounding error of
// that addition added to lo.
__device__ __forceinline__ void two_sum(float &hi, float &lo, float b) {
    const float s = hi + b;
    const float bb = s - hi;
    const float err = (hi - (s - bb)) + (b - bb);
    hi = s;
    lo = lo + err;
}

// One pair of the lane's k-th i-record with j-record jr; with SELF, the record of the
// lane's own particle (tile slot jj == self[k]) is replaced by Op::null_j of it.
template <class Op, bool FULL, bool SELF>
__device__ __forceinline__ void pair_k(const float *jr, int jj, int self_k,
                                       const typename Op::IState &is, float eps2,
                                       float (&acc)[Op::kOut]) {
    if constexpr (SELF) {
        float r[Op::kJWords];
        float z[Op::kJWords];
#pragma unroll
        for (int w = 0; w < Op::kJWords; ++w) r[w] = z[w] = jr[w];
        Op::null_j(z);
        const bool own = jj == self_k;
#pragma unroll
        for (int w = 0; w < Op::kJWords; ++w) r[w] = own ? z[w] : r[w];
        Op::template pair<FULL>(r, is, eps2, acc);
    } else {
        Op::template pair<FULL>(jr, is, eps2, acc);
    }
}

// One LDS tile: all JT j-records against the lane's IPL i-records.  With SELF, self[k]
// is the tile slot of the lane's k-th own particle (outside [0, JT) if not in it).
template <class Op, int IPL, int JT, int MODE, bool FULL, bool SELF = false>
__device__ __forceinline__ void tile_pass(const float4 *tl, const typename Op::IState (&is)[IPL],
                                          float eps2, float (&hs)[IPL][Op::kOut],
                                          float (&ls)[IPL][Op::kOut],
                                          double (&ds)[IPL][Op::kOut],
                                          const int (&self)[IPL]) {
    constexpr int W = Op::kJWords;
    constexpr int NO = Op::kOut;
    auto read = [&](int jj, float (&jr)[W]) {
#pragma unroll
        for (int v = 0; v < W / 4; ++v) {
            const float4 q4 = tl[jj * (W / 4) + v];
            jr[4 * v] = q4.x;
            jr[4 * v + 1] = q4.y;
            jr[4 * v + 2] = q4.z;
            jr[4 * v + 3] = q4.w;
        }
    };
    // The pass with the self test runs on a few tiles only: a shorter unroll keeps its
    // code small.
    constexpr int kUnrollPlain = SELF ? 4 : 8;
    if constexpr (MODE == NBODY_PLAIN) {
#pragma unroll kUnrollPlain
        for (int jj = 0; jj < JT; ++jj) {
            float jr[W];
            read(jj, jr);
#pragma unroll
            for (int k = 0; k < IPL; ++k)
                pair_k<Op, FULL, SELF>(jr, jj, self[k], is[k], eps2, hs[k]);
        }
    } else {
        constexpr int BJ = JT < Op::kBlockJ ? JT : Op::kBlockJ;
        static_assert(JT % BJ == 0, "blocks tile the j-tile");
        for (int jb = 0; jb < JT; jb += BJ) {
            float bs[IPL][NO];
#pragma unroll
            for (int k = 0; k < IPL; ++k)
#pragma unroll
                for (int c = 0; c < NO; ++c) bs[k][c] = -0.0f;
            // Unrolled 32 pairs deep: longer blocks loop over that body (a scalar
            // branch per 32 pairs) instead of growing the code and the build time.
            constexpr int kUnroll = SELF ? 8 : 32;
#pragma unroll kUnroll
            for (int jj = 0; jj < BJ; ++jj) {
                float jr[W];
                read(jb + jj, jr);
#pragma unroll
                for (int k = 0; k < IPL; ++k)
                    pair_k<Op, FULL, SELF>(jr, jb + jj, self[k], is[k], eps2, bs[k]);
            }
#pragma unroll
            for (int k = 0; k < IPL; ++k)
#pragma unroll
                for (int c = 0; c < NO; ++c) {
                    if constexpr (MODE == NBODY_COMP)
                        two_sum(hs[k][c], ls[k][c], bs[k][c]);
                    else
                        ds[k][c] += (double)bs[k][c];
                }
        }
    }
}

// One block's work: the i-tile [i0, i0 + ni) (ni <= 256 * IPL) against the j-range
// [j0, j0 + nj), partial sums written to planes out[word * plane + col0 + lane-slot].
// `tile` is the block's LDS staging area; every lane of the block must call this
// with the same arguments (it contains barriers).
template <class Op, int IPL, int JT, int MODE, bool FULL>
__device__ __forceinline__ void block_work(const typename Op::Args &a, float4 (*tile)[JT * (Op::kJWords / 4)],
                                           int i0, int ni, int j0, int nj, float eps2, void *out,
                                           size_t plane, size_t col0) {
    constexpr int W = Op::kJWords;
    constexpr int NO = Op::kOut;
    constexpr int LPT = (JT + kTPB - 1) / kTPB;  // j-records staged per lane
    static_assert(W % 4 == 0, "j-records are whole float4s");
    const int tid = threadIdx.x;
    const typename Op::Ctx ctx = Op::make_ctx(a, i0);

    typename Op::IState is[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const int r = k * kTPB + tid;
        is[k] = Op::load_i(a, ctx, i0 + (r < ni ? r : ni - 1));
    }

    float hs[IPL][NO], ls[IPL][NO];
    double ds[IPL][NO];
#pragma unroll
    for (int k = 0; k < IPL; ++k)
#pragma unroll
        for (int c = 0; c < NO; ++c) {
            hs[k][c] = 0.0f;
            ls[k][c] = 0.0f;
            ds[k][c] = 0.0;
        }

    const int j1 = j0 + nj;
    const int ntiles = nj > 0 ? (nj + JT - 1) / JT : 0;

    float stage[LPT][W];
    auto fetch = [&](int t) {
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const int jj = q * kTPB + tid;
            const int j = j0 + t * JT + jj;
            if (jj < JT) {
                if (j < j1)
                    Op::load_j(a, ctx, j, stage[q]);
                else
                    Op::pad_j(stage[q]);
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < LPT; ++q) {
            const int jj = q * kTPB + tid;
            if (jj < JT)
#pragma unroll
                for (int v = 0; v < W / 4; ++v)
                    tile[buf][jj * (W / 4) + v] =
                        make_float4(stage[q][4 * v], stage[q][4 * v + 1], stage[q][4 * v + 2],
                                    stage[q][4 * v + 3]);
        }
    };

    // Global index of the lane's k-th own particle (padding lanes of the last i-tile
    // get indices >= n, whose j-slots hold padding records or nothing).
    int own[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) own[k] = i0 + k * kTPB + tid;

    if (ntiles > 0) {
        fetch(0);
        store(0);
    }
    __syncthreads();
    __builtin_amdgcn_s_waitcnt(kWaitVmem);
    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        if (t + 1 < ntiles) fetch(t + 1);
        const int jt0 = j0 + t * JT;
        int self[IPL];
#pragma unroll
        for (int k = 0; k < IPL; ++k) self[k] = own[k] - jt0;
        if constexpr (Op::kSelf) {
            // Uniform over the block: does this tile hold any of the block's own i's?
            if (jt0 < i0 + kTPB * IPL && i0 < jt0 + JT)
                tile_pass<Op, IPL, JT, MODE, FULL, true>(tile[buf], is, eps2, hs, ls, ds, self);
            else
                tile_pass<Op, IPL, JT, MODE, FULL, false>(tile[buf], is, eps2, hs, ls, ds, self);
        } else {
            tile_pass<Op, IPL, JT, MODE, FULL, false>(tile[buf], is, eps2, hs, ls, ds, self);
        }
        if (t + 1 < ntiles) store(buf ^ 1);
        __syncthreads();
    }

#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        const size_t i = col0 + k * kTPB + tid;
        if constexpr (MODE == NBODY_FP64RED) {
            double *p = static_cast<double *>(out) + i;
#pragma unroll
            for (int c = 0; c < NO; ++c) p[c * plane] = ds[k][c];
        } else if constexpr (MODE == NBODY_COMP) {
            float *p = static_cast<float *>(out) + i;
#pragma unroll
            for (int c = 0; c < NO; ++c) {
                p[c * plane] = hs[k][c];
                p[(NO + c) * plane] = ls[k][c];
            }
        } else {
            float *p = static_cast<float *>(out) + i;
#pragma unroll
            for (int c = 0; c < NO; ++c) p[c * plane] = hs[k][c];
        }
    }
}

// Words (4 bytes) of partial sums per output, i-particle and segment.
template <int MODE>
constexpr int words_per_out() {
    return MODE == NBODY_PLAIN ? 1 : 2;
}

// Grid launch: blockIdx.x = i-tile, blockIdx.y = j-segment of a.seg_len j's.  Partial
// planes [seg][word][npad].
template <class Op, int IPL, int JT, int MODE, bool FULL>
__global__ __launch_bounds__(kTPB) void tile_kernel(typename Op::Args a) {
    __shared__ float4 tile[2][JT * (Op::kJWords / 4)];
    const int i0 = blockIdx.x * (kTPB * IPL);
    const int ni = min(kTPB * IPL, Op::n_i(a) - i0);
    const int j0 = blockIdx.y * a.seg_len;
    const int nj = max(0, min(a.seg_len, Op::n_j(a) - j0));
    const size_t plane = (size_t)a.npad;
    constexpr int WO = Op::kOut * words_per_out<MODE>();
    void *out = static_cast<float *>(a.part) + (size_t)blockIdx.y * WO * plane;
    block_work<Op, IPL, JT, MODE, FULL>(a, tile, i0, ni, j0, nj, a.eps2, out, plane, (size_t)i0);
}

// Persistent launch over a list of work items (ragged batches of independent
// systems).  Each block takes the next item from an atomic ticket until the list is
// exhausted; items are sorted by decreasing cost so the tail is short.  Every item
// writes its own partial slots, so results do not depend on which block ran it.
template <class Op, int IPL, int JT, int MODE, bool FULL>
__global__ __launch_bounds__(kTPB) void persistent_kernel(typename Op::Args a, BatchSched sc) {
    __shared__ float4 tile[2][JT * (Op::kJWords / 4)];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(sc.counter, 1u);
        __syncthreads();
        const int it = s_item;
        __syncthreads();  // all lanes hold `it` before lane 0 can overwrite s_item
        if (it >= sc.nitems) break;
        const BatchItem w = sc.items[it];
        const float e = sc.eps[w.sys];
        void *out = static_cast<float *>(sc.part) + w.part;
        block_work<Op, IPL, JT, MODE, FULL>(a, tile, w.i0, w.ni, w.j0, w.nj, e * e, out,
                                            (size_t)w.npad, (size_t)w.col0);
    }
}

// Fixed-order sums of the segment partials.  Segment s holds, per output c, the words
// [s][c][plane] (PLAIN: FP32; FP64RED: FP64) or [s][c][plane] = hi and [s][NO + c][plane]
// = lo (COMP: FP32), summed as r += hi; r += lo.  The loads run a batch of segments
// ahead of the additions, which stay strictly sequential in s: with few particles the
// finalize has few waves and is bound by load latency, not bandwidth.
template <int NO, int MODE>
struct PartialLayout {
    using T = typename std::conditional<MODE == NBODY_FP64RED, double, float>::type;
    static constexpr int kWords = MODE == NBODY_COMP ? 2 : 1;  // hi (, lo) per output
    static constexpr int kStride = kWords * NO;                 // words per segment and column
};

// Segments whose loads a finalize thread issues ahead of its additions: 8 when the
// finalize has under 4 waves per SIMD (bound by load latency: at N = 16384 the force
// finalize went from 18 to 6 us), 1 otherwise (bound by bandwidth; a deeper batch only
// scatters the DRAM accesses: at N = 131072 it went from 26 to 39 us).
inline int finalize_batch(int64_t n, int outputs) {
    return n * outputs < (int64_t)4 * 1024 * 64 ? 8 : 1;
}

// One output c of particle i (FP64 for FP64RED/COMP, FP32 for PLAIN, returned widened).
template <int NO, int MODE, int BATCH>
__device__ __forceinline__ double sum_partial_output(const void *part, int nseg, size_t plane,
                                                     int i, int c) {
    using L = PartialLayout<NO, MODE>;
    using T = typename L::T;
    const T *p = static_cast<const T *>(part) + i + (size_t)c * plane;
    const size_t step = (size_t)L::kStride * plane;
    const size_t lo = (size_t)NO * plane;  // COMP: offset of the lo word
    using Acc = typename std::conditional<MODE == NBODY_PLAIN, float, double>::type;
    Acc r = 0;
    int s = 0;
    for (; s + BATCH <= nseg; s += BATCH) {
        T v[BATCH][L::kWords];
#pragma unroll
        for (int b = 0; b < BATCH; ++b) {
            v[b][0] = p[(size_t)(s + b) * step];
            if constexpr (L::kWords == 2) v[b][L::kWords - 1] = p[(size_t)(s + b) * step + lo];
        }
#pragma unroll
        for (int b = 0; b < BATCH; ++b)
#pragma unroll
            for (int w = 0; w < L::kWords; ++w) r = r + (Acc)v[b][w];
    }
    for (; s < nseg; ++s) {
        r = r + (Acc)p[(size_t)s * step];
        if constexpr (L::kWords == 2) r = r + (Acc)p[(size_t)s * step + lo];
    }
    return (double)r;
}

// All NO outputs of particle i in r[0 .. NO), each with the rounding of the
// corresponding sum_partial_output.
template <int NO, int MODE, int BATCH>
__device__ __forceinline__ void sum_partials(const void *part, int nseg, size_t plane, int i,
                                             double (&r)[NO]) {
    using L = PartialLayout<NO, MODE>;
    using T = typename L::T;
    const T *p = static_cast<const T *>(part) + i;
    const size_t step = (size_t)L::kStride * plane;
    const size_t lo = (size_t)NO * plane;
    using Acc = typename std::conditional<MODE == NBODY_PLAIN, float, double>::type;
    Acc acc[NO];
#pragma unroll
    for (int c = 0; c < NO; ++c) acc[c] = 0;
    int s = 0;
    for (; s + BATCH <= nseg; s += BATCH) {
        T v[BATCH][NO][L::kWords];
#pragma unroll
        for (int b = 0; b < BATCH; ++b)
#pragma unroll
            for (int c = 0; c < NO; ++c) {
                v[b][c][0] = p[(size_t)(s + b) * step + (size_t)c * plane];
                if constexpr (L::kWords == 2)
                    v[b][c][L::kWords - 1] = p[(size_t)(s + b) * step + (size_t)c * plane + lo];
            }
#pragma unroll
        for (int b = 0; b < BATCH; ++b)
#pragma unroll
            for (int c = 0; c < NO; ++c)
#pragma unroll
                for (int w = 0; w < L::kWords; ++w) acc[c] = acc[c] + (Acc)v[b][c][w];
    }
    for (; s < nseg; ++s)
#pragma unroll
        for (int c = 0; c < NO; ++c) {
            acc[c] = acc[c] + (Acc)p[(size_t)s * step + (size_t)c * plane];
            if constexpr (L::kWords == 2)
                acc[c] = acc[c] + (Acc)p[(size_t)s * step + (size_t)c * plane + lo];
        }
#pragma unroll
    for (int c = 0; c < NO; ++c) r[c] = (double)acc[c];
}

// Launch-shape dispatch over the template parameters.
template <class Op>
using TileFn = void (*)(typename Op::Args);

template <class Op, int IPL, int JT, int MODE>
TileFn<Op> pick_full(bool full) {
    return full ? tile_kernel<Op, IPL, JT, MODE, true> : tile_kernel<Op, IPL, JT, MODE, false>;
}

template <class Op, int IPL, int JT>
TileFn<Op> pick_mode(int mode, bool full) {
    switch (mode) {
        case NBODY_PLAIN: return pick_full<Op, IPL, JT, NBODY_PLAIN>(full);
        case NBODY_FP64RED: return pick_full<Op, IPL, JT, NBODY_FP64RED>(full);
        case NBODY_COMP: return pick_full<Op, IPL, JT, NBODY_COMP>(full);
    }
    return nullptr;
}

template <class Op, int IPL>
TileFn<Op> pick_jt(int jt, int mode, bool full) {
    switch (jt) {
        case 64: return pick_mode<Op, IPL, 64>(mode, full);
        case 128: return pick_mode<Op, IPL, 128>(mode, full);
        case 256: return pick_mode<Op, IPL, 256>(mode, full);
        case 512: return pick_mode<Op, IPL, 512>(mode, full);
    }
    return nullptr;
}

template <class Op>
TileFn<Op> pick_tile(int ipl, int jt, int mode, bool full) {
    switch (ipl) {
        case 1: return pick_jt<Op, 1>(jt, mode, full);
        case 2: return pick_jt<Op, 2>(jt, mode, full);
        case 4: return pick_jt<Op, 4>(jt, mode, full);
        case 8: return pick_jt<Op, 8>(jt, mode, full);
    }
    return nullptr;
}

template <class Op>
using PersistFn = void (*)(typename Op::Args, BatchSched);

template <class Op, int IPL, int JT, int MODE>
PersistFn<Op> ppick_full(bool full) {
    return full ? persistent_kernel<Op, IPL, JT, MODE, true> : persistent_kernel<Op, IPL, JT, MODE, false>;
}

template <class Op, int IPL, int JT>
PersistFn<Op> ppick_mode(int mode, bool full) {
    switch (mode) {
        case NBODY_PLAIN: return ppick_full<Op, IPL, JT, NBODY_PLAIN>(full);
        case NBODY_FP64RED: return ppick_full<Op, IPL, JT, NBODY_FP64RED>(full);
        case NBODY_COMP: return ppick_full<Op, IPL, JT, NBODY_COMP>(full);
    }
    return nullptr;
}

template <class Op, int IPL>
PersistFn<Op> ppick_jt(int jt, int mode, bool full) {
    switch (jt) {
        case 64: return ppick_mode<Op, IPL, 64>(mode, full);
        case 128: return ppick_mode<Op, IPL, 128>(mode, full);
        case 256: return ppick_mode<Op, IPL, 256>(mode, full);
        case 512: return ppick_mode<Op, IPL, 512>(mode, full);
    }
    return nullptr;
}

template <class Op>
PersistFn<Op> pick_persistent(int ipl, int jt, int mode, bool full) {
    switch (ipl) {
        case 1: return ppick_jt<Op, 1>(jt, mode, full);
        case 2: return ppick_jt<Op, 2>(jt, mode, full);
        case 4: return ppick_jt<Op, 4>(jt, mode, full);
        case 8: return ppick_jt<Op, 8>(jt, mode, full);
    }
    return nullptr;
}

}  // namespace engine
}  // namespace nbody
