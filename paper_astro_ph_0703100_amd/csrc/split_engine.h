// Single-launch pair engine for systems too small to fill the chip with whole i-tiles
// (device code, header-only).  Same pipelines (Op) as the tile engine, but the j-range
// of each i-particle is split across lanes of one wavefront instead of across blocks:
//
//   * a wave holds G = 64 / Q i-groups; the Q lanes of a group share IPL i-records
//     and take every Q-th j-record of each staged tile (lane q: slots q, q + Q, ...),
//     so an i-particle's pairs are spread over Q lanes and the 4 waves of a block own
//     different i's: TI = 4 * G * IPL i-particles per block, every j in every block;
//   * j-tiles of JT records are staged in LDS exactly as in the tile engine (coalesced,
//     double-buffered, one barrier per tile); a read instruction of a wave touches Q
//     distinct records, each broadcast to the G lanes that hold different i's;
//   * each lane accumulates its share like the tile engine (PLAIN: FP32; FP64RED: FP32
//     blocks added in FP64; COMP: FP32 blocks added into an FP32 (hi, lo) pair by a
//     two-sum), the FP32 block being the lane's R = JT / Q pairs of one tile;
//   * the Q partial sums of every (i, output) are then added across the lanes of the
//     group in FP64 (PLAIN: FP32) by a butterfly of cross-lane moves: DPP quad
//     permutations and row mirrors for lane distances 1 to 8, v_permlane16_swap and
//     v_permlane32_swap for 16 and 32.  Both lanes of every exchange add the same two
//     values, so all Q lanes end with bitwise the same sum, and the order is fixed;
//   * the group's lanes then store the results through a Sink (lane q stores the slots
//     c with c % Q == q), which also applies what the FP64 finalize of the tile engine
//     applies (self potential, a fused leapfrog kick, the adjoint's own-cotangent term,
//     accumulation).
// No partial sums leave the chip and no second launch is needed; results are bitwise
// reproducible for a given launch shape (IPL, Q, JT).
//
// A Sink provides
//   struct Args;
//   static constexpr int kOutputs;          // the pipeline's outputs it reads
//   static constexpr int stores(bool full);  // store slots per particle
//   template <class Sum> static void put(const Args&, int i, int c, Sum sum);
//                                           // slot c of i-particle i; sum(o) is the FP64
//                                           // sum of output o
#pragma once

#include "tile_engine.h"

namespace nbody {
namespace split {

// Lane distance-M exchange partner value of v (xor butterfly step M), for 32-bit words.
// M = 4 and M = 8 use the row mirrors, which pair lane l with 7 - l (within 8 lanes)
// and 15 - l (within 16): after the steps M = 1, 2 (resp. 1, 2, 4) every lane of a
// quad (resp. of an 8-lane half row) holds the same value, so the mirror partner's
// value is the value of the lane at distance M.
template <int M>
__device__ __forceinline__ int partner_b32(int v) {
    static_assert(M == 1 || M == 2 || M == 4 || M == 8, "DPP steps within a row");
    constexpr int kCtrl = M == 1 ? 0xB1 :   // quad_perm [1, 0, 3, 2]
                          M == 2 ? 0x4E :   // quad_perm [2, 3, 0, 1]
                          M == 4 ? 0x141 :  // row_half_mirror
                                   0x140;   // row_mirror
    return __builtin_amdgcn_mov_dpp(v, kCtrl, 0xF, 0xF, false);
}

// One butterfly step on a float: v + (value of the partner at distance M).
template <int M>
__device__ __forceinline__ float step(float v) {
    if constexpr (M <= 8) {
        return v + __int_as_float(partner_b32<M>(__float_as_int(v)));
    } else if constexpr (M == 16) {
        // Rows 2r and 2r + 1 exchange: both lanes receive (row 2r value, row 2r+1 value)
        // in the same two registers, so both add them in the same order.
        const auto p = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v),
                                                        false, false);
        return __int_as_float(p[0]) + __int_as_float(p[1]);
    } else {
        static_assert(M == 32, "lane distances 1 to 32");
        const auto p = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v),
                                                        false, false);
        return __int_as_float(p[0]) + __int_as_float(p[1]);
    }
}

template <int M>
__device__ __forceinline__ double step(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = (int)(unsigned)(b & 0xffffffffll);
    const int hi = (int)(unsigned)((unsigned long long)b >> 32);
    auto join = [](int l, int h) {
        return __longlong_as_double((long long)(((unsigned long long)(unsigned)h << 32) |
                                                (unsigned)l));
    };
    if constexpr (M <= 8) {
        return v + join(partner_b32<M>(lo), partner_b32<M>(hi));
    } else if constexpr (M == 16) {
        const auto pl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto ph = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        return join(pl[0], ph[0]) + join(pl[1], ph[1]);
    } else {
        static_assert(M == 32, "lane distances 1 to 32");
        const auto pl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto ph = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        return join(pl[0], ph[0]) + join(pl[1], ph[1]);
    }
}

// Sum over the Q consecutive lanes of a group (Q a power of two, 1 to 64); every lane of
// the group returns bitwise the same value.  Must be called by all 64 lanes.
template <int Q, class T>
__device__ __forceinline__ T group_sum(T v) {
    if constexpr (Q >= 2) v = step<1>(v);
    if constexpr (Q >= 4) v = step<2>(v);
    if constexpr (Q >= 8) v = step<4>(v);
    if constexpr (Q >= 16) v = step<8>(v);
    if constexpr (Q >= 32) v = step<16>(v);
    if constexpr (Q >= 64) v = step<32>(v);
    return v;
}

// Records a lane reads from LDS before it runs their pairs: with few waves per SIMD
// (the small systems this engine is for) the LDS latency is not hidden by other waves,
// so each group of kAhead independent pairs is issued after one wait.
constexpr int kAhead = 4;

// One lane's share of an LDS tile: records q, q + Q, ..., q + (R - 1) Q against the
// lane's IPL i-records.  With SELF, self[k] is the tile slot of the lane's k-th own
// particle; that slot's record is swapped for Op::null_j of it.
template <class Op, int IPL, int Q, int JT, int MODE, bool FULL, bool SELF>
__device__ __forceinline__ void lane_pass(const float4 *tl, int q,
                                          const typename Op::IState (&is)[IPL], float eps2,
                                          float (&hs)[IPL][Op::kOut], float (&ls)[IPL][Op::kOut],
                                          double (&ds)[IPL][Op::kOut], const int (&self)[IPL]) {
    constexpr int W = Op::kJWords;
    constexpr int NO = Op::kOut;
    constexpr int R = JT / Q;
    constexpr int A = R < kAhead ? R : kAhead;
    static_assert(R % A == 0, "whole groups of records");
    // Pairs of records r0 .. r0 + A - 1 into acc (reads first, then the pair bodies).
    auto group = [&](int r0, float (&acc)[IPL][NO]) {
        float jr[A][W];
#pragma unroll
        for (int p = 0; p < A; ++p)
#pragma unroll
            for (int v = 0; v < W / 4; ++v) {
                const float4 q4 = tl[((r0 + p) * Q + q) * (W / 4) + v];
                jr[p][4 * v] = q4.x;
                jr[p][4 * v + 1] = q4.y;
                jr[p][4 * v + 2] = q4.z;
                jr[p][4 * v + 3] = q4.w;
            }
#pragma unroll
        for (int p = 0; p < A; ++p)
#pragma unroll
            for (int k = 0; k < IPL; ++k)
                engine::pair_k<Op, FULL, SELF>(jr[p], (r0 + p) * Q + q, self[k], is[k], eps2,
                                               acc[k]);
    };
    if constexpr (MODE == NBODY_PLAIN) {
#pragma unroll 2
        for (int r = 0; r < R; r += A) group(r, hs);
    } else {
        constexpr int BJ = R < Op::kBlockJ ? R : Op::kBlockJ;
        static_assert(R % BJ == 0 && BJ % A == 0, "blocks tile the lane's share");
        for (int rb = 0; rb < R; rb += BJ) {
            float bs[IPL][NO];
#pragma unroll
            for (int k = 0; k < IPL; ++k)
#pragma unroll
                for (int c = 0; c < NO; ++c) bs[k][c] = -0.0f;
#pragma unroll 4
            for (int r = 0; r < BJ; r += A) group(rb + r, bs);
#pragma unroll
            for (int k = 0; k < IPL; ++k)
#pragma unroll
                for (int c = 0; c < NO; ++c) {
                    if constexpr (MODE == NBODY_COMP)
                        engine::two_sum(hs[k][c], ls[k][c], bs[k][c]);
                    else
                        ds[k][c] += (double)bs[k][c];
                }
        }
    }
}

// i-particles per block of a split launch.
template <int IPL, int Q>
constexpr int block_i() {
    return 4 * (64 / Q) * IPL;
}

// Grid: ceil(n_i / block_i) blocks of kTPB lanes; f is the Sink's argument block.
template <class Op, class Sink, int IPL, int Q, int JT, int MODE, bool FULL>
__global__ __launch_bounds__(kTPB) void split_kernel(typename Op::Args a, typename Sink::Args f) {
    constexpr int W = Op::kJWords;
    constexpr int NO = Op::kOut;
    constexpr int G = 64 / Q;
    constexpr int TI = block_i<IPL, Q>();
    constexpr int LPT = (JT + kTPB - 1) / kTPB;  // j-records staged per lane and tile
    static_assert(Q >= 1 && Q <= 64 && (Q & (Q - 1)) == 0, "Q is a power of two");
    static_assert(JT % Q == 0, "every lane takes the same number of records per tile");
    static_assert(W % 4 == 0, "j-records are whole float4s");
    __shared__ float4 tile[2][JT * (W / 4)];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int q = lane % Q;
    const int g = lane / Q;
    const int ni = Op::n_i(a);
    const int nj = Op::n_j(a);
    const int i0 = blockIdx.x * TI;
    const typename Op::Ctx ctx = Op::make_ctx(a, i0);

    // The lane's k-th i-particle; lanes past the end load the last one and store nothing.
    int own[IPL];
    typename Op::IState is[IPL];
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        own[k] = i0 + (k * 4 + wave) * G + g;
        is[k] = Op::load_i(a, ctx, own[k] < ni ? own[k] : ni - 1);
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

    const int ntiles = (nj + JT - 1) / JT;
    float stage[LPT][W];
    auto fetch = [&](int t) {
#pragma unroll
        for (int p = 0; p < LPT; ++p) {
            const int jj = p * kTPB + tid;
            const int j = t * JT + jj;
            if (jj < JT) {
                if (j < nj)
                    Op::load_j(a, ctx, j, stage[p]);
                else
                    Op::pad_j(stage[p]);
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int p = 0; p < LPT; ++p) {
            const int jj = p * kTPB + tid;
            if (jj < JT)
#pragma unroll
                for (int v = 0; v < W / 4; ++v)
                    tile[buf][jj * (W / 4) + v] =
                        make_float4(stage[p][4 * v], stage[p][4 * v + 1], stage[p][4 * v + 2],
                                    stage[p][4 * v + 3]);
        }
    };

    if (ntiles > 0) {
        fetch(0);
        store(0);
    }
    __syncthreads();
    // Every load issued so far (the i-records, the first tile) has completed here; saying
    // so keeps the compiler from waiting on the i-record loads inside the tile loop,
    // where the in-order load counter would also hold back the next tile's loads.
    __builtin_amdgcn_s_waitcnt(engine::kWaitVmem);
    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        if (t + 1 < ntiles) fetch(t + 1);
        const int jt0 = t * JT;
        int self[IPL];
#pragma unroll
        for (int k = 0; k < IPL; ++k) self[k] = own[k] - jt0;
        if constexpr (Op::kSelf) {
            // Uniform over the block: does this tile hold any of the block's own i's?
            if (jt0 < i0 + TI && i0 < jt0 + JT)
                lane_pass<Op, IPL, Q, JT, MODE, FULL, true>(tile[buf], q, is, a.eps2, hs, ls,
                                                            ds, self);
            else
                lane_pass<Op, IPL, Q, JT, MODE, FULL, false>(tile[buf], q, is, a.eps2, hs,
                                                             ls, ds, self);
        } else {
            lane_pass<Op, IPL, Q, JT, MODE, FULL, false>(tile[buf], q, is, a.eps2, hs, ls,
                                                         ds, self);
        }
        if (t + 1 < ntiles) store(buf ^ 1);
        __syncthreads();
    }

    // Cross-lane sums of each (i, output), then the stores: lane q of a group stores the
    // slots c with c % Q == q (every lane of the group holds every sum).
    static_assert(Sink::kOutputs == NO, "the output stage reads the pipeline's outputs");
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
        double rr[NO];
#pragma unroll
        for (int c = 0; c < NO; ++c) {
            rr[c] = 0.0;
            if (!FULL && c == NO - 1) continue;
            if constexpr (MODE == NBODY_PLAIN) {
                rr[c] = (double)group_sum<Q>(hs[k][c]);
            } else if constexpr (MODE == NBODY_COMP) {
                rr[c] = group_sum<Q>((double)hs[k][c] + (double)ls[k][c]);
            } else {
                rr[c] = group_sum<Q>(ds[k][c]);
            }
        }
#pragma unroll
        for (int c = 0; c < Sink::stores(FULL); ++c)
            if (c % Q == q && own[k] < ni) Sink::put(f, own[k], c, [&](int o) { return rr[o]; });
    }
}

// Launch-shape dispatch: IPL in {1, 2}, Q in {8, 16, 32, 64}, JT in {256, 512, 1024,
// 2048} (JT * kJWords * 8 bytes of LDS: at most 32 KB, four or more blocks per CU; or
// 64 KB for 2048 16-byte records and Q >= 32, the tiny systems where one or two tiles
// hold every j and a block's loads should all be in flight at once).
template <class Op, class Sink>
using SplitFn = void (*)(typename Op::Args, typename Sink::Args);

template <class Op, class Sink, int IPL, int Q, int JT>
SplitFn<Op, Sink> spick_mode(int mode, bool full) {
    constexpr bool kFits = JT * Op::kJWords * 8 <= 32768 ||
                           (JT == 2048 && Op::kJWords == 4 && Q >= 32);
    if constexpr (!kFits) {
        return nullptr;
    } else {
        switch (mode) {
            case NBODY_PLAIN:
                return full ? split_kernel<Op, Sink, IPL, Q, JT, NBODY_PLAIN, true>
                            : split_kernel<Op, Sink, IPL, Q, JT, NBODY_PLAIN, false>;
            case NBODY_FP64RED:
                return full ? split_kernel<Op, Sink, IPL, Q, JT, NBODY_FP64RED, true>
                            : split_kernel<Op, Sink, IPL, Q, JT, NBODY_FP64RED, false>;
            case NBODY_COMP:
                return full ? split_kernel<Op, Sink, IPL, Q, JT, NBODY_COMP, true>
                            : split_kernel<Op, Sink, IPL, Q, JT, NBODY_COMP, false>;
        }
        return nullptr;
    }
}

template <class Op, class Sink, int IPL, int Q>
SplitFn<Op, Sink> spick_jt(int jt, int mode, bool full) {
    switch (jt) {
        case 256: return spick_mode<Op, Sink, IPL, Q, 256>(mode, full);
        case 512: return spick_mode<Op, Sink, IPL, Q, 512>(mode, full);
        case 1024: return spick_mode<Op, Sink, IPL, Q, 1024>(mode, full);
        case 2048: return spick_mode<Op, Sink, IPL, Q, 2048>(mode, full);
    }
    return nullptr;
}

template <class Op, class Sink, int IPL>
SplitFn<Op, Sink> spick_q(int q, int jt, int mode, bool full) {
    switch (q) {
        case 8: return spick_jt<Op, Sink, IPL, 8>(jt, mode, full);
        case 16: return spick_jt<Op, Sink, IPL, 16>(jt, mode, full);
        case 32: return spick_jt<Op, Sink, IPL, 32>(jt, mode, full);
        case 64: return spick_jt<Op, Sink, IPL, 64>(jt, mode, full);
    }
    return nullptr;
}

template <class Op, class Sink>
SplitFn<Op, Sink> pick_split(int ipl, int q, int jt, int mode, bool full) {
    switch (ipl) {
        case 1: return spick_q<Op, Sink, 1>(q, jt, mode, full);
        case 2: return spick_q<Op, Sink, 2>(q, jt, mode, full);
    }
    return nullptr;
}

}  // namespace split
}  // namespace nbody
