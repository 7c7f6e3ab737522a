// Symmetric pair engine for the single-set gravity force on FP32 positions (device
// code, header-only).  The pair term of eq. (1) is antisymmetric: particle j pulls i
// with m_j d / s^3 and i pulls j with -m_i d / s^3 (d = x_j - x_i), and the potential
// terms share the same 1 / s.  The ordered-pair engines form every separation,
// reciprocal square root and r^3 twice, once per direction; this engine forms them once
// per unordered pair {i, j} and adds the term to both particles.
//
//   * particles are grouped in block rows of BI = 64 W IPL (W waves of 64 lanes, IPL
//     per lane, lane-strided); row b's work is the one-sided pairs among its own
//     particles (the diagonal, j == i left out as in the tile engine) and the
//     symmetric pairs with every particle j >= (b + 1) BI, walked in LDS j-tiles of JT
//     records;
//   * a work item (one block) is (row b, segment s): segment s covers `segt` j-tiles
//     of the row's symmetric range, and segment 0 also runs the diagonal.  Items are
//     numbered segment-major, so the heaviest (s = 0, one per row) start first;
//   * within a tile a wave takes chunks of 64 records, staged as four rows of 16, each
//     row stored twice in a row (32 slots), so that the record k columns before any
//     column is at a fixed offset from it.  Lane (row r, column c) takes, in turn for
//     g = 0..3, chunk row (r + g) mod 4, and in steps k = 0..15 reads the record of
//     column c - k (mod 16) from LDS and pairs it with its IPL i-particles;
//   * the j-side sums travel with the records they belong to: at each step the lane's
//     four j-sums move one lane on within the row (DPP row rotation, folded into the
//     addition of the step's first term), the lane that held column c - k + 1's sums
//     passing them to the lane that meets column c - k next.  After step 15 each lane
//     holds the sums of column c + 1 and stores them in that record's slot of the
//     wave's LDS slice (the first record load of a chunk stores, the others add);
//   * i-side sums as in the tile engine: FP32 over each 64-record chunk, added in
//     FP64 (FP64RED) or into an FP32 (hi, lo) pair by a two-sum (COMP), or FP32
//     throughout (PLAIN); written at the end of the item to the i-plane of segment s;
//   * j-side sums: FP32 per wave (its 64 IPL terms per record), then, after the tile's
//     barrier, the W slices are added in a fixed order in FP64 (PLAIN: FP32) and
//     written to the j-plane of row b (which covers only j >= (b + 1) BI);
//   * the finalize adds, for a particle of row q, the segment partials of its row and
//     then the j-planes of rows 0 .. q - 1, in that fixed order.
// No atomics: every result is a fixed-order sum, bitwise reproducible per launch
// shape (W, IPL, JT, segt).
//
// Issue cost per unordered pair with the potential, in clocks per wavefront as measured
// on gfx950 (two-operand operations 2, FMACs about 2.6, an FMA with a scalar addend and
// any DPP-modified operation 4, v_rsq_f32 8): 3 separations, s^2 (one scalar-addend FMA,
// two FMACs), rsq, r^2, and per side m r, m r^3, three FMACs and one addition: about 53,
// against 2 x 39 for the two ordered pairs of the tile engine; the rotation of the
// j-sums adds about 12 per step, shared by the lane's IPL pairs of that step.
#pragma once

#include <utility>

#include "gravity.h"

namespace nbody {
namespace sym {

// Value of v in the lane K places away within the lane's row of 16 (DPP row_ror:K:
// lane c receives the value of lane c - K mod 16).  The uses below have an arithmetic
// consumer into which the compiler folds the move.
template <int K>
__device__ __forceinline__ float row_ror(float v) {
    static_assert(K > 0 && K < 16, "rotations within a row of 16 lanes");
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x120 + K, 0xF, 0xF, true));
}

// The lane's IPL i-particles: positions and -m (a padding particle has m = 0: its terms
// on the records it meets are exactly zero).
template <int IPL>
struct IRegs {
    float x[IPL], y[IPL], z[IPL], nm[IPL];
};

// Step K of a record load: the lane's IPL i-particles against record jr.  bi receives the
// i-side terms; aj holds the j-side sums of jr's record, moved one lane on by the first
// addition (K > 0: until then the lane held the sums of the record it met at step K - 1).
template <int K, int IPL, bool FULL>
__device__ __forceinline__ void step(const float4 &jr, const IRegs<IPL> &is, float eps2,
                                     float (&bi)[IPL][4], float (&aj)[4]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int p = 0; p < IPL; ++p) {
        const float dx = jr.x - is.x[p];
        const float dy = jr.y - is.y[p];
        const float dz = jr.z - is.z[p];
        float s2 = __builtin_fmaf(dx, dx, eps2);
        s2 = __builtin_fmaf(dy, dy, s2);
        s2 = __builtin_fmaf(dz, dz, s2);
        const float ri = __builtin_amdgcn_rsqf(s2);
        const float ri2 = ri * ri;
        // i side: the ordered pair body of the tile engine (a += m_j d / s^3, phi -= m_j / s).
        const float mjr = jr.w * ri;
        const float mjr3 = mjr * ri2;
        bi[p][0] = __builtin_fmaf(mjr3, dx, bi[p][0]);
        bi[p][1] = __builtin_fmaf(mjr3, dy, bi[p][1]);
        bi[p][2] = __builtin_fmaf(mjr3, dz, bi[p][2]);
        if constexpr (FULL) bi[p][3] = bi[p][3] - mjr;
        // j side: a_j += (-m_i) d / s^3, phi_j += (-m_i) / s.
        const float nmir = is.nm[p] * ri;
        const float nmir3 = nmir * ri2;
        if constexpr (K > 0) {
            if (p == 0) {
                // The rotated sum cannot be the addend of an FMA: product, then addition.
                const float tx = nmir3 * dx;
                const float ty = nmir3 * dy;
                const float tz = nmir3 * dz;
                aj[0] = row_ror<1>(aj[0]) + tx;
                aj[1] = row_ror<1>(aj[1]) + ty;
                aj[2] = row_ror<1>(aj[2]) + tz;
                if constexpr (FULL) aj[3] = row_ror<1>(aj[3]) + nmir;
                continue;
            }
        }
        aj[0] = __builtin_fmaf(nmir3, dx, aj[0]);
        aj[1] = __builtin_fmaf(nmir3, dy, aj[1]);
        aj[2] = __builtin_fmaf(nmir3, dz, aj[2]);
        if constexpr (FULL) aj[3] = aj[3] + nmir;
    }
}

// The 16 steps of one record load: row points at column c of the doubled chunk row, so
// column c - k (mod 16) is row[16 - k].  The next step's record is read before the
// current step runs.
template <int IPL, bool FULL, int... K>
__device__ __forceinline__ void steps(std::integer_sequence<int, K...>, const float4 *row,
                                      const IRegs<IPL> &is, float eps2, float (&bi)[IPL][4],
                                      float (&aj)[4]) {
    float4 cur = row[16];
    auto one = [&](auto kc) {
        constexpr int k = decltype(kc)::value;
        float4 nxt = cur;
        if constexpr (k < 15) nxt = row[15 - k];
        step<k, IPL, FULL>(cur, is, eps2, bi, aj);
        cur = nxt;
    };
    (one(std::integral_constant<int, K>{}), ...);
}

// One chunk of 64 records (tl: four doubled rows of 32 slots) against the wave's 64 IPL
// i-particles: i-side terms into bi, j-side sums into the wave's slice sl[0 .. 64)
// (stored for the first record load, added for the other three).
template <int IPL, bool FULL>
__device__ __forceinline__ void chunk(const float4 *tl, float4 *sl, int lane,
                                      const IRegs<IPL> &is, float eps2, float (&bi)[IPL][4]) {
    const int r = lane >> 4;
    const int c = lane & 15;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const int row = (r + g) & 3;
        // -0 + t == t exactly, so the first term of each sum needs no rounding step.
        float aj[4] = {-0.0f, -0.0f, -0.0f, -0.0f};
        steps<IPL, FULL>(std::make_integer_sequence<int, 16>{}, tl + row * 32 + c, is, eps2, bi,
                         aj);
        float4 *h = sl + row * 16 + ((c + 1) & 15);
        if (g == 0) {
            *h = make_float4(aj[0], aj[1], aj[2], aj[3]);
        } else {
            const float4 o = *h;
            *h = make_float4(o.x + aj[0], o.y + aj[1], o.z + aj[2], o.w + aj[3]);
        }
    }
}

// One symmetric j-tile of JT records (JT / 64 chunks of 128 slots).
template <int IPL, int JT, int MODE, bool FULL>
__device__ __forceinline__ void sym_tile(const float4 *tl, float4 *sl, int lane,
                                         const IRegs<IPL> &is, float eps2,
                                         float (&hs)[IPL][4], float (&ls)[IPL][4],
                                         double (&ds)[IPL][4]) {
    static_assert(JT % 64 == 0, "whole chunks");
#pragma unroll 1
    for (int h = 0; h < JT / 64; ++h) {
        if constexpr (MODE == NBODY_PLAIN) {
            chunk<IPL, FULL>(tl + h * 128, sl + h * 64, lane, is, eps2, hs);
        } else {
            float bs[IPL][4];
#pragma unroll
            for (int p = 0; p < IPL; ++p)
#pragma unroll
                for (int o = 0; o < 4; ++o) bs[p][o] = -0.0f;
            chunk<IPL, FULL>(tl + h * 128, sl + h * 64, lane, is, eps2, bs);
#pragma unroll
            for (int p = 0; p < IPL; ++p)
#pragma unroll
                for (int o = 0; o < 4; ++o) {
                    if constexpr (MODE == NBODY_COMP)
                        engine::two_sum(hs[p][o], ls[p][o], bs[p][o]);
                    else
                        ds[p][o] += (double)bs[p][o];
                }
        }
    }
}

template <int W, int IPL, int JT, int MODE, bool FULL>
__global__ __launch_bounds__(64 * W) void sym_kernel(SymArgs a) {
    constexpr int NT = 64 * W;
    constexpr int BI = NT * IPL;
    constexpr int NO = 4;
    static_assert(JT <= NT, "one staged record per lane at most");
    using JT_t = typename std::conditional<MODE == NBODY_PLAIN, float, double>::type;
    // Diagonal tiles: JT records in order; symmetric tiles: JT / 64 chunks of four doubled
    // rows (2 JT slots).
    __shared__ float4 tile[2][2 * JT];
    __shared__ float4 slices[2][W][JT];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;

    // Work item -> (row b, segment s).
    int it = blockIdx.x;
    int s = 0;
    for (;; ++s) {
        if (s >= a.smax) return;  // not reached: the grid has exactly the items
        const int cnt = items_of_segment(a.n, BI, JT, a.segt, a.nb, s);
        if (it < cnt) break;
        it -= cnt;
    }
    const int b = it;
    const int i0 = b * BI;
    const int ni = min(BI, a.n - i0);
    const int js = i0 + BI;
    const int t0 = s * a.segt;
    const int t1 = min(t0 + a.segt, row_tiles(a.n, BI, JT, b));
    const int ndiag = s == 0 ? (ni + JT - 1) / JT : 0;
    const int ntiles = ndiag + max(0, t1 - t0);

    IRegs<IPL> is;
    Gravity::IState ig[IPL];
    int own[IPL];
#pragma unroll
    for (int p = 0; p < IPL; ++p) {
        const int r = p * NT + tid;
        const int i = i0 + (r < ni ? r : ni - 1);
        is.x[p] = a.x[i];
        is.y[p] = a.y[i];
        is.z[p] = a.z[i];
        is.nm[p] = r < ni ? -a.m[i] : 0.0f;
        ig[p] = {is.x[p], is.y[p], is.z[p]};
        own[p] = i0 + r;
    }

    float hs[IPL][NO], ls[IPL][NO];
    double ds[IPL][NO];
#pragma unroll
    for (int p = 0; p < IPL; ++p)
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            hs[p][o] = 0.0f;
            ls[p][o] = 0.0f;
            ds[p][o] = 0.0;
        }

    // Tile t: the diagonal tiles [i0 + t JT, ...) (limit i0 + ni), then the symmetric
    // tiles [js + (t0 + t - ndiag) JT, ...) (limit n).
    auto tile_base = [&](int t) { return t < ndiag ? i0 + t * JT : js + (t0 + t - ndiag) * JT; };
    float4 stage = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    auto fetch = [&](int t) {
        if (tid < JT) {
            const int j = tile_base(t) + tid;
            const int lim = t < ndiag ? i0 + ni : a.n;
            if (j < lim)
                stage = make_float4(a.x[j], a.y[j], a.z[j], a.m[j]);
            else
                stage = make_float4(0.0f, 0.0f, 0.0f, 0.0f);  // adds exactly zero
        }
    };
    auto store = [&](int buf, int t) {
        if (tid < JT) {
            if (t < ndiag) {
                tile[buf][tid] = stage;
            } else {
                float4 *q = &tile[buf][(tid >> 6) * 128 + ((tid >> 4) & 3) * 32 + (tid & 15)];
                q[0] = stage;
                q[16] = stage;
            }
        }
    };

    if (ntiles > 0) {
        fetch(0);
        store(0, 0);
    }
    __syncthreads();
    __builtin_amdgcn_s_waitcnt(engine::kWaitVmem);
    for (int t = 0; t < ntiles; ++t) {
        const int buf = t & 1;
        if (t + 1 < ntiles) fetch(t + 1);
        if (t < ndiag) {
            int self[IPL];
#pragma unroll
            for (int p = 0; p < IPL; ++p) self[p] = own[p] - (i0 + t * JT);
            engine::tile_pass<Gravity, IPL, JT, MODE, FULL, true>(tile[buf], ig, a.eps2, hs, ls,
                                                                  ds, self);
        } else {
            sym_tile<IPL, JT, MODE, FULL>(tile[buf], slices[buf][wave], lane, is, a.eps2, hs, ls,
                                          ds);
        }
        if (t + 1 < ntiles) store(buf ^ 1, t + 1);
        __syncthreads();
        if (t >= ndiag) {
            // Fixed-order sum of the W wave slices of this tile, one (record, output)
            // per thread, into row b's j-plane.
            const int jt0 = tile_base(t);
            JT_t *jp = static_cast<JT_t *>(a.jpart) + jrow_base(a.nb, BI, b);
            const size_t len = jrow_len(a.nb, BI, b);
#pragma unroll
            for (int q = tid; q < NO * JT; q += NT) {
                const int o = q / JT;
                const int jj = q - o * JT;
                const int j = jt0 + jj;
                if (j < a.n) {
                    JT_t v = (JT_t)reinterpret_cast<const float *>(&slices[buf][0][jj])[o];
#pragma unroll
                    for (int w = 1; w < W; ++w)
                        v += (JT_t)reinterpret_cast<const float *>(&slices[buf][w][jj])[o];
                    jp[(size_t)o * len + (j - js)] = v;
                }
            }
        }
    }

    // i-side partials of this item: plane s, words [s][word][npad] as in the tile engine.
    constexpr int WO = NO * engine::words_per_out<MODE>();
    const size_t plane = (size_t)a.npad;
    float *base = static_cast<float *>(a.ipart) + (size_t)s * WO * plane;
#pragma unroll
    for (int p = 0; p < IPL; ++p) {
        const size_t i = (size_t)i0 + p * NT + tid;
        if constexpr (MODE == NBODY_FP64RED) {
            double *q = reinterpret_cast<double *>(base) + i;
#pragma unroll
            for (int o = 0; o < NO; ++o) q[o * plane] = ds[p][o];
        } else if constexpr (MODE == NBODY_COMP) {
            float *q = base + i;
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                q[o * plane] = hs[p][o];
                q[(NO + o) * plane] = ls[p][o];
            }
        } else {
            float *q = base + i;
#pragma unroll
            for (int o = 0; o < NO; ++o) q[o * plane] = hs[p][o];
        }
    }
}

}  // namespace sym
}  // namespace nbody
