// mvf_lane.h -- per-lane pieces of the subdomain bounding kernels shared by
// the interpreter kernels and the run-time-compiled specialised kernels:
// kernel-argument access, Step 1 (breakpoint table, subdomain decode;
// Sec. 3.1.1), and the Step 3 reduction of the subdomain bounds to their hull
// with the objective's argmin and the two branch-and-bound bounds (Sec. 3.1).
#pragma once
#include "mvf_device.h"
#include "mvf_kargs.h"

namespace mvf {
namespace dev {

// breakpoint b_j of [lo, hi] split in s (round to nearest; fp-contract off)
__device__ __forceinline__ double breakpoint(double lo, double hi, int s, int j) {
    if (j <= 0) return lo;
    if (j >= s) return hi;
    double w = hi - lo;
    double h = w / (double)s;
    double r = lo + (double)j * h;
    return r < hi ? r : hi;
}

// Kernel arguments are read through a pointer to the kernarg segment that the
// optimiser cannot see through: every use re-issues a scalar load (a
// scalar-cache hit) instead of keeping the loaded values in SGPRs across the
// interpreter loops.
template <typename K>
using KPtr = const __attribute__((address_space(4))) K *;

template <typename K>
__device__ __forceinline__ KPtr<K> kargs() {
    const uint64_t v = reinterpret_cast<uint64_t>(__builtin_amdgcn_kernarg_segment_ptr());
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    asm volatile("" : "+s"(lo), "+s"(hi));
    return reinterpret_cast<KPtr<K>>((uint64_t)hi << 32 | lo);
}

constexpr Iv kZero = {0.0, 0.0};
constexpr Iv kOne = {1.0, -1.0};

// Wave reductions with DPP lane moves (VALU, no LDS round trip): swaps within
// quads, mirrors within half-rows and rows (each lane then holds its row's
// result), then row 0 into row 1 and row 2 into row 3, then row 1 into rows 2
// and 3; lane 63 ends with the whole wave's, which is read back uniform.  A
// lane a move does not write keeps its own value, which the minimum ignores.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x) {
    const int lo = (int)(uint32_t)x, hi = (int)(uint32_t)(x >> 32);
    const int rlo = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xf, false);
    const int rhi = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xf, false);
    return (uint64_t)(uint32_t)rhi << 32 | (uint32_t)rlo;
}
__device__ __forceinline__ uint64_t lane63_u64(uint64_t x) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)x, 63);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), 63);
    return (uint64_t)hi << 32 | lo;
}
// the six moves: quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror,
// row_mirror, row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and 3
#define MVF_WAVE_STEPS(STEP) \
    STEP(0xB1, 0xf) STEP(0x4E, 0xf) STEP(0x141, 0xf) STEP(0x140, 0xf) STEP(0x142, 0xa) STEP(0x143, 0xc)

__device__ __forceinline__ double wave_min(double v) {
#define MVF_MIN_STEP(C, R) \
    v = fmin_(v, __builtin_bit_cast(double, dpp_u64<C, R>(__builtin_bit_cast(uint64_t, v))));
    MVF_WAVE_STEPS(MVF_MIN_STEP)
#undef MVF_MIN_STEP
    return __builtin_bit_cast(double, lane63_u64(__builtin_bit_cast(uint64_t, v)));
}

// (value, index) minimum, ties to the smaller index
__device__ __forceinline__ void wave_argmin(double &v, int64_t &k) {
#define MVF_ARGMIN_STEP(C, R)                                                                        \
    {                                                                                                \
        const double v2 = __builtin_bit_cast(double, dpp_u64<C, R>(__builtin_bit_cast(uint64_t, v))); \
        const int64_t k2 = (int64_t)dpp_u64<C, R>((uint64_t)k);                                       \
        const bool take = v2 < v || (v2 == v && k2 < k);                                             \
        v = take ? v2 : v;                                                                           \
        k = take ? k2 : k;                                                                           \
    }
    MVF_WAVE_STEPS(MVF_ARGMIN_STEP)
#undef MVF_ARGMIN_STEP
    v = __builtin_bit_cast(double, lane63_u64(__builtin_bit_cast(uint64_t, v)));
    k = (int64_t)lane63_u64((uint64_t)k);
}

// Where a lane's results go: the optional per-subdomain output and the wave's
// running reduction record in LDS.  The record holds, for each root r, the
// minimum lower endpoint and the minimum of -upper at [2r], [2r + 1]; the
// objective's argmin (value, subdomain) at [2m], [2m + 1]; the smallest
// flagged subdomain at [2m + 2]; the feasibility-filtered objective bound at
// [2m + 3] and the upper bound from feasible centres at [2m + 4].
struct LaneOut {
    double *per_sub;     // [m][2][S] or null
    int64_t S, k;
    double *w;           // the wave's record
    int lane;
    bool active;
    uint32_t ineq, eq;   // constraint roots (bit masks)
};

constexpr int wred_len(int m) { return 2 * m + 5; }

// Per-lane state of the two bounds a B&B needs besides the hulls: the
// objective's lower bound unless a constraint proves the subdomain infeasible
// (inequality lower bound > 0, or an equality bound excluding 0), and the
// objective's upper bound at the centre when every inequality's enclosure at
// the centre is <= 0 (no equality constraints).
struct FeasTrack {
    double obj_lo = 0.0, centre_hi = __builtin_inf();
    bool infeasible = false, centre_ok = true;
};

__device__ __forceinline__ void track_root(FeasTrack &F, int r, Iv B, Iv FC, bool have_fc, const LaneOut &o) {
    if (r == 0) {
        F.obj_lo = B.lo;
        F.centre_hi = -FC.nh;
        F.centre_ok &= have_fc && o.eq == 0;            // (combined, so the roots may come in any order)
        return;
    }
    if ((o.ineq >> r) & 1u) {
        F.infeasible |= B.lo > 0.0;
        F.centre_ok &= FC.nh >= 0.0;                         // hi(g(c)) <= 0; false for NaN
    }
    if ((o.eq >> r) & 1u) F.infeasible |= B.lo > 0.0 || B.nh > 0.0;   // 0 not in [lo, hi]
}

__device__ __forceinline__ int64_t wave_min_i64(int64_t v) {
#define MVF_MINI_STEP(C, R)                                \
    {                                                      \
        const int64_t u = (int64_t)dpp_u64<C, R>((uint64_t)v); \
        v = u < v ? u : v;                                 \
    }
    MVF_WAVE_STEPS(MVF_MINI_STEP)
#undef MVF_MINI_STEP
    return (int64_t)lane63_u64((uint64_t)v);
}

// Fold root r's bound on this lane's subdomain into the wave record.  A lane
// whose subdomain is flagged later is fixed up by finish_lane.
__device__ __forceinline__ void reduce_root(int r, int m, Iv B, const LaneOut &o) {
    if (o.active && o.per_sub) {
        o.per_sub[(int64_t)(2 * r) * o.S + o.k] = B.lo;
        o.per_sub[(int64_t)(2 * r + 1) * o.S + o.k] = -B.nh;
    }
    const double lo = o.active && B.lo == B.lo ? B.lo : __builtin_inf();
    const double nh = o.active && B.nh == B.nh ? B.nh : __builtin_inf();
    const double wl = wave_min(lo), wn = wave_min(nh);
    if (r == 0) {
        double v = lo;
        int64_t kk = o.active ? o.k : INT64_MAX;
        wave_argmin(v, kk);
        if (o.lane == 0) {
            const double pv = o.w[2 * m];
            const int64_t pk = reinterpret_cast<int64_t *>(o.w)[2 * m + 1];
            if (v < pv || (v == pv && kk < pk)) {
                o.w[2 * m] = v;
                reinterpret_cast<int64_t *>(o.w)[2 * m + 1] = kk;
            }
        }
    }
    if (o.lane == 0) {
        o.w[2 * r] = fmin(o.w[2 * r], wl);
        o.w[2 * r + 1] = fmin(o.w[2 * r + 1], wn);
    }
}

// After all roots: the domain flag, the per-subdomain bounds of a flagged
// subdomain ([-inf, +inf] for every root), and the wave's smallest flagged
// subdomain.
__device__ __forceinline__ void finish_lane(int m, uint32_t bad, const FeasTrack &F, const LaneOut &o,
                                            uint32_t *flags) {
    if (o.active && flags) flags[o.k] = bad;
    {
        const double inf = __builtin_inf();
        const double fl = !o.active ? inf : bad ? -inf : F.infeasible ? inf : F.obj_lo;
        const double ub = o.active && !bad && F.centre_ok && F.centre_hi == F.centre_hi ? F.centre_hi : inf;
        const double wfl = wave_min(fl), wub = wave_min(ub);
        if (o.lane == 0) {
            o.w[2 * m + 3] = fmin(o.w[2 * m + 3], wfl);
            o.w[2 * m + 4] = fmin(o.w[2 * m + 4], wub);
        }
    }
    if (o.active && bad && o.per_sub) {
        for (int r = 0; r < m; ++r) {
            o.per_sub[(int64_t)(2 * r) * o.S + o.k] = -__builtin_inf();
            o.per_sub[(int64_t)(2 * r + 1) * o.S + o.k] = __builtin_inf();
        }
    }
    const int64_t kb = wave_min_i64(o.active && bad ? o.k : INT64_MAX);
    if (o.lane == 0) {
        int64_t *wk = reinterpret_cast<int64_t *>(o.w);
        wk[2 * m + 2] = kb < wk[2 * m + 2] ? kb : wk[2 * m + 2];
    }
}

__device__ __forceinline__ void reset_wred(double *w, int m) {
    for (int r = 0; r < 2 * m + 1; ++r) w[r] = __builtin_inf();
    reinterpret_cast<int64_t *>(w)[2 * m + 1] = INT64_MAX;
    reinterpret_cast<int64_t *>(w)[2 * m + 2] = INT64_MAX;
    w[2 * m + 3] = __builtin_inf();
    w[2 * m + 4] = __builtin_inf();
}

// build the breakpoint table of one box (whole workgroup); tab_off in LDS
__device__ __forceinline__ void build_table(int n, const double *box, const int32_t *splits, const int32_t *tab_off,
                                            double4 *tab, int tid, int blk) {
    const int total = tab_off[n];
    for (int t = tid; t < total; t += blk) {
        int i = 0;
        while (tab_off[i + 1] <= t) ++i;
        const int j = t - tab_off[i], s = splits[i];
        const double lo = box[2 * i], hi = box[2 * i + 1];
        const double bl = breakpoint(lo, hi, s, j), bh = breakpoint(lo, hi, s, j + 1);
        const double c = 0.5 * (bl + bh);
        tab[t] = make_double4(bl, -bh, c, -c);
    }
}

// table index of dimension i for subdomain q (dimension 0 fastest)
__device__ __forceinline__ void decode_subdomain(int n, int64_t q, const int32_t *splits, const int32_t *tab_off,
                                                 uint16_t *vrec, int tid, int blk) {
    for (int i = 0; i < n; ++i) {
        const int s = splits[i];
        vrec[i * blk + tid] = (uint16_t)(tab_off[i] + (int)(q % s));
        q /= s;
    }
}

// Combine the waves' records into one partial (thread 0).  Any flagged
// subdomain makes every root's hull [-inf, +inf]; the objective's argmin is
// then the smallest subdomain whose lower bound is -inf.
__device__ __forceinline__ void write_partial(const double *wred, int waves, int m, double *part, double *plo0,
                                              int64_t *pk, double *pext) {
    double best = __builtin_inf();
    int64_t bk = INT64_MAX, kb = INT64_MAX;
    double fl = __builtin_inf(), ub = __builtin_inf();
    for (int w = 0; w < waves; ++w) {
        fl = fmin(fl, wred[w * wred_len(m) + 2 * m + 3]);
        ub = fmin(ub, wred[w * wred_len(m) + 2 * m + 4]);
    }
    pext[0] = fl;
    pext[1] = ub;
    for (int r = 0; r < m; ++r) {
        double l = __builtin_inf(), h = __builtin_inf();
        for (int w = 0; w < waves; ++w) {
            const double *wr = wred + w * wred_len(m);
            l = fmin(l, wr[2 * r]);
            h = fmin(h, wr[2 * r + 1]);
        }
        part[2 * r] = l;
        part[2 * r + 1] = h;
    }
    for (int w = 0; w < waves; ++w) {
        const double *wr = wred + w * wred_len(m);
        const double v = wr[2 * m];
        const int64_t kk = reinterpret_cast<const int64_t *>(wr)[2 * m + 1];
        if (v < best || (v == best && kk < bk)) { best = v; bk = kk; }
        const int64_t f = reinterpret_cast<const int64_t *>(wr)[2 * m + 2];
        kb = f < kb ? f : kb;
    }
    if (kb != INT64_MAX) {
        for (int r = 0; r < 2 * m; ++r) part[r] = -__builtin_inf();
        bk = best == -__builtin_inf() && bk < kb ? bk : kb;
        best = -__builtin_inf();
    }
    *plo0 = best;
    *pk = bk;
}

}  // namespace dev
}  // namespace mvf
