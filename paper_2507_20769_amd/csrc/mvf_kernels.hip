// mvf_kernels.hip -- subdomain MVF bounding kernels for gfx950.
//
// One lane = one subdomain.  A workgroup stages the register programs (one
// per root) and a per-dimension breakpoint table into LDS; every lane decodes
// its subdomain index, then interprets the programs instruction by
// instruction: the 16-byte instruction is broadcast from LDS to the wave and
// made wave-uniform, operands come from the lane's GPR-indexed slot file, the
// breakpoint table (variables) or the instruction (constants), and the result
// goes back to a slot.
//
// Per root (Sec. 3.1 Step 2; Sec. 2.2 Definition "Mean Value Form"):
//   * a point pass at the centre c gives [f(c)];
//   * forward (tangent) mode: passes over X_k give the NIE and C gradient
//     components at a time;
//   * reverse mode: one value pass over X_k gives the NIE and leaves the local
//     partials of every instruction on a per-lane global-memory tape; one
//     reverse sweep over the same program then accumulates the adjoints in
//     the (re-used) slot file and the variable gradients in LDS;
//   * MVF = [f(c)] + sum_i G_i * (X_i - c_i), i ascending, intersected with
//     the NIE.
// The subdomain bounds are min-reduced per wave with cross-lane shuffles, per
// workgroup through LDS and across workgroups by a second kernel (Sec. 3.1
// Step 3, the interval hull).  The batched form runs many B&B nodes of
// uneven size in one persistent launch: workgroups pull (node, chunk) work
// items from an atomic counter; a plan kernel derives the items from the
// device-resident splits, so the whole sequence can be replayed from a graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mvf.h"
#include "mvf_device.h"
#include "mvf_internal.h"
#include "mvf_kernels.h"

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

// Hide a pointer from the optimiser: loads through it are re-issued where they
// are used (scalar-cache hits) instead of being hoisted into SGPRs that stay
// live across the interpreter loop; SGPR pressure there spills into VGPR lanes.
template <typename P>
__device__ __forceinline__ const P *opaque(const P *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    asm volatile("" : "+s"(lo), "+s"(hi));
    lo = __builtin_amdgcn_readfirstlane(lo);          // keeps the pointer wave-uniform
    hi = __builtin_amdgcn_readfirstlane(hi);
    return reinterpret_cast<const P *>((uint64_t)hi << 32 | lo);
}

struct Ctx {
    const uint4 *prog;       // LDS program
    const double4 *tab;      // LDS: {lo, nh, c, -c} per (dim, j)
    const uint16_t *vrec;    // LDS: [dim][BLK] table index of the lane's subdomain
    double2 *G;              // reverse-mode gradient accumulators of this lane ([dim] with stride gstride),
                             // in LDS or global memory (flat addressing)
    int64_t gstride;
    double2 *rec;            // global reverse-mode tape of this lane ([record][lane])
    int64_t rec_stride;      // lanes sharing the tape (record stride, in records)
    double2 *spill;          // LDS spill slots of this lane ([slot][component][lane])
    uint32_t nreg;           // slot ids >= nreg are spilled (tangent passes)
    int tid, blk;
};

template <int C>
__device__ __forceinline__ void spill_read(const Ctx &X, uint32_t a, Iv &val, Iv (&tan)[C > 0 ? C : 1]) {
    const double2 *p = X.spill + (size_t)(a - X.nreg) * (1 + C) * X.blk;
    const double2 v = p[0];
    val = Iv{v.x, v.y};
#pragma unroll
    for (int t = 0; t < C; ++t) {
        const double2 w = p[(size_t)(t + 1) * X.blk];
        tan[t] = Iv{w.x, w.y};
    }
}

template <int C>
__device__ __forceinline__ void spill_write(const Ctx &X, uint32_t a, const Iv &val, const Iv (&tan)[C > 0 ? C : 1]) {
    double2 *p = X.spill + (size_t)(a - X.nreg) * (1 + C) * X.blk;
    p[0] = make_double2(val.lo, val.nh);
#pragma unroll
    for (int t = 0; t < C; ++t) p[(size_t)(t + 1) * X.blk] = make_double2(tan[t].lo, tan[t].nh);
}

__device__ __forceinline__ double4 var_rec(const Ctx &X, uint32_t i) {
    return X.tab[X.vrec[i * X.blk + X.tid]];
}

// fetch operand (kind, a): value and C tangent components [c0, c0 + C)
template <int C, bool POINT>
__device__ __forceinline__ void fetch(const Ctx &X, uint32_t kind, uint32_t a, double k, int c0, Iv &val,
                                      Iv (&tan)[C > 0 ? C : 1]) {
    constexpr uint32_t SD = 4 + 4 * C;
    if (kind == K_SLOT) {
        if (C > 0 && a >= X.nreg) spill_read<C>(X, a, val, tan);
        else slot_read<C>(a * SD, val, tan);
    } else if (kind == K_VAR) {
        double4 r = var_rec(X, a);
        val = POINT ? Iv{r.z, r.w} : Iv{r.x, r.y};
#pragma unroll
        for (int t = 0; t < C; ++t) {
            const bool hit = (int)a == c0 + t;
            tan[t] = Iv{hit ? 1.0 : 0.0, hit ? -1.0 : 0.0};
        }
    } else {
        val = Iv{k, -k};
#pragma unroll
        for (int t = 0; t < C; ++t) tan[t] = Iv{0.0, 0.0};
    }
}

struct Decoded {
    uint32_t op, ak, bk, ia, ib, a, b, d;
    double k;
};

__device__ __forceinline__ Decoded decode(const uint4 *P, int pc) {
    uint4 raw = P[pc];
    const uint32_t w0 = __builtin_amdgcn_readfirstlane(raw.x);
    const uint32_t w1 = __builtin_amdgcn_readfirstlane(raw.y);
    Decoded D;
    D.k = __hiloint2double((int)raw.w, (int)raw.z);
    D.op = w0 & 0xffu;
    D.ak = (w0 >> 8) & 3u;
    D.bk = (w0 >> 10) & 3u;
    D.ia = (w0 >> 12) & 1u;
    D.ib = (w0 >> 13) & 1u;
    D.a = w0 >> 16;
    D.b = w1 & 0xffffu;
    D.d = w1 >> 16;
    return D;
}

// Run one root program forward; returns the root's value interval and (C > 0)
// its tangent components [c0, c0 + C).  With TAPE, also writes the reverse-mode
// records of every instruction.
template <int C, bool POINT, bool TAPE>
__device__ Iv run_program(const Ctx &X, int begin, int len, int res_slot, int c0, Iv (&gout)[C > 0 ? C : 1],
                          uint32_t &bad) {
    constexpr uint32_t SD = 4 + 4 * C;
    int64_t rp = 0;                                    // record position
    for (int pc = begin; pc < begin + len; ++pc) {
        const Decoded I = decode(X.prog, pc);
        Iv U, V, Z;
        Iv dU[C > 0 ? C : 1], dV[C > 0 ? C : 1], dZ[C > 0 ? C : 1];
        fetch<C, POINT>(X, I.ak, I.a, I.k, c0, U, dU);
        if (I.op >= I_ADD && I.op <= I_DIV) fetch<C, POINT>(X, I.bk, I.b, I.k, c0, V, dV);
        Iv r0, r1;                                     // records of this instruction
        switch (I.op) {
        case I_ADD:
            Z = iadd(U, V);
#pragma unroll
            for (int t = 0; t < C; ++t) dZ[t] = iadd(dU[t], dV[t]);
            break;
        case I_SUB:
            Z = isub(U, V);
#pragma unroll
            for (int t = 0; t < C; ++t) dZ[t] = isub(dU[t], dV[t]);
            break;
        case I_MUL:
            Z = imul(U, V);
#pragma unroll
            for (int t = 0; t < C; ++t) dZ[t] = iadd(imul(V, dU[t]), imul(U, dV[t]));
            r0 = U;
            r1 = V;
            break;
        case I_DIV: {
            bad |= (V.lo <= 0.0 && V.nh <= 0.0) ? 1u : 0u;
            Z = idiv(U, V);
            if constexpr (C > 0 || TAPE) {
                Iv R = irecip(V);
#pragma unroll
                for (int t = 0; t < C; ++t) dZ[t] = imul(isub(dU[t], imul(Z, dV[t])), R);
                r0 = R;
                r1 = Z;
            }
            break;
        }
        case I_SQR: {
            Z = isqr(U);
            if constexpr (C > 0 || TAPE) {
                Iv T = itwice(U);
#pragma unroll
                for (int t = 0; t < C; ++t) dZ[t] = imul(T, dU[t]);
                r0 = T;
            }
            break;
        }
        case I_SQRT: {
            bad |= U.lo < 0.0 ? 1u : 0u;
            Z = isqrt(U);
            if constexpr (C > 0 || TAPE) {
                Iv R = isqrt_deriv(Z);
#pragma unroll
                for (int t = 0; t < C; ++t) dZ[t] = imul(dU[t], R);
                r0 = R;
            }
            break;
        }
        case I_EXP:
            Z = iexp(U);
#pragma unroll
            for (int t = 0; t < C; ++t) dZ[t] = imul(Z, dU[t]);
            r0 = Z;
            break;
        case I_LOG: {
            bad |= U.lo <= 0.0 ? 1u : 0u;
            Z = ilog(U);
            if constexpr (C > 0 || TAPE) {
                Iv R = irecip(U);
#pragma unroll
                for (int t = 0; t < C; ++t) dZ[t] = imul(dU[t], R);
                r0 = R;
            }
            break;
        }
        default:   // I_LOAD
            Z = U;
#pragma unroll
            for (int t = 0; t < C; ++t) dZ[t] = dU[t];
            break;
        }
        if (C > 0 && I.d >= X.nreg) spill_write<C>(X, I.d, Z, dZ);
        else slot_write<C>(I.d * SD, Z, dZ);
        if constexpr (TAPE) {
            // records in the order of n_records(): U then V, 1/V then Z, or the single partial
            if (I.op == I_MUL) {
                if (I.ak == K_SLOT && I.bk != K_CONST) X.rec[(rp++) * X.rec_stride] = make_double2(r0.lo, r0.nh);
                if (I.bk == K_SLOT && I.ak != K_CONST) X.rec[(rp++) * X.rec_stride] = make_double2(r1.lo, r1.nh);
            } else if (I.op == I_DIV) {
                X.rec[(rp++) * X.rec_stride] = make_double2(r0.lo, r0.nh);
                if (I.bk != K_CONST) X.rec[(rp++) * X.rec_stride] = make_double2(r1.lo, r1.nh);
            } else if (I.op >= I_SQR && I.op <= I_LOG) {
                X.rec[(rp++) * X.rec_stride] = make_double2(r0.lo, r0.nh);
            }
        }
    }
    Iv val;
    if (C > 0 && (uint32_t)res_slot >= X.nreg) spill_read<C>(X, (uint32_t)res_slot, val, gout);
    else slot_read<C>((uint32_t)res_slot * SD, val, gout);
    return val;
}

__device__ __forceinline__ Iv ld_rec(const Ctx &X, int64_t rp) {
    const double2 v = X.rec[rp * X.rec_stride];
    return Iv{v.x, v.y};
}

// adjoint contribution c to operand (kind, a); init: first contribution
// (the slot is written, not accumulated); neg: subtract instead of add
__device__ __forceinline__ void contribute(const Ctx &X, uint32_t kind, uint32_t a, uint32_t init, bool neg, Iv c) {
    if (kind == K_SLOT) {
        const uint32_t idx = a * 4;
        if (init) {
            slot_wr(idx, neg ? Iv{c.nh, c.lo} : c);    // 0 - [lo, hi] = [-hi, -lo]
        } else {
            const Iv s = slot_rd(idx);
            slot_wr(idx, neg ? isub(s, c) : iadd(s, c));
        }
    } else if (kind == K_VAR) {
        double2 *g = X.G + a * X.gstride;
        const double2 s = *g;
        const Iv gi = neg ? isub(Iv{s.x, s.y}, c) : iadd(Iv{s.x, s.y}, c);
        *g = make_double2(gi.lo, gi.nh);
    }
}

// Reverse sweep over one root program; the adjoint of the root is [1, 1].
__device__ void reverse_sweep(const Ctx &X, int begin, int len, int res_slot, int64_t n_rec) {
    slot_wr((uint32_t)res_slot * 4, Iv{1.0, -1.0});
    int64_t rp = n_rec;
    for (int pc = begin + len - 1; pc >= begin; --pc) {
        const Decoded I = decode(X.prog, pc);
        const Iv zb = slot_rd(I.d * 4);
        switch (I.op) {
        case I_ADD:
            contribute(X, I.ak, I.a, I.ia, false, zb);
            contribute(X, I.bk, I.b, I.ib, false, zb);
            break;
        case I_SUB:
            contribute(X, I.ak, I.a, I.ia, false, zb);
            contribute(X, I.bk, I.b, I.ib, true, zb);
            break;
        case I_MUL: {
            const bool hv = I.bk == K_SLOT && I.ak != K_CONST, hu = I.ak == K_SLOT && I.bk != K_CONST;
            Iv V = {0.0, 0.0}, U = {0.0, 0.0};
            if (hv) V = ld_rec(X, --rp);
            if (hu) U = ld_rec(X, --rp);
            if (I.ak != K_CONST) {
                if (I.bk == K_VAR) { const double4 r = var_rec(X, I.b); V = Iv{r.x, r.y}; }
                else if (I.bk == K_CONST) V = Iv{I.k, -I.k};
                contribute(X, I.ak, I.a, I.ia, false, imul(zb, V));
            }
            if (I.bk != K_CONST) {
                if (I.ak == K_VAR) { const double4 r = var_rec(X, I.a); U = Iv{r.x, r.y}; }
                else if (I.ak == K_CONST) U = Iv{I.k, -I.k};
                contribute(X, I.bk, I.b, I.ib, false, imul(zb, U));
            }
            break;
        }
        case I_DIV: {
            Iv Z = {0.0, 0.0};
            if (I.bk != K_CONST) Z = ld_rec(X, --rp);
            const Iv R = ld_rec(X, --rp);
            const Iv T = imul(zb, R);
            contribute(X, I.ak, I.a, I.ia, false, T);
            if (I.bk != K_CONST) contribute(X, I.bk, I.b, I.ib, true, imul(T, Z));
            break;
        }
        case I_SQR: case I_SQRT: case I_EXP: case I_LOG: {
            const Iv R = ld_rec(X, --rp);
            contribute(X, I.ak, I.a, I.ia, false, imul(zb, R));
            break;
        }
        default:   // I_LOAD
            contribute(X, I.ak, I.a, I.ia, false, zb);
            break;
        }
    }
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ void wave_argmin(double &v, int64_t &k) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        double v2 = __shfl_xor(v, o, 64);
        int64_t k2 = __shfl_xor(k, o, 64);
        const bool take = v2 < v || (v2 == v && k2 < k);
        v = take ? v2 : v;
        k = take ? k2 : k;
    }
}

// Bounds of every root on the lane's subdomain, written to the result slots.
// Returns the domain flag (violation or NaN).
template <int C, bool REV>
__device__ uint32_t bound_lane(const TapeArgs &T0, const Ctx &X) {
    const int m = opaque(&T0)->n_roots;
    const uint32_t res_base = (uint32_t)usable_dwords(m);
    mode_round_down();
    uint32_t bad = 0;
    for (int r = 0; r < m; ++r) {
        const TapeArgs &T = *opaque(&T0);
        const int n = T.n;
        const int pb = T.root_begin[r], pl = T.root_len[r], rs = T.root_slot[r];
        Iv B;
        Iv g0[1];
        if (T.mode == MVF_MODE_NIE) {
            B = run_program<0, false, false>(X, pb, pl, rs, 0, g0, bad);
        } else if constexpr (REV) {
            const Iv FC = run_program<0, true, false>(X, pb, pl, rs, 0, g0, bad);
            const Iv nie = run_program<0, false, true>(X, pb, pl, rs, 0, g0, bad);
            for (int i = 0; i < n; ++i) X.G[i * X.gstride] = make_double2(0.0, 0.0);
            reverse_sweep(X, pb, pl, rs, T.root_rec[r]);
            Iv acc = FC;
            for (int i = 0; i < n; ++i) {
                const double4 rec = var_rec(X, (uint32_t)i);
                const Iv D = {fadd(rec.x, rec.w), fadd(rec.y, rec.z)};   // X_i - c_i
                const double2 g = X.G[i * X.gstride];
                acc = iadd(acc, imul(Iv{g.x, g.y}, D));
            }
            B = T.mode == MVF_MODE_MVF ? acc : Iv{fmax_(acc.lo, nie.lo), fmax_(acc.nh, nie.nh)};
        } else {
            Iv G[C > 0 ? C : 1];
            const Iv FC = run_program<0, true, false>(X, pb, pl, rs, 0, g0, bad);
            Iv acc = FC, nie = {0.0, 0.0};
            for (int c0 = 0; c0 < n; c0 += C) {
                Iv v = run_program<C, false, false>(X, pb, pl, rs, c0, G, bad);
                if (c0 == 0) nie = v;
#pragma unroll
                for (int t = 0; t < C; ++t) {
                    if (c0 + t < n) {
                        const double4 rec = var_rec(X, (uint32_t)(c0 + t));
                        const Iv D = {fadd(rec.x, rec.w), fadd(rec.y, rec.z)};   // X_i - c_i
                        acc = iadd(acc, imul(G[t], D));
                    }
                }
            }
            B = T.mode == MVF_MODE_MVF ? acc : Iv{fmax_(acc.lo, nie.lo), fmax_(acc.nh, nie.nh)};
        }
        slot_wr(res_base + 4 * r, B);
    }
    mode_round_nearest();
    for (int r = 0; r < m; ++r) {
        Iv B = slot_rd(res_base + 4 * r);
        if (B.lo != B.lo || B.nh != B.nh) bad = 1;
    }
    return bad;
}

// stage the programs into LDS (whole workgroup)
__device__ __forceinline__ void stage_program(const TapeArgs &T, uint4 *lprog, int tid, int blk) {
    const uint4 *src = reinterpret_cast<const uint4 *>(T.prog);
    for (int i = tid; i < T.n_instr; i += blk) lprog[i] = src[i];
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

struct Smem {
    uint4 *prog;
    double4 *tab;
    uint16_t *vrec;
    double2 *G;
    double2 *spill;
    double *wred;
    int32_t *ints;     // splits[MVF_MAX_VARS], tab_off[MVF_MAX_VARS + 1], scratch
};

__device__ __forceinline__ Smem carve(uint8_t *smem, const TapeArgs &T, int tab_cap, int blk, bool g_lds, int chunk) {
    Smem s;
    uint8_t *p = smem;
    s.prog = reinterpret_cast<uint4 *>(p);
    p += (size_t)T.n_instr * 16;
    s.tab = reinterpret_cast<double4 *>(p);
    p += (size_t)tab_cap * 32;
    s.G = reinterpret_cast<double2 *>(p);
    if (g_lds) p += (size_t)T.n * blk * 16;
    s.spill = reinterpret_cast<double2 *>(p);
    p += (size_t)T.spill_slots * (1 + chunk) * 16 * blk;
    s.wred = reinterpret_cast<double *>(p);
    p += (size_t)(blk / 64) * (2 * T.n_roots + 2) * 8;
    s.ints = reinterpret_cast<int32_t *>(p);
    p += (2 * MVF_MAX_VARS + 8) * 4;
    p = reinterpret_cast<uint8_t *>((reinterpret_cast<uintptr_t>(p) + 15) & ~uintptr_t(15));
    s.vrec = reinterpret_cast<uint16_t *>(p);
    return s;
}

// Per-wave reduction of the lanes' result slots into the wave's LDS record
// (running min over calls); per_sub/flags written for active lanes.
__device__ __forceinline__ void reduce_lane(const TapeArgs &T, double *w, bool active, int64_t k, uint32_t bad,
                                            double *per_sub, int64_t S, uint32_t *flags, int lane) {
    const int m = T.n_roots;
    const uint32_t res_base = (uint32_t)usable_dwords(m);
    for (int r = 0; r < m; ++r) {
        Iv B = slot_rd(res_base + 4 * r);
        if (bad) B = Iv{-__builtin_inf(), -__builtin_inf()};
        if (active && per_sub) {
            per_sub[(int64_t)(2 * r) * S + k] = B.lo;
            per_sub[(int64_t)(2 * r + 1) * S + k] = -B.nh;
        }
        const double lo = active ? B.lo : __builtin_inf();
        const double nh = active ? B.nh : __builtin_inf();
        const double wl = wave_min(lo), wn = wave_min(nh);
        if (r == 0) {
            double v = lo;
            int64_t kk = active ? k : INT64_MAX;
            wave_argmin(v, kk);
            if (lane == 0) {
                const double pv = w[2 * m];
                const int64_t pk = reinterpret_cast<int64_t *>(w)[2 * m + 1];
                if (v < pv || (v == pv && kk < pk)) {
                    w[2 * m] = v;
                    reinterpret_cast<int64_t *>(w)[2 * m + 1] = kk;
                }
            }
        }
        if (lane == 0) {
            w[2 * r] = fmin(w[2 * r], wl);
            w[2 * r + 1] = fmin(w[2 * r + 1], wn);
        }
    }
    if (active && flags) flags[k] = bad;
}

__device__ __forceinline__ void reset_wred(double *w, int m) {
    for (int r = 0; r < 2 * m + 1; ++r) w[r] = __builtin_inf();
    reinterpret_cast<int64_t *>(w)[2 * m + 1] = INT64_MAX;
}

// combine the waves' records into one partial (thread 0)
__device__ __forceinline__ void write_partial(const double *wred, int waves, int m, double *part, double *plo0,
                                              int64_t *pk) {
    double best = __builtin_inf();
    int64_t bk = INT64_MAX;
    for (int r = 0; r < m; ++r) {
        double l = __builtin_inf(), h = __builtin_inf();
        for (int w = 0; w < waves; ++w) {
            const double *wr = wred + w * (2 * m + 2);
            l = fmin(l, wr[2 * r]);
            h = fmin(h, wr[2 * r + 1]);
        }
        part[2 * r] = l;
        part[2 * r + 1] = h;
    }
    for (int w = 0; w < waves; ++w) {
        const double *wr = wred + w * (2 * m + 2);
        const double v = wr[2 * m];
        const int64_t kk = reinterpret_cast<const int64_t *>(wr)[2 * m + 1];
        if (v < best || (v == best && kk < bk)) { best = v; bk = kk; }
    }
    *plo0 = best;
    *pk = bk;
}

}  // namespace dev

// ---------------------------------------------------------------------------
// single box
// ---------------------------------------------------------------------------
template <int C, bool REV>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_num_vgpr(SLOT_BASE), amdgpu_waves_per_eu(5, 5))) void bound_kernel(TapeArgs T,
                                                                                               BoxArgs B) {
    using namespace dev;
    extern __shared__ __align__(16) uint8_t smem[];
    claim_slot_file();
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = T.n_roots, n = T.n;
    const bool g_lds = B.gacc == nullptr;
    Smem s = carve(smem, T, B.tab_off[n], BLK, REV && g_lds, C);
    stage_program(T, s.prog, tid, BLK);
    if (tid <= n) s.ints[MVF_MAX_VARS + tid] = B.tab_off[tid];
    if (tid < n) s.ints[tid] = B.splits[tid];
    __syncthreads();
    build_table(n, B.box, s.ints, s.ints + MVF_MAX_VARS, s.tab, tid, BLK);
    if (lane == 0) reset_wred(s.wred + wave * (2 * m + 2), m);
    __syncthreads();

    Ctx X;
    X.prog = s.prog;
    X.tab = s.tab;
    X.vrec = s.vrec;
    X.G = g_lds ? s.G + tid : B.gacc + (int64_t)blockIdx.x * BLK + tid;
    X.gstride = g_lds ? BLK : (int64_t)gridDim.x * BLK;
    X.tid = tid;
    X.blk = BLK;
    X.rec_stride = (int64_t)gridDim.x * BLK;
    X.rec = B.rec + (int64_t)blockIdx.x * BLK + tid;
    X.spill = s.spill + tid;
    X.nreg = (uint32_t)T.nreg;
    for (int64_t base = (int64_t)blockIdx.x * BLK; base < B.S; base += (int64_t)gridDim.x * BLK) {
        const int64_t k = base + tid;
        const bool active = k < B.S;
        decode_subdomain(n, active ? k : B.S - 1, s.ints, s.ints + MVF_MAX_VARS, s.vrec, tid, BLK);
        const uint32_t bad = bound_lane<C, REV>(T, X);
        reduce_lane(T, s.wred + wave * (2 * m + 2), active, k, bad, B.per_sub, B.S, B.flags, lane);
    }
    __syncthreads();
    if (tid == 0)
        write_partial(s.wred, BLK / 64, m, B.partial + (size_t)blockIdx.x * m * 2, B.partial_lo0 + blockIdx.x,
                      B.partial_k + blockIdx.x);
}

// Reduce per-block partials [nblocks][m][2] into reduced[m][2] (lo, hi) and argmin.
__global__ __launch_bounds__(256) void finish_kernel(const double *partial, const double *plo0, const int64_t *pk,
                                                     int nblocks, int m, double *reduced, int64_t *argmin) {
    __shared__ double sv[256];
    __shared__ int64_t sk[256];
    const int tid = threadIdx.x;
    for (int r = 0; r < m; ++r) {
        for (int c = 0; c < 2; ++c) {
            double v = __builtin_inf();
            for (int b = tid; b < nblocks; b += 256) v = fmin(v, partial[((size_t)b * m + r) * 2 + c]);
            sv[tid] = v;
            __syncthreads();
            for (int st = 128; st > 0; st >>= 1) {
                if (tid < st) sv[tid] = fmin(sv[tid], sv[tid + st]);
                __syncthreads();
            }
            if (tid == 0) reduced[r * 2 + c] = c == 0 ? sv[0] : -sv[0];
            __syncthreads();
        }
    }
    if (argmin) {
        double v = __builtin_inf();
        int64_t k = INT64_MAX;
        for (int b = tid; b < nblocks; b += 256) {
            const double v2 = plo0[b];
            const int64_t k2 = pk[b];
            if (v2 < v || (v2 == v && k2 < k)) { v = v2; k = k2; }
        }
        sv[tid] = v;
        sk[tid] = k;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (tid < st) {
                const double v2 = sv[tid + st];
                const int64_t k2 = sk[tid + st];
                if (v2 < sv[tid] || (v2 == sv[tid] && k2 < sk[tid])) { sv[tid] = v2; sk[tid] = k2; }
            }
            __syncthreads();
        }
        if (tid == 0) *argmin = sk[0];
    }
}

// ---------------------------------------------------------------------------
// batched: many nodes in one persistent launch
// ---------------------------------------------------------------------------

// One workgroup: validate every node, count its work items (chunks of BLK
// subdomains), exclusive prefix sum into item_off[N + 1], reset the work
// counter.  Invalid nodes (split outside [1, 65535], table above the LDS
// table capacity, more than 2^40 subdomains) get no items and status 1; if
// the total exceeds the workspace's item capacity no node runs (status 2).
__global__ __launch_bounds__(256) void batch_plan_kernel(BatchArgs A) {
    __shared__ int64_t part[256];
    const int tid = threadIdx.x;
    const int N = node_count(A);
    const int n = A.n;
    const int per = (N + 255) / 256;
    int64_t local = 0;
    for (int q = 0; q < per; ++q) {
        const int node = tid * per + q;
        if (node >= N) break;
        int64_t S = 1;
        int tab = 0;
        int ok = 1;
        for (int i = 0; i < n; ++i) {
            const int s = A.splits[(int64_t)node * n + i];
            if (s < 1 || s > 65535) { ok = 0; break; }
            tab += s;
            if (S > (INT64_C(1) << 40) / s) { ok = 0; break; }
            S *= s;
        }
        if (tab > A.tab_cap) ok = 0;
        A.node_S[node] = ok ? S : 0;
        A.status[node] = ok ? 0 : 1;
        local += ok ? (S + BLK - 1) / BLK : 0;
    }
    part[tid] = local;
    __syncthreads();
    __shared__ int over;
    if (tid == 0) {
        int64_t run = 0;
        for (int t = 0; t < 256; ++t) {
            const int64_t v = part[t];
            part[t] = run;
            run += v;
        }
        over = run > A.item_cap;             // more work than the workspace holds: run nothing
        A.item_off[N] = over ? 0 : run;
        *A.counter = 0;
    }
    __syncthreads();
    int64_t run = over ? 0 : part[tid];
    for (int q = 0; q < per; ++q) {
        const int node = tid * per + q;
        if (node >= N) break;
        A.item_off[node] = run;
        if (over) {
            A.node_S[node] = 0;
            A.status[node] = 2;
        }
        const int64_t S = A.node_S[node];
        run += (S + BLK - 1) / BLK;
    }
}

template <int C, bool REV>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_num_vgpr(SLOT_BASE), amdgpu_waves_per_eu(5, 5))) void batch_kernel(TapeArgs T,
                                                                                               BatchArgs A0) {
    using namespace dev;
    extern __shared__ __align__(16) uint8_t smem[];
    claim_slot_file();
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = T.n_roots, n = T.n;
    const int N = node_count(A0);
    const bool g_lds = A0.gacc == nullptr;
    Smem s = carve(smem, T, A0.tab_cap, BLK, REV && g_lds, C);
    __shared__ int64_t sh_item;
    __shared__ int sh_node;
    stage_program(T, s.prog, tid, BLK);

    Ctx X;
    X.prog = s.prog;
    X.tab = s.tab;
    X.vrec = s.vrec;
    X.G = g_lds ? s.G + tid : A0.gacc + (int64_t)blockIdx.x * BLK + tid;
    X.gstride = g_lds ? BLK : (int64_t)gridDim.x * BLK;
    X.tid = tid;
    X.blk = BLK;
    X.rec_stride = (int64_t)gridDim.x * BLK;
    X.rec = A0.rec + (int64_t)blockIdx.x * BLK + tid;
    X.spill = s.spill + tid;
    X.nreg = (uint32_t)T.nreg;
    const int64_t total = A0.item_off[N];
    int cur = -1;
    for (;;) {
        const BatchArgs &A = *opaque(&A0);
        if (tid == 0) sh_item = atomicAdd(reinterpret_cast<unsigned long long *>(A.counter), 1ull);
        __syncthreads();
        const int64_t item = sh_item;
        if (item >= total) break;                       // uniform exit: every wave reaches it
        if (tid == 0) {                                 // node owning the item: last node with item_off <= item
            int lo = 0, hi = N - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (A.item_off[mid] <= item) lo = mid; else hi = mid - 1;
            }
            while (lo < N - 1 && A.item_off[lo + 1] <= item) ++lo;   // skip nodes without items
            sh_node = lo;
        }
        __syncthreads();
        const int node = sh_node;
        if (node != cur) {                              // new node: splits, offsets, breakpoint table
            if (tid < n) s.ints[tid] = A.splits[(int64_t)node * n + tid];
            __syncthreads();
            if (tid == 0) {
                int acc = 0;
                for (int i = 0; i < n; ++i) { s.ints[MVF_MAX_VARS + i] = acc; acc += s.ints[i]; }
                s.ints[MVF_MAX_VARS + n] = acc;
            }
            __syncthreads();
            build_table(n, A.boxes + (int64_t)node * n * 2, s.ints, s.ints + MVF_MAX_VARS, s.tab, tid, BLK);
            cur = node;
        }
        if (lane == 0) reset_wred(s.wred + wave * (2 * m + 2), m);
        __syncthreads();
        const int64_t S = A.node_S[node];
        const int64_t k = (item - A.item_off[node]) * BLK + tid;
        const bool active = k < S;
        decode_subdomain(n, active ? k : S - 1, s.ints, s.ints + MVF_MAX_VARS, s.vrec, tid, BLK);
        const uint32_t bad = bound_lane<C, REV>(T, X);
        reduce_lane(T, s.wred + wave * (2 * m + 2), active, k, bad, nullptr, S, nullptr, lane);
        __syncthreads();
        if (tid == 0)
            write_partial(s.wred, BLK / 64, m, A.partial + (size_t)item * m * 2, A.partial_lo0 + item,
                          A.partial_k + item);
    }
}

// one workgroup per node: reduce the node's item partials
__global__ __launch_bounds__(256) void batch_finish_kernel(BatchArgs A, int m) {
    __shared__ double sv[256];
    __shared__ int64_t sk[256];
    const int node = blockIdx.x, tid = threadIdx.x;
    if (node >= node_count(A)) return;                    // uniform per block
    const int64_t b0 = A.item_off[node], b1 = A.item_off[node + 1];
    const bool ok = A.status[node] == 0;
    for (int r = 0; r < m; ++r) {
        for (int c = 0; c < 2; ++c) {
            double v = __builtin_inf();
            for (int64_t b = b0 + tid; b < b1; b += 256) v = fmin(v, A.partial[((size_t)b * m + r) * 2 + c]);
            sv[tid] = v;
            __syncthreads();
            for (int st = 128; st > 0; st >>= 1) {
                if (tid < st) sv[tid] = fmin(sv[tid], sv[tid + st]);
                __syncthreads();
            }
            if (tid == 0) A.reduced[((size_t)node * m + r) * 2 + c] = ok ? (c == 0 ? sv[0] : -sv[0]) : __builtin_nan("");
            __syncthreads();
        }
    }
    if (A.argmin) {
        double v = __builtin_inf();
        int64_t k = INT64_MAX;
        for (int64_t b = b0 + tid; b < b1; b += 256) {
            const double v2 = A.partial_lo0[b];
            const int64_t k2 = A.partial_k[b];
            if (v2 < v || (v2 == v && k2 < k)) { v = v2; k = k2; }
        }
        sv[tid] = v;
        sk[tid] = k;
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (tid < st) {
                const double v2 = sv[tid + st];
                const int64_t k2 = sk[tid + st];
                if (v2 < sv[tid] || (v2 == sv[tid] && k2 < sk[tid])) { sv[tid] = v2; sk[tid] = k2; }
            }
            __syncthreads();
        }
        if (tid == 0) A.argmin[node] = ok ? sk[0] : -1;
    }
}

// ---------------------------------------------------------------------------
// launch helpers (host)
// ---------------------------------------------------------------------------

template <typename K>
static hipError_t allow_lds(K kernel) {
    // leave room for the kernels' small static LDS variables
    return hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(LDS_BUDGET - 1024));
}

#define MVF_DISPATCH(C_, REV_, CALL)                       \
    do {                                                   \
        if (REV_) {                                        \
            constexpr int Cx = 0; constexpr bool Rx = true; \
            CALL;                                          \
        } else if ((C_) == 0) {                            \
            constexpr int Cx = 0; constexpr bool Rx = false; \
            CALL;                                          \
        } else if ((C_) == 1) {                            \
            constexpr int Cx = 1; constexpr bool Rx = false; \
            CALL;                                          \
        } else {                                           \
            constexpr int Cx = 2; constexpr bool Rx = false; \
            CALL;                                          \
        }                                                  \
    } while (0)

hipError_t launch_bound(const TapeArgs &T, const BoxArgs &B, int chunk, bool rev, int grid, size_t lds,
                        hipStream_t stream) {
    static_assert(MAX_CHUNK == 2, "one kernel instance per chunk size");
    hipError_t e = hipSuccess;
    MVF_DISPATCH(chunk, rev, {
        static std::once_flag once;
        static hipError_t ae = hipSuccess;
        std::call_once(once, [] { ae = allow_lds(bound_kernel<Cx, Rx>); });
        if (ae != hipSuccess) return ae;
        hipLaunchKernelGGL((bound_kernel<Cx, Rx>), dim3(grid), dim3(BLK), lds, stream, T, B);
    });
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, stream, B.partial, B.partial_lo0, B.partial_k, grid,
                       T.n_roots, B.reduced, B.argmin);
    return hipGetLastError();
}

hipError_t launch_batch(const TapeArgs &T, const BatchArgs &A, int chunk, bool rev, int grid, size_t lds,
                        int max_nodes, hipStream_t stream) {
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(256), 0, stream, A);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    MVF_DISPATCH(chunk, rev, {
        static std::once_flag once;
        static hipError_t ae = hipSuccess;
        std::call_once(once, [] { ae = allow_lds(batch_kernel<Cx, Rx>); });
        if (ae != hipSuccess) return ae;
        hipLaunchKernelGGL((batch_kernel<Cx, Rx>), dim3(grid), dim3(BLK), lds, stream, T, A);
    });
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_finish_kernel, dim3(max_nodes), dim3(256), 0, stream, A, T.n_roots);
    return hipGetLastError();
}

}  // namespace mvf
