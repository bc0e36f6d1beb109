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
// The subdomain bounds are min-reduced per wave with DPP lane moves, per
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
#include "mvf_lane.h"

namespace mvf {
namespace dev {

struct Ctx {
    const uint4 *prog;       // LDS program (root programs, then auxiliary records)
    const double4 *tab;      // LDS: {lo, nh, c, -c} per (dim, j)
    const uint16_t *vrec;    // LDS: [dim][BLK] table index of the lane's subdomain
    double2 *G;              // reverse-mode gradient accumulators of this lane ([dim] with stride gstride),
                             // in LDS or global memory (flat addressing)
    int64_t gstride;
    double2 *rec;            // global reverse-mode tape of this lane ([record][lane])
    int64_t rec_stride;      // lanes sharing the tape (record stride, in records)
    double2 *spill;          // LDS spill slots of this lane ([slot][component][lane])
    const double *vsrc;      // this lane's point [n] or box [n][2] (point and box entry points)
    uint32_t nreg;           // slot ids >= nreg are spilled (tangent passes)
    int tid, blk;
};

__device__ __forceinline__ double4 var_rec(const Ctx &X, uint32_t i) {
    return X.tab[X.vrec[i * X.blk + X.tid]];
}

// Where variable values come from: the breakpoint table of the lane's
// subdomain, the lane's point [x_i, x_i], or the lane's box.
enum : int { VS_TABLE = 0, VS_POINT = 1, VS_BOX = 2 };

template <int VS, bool POINT>
__device__ __forceinline__ Iv var_val(const Ctx &X, uint32_t i) {
    if constexpr (VS == VS_TABLE) {
        const double4 r = var_rec(X, i);
        return POINT ? Iv{r.z, r.w} : Iv{r.x, r.y};
    } else if constexpr (VS == VS_POINT) {
        const double x = X.vsrc[i];
        return Iv{x, -x};
    } else {
        return Iv{X.vsrc[2 * i], -X.vsrc[2 * i + 1]};
    }
}

__device__ __forceinline__ Iv aux_rec(const Ctx &X, uint32_t i) {
    const uint4 r = X.prog[i];
    return Iv{__hiloint2double((int)r.y, (int)r.x), __hiloint2double((int)r.w, (int)r.z)};
}

// Slot access for a pass carrying C tangent components: a slot holds the value
// then the components, 4 dwords each, and is moved as a whole (one GPR-index
// session); ids >= nreg live in LDS (tangent passes).
template <int C>
__device__ __forceinline__ void load_slot(const Ctx &X, uint32_t s, Iv (&A)[1 + C]) {
    if (C > 0 && s >= X.nreg) {
        const double2 *p = X.spill + (size_t)(s - X.nreg) * (1 + C) * X.blk;
#pragma unroll
        for (int i = 0; i <= C; ++i) {
            const double2 v = p[(size_t)i * X.blk];
            A[i] = Iv{v.x, v.y};
        }
        return;
    }
    slot_rd_n<1 + C>(s * (4 + 4 * C), A);
}
template <int C>
__device__ __forceinline__ void store_slot(const Ctx &X, uint32_t s, const Iv (&Z)[1 + C]) {
    if (C > 0 && s >= X.nreg) {
        double2 *p = X.spill + (size_t)(s - X.nreg) * (1 + C) * X.blk;
#pragma unroll
        for (int i = 0; i <= C; ++i) p[(size_t)i * X.blk] = make_double2(Z[i].lo, Z[i].nh);
        return;
    }
    slot_wr_n<1 + C>(s * (4 + 4 * C), Z);
}

// Operand (kind, a): value in A[0]; for a slot the C tangent components in
// A[1..C] (dense); for a variable, hit = its component index within
// [c0, c0 + C) (its tangent is one there and zero elsewhere), -1 otherwise;
// constants have zero tangents.
template <int C, bool POINT, int VS>
__device__ __forceinline__ void fetch(const Ctx &X, uint32_t kind, uint32_t a, double k, int c0, Iv (&A)[1 + C],
                                      bool &dense, int &hit) {
    dense = false;
    hit = -1;
    if (kind == K_SLOT) {
        dense = true;
        load_slot<C>(X, a, A);
    } else if (kind == K_VAR) {
        A[0] = var_val<VS, POINT>(X, a);
        const int h = (int)a - c0;
        hit = h >= 0 && h < C ? h : -1;
    } else {
        A[0] = Iv{k, -k};
    }
}

struct Dec {
    uint32_t w0, op, ak, bk, a, b, d;
    double k;
};

__device__ __forceinline__ Dec decode(uint4 raw) {
    Dec D;
    D.w0 = __builtin_amdgcn_readfirstlane(raw.x);
    const uint32_t w1 = __builtin_amdgcn_readfirstlane(raw.y);
    D.k = __hiloint2double((int)raw.w, (int)raw.z);
    D.op = D.w0 & 31u;
    D.ak = (D.w0 >> 5) & 3u;
    D.bk = (D.w0 >> 7) & 3u;
    D.a = D.w0 >> 16;
    D.b = w1 & 0xffffu;
    D.d = w1 >> 16;
    return D;
}

// Z[1 + h] = f(Z[1 + h]) for the hit component h of a variable operand
#define MVF_AT_HIT(h, EXPR)                                 \
    do {                                                    \
        _Pragma("unroll") for (int t_ = 0; t_ < C; ++t_) {  \
            if (t_ == (h)) { Iv &z = Z[1 + t_]; z = (EXPR); } \
        }                                                   \
    } while (0)

// Run one root program forward; returns the root's value interval and (C > 0)
// its tangent components [c0, c0 + C).  Each instruction moves its operands
// and its result as whole slots (value and components).  With TAPE, writes
// the reverse-mode records.
template <int C, bool POINT, bool TAPE, int VS = VS_TABLE>
__device__ Iv run_program(const Ctx &X, int begin, int len, int res_slot, int c0, Iv (&gout)[C > 0 ? C : 1],
                          uint32_t &bad) {
    constexpr int N = 1 + C;
    int64_t rp = 0;                                    // record position
    const int end = begin + len;
    uint4 nxt = X.prog[begin];
    for (int pc = begin; pc < end; ++pc) {
        const Dec I = decode(nxt);
        Iv A[N], B[N], Z[N];
        bool ad, bd = false;
        int ha, hb = -1;
        fetch<C, POINT, VS>(X, I.ak, I.a, I.k, c0, A, ad, ha);
        if (I.op <= I_DIV) fetch<C, POINT, VS>(X, I.bk, I.b, I.k, c0, B, bd, hb);
        nxt = X.prog[pc + 1 < end ? pc + 1 : pc];      // prefetch the next instruction
        const Iv U = A[0], V = B[0];
#pragma unroll
        for (int t = 1; t < N; ++t) Z[t] = kZero;
        switch (I.op) {
        case I_ADD:
            Z[0] = iadd(U, V);
            if constexpr (C > 0) {
                if (ad) {
#pragma unroll
                    for (int t = 1; t < N; ++t) Z[t] = A[t];
                }
                if (bd) {
#pragma unroll
                    for (int t = 1; t < N; ++t) Z[t] = iadd(Z[t], B[t]);     // exact when Z[t] is zero
                }
                if (ha >= 0) MVF_AT_HIT(ha, iadd(z, kOne));
                if (hb >= 0) MVF_AT_HIT(hb, iadd(z, kOne));
            }
            break;
        case I_SUB:
            Z[0] = isub(U, V);
            if constexpr (C > 0) {
                if (ad) {
#pragma unroll
                    for (int t = 1; t < N; ++t) Z[t] = A[t];
                }
                if (bd) {
#pragma unroll
                    for (int t = 1; t < N; ++t) Z[t] = isub(Z[t], B[t]);     // exact negation when Z[t] is zero
                }
                if (ha >= 0) MVF_AT_HIT(ha, iadd(z, kOne));
                if (hb >= 0) MVF_AT_HIT(hb, isub(z, kOne));
            }
            break;
        case I_MUL:
            Z[0] = imul(U, V);
            if constexpr (TAPE) {
                if (is_reg_kind(I.ak) && I.bk != K_CONST) X.rec[(rp++) * X.rec_stride] = make_double2(U.lo, U.nh);
                if (is_reg_kind(I.bk) && I.ak != K_CONST) X.rec[(rp++) * X.rec_stride] = make_double2(V.lo, V.nh);
            }
            if constexpr (C > 0) {
                if (ad) {
#pragma unroll
                    for (int t = 1; t < N; ++t) Z[t] = imul(V, A[t]);
                }
                if (bd) {
#pragma unroll
                    for (int t = 1; t < N; ++t) Z[t] = iadd(Z[t], imul(U, B[t]));   // exact when Z[t] is zero
                }
                if (ha >= 0) MVF_AT_HIT(ha, iadd(z, V));
                if (hb >= 0) MVF_AT_HIT(hb, iadd(z, U));
            }
            break;
        case I_DIV: {
            bad |= (V.lo <= 0.0 && V.nh <= 0.0) ? 1u : 0u;
            Z[0] = idiv(U, V);
            if constexpr (C > 0 || TAPE) {
                const Iv R = irecip(V);
                if constexpr (TAPE) {
                    X.rec[(rp++) * X.rec_stride] = make_double2(R.lo, R.nh);
                    if (I.bk != K_CONST) X.rec[(rp++) * X.rec_stride] = make_double2(Z[0].lo, Z[0].nh);
                }
                if constexpr (C > 0) {
                    // q = dU - Z dV, then dZ = q / V (times the enclosure of 1/V)
                    if (ad) {
#pragma unroll
                        for (int t = 1; t < N; ++t) Z[t] = A[t];
                    }
                    if (bd) {
#pragma unroll
                        for (int t = 1; t < N; ++t) Z[t] = isub(Z[t], imul(Z[0], B[t]));
                    }
                    if (ha >= 0) MVF_AT_HIT(ha, iadd(z, kOne));
                    if (hb >= 0) MVF_AT_HIT(hb, isub(z, Z[0]));
                    if (ad || bd || ha >= 0 || hb >= 0) {
#pragma unroll
                        for (int t = 1; t < N; ++t) Z[t] = imul(Z[t], R);
                    }
                }
            }
            break;
        }
        case I_SQR: case I_SQRT: case I_EXP: case I_LOG: case I_TANH: case I_SIN: case I_COS: {
            Iv D = kZero;                               // local derivative
            if (I.op == I_SQR) {
                Z[0] = isqr(U);
                if constexpr (C > 0 || TAPE) D = itwice(U);
            } else if (I.op == I_SQRT) {
                bad |= U.lo < 0.0 ? 1u : 0u;
                Z[0] = isqrt(U);
                if constexpr (C > 0 || TAPE) D = isqrt_deriv(Z[0]);
            } else if (I.op == I_EXP) {
                Z[0] = iexp(U);
                D = Z[0];
            } else if (I.op == I_LOG) {
                bad |= U.lo <= 0.0 ? 1u : 0u;
                Z[0] = ilog(U);
                if constexpr (C > 0 || TAPE) D = irecip(U);
            } else if (I.op == I_TANH) {
                Z[0] = itanh(U);
                if constexpr (C > 0 || TAPE) D = itanh_deriv(Z[0]);
            } else if (I.op == I_SIN) {
                Z[0] = isin(U);
                if constexpr (C > 0 || TAPE) D = isin_deriv(U);
            } else {
                Z[0] = icos(U);
                if constexpr (C > 0 || TAPE) D = icos_deriv(U);
            }
            if constexpr (TAPE) {
                if (I.ak != K_CONST) X.rec[(rp++) * X.rec_stride] = make_double2(D.lo, D.nh);
            }
            if constexpr (C > 0) {
                if (ad) {
#pragma unroll
                    for (int t = 1; t < N; ++t) Z[t] = imul(D, A[t]);
                }
                if (ha >= 0) MVF_AT_HIT(ha, D);
            }
            break;
        }
        case I_ADDK: case I_KSUB: case I_LOAD: {
            const bool ks = I.op == I_KSUB;
            Z[0] = I.op == I_ADDK ? Iv{fadd(U.lo, I.k), fsub(U.nh, I.k)} : ks ? Iv{fadd(I.k, U.nh), fsub(U.lo, I.k)} : U;
            if constexpr (C > 0) {
                if (ad) {
#pragma unroll
                    for (int t = 1; t < N; ++t) Z[t] = ks ? ineg(A[t]) : A[t];
                }
                if (ha >= 0) MVF_AT_HIT(ha, ks ? ineg(kOne) : kOne);
            }
            break;
        }
        case I_MULK: case I_MULKN: {
            const bool ng = I.op == I_MULKN;
            Z[0] = imulk(ng ? ineg(U) : U, I.k);
            if constexpr (C > 0) {
                if (ad) {
#pragma unroll
                    for (int t = 1; t < N; ++t) Z[t] = imulk(ng ? ineg(A[t]) : A[t], I.k);
                }
                if (ha >= 0) MVF_AT_HIT(ha, imulk(ng ? ineg(kOne) : kOne, I.k));
            }
            break;
        }
        default: {   // I_DIVK, I_DIVKN
            const bool ng = I.op == I_DIVKN;
            Z[0] = idivk(ng ? ineg(U) : U, I.k);
            if constexpr (C > 0) {
                const Iv R = aux_rec(X, I.b);
                if (ad) {
#pragma unroll
                    for (int t = 1; t < N; ++t) Z[t] = imul_pos(ng ? ineg(A[t]) : A[t], R);
                }
                if (ha >= 0) MVF_AT_HIT(ha, imul_pos(ng ? ineg(kOne) : kOne, R));
            }
            break;
        }
        }
        store_slot<C>(X, I.d, Z);
    }
    if (res_slot < 0) return kZero;                    // the union program: roots are read by the caller
    Iv R[N];
    load_slot<C>(X, (uint32_t)res_slot, R);
#pragma unroll
    for (int t = 0; t < C; ++t) gout[t] = R[1 + t];
    return R[0];
}
#undef MVF_AT_HIT

__device__ __forceinline__ Iv ld_rec(const Ctx &X, int64_t rp) {
    const double2 v = X.rec[rp * X.rec_stride];
    return Iv{v.x, v.y};
}

// adjoint contribution c to operand (kind, a); init: first contribution
// (written, not accumulated; 0 - [lo, hi] = [-hi, -lo]); neg: subtract
__device__ __forceinline__ void contribute(const Ctx &X, uint32_t kind, uint32_t a, bool init, bool neg, Iv c) {
    if (kind == K_SLOT) {
        const uint32_t idx = a * 4;
        if (init) {
            slot_wr(idx, neg ? ineg(c) : c);
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

// Reverse sweep over one program.  The caller seeds the adjoints of the
// program's results (for a root program: [1, 1] in its result slot).
template <int VS = VS_TABLE>
__device__ void reverse_sweep(const Ctx &X, int begin, int len, int64_t n_rec) {
    int64_t rp = n_rec;
    uint4 nxt = X.prog[begin + len - 1];
    for (int pc = begin + len - 1; pc >= begin; --pc) {
        const uint4 raw = nxt;
        nxt = X.prog[pc > begin ? pc - 1 : pc];        // prefetch the next instruction
        const Dec I = decode(raw);
        const bool ia = (I.w0 & W0_INIT_A) != 0, ib = (I.w0 & W0_INIT_B) != 0;
        const Iv zb = slot_rd(I.d * 4);
        switch (I.op) {
        case I_ADD: case I_SUB:
            contribute(X, I.ak, I.a, ia, false, zb);
            contribute(X, I.bk, I.b, ib, I.op == I_SUB, zb);
            break;
        case I_MUL: {
            const bool hv = is_reg_kind(I.bk) && I.ak != K_CONST, hu = is_reg_kind(I.ak) && I.bk != K_CONST;
            Iv V = kZero, U = kZero;
            if (hv) V = ld_rec(X, --rp);
            if (hu) U = ld_rec(X, --rp);
            if (I.ak != K_CONST) {
                if (I.bk == K_VAR) V = var_val<VS, false>(X, I.b);
                else if (I.bk == K_CONST) V = Iv{I.k, -I.k};
                contribute(X, I.ak, I.a, ia, false, imul(zb, V));
            }
            if (I.bk != K_CONST) {
                if (I.ak == K_VAR) U = var_val<VS, false>(X, I.a);
                else if (I.ak == K_CONST) U = Iv{I.k, -I.k};
                contribute(X, I.bk, I.b, ib, false, imul(zb, U));
            }
            break;
        }
        case I_DIV: {
            Iv Z = kZero;
            if (I.bk != K_CONST) Z = ld_rec(X, --rp);
            const Iv R = ld_rec(X, --rp);
            const Iv T = imul(zb, R);
            contribute(X, I.ak, I.a, ia, false, T);
            if (I.bk != K_CONST) contribute(X, I.bk, I.b, ib, true, imul(T, Z));
            break;
        }
        case I_SQR: case I_SQRT: case I_EXP: case I_LOG: case I_TANH: case I_SIN: case I_COS:
            if (I.ak != K_CONST) {
                const Iv R = ld_rec(X, --rp);
                contribute(X, I.ak, I.a, ia, false, imul(zb, R));
            }
            break;
        case I_ADDK: case I_KSUB: case I_LOAD:
            contribute(X, I.ak, I.a, ia, I.op == I_KSUB, zb);
            break;
        case I_MULK: case I_MULKN:
            contribute(X, I.ak, I.a, ia, false, imulk(I.op == I_MULKN ? ineg(zb) : zb, I.k));
            break;
        default:     // I_DIVK, I_DIVKN
            contribute(X, I.ak, I.a, ia, false, imul_pos(I.op == I_DIVKN ? ineg(zb) : zb, aux_rec(X, I.b)));
            break;
        }
    }
}

// Bounds of every root on the lane's subdomain, each folded into the wave's
// reduction record as soon as it is known.  Returns the domain flag
// (violation or NaN).
template <int C, bool REV>
__device__ uint32_t bound_lane(int m, int n, int mode, int root_base, const Ctx &X, const LaneOut &o,
                               FeasTrack &F) {
    mode_round_down();
    uint32_t bad = 0;
    for (int r = 0; r < m; ++r) {
        const uint4 ri = X.prog[root_base + r];
        const int pb = (int)__builtin_amdgcn_readfirstlane(ri.x), pl = (int)__builtin_amdgcn_readfirstlane(ri.y);
        const int rs = (int)__builtin_amdgcn_readfirstlane(ri.z);
        Iv B, FC = kZero;
        Iv g0[1];
        if (mode == MVF_MODE_NIE) {
            B = run_program<0, false, false>(X, pb, pl, rs, 0, g0, bad);
        } else if constexpr (REV) {
            FC = run_program<0, true, false>(X, pb, pl, rs, 0, g0, bad);
            const Iv nie = run_program<0, false, true>(X, pb, pl, rs, 0, g0, bad);
            for (int i = 0; i < n; ++i) X.G[i * X.gstride] = make_double2(0.0, 0.0);
            slot_wr((uint32_t)rs * 4, kOne);
            reverse_sweep(X, pb, pl, (int64_t)__builtin_amdgcn_readfirstlane(ri.w));
            Iv acc = FC;
            for (int i = 0; i < n; ++i) {
                const double4 rec = var_rec(X, (uint32_t)i);
                const Iv D = {fadd(rec.x, rec.w), fadd(rec.y, rec.z)};   // X_i - c_i
                const double2 g = X.G[i * X.gstride];
                acc = iadd(acc, imul(Iv{g.x, g.y}, D));
            }
            B = mode == MVF_MODE_MVF ? acc : Iv{fmax_(acc.lo, nie.lo), fmax_(acc.nh, nie.nh)};
        } else if constexpr (C > 0) {
            Iv G[C];
            FC = run_program<0, true, false>(X, pb, pl, rs, 0, g0, bad);
            Iv acc = FC, nie = kZero;
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
            B = mode == MVF_MODE_MVF ? acc : Iv{fmax_(acc.lo, nie.lo), fmax_(acc.nh, nie.nh)};
        } else {
            B = kZero;   // not launched: a forward gradient needs tangent components
        }
        if (B.lo != B.lo || B.nh != B.nh) bad = 1;
        reduce_root(r, m, B, o);
        track_root(F, r, B, FC, mode != MVF_MODE_NIE, o);
    }
    mode_round_nearest();
    return bad;
}

// stage the programs into LDS (whole workgroup)
template <typename TA>
__device__ __forceinline__ void stage_program(const TA &T, uint4 *lprog, int tid, int blk) {
    const uint4 *src = reinterpret_cast<const uint4 *>(T.prog);
    for (int i = tid; i < T.n_instr; i += blk) lprog[i] = src[i];
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

template <typename TA>     // TapeArgs in any address space
__device__ __forceinline__ Smem carve(uint8_t *smem, const TA &T, int tab_cap, int blk, bool g_lds, int chunk) {
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
    p += (size_t)(blk / 64) * wred_len(T.n_roots) * 8;       // 32 (2m + 3) bytes: 16-byte aligned
    s.ints = reinterpret_cast<int32_t *>(p);
    p += (2 * MVF_MAX_VARS + 8) * 4;       // every region above is a multiple of 16 bytes
    s.vrec = reinterpret_cast<uint16_t *>(p);
    return s;
}

}  // namespace dev

// ---------------------------------------------------------------------------
// single box
// ---------------------------------------------------------------------------
template <int C, bool REV>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_num_vgpr(SLOT_BASE), amdgpu_waves_per_eu(4, 4))) void bound_kernel(
    BoundKArgs /* read through kargs() */) {
    using namespace dev;
    extern __shared__ __align__(16) uint8_t smem[];
    claim_slot_file();
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    Smem s;
    Ctx X;
    int m, n;
    {
        const auto K = kargs<BoundKArgs>();
        m = K->T.n_roots;
        n = K->T.n;
        const bool g_lds = K->B.gacc == nullptr;
        s = carve(smem, K->T, K->B.tab_off[n], BLK, REV && g_lds, C);
        stage_program(K->T, s.prog, tid, BLK);
        if (tid <= n) s.ints[MVF_MAX_VARS + tid] = K->B.tab_off[tid];
        if (tid < n) s.ints[tid] = K->B.splits[tid];
        __syncthreads();
        build_table(n, K->B.box, s.ints, s.ints + MVF_MAX_VARS, s.tab, tid, BLK);
        if (lane == 0) reset_wred(s.wred + wave * wred_len(m), m);
        X.G = g_lds ? s.G + tid : K->B.gacc + ((int64_t)blockIdx.x * BLK + wave * 64) * n + lane;
        X.gstride = g_lds ? BLK : 64;
        X.rec = K->B.rec + ((int64_t)blockIdx.x * BLK + wave * 64) * K->B.rec_lane + lane;
        X.nreg = (uint32_t)K->T.nreg;
    }
    __syncthreads();
    X.prog = s.prog;
    X.tab = s.tab;
    X.vrec = s.vrec;
    X.tid = tid;
    X.blk = BLK;
    X.rec_stride = 64;
    X.spill = s.spill + tid;
    for (int64_t base = (int64_t)blockIdx.x * BLK;; base += (int64_t)gridDim.x * BLK) {
        const int64_t S = kargs<BoundKArgs>()->B.S;
        if (base >= S) break;
        const int64_t k = base + tid;
        const bool active = k < S;
        decode_subdomain(n, active ? k : S - 1, s.ints, s.ints + MVF_MAX_VARS, s.vrec, tid, BLK);
        LaneOut o;
        FeasTrack F;
        uint32_t bad;
        {
            const auto K = kargs<BoundKArgs>();
            o.per_sub = K->B.per_sub;
            o.S = S;
            o.k = k;
            o.w = s.wred + wave * wred_len(m);
            o.lane = lane;
            o.active = active;
            o.ineq = K->T.ineq_mask;
            o.eq = K->T.eq_mask;
            bad = bound_lane<C, REV>(m, n, K->T.mode, K->T.root_base, X, o, F);
        }
        finish_lane(m, bad, F, o, kargs<BoundKArgs>()->B.flags);
    }
    __syncthreads();
    if (tid == 0) {
        const auto K = kargs<BoundKArgs>();
        write_partial(s.wred, BLK / 64, m, K->B.partial + (size_t)blockIdx.x * m * 2, K->B.partial_lo0 + blockIdx.x,
                      K->B.partial_k + blockIdx.x, K->B.partial_ext + 2 * (size_t)blockIdx.x);
    }
}

// minimum over the workgroup of one value per thread (all threads get it)
__device__ __forceinline__ double block_min(double v, double *sv, int tid) {
    sv[tid] = v;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) sv[tid] = fmin(sv[tid], sv[tid + st]);
        __syncthreads();
    }
    const double r = sv[0];
    __syncthreads();
    return r;
}

// Reduce per-block partials [nblocks][m][2] into reduced[m][2] (lo, hi), argmin,
// and the two B&B bounds (extra, nullable): every thread takes the minima of
// all quantities over its share of the blocks (one block each up to 1024
// blocks, so all loads are in flight at once), each wave reduces them with
// DPP lane moves, and the last step combines the waves.
constexpr int FIN_BLK = 1024;
__global__ __launch_bounds__(FIN_BLK) void finish_kernel(const double *partial, const double *plo0, const int64_t *pk,
                                                         const double *pext, int nblocks, int m, double *reduced,
                                                         int64_t *argmin, double *extra) {
    using namespace dev;
    constexpr int Q = 2 * MVF_MAX_ROOTS;
    constexpr int W = FIN_BLK / 64;
    __shared__ double sv[W][Q + 2];
    __shared__ double sav[W];
    __shared__ int64_t sak[W];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    double v[Q], e0 = __builtin_inf(), e1 = __builtin_inf(), av = __builtin_inf();
    int64_t ak = INT64_MAX;
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = __builtin_inf();
    for (int b = tid; b < nblocks; b += FIN_BLK) {
        const double *pb = partial + (size_t)b * m * 2;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (q < 2 * m) v[q] = fmin(v[q], pb[q]);
        if (extra) {
            e0 = fmin(e0, pext[2 * (size_t)b]);
            e1 = fmin(e1, pext[2 * (size_t)b + 1]);
        }
        if (argmin) {
            const double v2 = plo0[b];
            const int64_t k2 = pk[b];
            if (v2 < av || (v2 == av && k2 < ak)) {
                av = v2;
                ak = k2;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < Q; ++q)
        if (q < 2 * m) v[q] = wave_min(v[q]);
    if (extra) {
        e0 = wave_min(e0);
        e1 = wave_min(e1);
    }
    if (argmin) wave_argmin(av, ak);
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (q < 2 * m) sv[wave][q] = v[q];
        sv[wave][Q] = e0;
        sv[wave][Q + 1] = e1;
        sav[wave] = av;
        sak[wave] = ak;
    }
    __syncthreads();
    if (tid < 2 * m || (extra && (tid == Q || tid == Q + 1))) {
        double r = sv[0][tid];
        for (int w = 1; w < W; ++w) r = fmin(r, sv[w][tid]);
        if (tid < 2 * m) reduced[tid] = (tid & 1) ? -r : r;
        else extra[tid - Q] = r;
    }
    if (argmin && tid == 0) {
        double a = sav[0];
        int64_t k = sak[0];
        for (int w = 1; w < W; ++w)
            if (sav[w] < a || (sav[w] == a && sak[w] < k)) {
                a = sav[w];
                k = sak[w];
            }
        *argmin = k;
    }
}

// ---------------------------------------------------------------------------
// batched: many nodes in one persistent launch
// ---------------------------------------------------------------------------

// One workgroup: validate every node, count its work items (chunks of spl * BLK
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
    const int64_t isz = (int64_t)A.spl * BLK;      // subdomains per work item
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
        local += ok ? (S + isz - 1) / isz : 0;
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
        run += (S + isz - 1) / isz;
    }
}

template <int C, bool REV>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_num_vgpr(SLOT_BASE), amdgpu_waves_per_eu(4, 4))) void batch_kernel(
    BatchKArgs /* read through kargs() */) {
    using namespace dev;
    extern __shared__ __align__(16) uint8_t smem[];
    claim_slot_file();
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    __shared__ int64_t sh_item;
    __shared__ int sh_node;
    Smem s;
    Ctx X;
    int m, n;
    {
        const auto K = kargs<BatchKArgs>();
        m = K->T.n_roots;
        n = K->T.n;
        const bool g_lds = K->A.gacc == nullptr;
        s = carve(smem, K->T, K->A.tab_cap, BLK, REV && g_lds, C);
        stage_program(K->T, s.prog, tid, BLK);
        X.G = g_lds ? s.G + tid : K->A.gacc + ((int64_t)blockIdx.x * BLK + wave * 64) * n + lane;
        X.gstride = g_lds ? BLK : 64;
        X.rec = K->A.rec + ((int64_t)blockIdx.x * BLK + wave * 64) * K->A.rec_lane + lane;
        X.nreg = (uint32_t)K->T.nreg;
    }
    X.prog = s.prog;
    X.tab = s.tab;
    X.vrec = s.vrec;
    X.tid = tid;
    X.blk = BLK;
    X.rec_stride = 64;
    X.spill = s.spill + tid;
    int cur = -1;
    for (;;) {
        {
            const auto K = kargs<BatchKArgs>();
            if (tid == 0) sh_item = atomicAdd(reinterpret_cast<unsigned long long *>(K->A.counter), 1ull);
        }
        __syncthreads();
        const int64_t item = sh_item;
        int N;
        {
            const auto K = kargs<BatchKArgs>();
            N = node_count(K->A);
            if (item >= K->A.item_off[N]) break;           // uniform exit: every wave reaches it
            if (tid == 0) {                                 // node owning the item: last node with item_off <= item
                int lo = 0, hi = N - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (K->A.item_off[mid] <= item) lo = mid; else hi = mid - 1;
                }
                while (lo < N - 1 && K->A.item_off[lo + 1] <= item) ++lo;   // skip nodes without items
                sh_node = lo;
            }
        }
        __syncthreads();
        const int node = sh_node;
        if (node != cur) {                              // new node: splits, offsets, breakpoint table
            const auto K = kargs<BatchKArgs>();
            if (tid < n) s.ints[tid] = K->A.splits[(int64_t)node * n + tid];
            __syncthreads();
            if (tid == 0) {
                int acc = 0;
                for (int i = 0; i < n; ++i) { s.ints[MVF_MAX_VARS + i] = acc; acc += s.ints[i]; }
                s.ints[MVF_MAX_VARS + n] = acc;
            }
            __syncthreads();
            build_table(n, K->A.boxes + (int64_t)node * n * 2, s.ints, s.ints + MVF_MAX_VARS, s.tab, tid, BLK);
            cur = node;
        }
        if (lane == 0) reset_wred(s.wred + wave * wred_len(m), m);
        __syncthreads();
        int64_t S, base;
        int spl;
        {
            const auto K = kargs<BatchKArgs>();
            S = K->A.node_S[node];
            spl = K->A.spl;
            base = (item - K->A.item_off[node]) * spl * BLK;
        }
        for (int j = 0; j < spl && base + (int64_t)j * BLK < S; ++j) {      // uniform over the workgroup
            const int64_t k = base + (int64_t)j * BLK + tid;
            const bool active = k < S;
            decode_subdomain(n, active ? k : S - 1, s.ints, s.ints + MVF_MAX_VARS, s.vrec, tid, BLK);
            LaneOut o;
            o.per_sub = nullptr;
            o.S = S;
            o.k = k;
            o.w = s.wred + wave * wred_len(m);
            o.lane = lane;
            o.active = active;
            FeasTrack F;
            uint32_t bad;
            {
                const auto K = kargs<BatchKArgs>();
                o.ineq = K->T.ineq_mask;
                o.eq = K->T.eq_mask;
                bad = bound_lane<C, REV>(m, n, K->T.mode, K->T.root_base, X, o, F);
            }
            finish_lane(m, bad, F, o, nullptr);
        }
        __syncthreads();
        if (tid == 0) {
            const auto K = kargs<BatchKArgs>();
            write_partial(s.wred, BLK / 64, m, K->A.partial + (size_t)item * m * 2, K->A.partial_lo0 + item,
                          K->A.partial_k + item, K->A.partial_ext + 2 * (size_t)item);
        }
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
    if (A.extra) {
        for (int c = 0; c < 2; ++c) {
            double v = __builtin_inf();
            for (int64_t b = b0 + tid; b < b1; b += 256) v = fmin(v, A.partial_ext[2 * b + c]);
            v = block_min(v, sv, tid);
            if (tid == 0) A.extra[2 * (size_t)node + c] = ok ? v : __builtin_nan("");
        }
    }
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
// points and boxes: values and vector-Jacobian products at points, interval
// gradients on boxes (one lane per point or box, grid-stride)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t u4_at(uint4 q, int j) { return j == 0 ? q.x : j == 1 ? q.y : j == 2 ? q.z : q.w; }

template <int OP, int C>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_num_vgpr(SLOT_BASE), amdgpu_waves_per_eu(4, 4))) void points_kernel(
    PointsKArgs /* read through kargs() */) {
    using namespace dev;
    extern __shared__ __align__(16) uint8_t smem[];
    claim_slot_file();
    const int tid = threadIdx.x;
    uint4 *lprog = reinterpret_cast<uint4 *>(smem);
    Ctx X;
    int m, n;
    {
        const auto K = kargs<PointsKArgs>();
        m = K->P.n_roots;
        n = K->P.n;
        const int nr = K->P.n_records;
        const uint4 *src = reinterpret_cast<const uint4 *>(K->P.prog);
        for (int i = tid; i < nr; i += BLK) lprog[i] = src[i];
        uint8_t *p = smem + (size_t)nr * 16;
        // gradient accumulators exist only for the reverse-mode entry points (the
        // host sizes the LDS the same way: programs, accumulators, spill slots)
        constexpr bool REVOP = OP == PT_VJP || OP == PT_GRAD_REV;
        const bool g_lds = REVOP && K->P.gacc == nullptr;
        X.G = g_lds ? reinterpret_cast<double2 *>(p) + tid
                    : K->P.gacc + ((int64_t)blockIdx.x * BLK + (tid >> 6) * 64) * n + (tid & 63);
        X.gstride = g_lds ? BLK : 64;
        if (g_lds) p += (size_t)n * BLK * 16;
        X.spill = reinterpret_cast<double2 *>(p) + tid;
        X.rec = K->P.rec + ((int64_t)blockIdx.x * BLK + (tid >> 6) * 64) * K->P.rec_lane + (tid & 63);
        X.nreg = (uint32_t)K->P.nreg;
    }
    __syncthreads();
    X.prog = lprog;
    X.tab = nullptr;
    X.vrec = nullptr;
    X.tid = tid;
    X.blk = BLK;
    X.rec_stride = 64;
    constexpr int VS = OP >= PT_GRAD_FWD ? VS_BOX : VS_POINT;
    for (int64_t base = (int64_t)blockIdx.x * BLK;; base += (int64_t)gridDim.x * BLK) {
        int64_t B, k, kk;
        int ub, ul, urec, root_rec;
        {
            const auto K = kargs<PointsKArgs>();
            B = K->P.B;
            if (base >= B) break;
            k = base + tid;
            kk = k < B ? k : B - 1;                  // lanes past the end repeat the last item; nothing is stored
            X.vsrc = K->P.x + kk * n * (VS == VS_BOX ? 2 : 1);
            const uint4 ur = X.prog[K->P.union_base];
            ub = (int)__builtin_amdgcn_readfirstlane(ur.x);
            ul = (int)__builtin_amdgcn_readfirstlane(ur.y);
            urec = (int)__builtin_amdgcn_readfirstlane(ur.z);
            root_rec = K->P.root_base + K->P.root;
        }
        const bool active = k < B;
        const int ubase = kargs<PointsKArgs>()->P.union_base;
        mode_round_down();
        uint32_t bad = 0;
        Iv g0[1];
        if constexpr (OP == PT_EVAL) {
            run_program<0, true, false, VS>(X, ub, ul, -1, 0, g0, bad);
            double *f = kargs<PointsKArgs>()->P.out;
            for (int r = 0; r < m; ++r) {
                const uint4 q = X.prog[ubase + 1 + r / 4];
                const uint32_t sl = __builtin_amdgcn_readfirstlane(u4_at(q, r & 3));
                const Iv v = slot_rd(sl * 4);
                if (active) {
                    f[(kk * m + r) * 2] = bad ? -__builtin_inf() : v.lo;
                    f[(kk * m + r) * 2 + 1] = bad ? __builtin_inf() : -v.nh;
                }
            }
        } else if constexpr (OP == PT_VJP) {
            run_program<0, true, true, VS>(X, ub, ul, -1, 0, g0, bad);
            for (int i = 0; i < n; ++i) X.G[i * X.gstride] = make_double2(0.0, 0.0);
            const double *gout = kargs<PointsKArgs>()->P.gout;
            for (int r = 0; r < m; ++r) {                // seeds, roots in order; a repeated root accumulates
                const uint4 q = X.prog[ubase + 1 + r / 4];
                const uint32_t sl = __builtin_amdgcn_readfirstlane(u4_at(q, r & 3));
                bool seen = false;
                for (int r2 = 0; r2 < r; ++r2) {
                    const uint4 q2 = X.prog[ubase + 1 + r2 / 4];
                    seen |= __builtin_amdgcn_readfirstlane(u4_at(q2, r2 & 3)) == sl;
                }
                const double g = gout[kk * m + r];
                const Iv seed = {g, -g};
                slot_wr(sl * 4, seen ? iadd(slot_rd(sl * 4), seed) : seed);
            }
            reverse_sweep<VS>(X, ub, ul, urec);
        } else {
            run_program<0, false, false, VS>(X, ub, ul, -1, 0, g0, bad);   // domain of every live node
            const uint4 ri = X.prog[root_rec];
            const int pb = (int)__builtin_amdgcn_readfirstlane(ri.x), pl = (int)__builtin_amdgcn_readfirstlane(ri.y);
            const int rs = (int)__builtin_amdgcn_readfirstlane(ri.z);
            uint32_t bad2 = 0;
            double *Gout = kargs<PointsKArgs>()->P.out;
            if constexpr (OP == PT_GRAD_REV) {
                run_program<0, false, true, VS>(X, pb, pl, rs, 0, g0, bad2);
                for (int i = 0; i < n; ++i) X.G[i * X.gstride] = make_double2(0.0, 0.0);
                slot_wr((uint32_t)rs * 4, kOne);
                reverse_sweep<VS>(X, pb, pl, (int64_t)__builtin_amdgcn_readfirstlane(ri.w));
            } else {
                for (int c0 = 0; c0 < n; c0 += C) {
                    Iv G[C];
                    run_program<C, false, false, VS>(X, pb, pl, rs, c0, G, bad2);
#pragma unroll
                    for (int t = 0; t < C; ++t) {
                        if (active && c0 + t < n) {
                            Gout[(kk * n + c0 + t) * 2] = bad ? -__builtin_inf() : G[t].lo;
                            Gout[(kk * n + c0 + t) * 2 + 1] = bad ? __builtin_inf() : -G[t].nh;
                        }
                    }
                }
            }
        }
        mode_round_nearest();
        if constexpr (OP == PT_VJP || OP == PT_GRAD_REV) {
            double *o = kargs<PointsKArgs>()->P.out;
            for (int i = 0; i < n; ++i) {
                const double2 g = X.G[i * X.gstride];
                if (active) {
                    o[(kk * n + i) * 2] = bad ? -__builtin_inf() : g.x;
                    o[(kk * n + i) * 2 + 1] = bad ? __builtin_inf() : -g.y;
                }
            }
        }
        uint32_t *flags = kargs<PointsKArgs>()->P.flags;
        if (active && flags) flags[kk] = bad;
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

// ---------------------------------------------------------------------------
// constraint propagation (forward-backward bound tightening) of node boxes
// ---------------------------------------------------------------------------
//
// The bound tightening the paper reports compatible with its method
// (constraint propagation, Sec. 3.2; its effect, Sec. 4.3): one lane per box
// walks the tape's DAG forward (the bounding interval
// extension of every live node; a violated domain gives [-inf, inf] and marks
// the node as carrying no information), cuts the roots to their feasible
// ranges (g <= 0, h = 0, objective <= ub), then backward in descending node
// order intersects each operand with the outward-rounded inverse of its
// operation, and finally meets every variable with its variable nodes.  An
// empty intersection proves the box infeasible.  Rounds repeat on the
// tightened box.  Node intervals live in global scratch [node][lane], the
// no-information marks in the rows after them.
namespace dev {

__device__ __forceinline__ Iv imeet(Iv a, Iv b) { return {fmax_(a.lo, b.lo), fmax_(a.nh, b.nh)}; }
__device__ __forceinline__ bool iempty(Iv a) { return !(a.lo <= -a.nh); }
__device__ __forceinline__ bool has_zero(Iv a) { return a.lo <= 0.0 && a.nh <= 0.0; }

// returns 1 when the box is proven infeasible (X then undefined)
__device__ uint32_t fbbt_lane(const FbbtArgs &A, double2 *val, int64_t stride, Iv *X) {
    constexpr double inf = __builtin_inf();
    const Iv nonneg = {0.0, -inf}, unit = {-1.0, -1.0};
    for (int round = 0; round < A.rounds; ++round) {
        // forward
        for (int i = 0; i < A.n_nodes; ++i) {
            const DagNode nd = A.nodes[i];
            if (!nd.live) continue;
            const Iv U = nd.op >= MVF_ADD ? Iv{val[(int64_t)nd.a * stride].x, val[(int64_t)nd.a * stride].y} : kZero;
            const Iv V = nd.op >= MVF_ADD && nd.op <= MVF_DIV
                             ? Iv{val[(int64_t)nd.b * stride].x, val[(int64_t)nd.b * stride].y} : kZero;
            Iv Z = kZero;
            int info = 1;
            switch (nd.op) {
            case MVF_VAR: Z = X[nd.a]; break;
            case MVF_CONST: Z = Iv{A.consts[nd.a], -A.consts[nd.a]}; break;
            case MVF_ADD: Z = iadd(U, V); break;
            case MVF_SUB: Z = isub(U, V); break;
            case MVF_MUL: Z = imul(U, V); break;
            case MVF_DIV:
                if (has_zero(V)) { info = 0; Z = Iv{-inf, -inf}; } else Z = idiv(U, V);
                break;
            case MVF_SQR: Z = isqr(U); break;
            case MVF_SQRT:
                if (U.lo < 0.0) { info = 0; Z = Iv{-inf, -inf}; } else Z = isqrt(U);
                break;
            case MVF_EXP: Z = iexp(U); break;
            case MVF_LOG:
                if (U.lo <= 0.0) { info = 0; Z = Iv{-inf, -inf}; } else Z = ilog(U);
                break;
            case MVF_TANH: Z = itanh(U); break;
            case MVF_SIN: Z = isin(U); break;
            default: Z = icos(U); break;
            }
            val[(int64_t)i * stride] = make_double2(Z.lo, Z.nh);
            val[((int64_t)A.n_nodes + i) * stride].x = info ? 1.0 : 0.0;    // rows n_nodes..: the marks
        }
        // the roots' feasible ranges
        for (int r = 0; r < A.m; ++r) {
            double2 &z = val[(int64_t)A.roots[r] * stride];
            Iv c = {-inf, -inf};
            if ((A.ineq_mask >> r) & 1u) c = Iv{-inf, -0.0};
            else if ((A.eq_mask >> r) & 1u) c = Iv{0.0, -0.0};
            else if (r == 0 && A.ub < inf) c = Iv{-inf, -A.ub};
            const Iv m = imeet(Iv{z.x, z.y}, c);
            z = make_double2(m.lo, m.nh);
        }
        // backward
        for (int i = A.n_nodes - 1; i >= 0; --i) {
            const DagNode nd = A.nodes[i];
            if (!nd.live) continue;
            const double2 zv = val[(int64_t)i * stride];
            Iv Z = {zv.x, zv.y};
            if (iempty(Z)) return 1;
            if (nd.op < MVF_ADD || val[((int64_t)A.n_nodes + i) * stride].x == 0.0) continue;
            double2 &us = val[(int64_t)nd.a * stride];
            Iv U = {us.x, us.y};
            const bool bin = nd.op <= MVF_DIV;
            Iv V = kZero;
            if (bin) {
                const double2 vs = val[(int64_t)nd.b * stride];
                V = Iv{vs.x, vs.y};
            }
            switch (nd.op) {
            // operands a and b may be one node: the second narrowing then starts from the first
            case MVF_ADD:
                U = imeet(U, isub(Z, V));
                if (nd.a == nd.b) V = U;
                V = imeet(V, isub(Z, U));
                if (nd.a == nd.b) U = V;
                break;
            case MVF_SUB:
                U = imeet(U, iadd(Z, V));
                if (nd.a == nd.b) V = U;
                V = imeet(V, isub(U, Z));
                if (nd.a == nd.b) U = V;
                break;
            case MVF_MUL:
                if (!has_zero(V)) U = imeet(U, idiv(Z, V));
                if (nd.a == nd.b) V = U;
                if (!iempty(U) && !has_zero(U)) V = imeet(V, idiv(Z, U));
                if (nd.a == nd.b) U = V;
                break;
            case MVF_DIV:
                U = imeet(U, imul(Z, V));
                if (nd.a == nd.b) V = U;
                if (!has_zero(Z)) V = imeet(V, idiv(U, Z));
                if (nd.a == nd.b) U = V;
                break;
            case MVF_SQR: {
                Z = imeet(Z, nonneg);
                if (iempty(Z)) return 1;
                const Iv R = isqrt(Z);
                if (U.lo >= 0.0) U = imeet(U, R);
                else if (U.nh >= 0.0) U = imeet(U, ineg(R));
                else U = imeet(U, Iv{R.nh, R.nh});
                break;
            }
            case MVF_SQRT:
                Z = imeet(Z, nonneg);
                if (iempty(Z)) return 1;
                U = imeet(U, isqr(Z));
                break;
            case MVF_EXP:
                Z = imeet(Z, nonneg);
                if (iempty(Z) || -Z.nh <= 0.0) return 1;    // exp > 0
                U = imeet(U, ilog(Z));
                break;
            case MVF_LOG: U = imeet(U, iexp(Z)); break;
            case MVF_TANH: {
                Z = imeet(Z, unit);
                if (iempty(Z)) return 1;
                double a = Z.lo, b = -Z.nh;
                lib2<LIB_ATANH>(a, b);
                const Iv R = {Z.lo <= -1.0 ? -inf : pred4(a), Z.nh <= -1.0 ? -inf : pred4(-b)};
                U = imeet(U, R);
                break;
            }
            default:     // sin, cos: only the range check
                if (iempty(imeet(Z, unit))) return 1;
                break;
            }
            if (iempty(U) || (bin && iempty(V))) return 1;
            us = make_double2(U.lo, U.nh);
            if (bin) val[(int64_t)nd.b * stride] = make_double2(V.lo, V.nh);
        }
        // the box
        for (int i = 0; i < A.n_nodes; ++i) {
            const DagNode nd = A.nodes[i];
            if (!nd.live || nd.op != MVF_VAR) continue;
            const double2 v = val[(int64_t)i * stride];
            X[nd.a] = imeet(X[nd.a], Iv{v.x, v.y});
        }
        for (int j = 0; j < A.n; ++j)
            if (iempty(X[j])) return 1;
    }
    return 0;
}

}  // namespace dev

// One lane per box; LDS: the node values and marks of the workgroup's lanes
// (lane-interleaved) in LDS, else in the workspace (lane-interleaved over all
// boxes).  The propagation walks the DAG node by node, each step reading what
// the previous ones wrote, so the latency of those accesses is its time.
template <bool LDS>
__global__ __launch_bounds__(64) void fbbt_kernel(FbbtArgs A) {
    using namespace dev;
    extern __shared__ __align__(16) double2 sval[];
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= A.N) return;
    Iv X[MVF_MAX_VARS];
    for (int j = 0; j < A.n; ++j) X[j] = Iv{A.boxes[(b * A.n + j) * 2], -A.boxes[(b * A.n + j) * 2 + 1]};
    mode_round_down();
    const uint32_t bad = LDS ? fbbt_lane(A, sval + threadIdx.x, blockDim.x, X) : fbbt_lane(A, A.val + b, A.stride, X);
    mode_round_nearest();
    A.status[b] = (int32_t)bad;
    for (int j = 0; j < A.n; ++j) {
        A.out[(b * A.n + j) * 2] = bad ? 0.0 : X[j].lo;
        A.out[(b * A.n + j) * 2 + 1] = bad ? 0.0 : -X[j].nh;
    }
}

hipError_t launch_fbbt(const FbbtArgs &A, hipStream_t stream) {
    if (A.N == 0) return hipSuccess;
    // LDS when a lane's values and marks (2 x n_nodes x 16 bytes) fit: as many
    // lanes per workgroup as keep it within 64 KB (two or more workgroups per
    // CU), at least one
    const size_t lane_bytes = (size_t)2 * A.n_nodes * 16;
    if (lane_bytes <= LDS_BUDGET - 1024) {
        static std::once_flag once;
        static hipError_t ae = hipSuccess;
        std::call_once(once, [] { ae = allow_lds(fbbt_kernel<true>); });
        if (ae != hipSuccess) return ae;
        const int lanes = (int)std::max<size_t>(1, std::min<size_t>(64, (64 * 1024) / lane_bytes));
        hipLaunchKernelGGL(fbbt_kernel<true>, dim3((unsigned)((A.N + lanes - 1) / lanes)), dim3(lanes),
                           lane_bytes * lanes, stream, A);
    } else {
        hipLaunchKernelGGL(fbbt_kernel<false>, dim3((unsigned)((A.N + 63) / 64)), dim3(64), 0, stream, A);
    }
    return hipGetLastError();
}

#define MVF_DISPATCH(C_, REV_, CALL)                            \
    do {                                                        \
        if (REV_) {                                             \
            constexpr int Cx = 0; constexpr bool Rx = true;     \
            CALL;                                               \
        } else if ((C_) == 0) {                                 \
            constexpr int Cx = 0; constexpr bool Rx = false;    \
            CALL;                                               \
        } else if ((C_) == 1) {                                 \
            constexpr int Cx = 1; constexpr bool Rx = false;    \
            CALL;                                               \
        } else if ((C_) == 2) {                                 \
            constexpr int Cx = 2; constexpr bool Rx = false;    \
            CALL;                                               \
        } else if ((C_) == 3) {                                 \
            constexpr int Cx = 3; constexpr bool Rx = false;    \
            CALL;                                               \
        } else {                                                \
            constexpr int Cx = 4; constexpr bool Rx = false;    \
            CALL;                                               \
        }                                                       \
    } while (0)

hipError_t launch_bound(const TapeArgs &T, const BoxArgs &B, int chunk, bool rev, int grid, size_t lds,
                        hipStream_t stream, hipEvent_t after) {
    static_assert(MAX_CHUNK == 4, "one kernel instance per chunk size");
    hipError_t e = hipSuccess;
    MVF_DISPATCH(chunk, rev, {
        static std::once_flag once;
        static hipError_t ae = hipSuccess;
        std::call_once(once, [] { ae = allow_lds(bound_kernel<Cx, Rx>); });
        if (ae != hipSuccess) return ae;
        hipLaunchKernelGGL((bound_kernel<Cx, Rx>), dim3(grid), dim3(BLK), lds, stream, BoundKArgs{T, B});
    });
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (after && (e = hipEventRecord(after, stream)) != hipSuccess) return e;
    return launch_finish(B, grid, T.n_roots, stream);
}

hipError_t launch_finish(const BoxArgs &B, int grid, int m, hipStream_t stream) {
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(FIN_BLK), 0, stream, B.partial, B.partial_lo0, B.partial_k,
                       B.partial_ext, grid, m, B.reduced, B.argmin, B.extra);
    return hipGetLastError();
}

hipError_t launch_batch_plan(const BatchArgs &A, hipStream_t stream) {
    hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(256), 0, stream, A);
    return hipGetLastError();
}

hipError_t launch_batch_finish(const BatchArgs &A, int m, int max_nodes, hipStream_t stream) {
    hipLaunchKernelGGL(batch_finish_kernel, dim3(max_nodes), dim3(256), 0, stream, A, m);
    return hipGetLastError();
}

hipError_t launch_batch(const TapeArgs &T, const BatchArgs &A, int chunk, bool rev, int grid, size_t lds,
                        int max_nodes, hipStream_t stream) {
    hipError_t e = launch_batch_plan(A, stream);
    if (e != hipSuccess) return e;
    MVF_DISPATCH(chunk, rev, {
        static std::once_flag once;
        static hipError_t ae = hipSuccess;
        std::call_once(once, [] { ae = allow_lds(batch_kernel<Cx, Rx>); });
        if (ae != hipSuccess) return ae;
        hipLaunchKernelGGL((batch_kernel<Cx, Rx>), dim3(grid), dim3(BLK), lds, stream, BatchKArgs{T, A});
    });
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_batch_finish(A, T.n_roots, max_nodes, stream);
}

hipError_t launch_points(const PointsArgs &A, int op, int chunk, int grid, size_t lds, hipStream_t stream) {
    static_assert(MAX_CHUNK == 4, "one kernel instance per chunk size");
    auto go = [&](auto kernel) -> hipError_t {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)(LDS_BUDGET - 1024));
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(kernel, dim3(grid), dim3(BLK), lds, stream, PointsKArgs{A});
        return hipGetLastError();
    };
    switch (op) {
    case PT_EVAL: return go(points_kernel<PT_EVAL, 0>);
    case PT_VJP: return go(points_kernel<PT_VJP, 0>);
    case PT_GRAD_REV: return go(points_kernel<PT_GRAD_REV, 0>);
    default:
        switch (chunk) {
        case 1: return go(points_kernel<PT_GRAD_FWD, 1>);
        case 2: return go(points_kernel<PT_GRAD_FWD, 2>);
        case 3: return go(points_kernel<PT_GRAD_FWD, 3>);
        default: return go(points_kernel<PT_GRAD_FWD, 4>);
        }
    }
}

// ---------------------------------------------------------------------------
// the no-allocation entry point's scratch: one file-scope device array per
// device (each GPU the library runs on holds its own copy until the process
// ends), shared by every call on that device
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[MVF_NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch(int device, void **ptr) {
    constexpr int MAX_DEVICES = 64;
    static std::mutex mu;
    static void *addr[MAX_DEVICES] = {};
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        // the host-side name of the array is not a device address: look up this
        // device's copy once, with the device current
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (cur != device) hipSetDevice(cur);
        if (e != hipSuccess) return e;
        addr[device] = a;
    }
    *ptr = addr[device];
    return hipSuccess;
}

}  // namespace mvf
