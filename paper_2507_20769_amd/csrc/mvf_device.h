// mvf_device.h -- gfx950 device primitives: directed-rounding FP64 interval
// arithmetic and the GPR-indexed register slot file.
//
// Rounding.  Interval endpoints must be rounded outward (Sec. 2.2 "Interval
// Arithmetic"; Sec. 3.2: + - * / sqrt directly rounded, other intrinsics
// widened on both sides).  gfx950 has no per-instruction rounding mode, so the
// kernels set the wave's FP64 rounding mode to "toward -inf" (MODE register,
// FP_ROUND bits [3:2] = 2) once, and store every interval as (lo, nh) with
// nh = -hi.  Then both stored endpoints are rounded down:
//     RD(x op y)  for lo,      -RU(x op y) = RD(-(x op y))  for nh,
// and negation is a free source modifier.  Every rounding-sensitive
// instruction is written as volatile inline asm, so the compiler neither
// folds it under round-to-nearest assumptions nor moves it across a mode
// change.  Division and square root start from the compiler's estimate and are
// corrected with exact-sign residual tests (fma rounded down keeps the sign of
// the exact residual), which yields the correctly rounded-down result.
//
// Slot file.  VGPRs [SLOT_BASE, 256) hold the interpreter's register slots;
// the compiler is restricted to VGPRs below SLOT_BASE (the kernels declare a
// VGPR limit and a 5-waves-per-SIMD target, which also keeps SGPR-spill lanes
// below the slot file; the build verifies the ISA).  A slot is read or written
// with s_set_gpr_idx_on (index in M0) and v_mov_b64.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mvf_internal.h"

namespace mvf {
namespace dev {

struct Iv {
    double lo, nh;   // the interval [lo, -nh]
};

#define MVF_STR2(x) #x
#define MVF_STR(x) MVF_STR2(x)

// ---- FP64 rounding mode -------------------------------------------------
__device__ __forceinline__ void mode_round_down() {
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2\n\ts_nop 1" ::: "memory");
}
__device__ __forceinline__ void mode_round_nearest() {
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0\n\ts_nop 1" ::: "memory");
}

// ---- single FP64 instructions under the current (round-down) mode ----------
__device__ __forceinline__ double fadd(double a, double b) {
    double r;
    asm volatile("v_add_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double fadd_nn(double a, double b) {       // RD(-a - b)
    double r;
    asm volatile("v_add_f64 %0, -%1, -%2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double fadd_s(double a, double s) {        // s in an SGPR pair
    double r;
    asm volatile("v_add_f64 %0, %1, %2" : "=v"(r) : "v"(a), "s"(s));
    return r;
}
__device__ __forceinline__ double fadd_ns(double a, double s) {       // RD(-a + s)
    double r;
    asm volatile("v_add_f64 %0, -%1, %2" : "=v"(r) : "v"(a), "s"(s));
    return r;
}
__device__ __forceinline__ double fmul(double a, double b) {
    double r;
    asm volatile("v_mul_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double fmul_n(double a, double b) {        // RD(a * -b)
    double r;
    asm volatile("v_mul_f64 %0, %1, -%2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double ffma_n(double a, double b, double c) {   // RD(-a*b + c)
    double r;
    asm volatile("v_fma_f64 %0, -%1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ double ffma_nn(double a, double b, double c) {  // RD(a*b - c)
    double r;
    asm volatile("v_fma_f64 %0, %1, %2, -%3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ double fmin_(double a, double b) {
    double r;
    asm volatile("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double fmax_(double a, double b) {
    double r;
    asm volatile("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

constexpr double kTiny = 4.9406564584124654e-324;     // 2^-1074
constexpr double kMax = 1.7976931348623157e308;

// next double below x (x != NaN); +inf steps to the largest finite double
__device__ __forceinline__ double pred(double x) {
    double r = fadd_s(x, -kTiny);
    return x == __builtin_inf() ? kMax : r;
}
// next double above x; -inf steps to the most negative finite double
__device__ __forceinline__ double succ(double x) {
    double r = -fadd_ns(x, -kTiny);       // -RD(-x - tiny)
    return x == -__builtin_inf() ? -kMax : r;
}

// Correctly rounded-down quotient x / y.
__device__ __forceinline__ double div_rd(double x, double y) {
    double q = x / y;                     // estimate (a few ulps at most in any mode)
    const bool neg = y < 0.0;
    const double xs = neg ? -x : x, ys = neg ? -y : y;   // now ys > 0
    if (q == __builtin_inf() && __builtin_isfinite(x) && __builtin_isfinite(y)) q = kMax;
#pragma unroll
    for (int it = 0; it < 2; ++it) {      // step down while q * ys > xs
        double r = ffma_n(q, ys, xs);     // RD(xs - q*ys): negative iff the exact residual is
        double qd = pred(q);
        q = r < 0.0 ? qd : q;
    }
#pragma unroll
    for (int it = 0; it < 2; ++it) {      // step up while succ(q) * ys <= xs
        double q1 = succ(q);
        double r1 = ffma_n(q1, ys, xs);
        q = r1 >= 0.0 ? q1 : q;
    }
    return q;
}

// Correctly rounded-down square root of a >= 0.
__device__ __forceinline__ double sqrt_rd(double a) {
    double s = __builtin_sqrt(a);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        double r = ffma_n(s, s, a);       // RD(a - s*s)
        double sd = pred(s);
        s = r < 0.0 ? sd : s;
    }
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        double s1 = succ(s);
        double r1 = ffma_n(s1, s1, a);
        s = r1 >= 0.0 ? s1 : s;
    }
    return s;
}
// -RU(sqrt(b)): the negated correctly rounded-up square root
__device__ __forceinline__ double sqrt_ru_neg(double b) {
    double s = sqrt_rd(b);
    double r = ffma_nn(s, s, b);          // RD(s*s - b) < 0 iff s*s < b
    double su = succ(s);
    return -(r < 0.0 ? su : s);
}

// ---- interval operations on (lo, nh) -------------------------------------
__device__ __forceinline__ Iv iadd(Iv u, Iv v) { return {fadd(u.lo, v.lo), fadd(u.nh, v.nh)}; }
__device__ __forceinline__ Iv isub(Iv u, Iv v) { return {fadd(u.lo, v.nh), fadd(u.nh, v.lo)}; }

// hull of the four endpoint products; hi = -nh, so lo*hi = RD(lo * -nh) etc.
__device__ __forceinline__ Iv imul(Iv u, Iv v) {
    double p0 = fmul(u.lo, v.lo), p1 = fmul_n(u.lo, v.nh), p2 = fmul_n(u.nh, v.lo), p3 = fmul(u.nh, v.nh);
    double q0 = fmul_n(u.lo, v.lo), q1 = fmul(u.lo, v.nh), q2 = fmul(u.nh, v.lo), q3 = fmul_n(u.nh, v.nh);
    return {fmin_(fmin_(p0, p1), fmin_(p2, p3)), fmin_(fmin_(q0, q1), fmin_(q2, q3))};
}

__device__ __forceinline__ Iv isqr(Iv u) {
    double plo = fmul(u.lo, u.lo), pnh = fmul(u.nh, u.nh);
    double qlo = fmul_n(u.lo, u.lo), qnh = fmul_n(u.nh, u.nh);
    const bool pos = u.lo >= 0.0, negv = u.nh >= 0.0;      // lo >= 0, or hi <= 0
    double mn = fmin_(qlo, qnh);
    Iv z;
    z.lo = pos ? plo : (negv ? pnh : 0.0);
    z.nh = pos ? qnh : (negv ? qlo : mn);
    return z;
}

// U / V with 0 not in V: the extreme quotients are picked by the signs
// (branch-free, lanes disagree on the signs).
__device__ __forceinline__ Iv idiv(Iv u, Iv v) {
    const double a = u.lo, b = -u.nh, c = v.lo, d = -v.nh;
    const bool vpos = c > 0.0;
    const double nl = vpos ? a : b;
    const double dl = vpos ? (a >= 0.0 ? d : c) : (b >= 0.0 ? d : c);
    const double nn = vpos ? -b : -a;
    const double dn = vpos ? (b >= 0.0 ? c : d) : (a >= 0.0 ? c : d);
    return {div_rd(nl, dl), div_rd(nn, dn)};
}

// 1 / V with 0 not in V: [RD(1/d), RU(1/c)]
__device__ __forceinline__ Iv irecip(Iv v) { return {div_rd(1.0, -v.nh), div_rd(-1.0, v.lo)}; }

__device__ __forceinline__ Iv isqrt(Iv u) { return {sqrt_rd(u.lo), sqrt_ru_neg(-u.nh)}; }

// 2U (exact up to overflow)
__device__ __forceinline__ Iv itwice(Iv u) { return {fadd(u.lo, u.lo), fadd(u.nh, u.nh)}; }

// enclosure of 1/(2 sqrt(u)) from Z = sqrt(U); unbounded above when z_lo is 0
__device__ __forceinline__ Iv isqrt_deriv(Iv z) {
    Iv t = itwice(z);
    if (t.lo <= 0.0) return {div_rd(1.0, -t.nh), -__builtin_inf()};
    return irecip(t);
}

// exp and log: library value in round-to-nearest, widened by two ulps per side
__device__ __forceinline__ Iv iexp(Iv u) {
    double xl = u.lo, xh = -u.nh;
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0\n\ts_nop 1" : "+v"(xl), "+v"(xh));
    double el = exp(xl), eh = exp(xh);
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2\n\ts_nop 1" : "+v"(el), "+v"(eh));
    double lo = pred(pred(el));
    return {lo > 0.0 ? lo : 0.0, pred(pred(-eh))};
}
__device__ __forceinline__ Iv ilog(Iv u) {
    double xl = u.lo, xh = -u.nh;
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0\n\ts_nop 1" : "+v"(xl), "+v"(xh));
    double ll = log(xl), lh = log(xh);
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2\n\ts_nop 1" : "+v"(ll), "+v"(lh));
    return {pred(pred(ll)), pred(pred(-lh))};
}

// ---- slot file (GPR index mode) -------------------------------------------
#define MVF_SB 96
static_assert(MVF_SB == mvf::SLOT_BASE, "slot base");

// Slot indices are wave-uniform; readfirstlane pins them to an SGPR as the
// index operand of s_set_gpr_idx_on requires.
__device__ __forceinline__ uint32_t sidx(uint32_t idx) { return __builtin_amdgcn_readfirstlane(idx); }

// read one interval at dword offset idx of the slot file
__device__ __forceinline__ Iv slot_rd(uint32_t idx) {
    idx = sidx(idx);
    Iv x;
    asm volatile("s_set_gpr_idx_on %2, gpr_idx(SRC0)\n\t"
                 "v_mov_b64 %0, v[96:97]\n\t"
                 "v_mov_b64 %1, v[98:99]\n\t"
                 "s_set_gpr_idx_off"
                 : "=v"(x.lo), "=v"(x.nh) : "s"(idx) : "m0");
    return x;
}
// read two consecutive intervals
__device__ __forceinline__ void slot_rd2(uint32_t idx, Iv &x, Iv &y) {
    idx = sidx(idx);
    asm volatile("s_set_gpr_idx_on %4, gpr_idx(SRC0)\n\t"
                 "v_mov_b64 %0, v[96:97]\n\t"
                 "v_mov_b64 %1, v[98:99]\n\t"
                 "v_mov_b64 %2, v[100:101]\n\t"
                 "v_mov_b64 %3, v[102:103]\n\t"
                 "s_set_gpr_idx_off"
                 : "=v"(x.lo), "=v"(x.nh), "=v"(y.lo), "=v"(y.nh) : "s"(idx) : "m0");
}
__device__ __forceinline__ void slot_wr(uint32_t idx, Iv x) {
    idx = sidx(idx);
    asm volatile("s_set_gpr_idx_on %0, gpr_idx(DST)\n\t"
                 "v_mov_b64 v[96:97], %1\n\t"
                 "v_mov_b64 v[98:99], %2\n\t"
                 "s_set_gpr_idx_off"
                 :: "s"(idx), "v"(x.lo), "v"(x.nh) : "m0");
}
__device__ __forceinline__ void slot_wr2(uint32_t idx, Iv x, Iv y) {
    idx = sidx(idx);
    asm volatile("s_set_gpr_idx_on %0, gpr_idx(DST)\n\t"
                 "v_mov_b64 v[96:97], %1\n\t"
                 "v_mov_b64 v[98:99], %2\n\t"
                 "v_mov_b64 v[100:101], %3\n\t"
                 "v_mov_b64 v[102:103], %4\n\t"
                 "s_set_gpr_idx_off"
                 :: "s"(idx), "v"(x.lo), "v"(x.nh), "v"(y.lo), "v"(y.nh) : "m0");
}
// make the slot file part of the kernel's register allocation
__device__ __forceinline__ void claim_slot_file() { asm volatile("" ::: "v255"); }

// read a slot of 1 + C intervals (value then C tangent components)
template <int C>
__device__ __forceinline__ void slot_read(uint32_t idx, Iv &val, Iv (&tan)[C > 0 ? C : 1]) {
    if constexpr (C == 0) {
        val = slot_rd(idx);
    } else if constexpr (C == 1) {
        slot_rd2(idx, val, tan[0]);
    } else {
        slot_rd2(idx, val, tan[0]);
#pragma unroll
        for (int t = 1; t < C; t += 2) {
            if (t + 1 < C) slot_rd2(idx + 4 * (t + 1), tan[t], tan[t + 1]);
            else tan[t] = slot_rd(idx + 4 * (t + 1));
        }
    }
}
template <int C>
__device__ __forceinline__ void slot_write(uint32_t idx, const Iv &val, const Iv (&tan)[C > 0 ? C : 1]) {
    if constexpr (C == 0) {
        slot_wr(idx, val);
    } else if constexpr (C == 1) {
        slot_wr2(idx, val, tan[0]);
    } else {
        slot_wr2(idx, val, tan[0]);
#pragma unroll
        for (int t = 1; t < C; t += 2) {
            if (t + 1 < C) slot_wr2(idx + 4 * (t + 1), tan[t], tan[t + 1]);
            else slot_wr(idx + 4 * (t + 1), tan[t]);
        }
    }
}

}  // namespace dev
}  // namespace mvf
