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
// change.  Minimum and maximum are exact in every mode: their asm is plain,
// so the compiler may schedule them freely.  Division and square root start from the compiler's correctly
// rounded estimate, computed in a short round-to-nearest window, and are
// corrected with exact-sign residual tests (fma rounded down keeps the sign of
// the exact residual), which yields the correctly rounded-down result.
//
// Slot file.  VGPRs [SLOT_BASE, 256) hold the interpreter's register slots;
// the compiler is restricted to VGPRs below SLOT_BASE (the kernels declare a
// VGPR limit and a 5-waves-per-SIMD target, which also keeps SGPR-spill lanes
// below the slot file; the build verifies the ISA).  A slot is read or written
// with s_set_gpr_idx_on (index in M0) and v_mov_b64.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

#include "mvf_isa.h"

namespace mvf {
namespace dev {

struct Iv {
    double lo, nh;   // the interval [lo, -nh]
};

#define MVF_STR2(x) #x
#define MVF_STR(x) MVF_STR2(x)

// ---- FP64 rounding mode -------------------------------------------------
// A MODE write takes effect for the next VALU instruction of the wave, and an
// instruction issued before it keeps the mode it was issued under (the
// compiler's own single-precision division relies on both when it toggles the
// denormal bits of the same register), so a switch needs no wait states
// around it.  Two MODE writes need two wait states between them; every switch
// pair here encloses or is followed by at least two VALU instructions (the
// build checks the compiled interpreter kernels for this on every path, a
// test the compiled code of generated specialised kernels).
__device__ __forceinline__ void mode_round_down() {
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2" ::: "memory");
}
__device__ __forceinline__ void mode_round_nearest() {
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0" ::: "memory");
}

// ---- single FP64 instructions under the current (round-down) mode ----------
__device__ __forceinline__ double fadd(double a, double b) {
    double r;
    asm volatile("v_add_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double fadd_s(double a, double s) {        // s in an SGPR pair
    double r;
    asm volatile("v_add_f64 %0, %1, %2" : "=v"(r) : "v"(a), "s"(s));
    return r;
}
__device__ __forceinline__ double fsub(double a, double b) {          // RD(a - b)
    double r;
    asm volatile("v_add_f64 %0, %1, -%2" : "=v"(r) : "v"(a), "v"(b));
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
__device__ __forceinline__ double fmin_(double a, double b) {
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}
__device__ __forceinline__ double fmax_(double a, double b) {
    double r;
    asm("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

constexpr double kTiny = 4.9406564584124654e-324;     // 2^-1074
constexpr double kMax = 1.7976931348623157e308;

// next double below x (x != NaN); +inf steps to the largest finite double
__device__ __forceinline__ double pred(double x) {
    double r = fadd_s(x, -kTiny);
    return x == __builtin_inf() ? kMax : r;
}

// x with its sign flipped where y is negative (x * sign(y), exact): two
// 32-bit logic operations on the high words instead of two selects
__device__ __forceinline__ double flip_by(double x, double y) {
    const uint64_t xb = __builtin_bit_cast(uint64_t, x), yb = __builtin_bit_cast(uint64_t, y);
    return __builtin_bit_cast(double, xb ^ (yb & 0x8000000000000000ull));
}
// next double below a finite x (fadd_s rounds down; +inf stays +inf)
__device__ __forceinline__ double pred_finite(double x) { return fadd_s(x, -kTiny); }

// Correctly rounded-down quotients x0 / y0 and x1 / y1 (y != 0).  The
// estimate q is the correctly rounded-to-nearest quotient, so no double lies
// strictly between q and the exact quotient t: RD(t) is q when q <= t and the
// predecessor of q otherwise.  q > t exactly when the residual x*sign(y) -
// q*|y| is negative, and an fma rounded down keeps the sign of the exact
// residual.  A finite quotient that overflows to +inf in round-to-nearest
// has a residual of -inf and steps down to the largest finite double (the
// predecessor is capped there); an infinite dividend gives a NaN residual and
// keeps its infinite quotient.  POS: the divisors are known positive (no sign
// fold).
//
// The estimates come from the compiler's IEEE division sequence, correctly
// rounded in round-to-nearest, run between two mode switches.  The switch to
// nearest takes the operands as asm operands and the switch back takes the
// estimates, so the estimates are computed inside the window and nothing else
// is.  The switch back, the two residuals and the two capped predecessors are
// one asm statement: the compiler pads an instruction that reads a result of
// the inline asm just before it, and here the first instructions after the
// switch read its operands.
#define MVF_CLOSE_AND_TEST2(N0, N1)                                                    \
    "s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2\n\t"                               \
    "v_fma_f64 %0, -%4, |%6|, " N0 "\n\t"        /* e0 = RD(n0 - q0 |y0|) */        \
    "v_fma_f64 %1, -%5, |%7|, " N1 "\n\t"        /* e1 = RD(n1 - q1 |y1|) */        \
    "v_add_f64 %2, %4, %8\n\t"                   /* d0 = RD(q0 - 2^-1074) */        \
    "v_add_f64 %3, %5, %8\n\t"                                                       \
    "v_min_f64 %2, %2, %9\n\t"                   /* capped at the largest double */ \
    "v_min_f64 %3, %3, %9"
__device__ __forceinline__ void close_and_test2(double q0, double q1, double y0, double y1, double n0, double n1,
                                                double &e0, double &e1, double &d0, double &d1) {
    asm volatile(MVF_CLOSE_AND_TEST2("%10", "%11")
                 : "=&v"(e0), "=&v"(e1), "=&v"(d0), "=v"(d1)
                 : "v"(q0), "v"(q1), "v"(y0), "v"(y1), "s"(-kTiny), "s"(kMax), "v"(n0), "v"(n1));
}
// the same with the numerators 1 and -1 (inline constants)
__device__ __forceinline__ void close_and_test2_pm1(double q0, double q1, double y0, double y1,
                                                    double &e0, double &e1, double &d0, double &d1) {
    asm volatile(MVF_CLOSE_AND_TEST2("1.0", "-1.0")
                 : "=&v"(e0), "=&v"(e1), "=&v"(d0), "=v"(d1)
                 : "v"(q0), "v"(q1), "v"(y0), "v"(y1), "s"(-kTiny), "s"(kMax));
}
template <bool POS = false>
__device__ __forceinline__ void div_rd2(double x0, double y0, double x1, double y1, double &r0, double &r1) {
    double q0, q1;
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0" : "+v"(x0), "+v"(y0), "+v"(x1), "+v"(y1));
    q0 = x0 / y0;
    q1 = x1 / y1;
    const double xs0 = POS ? x0 : flip_by(x0, y0), xs1 = POS ? x1 : flip_by(x1, y1);
    double e0, e1, d0, d1;
    close_and_test2(q0, q1, y0, y1, xs0, xs1, e0, e1, d0, d1);
    r0 = e0 < 0.0 ? d0 : q0;
    r1 = e1 < 0.0 ? d1 : q1;
}
// RD(1/y0) and RD(-1/y1): div_rd2 with the constant numerators
template <bool POS = false>
__device__ __forceinline__ void rcp_rd2(double y0, double y1, double &r0, double &r1) {
    double q0, q1;
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0" : "+v"(y0), "+v"(y1));
    q0 = 1.0 / y0;
    q1 = -1.0 / y1;
    double e0, e1, d0, d1;
    if constexpr (POS)
        close_and_test2_pm1(q0, q1, y0, y1, e0, e1, d0, d1);
    else
        close_and_test2(q0, q1, y0, y1, flip_by(1.0, y0), flip_by(-1.0, y1), e0, e1, d0, d1);
    r0 = e0 < 0.0 ? d0 : q0;
    r1 = e1 < 0.0 ? d1 : q1;
}

// [RD(sqrt(a)), -RU(sqrt(b))] for a, b >= 0 from the correctly rounded-to-
// nearest roots s: the lower end is s, or its predecessor when s*s > a; the
// upper end s, or its successor when s*s < b (residual signs as in div_rd2;
// the switch back and the tests again one asm statement).
__device__ __forceinline__ void sqrt_rd_ru2(double a, double b, double &lo, double &nh) {
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0" : "+v"(a), "+v"(b));
    const double s0 = __builtin_sqrt(a), s1 = __builtin_sqrt(b);
    double e0, g, d0, m1;
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2\n\t"
                 "v_fma_f64 %0, -%4, %4, %6\n\t"        // e0 = RD(a - s0*s0)
                 "v_fma_f64 %1, %5, %5, -%7\n\t"        // g = RD(s1*s1 - b)
                 "v_add_f64 %2, %4, %8\n\t"             // d0 = pred(s0)
                 "v_add_f64 %3, -%5, %8"                // m1 = pred(-s1)
                 : "=&v"(e0), "=&v"(g), "=&v"(d0), "=v"(m1)
                 : "v"(s0), "v"(s1), "v"(a), "v"(b), "s"(-kTiny));
    lo = e0 < 0.0 ? d0 : s0;
    nh = g < 0.0 ? m1 : -s1;
}

// ---- interval operations on (lo, nh) -------------------------------------
__device__ __forceinline__ Iv iadd(Iv u, Iv v) { return {fadd(u.lo, v.lo), fadd(u.nh, v.nh)}; }
__device__ __forceinline__ Iv isub(Iv u, Iv v) { return {fadd(u.lo, v.nh), fadd(u.nh, v.lo)}; }

// hull of the four endpoint products; hi = -nh, so lo*hi = RD(lo * -nh) etc.
// One asm statement for the whole hull: the compiler pads an instruction that
// reads a result of the inline asm just before it (it cannot see what the asm
// does), so the minima sit inside the statement with their products.  Each
// minimum follows its two products, so two temporaries suffice.
__device__ __forceinline__ Iv imul(Iv u, Iv v) {
    double lo, nh, t, w;
    asm volatile("v_mul_f64 %0, %4, %6\n\t"          // lo = a c
                 "v_mul_f64 %1, %4, -%6\n\t"         // nh = -(a c)
                 "v_mul_f64 %2, %4, -%7\n\t"         // a d
                 "v_mul_f64 %3, %4, %7\n\t"          // -(a d)
                 "v_min_f64 %0, %0, %2\n\t"
                 "v_min_f64 %1, %1, %3\n\t"
                 "v_mul_f64 %2, %5, -%6\n\t"         // b c
                 "v_mul_f64 %3, %5, %6\n\t"          // -(b c)
                 "v_min_f64 %0, %0, %2\n\t"
                 "v_min_f64 %1, %1, %3\n\t"
                 "v_mul_f64 %2, %5, %7\n\t"          // b d
                 "v_mul_f64 %3, %5, -%7\n\t"         // -(b d)
                 "v_min_f64 %0, %0, %2\n\t"
                 "v_min_f64 %1, %1, %3"
                 : "=&v"(lo), "=&v"(nh), "=&v"(t), "=&v"(w)
                 : "v"(u.lo), "v"(u.nh), "v"(v.lo), "v"(v.nh));
    return {lo, nh};
}

// [a, b]^2: the upper end is the square of max(|a|, |b|); the lower end the
// square of max(a, -b, 0), which is min(|a|, |b|) when 0 is not in [a, b]
// and 0 when it is (a square of a zero is +0 in every rounding mode).  One
// asm statement; nh = -b, so max(a, -b) is max(lo, nh).
__device__ __forceinline__ Iv isqr(Iv u) {
    double lo, nh;
    asm volatile("v_max_f64 %1, |%2|, |%3|\n\t"
                 "v_max_f64 %0, %2, %3\n\t"
                 "v_mul_f64 %1, %1, -%1\n\t"
                 "v_max_f64 %0, %0, 0\n\t"
                 "v_mul_f64 %0, %0, %0"
                 : "=v"(lo), "=&v"(nh)
                 : "v"(u.lo), "v"(u.nh));
    return {lo, nh};
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
    Iv z;
    div_rd2(nl, dl, nn, dn, z.lo, z.nh);
    return z;
}

// U / V for V > 0: the selection idiv makes for a positive denominator
__device__ __forceinline__ Iv idiv_pos(Iv u, Iv v) {
    const double a = u.lo, b = -u.nh, c = v.lo, d = -v.nh;
    Iv z;
    div_rd2<true>(a, a >= 0.0 ? d : c, -b, b >= 0.0 ? c : d, z.lo, z.nh);
    return z;
}

// 1 / V with 0 not in V: [RD(1/d), RU(1/c)]
__device__ __forceinline__ Iv irecip(Iv v) {
    Iv z;
    rcp_rd2(-v.nh, v.lo, z.lo, z.nh);
    return z;
}
// the same for V > 0
__device__ __forceinline__ Iv irecip_pos(Iv v) {
    Iv z;
    rcp_rd2<true>(-v.nh, v.lo, z.lo, z.nh);
    return z;
}

__device__ __forceinline__ Iv isqrt(Iv u) {
    Iv z;
    sqrt_rd_ru2(u.lo, -u.nh, z.lo, z.nh);
    return z;
}

// 2U (exact up to overflow)
// U + k and k - U for a constant k, each one asm statement with k read from
// scalar registers (the same two sums as iadd and isub with [k, k])
__device__ __forceinline__ Iv iaddk(Iv u, double k) {
    double lo, nh;
    asm volatile("v_add_f64 %0, %2, %4\n\tv_add_f64 %1, %3, -%4" : "=&v"(lo), "=v"(nh) : "v"(u.lo), "v"(u.nh), "s"(k));
    return {lo, nh};
}
__device__ __forceinline__ Iv iksub(double k, Iv u) {
    double lo, nh;
    asm volatile("v_add_f64 %0, %4, %3\n\tv_add_f64 %1, %2, -%4" : "=&v"(lo), "=v"(nh) : "v"(u.lo), "v"(u.nh), "s"(k));
    return {lo, nh};
}
__device__ __forceinline__ Iv itwice(Iv u) { return {fadd(u.lo, u.lo), fadd(u.nh, u.nh)}; }

// enclosure of 1/(2 sqrt(u)) from Z = sqrt(U); unbounded above when z_lo is 0
__device__ __forceinline__ Iv isqrt_deriv(Iv z) {
    const Iv t = itwice(z);
    double lo, nh;
    rcp_rd2<true>(-t.nh, t.lo, lo, nh);               // branch-free: lanes differ in the sign test
    return {lo, t.lo <= 0.0 ? -__builtin_inf() : nh};
}

// exp: library value in round-to-nearest, widened by two ulps per side
__device__ __forceinline__ Iv iexp(Iv u) {
    double xl = u.lo, xh = -u.nh;
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0" : "+v"(xl), "+v"(xh));
    double el = exp(xl), eh = exp(xh);
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2" : "+v"(el), "+v"(eh));
    // two predecessor steps (-eh is never +inf, so its steps need no stand-in)
    const double lo = pred(pred(el));
    return {lo > 0.0 ? lo : 0.0, pred_finite(pred_finite(-eh))};
}

// Natural logarithm in round-to-nearest arithmetic (inside a round-to-nearest
// window), written out from the series of atanh:
//   x = m 2^e with m in [sqrt(1/2), sqrt(2)), f = m - 1 (exact), s = f/(1+m),
//   |s| <= 0.1716, w = s^2, log m = 2 atanh s = 2s + 2s w Q(w) with
//   Q(w) = sum_{k=1..10} w^(k-1)/(2k+1) (the omitted tail is below 2^-60 of
//   log m), and log x = (e ln2_hi + 2s) + (2s w Q(w) + e ln2_lo), where
//   ln2_hi has 42 significant bits so that e ln2_hi is exact for every
//   exponent.
// Error (u = 2^-53): s carries at most 2u relative error (1 + m and the
// quotient are rounded), 2s is exact, 2s w Q(w) is at most 0.01 |2s| with
// about 12u relative error, and each of the three sums rounds once.  Since
// |2s| <= |log m| <= 0.347 and |log x| >= 0.346 whenever e != 0, the result is
// within 7u |log x| of log x (log 1 = 0 exactly).  0 gives -inf, +inf gives
// +inf, negative or NaN arguments NaN.
__device__ __forceinline__ double log_rn(double x) {
    constexpr double kLn2Hi = 0x1.62e42fefa3800p-1, kLn2Lo = 0x1.ef35793c76730p-45;
    constexpr double kSqrtHalf = 0x1.6a09e667f3bcdp-1;
    int e;
    double m = __builtin_frexp(x, &e);
    if (m < kSqrtHalf) {
        m += m;
        --e;
    }
    const double f = m - 1.0;
    const double s = f / (1.0 + m);
    const double s2 = s + s;
    const double w = s * s;
    // Q(w) by Horner's rule in one asm statement (the compiler pads each
    // instruction that reads the result of the inline asm just before it)
    double q;
    asm("v_fma_f64 %0, %1, %2, %3\n\t"
        "v_fma_f64 %0, %0, %1, %4\n\t"
        "v_fma_f64 %0, %0, %1, %5\n\t"
        "v_fma_f64 %0, %0, %1, %6\n\t"
        "v_fma_f64 %0, %0, %1, %7\n\t"
        "v_fma_f64 %0, %0, %1, %8\n\t"
        "v_fma_f64 %0, %0, %1, %9\n\t"
        "v_fma_f64 %0, %0, %1, %10\n\t"
        "v_fma_f64 %0, %0, %1, %11"
        : "=&v"(q)
        : "v"(w), "v"(1.0 / 21), "s"(1.0 / 19), "s"(1.0 / 17), "s"(1.0 / 15), "s"(1.0 / 13), "s"(1.0 / 11),
          "s"(1.0 / 9), "s"(1.0 / 7), "s"(1.0 / 5), "s"(1.0 / 3));
    const double de = (double)e;
    const double t = __builtin_fma(s2 * w, q, de * kLn2Lo);
    const double r = __builtin_fma(de, kLn2Hi, s2) + t;
    const double special = x == 0.0 ? -__builtin_inf() : x == __builtin_inf() ? x : __builtin_nan("");
    return x > 0.0 && x < __builtin_inf() ? r : special;     // selects, no branch
}

// log: log_rn of both ends, each widened outward by 2^-48 of its magnitude
// (32u, more than the 7u error bound) with the widening rounded outward too
__device__ __forceinline__ Iv ilog(Iv u) {
    double xl = u.lo, xh = -u.nh;
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0" : "+v"(xl), "+v"(xh));
    double ll = log_rn(xl), lh = log_rn(xh);
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2" : "+v"(ll), "+v"(lh));
    double lo, nh;
    asm volatile("v_fma_f64 %0, -|%1|, %2, %1" : "=v"(lo) : "v"(ll), "s"(0x1p-48));          // RD(l - |l| 2^-48)
    asm volatile("v_fma_f64 %0, -|%1|, %2, -%1" : "=v"(nh) : "v"(lh), "s"(0x1p-48));         // RD(-h - |h| 2^-48)
    return {ll == __builtin_inf() ? kMax : lo, nh};
}

// tanh, sin, cos (and atanh, for bound tightening): the library value of both
// endpoints in round-to-nearest (mode switches tied to the operands and
// results), widened by four ulps by the callers
enum : int { LIB_TANH = 0, LIB_SIN = 1, LIB_COS = 2, LIB_ATANH = 3 };
template <int F>
__device__ __forceinline__ void lib2(double &x0, double &x1) {
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 0" : "+v"(x0), "+v"(x1));
    if constexpr (F == LIB_TANH) {
        x0 = tanh(x0);
        x1 = tanh(x1);
    } else if constexpr (F == LIB_SIN) {
        x0 = sin(x0);
        x1 = sin(x1);
    } else if constexpr (F == LIB_ATANH) {
        x0 = atanh(x0);
        x1 = atanh(x1);
    } else {
        x0 = cos(x0);
        x1 = cos(x1);
    }
    asm volatile("s_setreg_imm32_b32 hwreg(HW_REG_MODE, 2, 2), 2" : "+v"(x0), "+v"(x1));
}
__device__ __forceinline__ double pred4(double x) { return pred(pred(pred(pred(x)))); }
// four predecessor steps of a value that is finite or NaN (library values of tanh, sin, cos)
__device__ __forceinline__ double pred4_finite(double x) {
    return pred_finite(pred_finite(pred_finite(pred_finite(x))));
}

// tanh is increasing with values in (-1, 1)
__device__ __forceinline__ Iv itanh(Iv u) {
    double a = u.lo, b = -u.nh;
    lib2<LIB_TANH>(a, b);
    return {fmax_(pred4_finite(a), -1.0), fmax_(pred4_finite(-b), -1.0)};
}
// pi lies between these neighbouring doubles
constexpr double kPiLo = 3.141592653589793, kPiHi = 3.1415926535897936;

// Can U contain c + 2 k pi for an integer k?  T = (U - C) / [2 pi] in outward
// rounding; true when T contains an integer or is not finite (so a "no" is
// rigorous and a "yes" at worst loosens the bound).
__device__ __forceinline__ bool may_contain(Iv u, Iv c) {
    const Iv t = idiv(isub(u, c), Iv{2.0 * kPiLo, -2.0 * kPiHi});
    const double lo = t.lo, hi = -t.nh;
    return !(__builtin_isfinite(lo) && __builtin_isfinite(hi)) || __builtin_ceil(lo) <= hi;
}

// sin or cos over U: the endpoint values widened by four ulps, +-1 where an
// extremum may lie inside (sin: maxima at pi/2 + 2 k pi, minima at
// -pi/2 + 2 k pi; cos: maxima at 2 k pi, minima at pi + 2 k pi), the whole
// [-1, 1] from a width of 6.28 on; branch-free (lanes differ)
template <int F>
__device__ __forceinline__ Iv itrig(Iv u) {
    double a = u.lo, b = -u.nh;
    lib2<F>(a, b);
    double lo = fmin_(pred4_finite(a), pred4_finite(b)), nh = fmin_(pred4_finite(-a), pred4_finite(-b));
    const Iv cmax = F == LIB_SIN ? Iv{kPiLo / 2, -kPiHi / 2} : Iv{0.0, -0.0};
    const Iv cmin = F == LIB_SIN ? Iv{-kPiHi / 2, kPiLo / 2} : Iv{kPiLo, -kPiHi};
    const bool hi1 = may_contain(u, cmax), lo1 = may_contain(u, cmin);
    const bool full = !(-fadd(u.lo, u.nh) < 6.28);             // RU(hi - lo) >= 6.28 (or NaN)
    nh = hi1 || full ? -1.0 : nh;
    lo = lo1 || full ? -1.0 : lo;
    return {fmax_(lo, -1.0), fmax_(nh, -1.0)};
}
__device__ __forceinline__ Iv isin(Iv u) { return itrig<LIB_SIN>(u); }
__device__ __forceinline__ Iv icos(Iv u) { return itrig<LIB_COS>(u); }

// -U = [-hi, -lo]: the two stored endpoints trade places (exact)
__device__ __forceinline__ Iv ineg(Iv u) { return {u.nh, u.lo}; }

// local derivative enclosures: 1 - Z^2 for Z = tanh(U); cos(U); -sin(U)
__device__ __forceinline__ Iv itanh_deriv(Iv z) { return isub(Iv{1.0, -1.0}, isqr(z)); }
__device__ __forceinline__ Iv isin_deriv(Iv u) { return icos(u); }
__device__ __forceinline__ Iv icos_deriv(Iv u) { return ineg(isin(u)); }

// ---- constant-operand forms ---------------------------------------------
// Each equals the general operation with a point interval [k, k] (k != 0)
// bit for bit, up to the sign of zero endpoints: the general hull's other
// candidates are never smaller, by monotonicity of rounding.



// U * k for k > 0
__device__ __forceinline__ Iv imulk(Iv u, double k) { return {fmul(u.lo, k), fmul(u.nh, k)}; }
// the same for a compile-time constant k: one asm statement, k from scalar registers
__device__ __forceinline__ Iv imulks(Iv u, double k) {
    double lo, nh;
    asm volatile("v_mul_f64 %0, %2, %4\n\tv_mul_f64 %1, %3, %4" : "=&v"(lo), "=v"(nh) : "v"(u.lo), "v"(u.nh), "s"(k));
    return {lo, nh};
}

// U * R for an interval R > 0 (stored (r_lo, -r_hi)): each endpoint of the
// result comes from one endpoint of U and either endpoint of R
__device__ __forceinline__ Iv imul_pos(Iv u, Iv r) {
    double lo, nh, t, w;
    asm volatile("v_mul_f64 %0, %4, %6\n\t"
                 "v_mul_f64 %2, %4, -%7\n\t"
                 "v_mul_f64 %1, %5, %6\n\t"
                 "v_mul_f64 %3, %5, -%7\n\t"
                 "v_min_f64 %0, %0, %2\n\t"
                 "v_min_f64 %1, %1, %3"
                 : "=&v"(lo), "=&v"(nh), "=&v"(t), "=v"(w)
                 : "v"(u.lo), "v"(u.nh), "v"(r.lo), "v"(r.nh));
    return {lo, nh};
}

// [c, c]^2: both ends are the one product c*c rounded each way (equals isqr)
__device__ __forceinline__ Iv isqr_deg(Iv u) { return {fmul(u.lo, u.lo), fmul_n(u.lo, u.lo)}; }
// U * [k, k] (a degenerate factor, c.lo = -c.nh = k): the four endpoint
// products of imul are two distinct ones, so this equals imul(u, c)
__device__ __forceinline__ Iv imul_deg(Iv u, Iv c) {
    double lo, nh, t, w;
    asm volatile("v_mul_f64 %0, %4, %6\n\t"
                 "v_mul_f64 %1, %4, -%6\n\t"
                 "v_mul_f64 %2, %5, -%6\n\t"
                 "v_mul_f64 %3, %5, %6\n\t"
                 "v_min_f64 %0, %0, %2\n\t"
                 "v_min_f64 %1, %1, %3"
                 : "=&v"(lo), "=&v"(nh), "=&v"(t), "=v"(w)
                 : "v"(u.lo), "v"(u.nh), "v"(c.lo));
    return {lo, nh};
}
// G * D for D = [dl, dh] with dl <= 0 <= dh (X - c with c in X): the lowest
// of the four endpoint products is gh dl or gl dh, the highest gl dl or gh dh,
// so this equals imul(g, d)
__device__ __forceinline__ Iv imul_dx(Iv g, Iv d) {
    double lo, nh, t, w;
    asm volatile("v_mul_f64 %0, %5, -%6\n\t"         // gh dl
                 "v_mul_f64 %2, %4, -%7\n\t"         // gl dh
                 "v_mul_f64 %1, %4, -%6\n\t"         // -(gl dl)
                 "v_mul_f64 %3, %5, -%7\n\t"         // -(gh dh)
                 "v_min_f64 %0, %0, %2\n\t"
                 "v_min_f64 %1, %1, %3"
                 : "=&v"(lo), "=&v"(nh), "=&v"(t), "=v"(w)
                 : "v"(g.lo), "v"(g.nh), "v"(d.lo), "v"(d.nh));
    return {lo, nh};
}

// Two independent products (the code generator pairs them; each is one asm
// statement, so the pair is two in a row)
__device__ __forceinline__ void imul2(Iv u, Iv v, Iv w, Iv x, Iv &r, Iv &s) {
    r = imul(u, v);
    s = imul(w, x);
}
__device__ __forceinline__ void imul_pos2(Iv u, Iv r, Iv w, Iv q, Iv &a, Iv &b) {
    a = imul_pos(u, r);
    b = imul_pos(w, q);
}

// U / k for k > 0
__device__ __forceinline__ Iv idivk(Iv u, double k) {
    Iv z;
    div_rd2<true>(u.lo, k, u.nh, k, z.lo, z.nh);
    return z;
}

// ---- slot file (GPR index mode) -------------------------------------------
#define MVF_SB 128
// the first four register pairs of the slot file (GPR-index base operands)
#define MVF_P0 "v[128:129]"
#define MVF_P1 "v[130:131]"
#define MVF_P2 "v[132:133]"
#define MVF_P3 "v[134:135]"
static_assert(MVF_SB == mvf::SLOT_BASE, "slot base");

// Slot indices are wave-uniform; readfirstlane pins them to an SGPR as the
// index operand of s_set_gpr_idx_on requires.
__device__ __forceinline__ uint32_t sidx(uint32_t idx) { return __builtin_amdgcn_readfirstlane(idx); }

// read one interval at dword offset idx of the slot file
__device__ __forceinline__ Iv slot_rd(uint32_t idx) {
    idx = sidx(idx);
    Iv x;
    asm volatile("s_set_gpr_idx_on %2, gpr_idx(SRC0)\n\t"
                 "v_mov_b64 %0, " MVF_P0 "\n\t"
                 "v_mov_b64 %1, " MVF_P1 "\n\t"
                 "s_set_gpr_idx_off"
                 : "=v"(x.lo), "=v"(x.nh) : "s"(idx) : "m0");
    return x;
}
// read two consecutive intervals
__device__ __forceinline__ void slot_rd2(uint32_t idx, Iv &x, Iv &y) {
    idx = sidx(idx);
    asm volatile("s_set_gpr_idx_on %4, gpr_idx(SRC0)\n\t"
                 "v_mov_b64 %0, " MVF_P0 "\n\t"
                 "v_mov_b64 %1, " MVF_P1 "\n\t"
                 "v_mov_b64 %2, " MVF_P2 "\n\t"
                 "v_mov_b64 %3, " MVF_P3 "\n\t"
                 "s_set_gpr_idx_off"
                 : "=v"(x.lo), "=v"(x.nh), "=v"(y.lo), "=v"(y.nh) : "s"(idx) : "m0");
}
__device__ __forceinline__ void slot_wr(uint32_t idx, Iv x) {
    idx = sidx(idx);
    asm volatile("s_set_gpr_idx_on %0, gpr_idx(DST)\n\t"
                 "v_mov_b64 " MVF_P0 ", %1\n\t"
                 "v_mov_b64 " MVF_P1 ", %2\n\t"
                 "s_set_gpr_idx_off"
                 :: "s"(idx), "v"(x.lo), "v"(x.nh) : "m0");
}
__device__ __forceinline__ void slot_wr2(uint32_t idx, Iv x, Iv y) {
    idx = sidx(idx);
    asm volatile("s_set_gpr_idx_on %0, gpr_idx(DST)\n\t"
                 "v_mov_b64 " MVF_P0 ", %1\n\t"
                 "v_mov_b64 " MVF_P1 ", %2\n\t"
                 "v_mov_b64 " MVF_P2 ", %3\n\t"
                 "v_mov_b64 " MVF_P3 ", %4\n\t"
                 "s_set_gpr_idx_off"
                 :: "s"(idx), "v"(x.lo), "v"(x.nh), "v"(y.lo), "v"(y.nh) : "m0");
}
// n consecutive intervals (a slot's value then its tangent components) at
// dword offset idx, in one GPR-index session
#define MVF_Q0 "v[128:129]"
#define MVF_Q1 "v[130:131]"
#define MVF_Q2 "v[132:133]"
#define MVF_Q3 "v[134:135]"
#define MVF_Q4 "v[136:137]"
#define MVF_Q5 "v[138:139]"
#define MVF_Q6 "v[140:141]"
#define MVF_Q7 "v[142:143]"
#define MVF_Q8 "v[144:145]"
#define MVF_Q9 "v[146:147]"
static_assert(MVF_SB == 128, "register names of the slot-file sessions");

template <int N>
__device__ __forceinline__ void slot_rd_n(uint32_t idx, Iv (&x)[N]) {
    idx = sidx(idx);
    static_assert(N >= 1 && N <= 5, "1 to 5 intervals");
    if constexpr (N == 1) {
        asm volatile("s_set_gpr_idx_on %2, gpr_idx(SRC0)\n\tv_mov_b64 %0, " MVF_Q0 "\n\tv_mov_b64 %1, " MVF_Q1
                     "\n\ts_set_gpr_idx_off"
                     : "=v"(x[0].lo), "=v"(x[0].nh) : "s"(idx) : "m0");
    } else if constexpr (N == 2) {
        asm volatile("s_set_gpr_idx_on %4, gpr_idx(SRC0)\n\tv_mov_b64 %0, " MVF_Q0 "\n\tv_mov_b64 %1, " MVF_Q1
                     "\n\tv_mov_b64 %2, " MVF_Q2 "\n\tv_mov_b64 %3, " MVF_Q3 "\n\ts_set_gpr_idx_off"
                     : "=v"(x[0].lo), "=v"(x[0].nh), "=v"(x[1].lo), "=v"(x[1].nh) : "s"(idx) : "m0");
    } else if constexpr (N == 3) {
        asm volatile("s_set_gpr_idx_on %6, gpr_idx(SRC0)\n\tv_mov_b64 %0, " MVF_Q0 "\n\tv_mov_b64 %1, " MVF_Q1
                     "\n\tv_mov_b64 %2, " MVF_Q2 "\n\tv_mov_b64 %3, " MVF_Q3 "\n\tv_mov_b64 %4, " MVF_Q4
                     "\n\tv_mov_b64 %5, " MVF_Q5 "\n\ts_set_gpr_idx_off"
                     : "=v"(x[0].lo), "=v"(x[0].nh), "=v"(x[1].lo), "=v"(x[1].nh), "=v"(x[2].lo), "=v"(x[2].nh)
                     : "s"(idx) : "m0");
    } else if constexpr (N == 4) {
        asm volatile("s_set_gpr_idx_on %8, gpr_idx(SRC0)\n\tv_mov_b64 %0, " MVF_Q0 "\n\tv_mov_b64 %1, " MVF_Q1
                     "\n\tv_mov_b64 %2, " MVF_Q2 "\n\tv_mov_b64 %3, " MVF_Q3 "\n\tv_mov_b64 %4, " MVF_Q4
                     "\n\tv_mov_b64 %5, " MVF_Q5 "\n\tv_mov_b64 %6, " MVF_Q6 "\n\tv_mov_b64 %7, " MVF_Q7
                     "\n\ts_set_gpr_idx_off"
                     : "=v"(x[0].lo), "=v"(x[0].nh), "=v"(x[1].lo), "=v"(x[1].nh), "=v"(x[2].lo), "=v"(x[2].nh),
                       "=v"(x[3].lo), "=v"(x[3].nh)
                     : "s"(idx) : "m0");
    } else {
        asm volatile("s_set_gpr_idx_on %10, gpr_idx(SRC0)\n\tv_mov_b64 %0, " MVF_Q0 "\n\tv_mov_b64 %1, " MVF_Q1
                     "\n\tv_mov_b64 %2, " MVF_Q2 "\n\tv_mov_b64 %3, " MVF_Q3 "\n\tv_mov_b64 %4, " MVF_Q4
                     "\n\tv_mov_b64 %5, " MVF_Q5 "\n\tv_mov_b64 %6, " MVF_Q6 "\n\tv_mov_b64 %7, " MVF_Q7
                     "\n\tv_mov_b64 %8, " MVF_Q8 "\n\tv_mov_b64 %9, " MVF_Q9 "\n\ts_set_gpr_idx_off"
                     : "=v"(x[0].lo), "=v"(x[0].nh), "=v"(x[1].lo), "=v"(x[1].nh), "=v"(x[2].lo), "=v"(x[2].nh),
                       "=v"(x[3].lo), "=v"(x[3].nh), "=v"(x[4].lo), "=v"(x[4].nh)
                     : "s"(idx) : "m0");
    }
}

template <int N>
__device__ __forceinline__ void slot_wr_n(uint32_t idx, const Iv (&x)[N]) {
    idx = sidx(idx);
    static_assert(N >= 1 && N <= 5, "1 to 5 intervals");
    if constexpr (N == 1) {
        asm volatile("s_set_gpr_idx_on %0, gpr_idx(DST)\n\tv_mov_b64 " MVF_Q0 ", %1\n\tv_mov_b64 " MVF_Q1
                     ", %2\n\ts_set_gpr_idx_off"
                     :: "s"(idx), "v"(x[0].lo), "v"(x[0].nh) : "m0");
    } else if constexpr (N == 2) {
        asm volatile("s_set_gpr_idx_on %0, gpr_idx(DST)\n\tv_mov_b64 " MVF_Q0 ", %1\n\tv_mov_b64 " MVF_Q1
                     ", %2\n\tv_mov_b64 " MVF_Q2 ", %3\n\tv_mov_b64 " MVF_Q3 ", %4\n\ts_set_gpr_idx_off"
                     :: "s"(idx), "v"(x[0].lo), "v"(x[0].nh), "v"(x[1].lo), "v"(x[1].nh) : "m0");
    } else if constexpr (N == 3) {
        asm volatile("s_set_gpr_idx_on %0, gpr_idx(DST)\n\tv_mov_b64 " MVF_Q0 ", %1\n\tv_mov_b64 " MVF_Q1
                     ", %2\n\tv_mov_b64 " MVF_Q2 ", %3\n\tv_mov_b64 " MVF_Q3 ", %4\n\tv_mov_b64 " MVF_Q4
                     ", %5\n\tv_mov_b64 " MVF_Q5 ", %6\n\ts_set_gpr_idx_off"
                     :: "s"(idx), "v"(x[0].lo), "v"(x[0].nh), "v"(x[1].lo), "v"(x[1].nh), "v"(x[2].lo), "v"(x[2].nh)
                     : "m0");
    } else if constexpr (N == 4) {
        asm volatile("s_set_gpr_idx_on %0, gpr_idx(DST)\n\tv_mov_b64 " MVF_Q0 ", %1\n\tv_mov_b64 " MVF_Q1
                     ", %2\n\tv_mov_b64 " MVF_Q2 ", %3\n\tv_mov_b64 " MVF_Q3 ", %4\n\tv_mov_b64 " MVF_Q4
                     ", %5\n\tv_mov_b64 " MVF_Q5 ", %6\n\tv_mov_b64 " MVF_Q6 ", %7\n\tv_mov_b64 " MVF_Q7
                     ", %8\n\ts_set_gpr_idx_off"
                     :: "s"(idx), "v"(x[0].lo), "v"(x[0].nh), "v"(x[1].lo), "v"(x[1].nh), "v"(x[2].lo), "v"(x[2].nh),
                        "v"(x[3].lo), "v"(x[3].nh)
                     : "m0");
    } else {
        asm volatile("s_set_gpr_idx_on %0, gpr_idx(DST)\n\tv_mov_b64 " MVF_Q0 ", %1\n\tv_mov_b64 " MVF_Q1
                     ", %2\n\tv_mov_b64 " MVF_Q2 ", %3\n\tv_mov_b64 " MVF_Q3 ", %4\n\tv_mov_b64 " MVF_Q4
                     ", %5\n\tv_mov_b64 " MVF_Q5 ", %6\n\tv_mov_b64 " MVF_Q6 ", %7\n\tv_mov_b64 " MVF_Q7
                     ", %8\n\tv_mov_b64 " MVF_Q8 ", %9\n\tv_mov_b64 " MVF_Q9 ", %10\n\ts_set_gpr_idx_off"
                     :: "s"(idx), "v"(x[0].lo), "v"(x[0].nh), "v"(x[1].lo), "v"(x[1].nh), "v"(x[2].lo), "v"(x[2].nh),
                        "v"(x[3].lo), "v"(x[3].nh), "v"(x[4].lo), "v"(x[4].nh)
                     : "m0");
    }
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
