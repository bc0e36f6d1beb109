// mvf_isa.h -- register-program format and launch constants shared by the
// tape compiler (host), the interpreter kernels and the run-time-compiled
// specialised kernels (device).  No host-library dependencies.
#pragma once
#ifdef __HIPCC_RTC__
#include "mvf_rtc_prelude.h"
#else
#include <stdint.h>
#endif

#include "mvf.h"

namespace mvf {

// Register slot file: VGPRs [SLOT_BASE, 256) of every lane, addressed through
// GPR index mode.  The compiler is limited to VGPRs [0, SLOT_BASE).
constexpr int SLOT_BASE = 128;
constexpr int SLOT_DWORDS = 256 - SLOT_BASE;        // 128
constexpr int MAX_CHUNK = 4;                        // tangent components per pass

// Instruction opcodes: the tape ops, a load, and constant-operand forms of
// + - * / (the non-constant operand is always operand a).
enum : uint32_t {
    I_ADD = MVF_ADD, I_SUB = MVF_SUB, I_MUL = MVF_MUL, I_DIV = MVF_DIV,
    I_SQR = MVF_SQR, I_SQRT = MVF_SQRT, I_EXP = MVF_EXP, I_LOG = MVF_LOG,
    I_LOAD = 10,      // dst = operand a (a variable or constant root, or a materialised constant)
    I_ADDK = 11,      // U + k      (also U - k, with k negated)
    I_KSUB = 12,      // k - U
    I_MULK = 13,      // U * k      (k finite, nonzero, sign bit clear)
    I_MULKN = 14,     // U * (-k)   (k stored as its magnitude)
    I_DIVK = 15,      // U / k      (k > 0); operand b indexes the enclosure of 1/k
    I_DIVKN = 16,     // U / (-k)   (k stored as its magnitude)
    I_TANH = 17, I_SIN = 18, I_COS = 19,   // the tape's TANH, SIN, COS
    I_NOPS = 20,
};

// unary functions with a local derivative interval: sqr sqrt exp log tanh sin cos
constexpr bool is_unary_fn(uint32_t op) { return (op >= I_SQR && op <= I_LOG) || (op >= I_TANH && op <= I_COS); }
// Operand kinds.  A result whose only consumer is the next instruction goes
// to slot 0, which the allocator keeps for such short-lived values (its
// adjoint in the reverse sweep lands in slot 0 the same way); K_PREV is not
// emitted.
enum : uint32_t { K_SLOT = 0, K_VAR = 1, K_CONST = 2, K_PREV = 3 };

// 16-byte instruction, read from LDS by all lanes of a wave (broadcast):
//   w0 = op | akind << 5 | bkind << 7 | init_a << 9 | init_b << 10 | nowrite << 11 | a << 16
//   w1 = b | dst << 16
//   k  = the constant operand (at most one operand is a constant)
// init_x: this instruction is the last consumer of operand x, so in the
// reverse sweep it makes the first contribution to that adjoint (written, not
// accumulated).  nowrite: the result is only consumed by the next instruction
// (it is written to slot 0).  For I_DIVK/I_DIVKN, b is the index of a 16-byte record after
// the programs holding the enclosure of 1/|k| as (lo, -hi).
struct Instr {
    uint32_t w0, w1;
    double k;
};
static_assert(sizeof(Instr) == 16, "instruction record is 16 bytes");

constexpr uint32_t W0_INIT_A = 1u << 9, W0_INIT_B = 1u << 10, W0_NOWRITE = 1u << 11;

inline Instr make_instr(uint32_t op, uint32_t ak, uint32_t a, uint32_t bk, uint32_t b, uint32_t dst, double k) {
    Instr I;
    I.w0 = op | (ak << 5) | (bk << 7) | (a << 16);
    I.w1 = (b & 0xffffu) | (dst << 16);
    I.k = k;
    return I;
}

constexpr bool is_reg_kind(uint32_t k) { return k == K_SLOT || k == K_PREV; }

// Interval records one instruction leaves on the reverse-mode tape: the local
// partials its adjoint rule needs (operand values of a product, 1/V and Z of a
// quotient, 2U, 1/(2Z), Z, 1/U, 1 - Z^2, cos U, -sin U).  Variable and constant operands are not
// recorded (they are known again in the reverse sweep), nor are the partials
// of the constant-operand forms.
// Order within an instruction: U then V for a product, 1/V then Z for a quotient.
constexpr uint32_t n_records(uint32_t op, uint32_t ak, uint32_t bk) {
    return op == I_MUL ? (is_reg_kind(ak) && bk != K_CONST) + (is_reg_kind(bk) && ak != K_CONST)
         : op == I_DIV ? 1u + (bk != K_CONST)
         : is_unary_fn(op) ? (ak != K_CONST ? 1u : 0u) : 0u;
}

}  // namespace mvf
