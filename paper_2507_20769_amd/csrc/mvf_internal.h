// mvf_internal.h -- register-program format shared by the tape compiler and the kernels.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

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
    I_NOPS = 17,
};
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
// quotient, 2U, 1/(2Z), Z, 1/U).  Variable and constant operands are not
// recorded (they are known again in the reverse sweep), nor are the partials
// of the constant-operand forms.
// Order within an instruction: U then V for a product, 1/V then Z for a quotient.
constexpr uint32_t n_records(uint32_t op, uint32_t ak, uint32_t bk) {
    return op == I_MUL ? (is_reg_kind(ak) && bk != K_CONST) + (is_reg_kind(bk) && ak != K_CONST)
         : op == I_DIV ? 1u + (bk != K_CONST)
         : (op >= I_SQR && op <= I_LOG) ? (ak != K_CONST ? 1u : 0u) : 0u;
}

// One compiled root program.
struct RootProg {
    int32_t begin = 0, len = 0;      // range in the instruction array
    int32_t result_slot = 0;         // slot holding the root after the last instruction
    int32_t n_slots = 0;             // live-set size
    int32_t n_rec = 0;               // reverse-mode records per subdomain
};

struct Compiled {
    int32_t n_vars = 0;
    int32_t n_prog = 0;              // instructions of the root programs (auxiliary records follow)
    int32_t root_base = 0;           // index of the per-root records {begin, len, result slot, records},
                                     // followed by the union program's record and its root slots
    RootProg uprog;                  // union of all root cones, every root live to its end
    std::vector<int32_t> union_slots;  // slot of each root at the end of the union program
    bool union_ok = false;           // the union program's live set fits the slot file
    int32_t n_bound = 0;             // records the bounding kernels stage (programs, aux, root records)
    int32_t union_base = 0;          // index of the union record
    std::vector<RootProg> roots;
    std::vector<Instr> instr;
    int32_t max_slots = 0;
    int32_t max_rec = 0;             // largest record count of a root program
    int32_t chunk = 0;               // tangent components per forward pass (set by the library)
    int32_t spill = 0;               // LDS spill slots per lane at that chunk
    int64_t ref_fwd = 0, ref_rev = 0;
};

// Records the message returned by mvf_last_error() and returns code.
int set_error(int code, const std::string &msg);

// Validates and compiles; returns an MVF_* code and fills err on failure.
int compile_tape(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts, int32_t n_vars,
                 const int32_t *roots, int32_t n_roots, Compiled *out, std::string *err);

// Dwords of the slot file available to a program (root results are kept in LDS).
constexpr int usable_dwords(int /*n_roots*/) { return SLOT_DWORDS; }

}  // namespace mvf
