// mvf_internal.h -- register-program format shared by the tape compiler and the kernels.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "mvf.h"

namespace mvf {

// Register slot file: VGPRs [SLOT_BASE, 256) of every lane, addressed through
// GPR index mode.  The compiler is limited to VGPRs [0, SLOT_BASE).
constexpr int SLOT_BASE = 96;
constexpr int SLOT_DWORDS = 256 - SLOT_BASE;        // 160
constexpr int MAX_CHUNK = 2;                        // tangent components per pass

// Instruction opcodes: the tape ops plus two loads.
enum : uint32_t {
    I_ADD = MVF_ADD, I_SUB = MVF_SUB, I_MUL = MVF_MUL, I_DIV = MVF_DIV,
    I_SQR = MVF_SQR, I_SQRT = MVF_SQRT, I_EXP = MVF_EXP, I_LOG = MVF_LOG,
    I_LOAD = 10,      // dst = operand a (a variable or constant root)
};
// Operand kinds.
enum : uint32_t { K_SLOT = 0, K_VAR = 1, K_CONST = 2 };

// 16-byte instruction, read from LDS by all lanes of a wave (broadcast):
//   w0 = op | akind << 8 | bkind << 10 | init_a << 12 | init_b << 13 | a << 16
//   w1 = b | dst << 16
//   k  = the constant operand (at most one operand is a constant)
struct Instr {
    uint32_t w0, w1;
    double k;
};
static_assert(sizeof(Instr) == 16, "instruction record is 16 bytes");

inline Instr make_instr(uint32_t op, uint32_t ak, uint32_t a, uint32_t bk, uint32_t b, uint32_t dst, double k) {
    Instr I;
    I.w0 = op | (ak << 8) | (bk << 10) | (a << 16);
    I.w1 = (b & 0xffffu) | (dst << 16);
    I.k = k;
    return I;
}

// Interval records one instruction leaves on the reverse-mode tape: the local
// partials its adjoint rule needs (operand values of a product, 1/V and Z of a
// quotient, 2U, 1/(2Z), Z, 1/U).  Variable and constant operands are not
// recorded; they are known again in the reverse sweep.
// Order within an instruction: U then V for a product, 1/V then Z for a quotient.
constexpr uint32_t n_records(uint32_t op, uint32_t ak, uint32_t bk) {
    return op == MVF_MUL ? (ak == K_SLOT && bk != K_CONST) + (bk == K_SLOT && ak != K_CONST)
         : op == MVF_DIV ? 1u + (bk != K_CONST)
         : (op >= MVF_SQR && op <= MVF_LOG) ? 1u : 0u;
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
    std::vector<RootProg> roots;
    std::vector<Instr> instr;
    int32_t max_slots = 0;
    int32_t max_rec = 0;             // largest record count of a root program
    int32_t chunk = 0;               // tangent components per forward pass (set by the library)
    int32_t spill = 0;               // LDS spill slots per lane at that chunk
    int64_t ref_fwd = 0, ref_rev = 0;
};

// Validates and compiles; returns an MVF_* code and fills err on failure.
int compile_tape(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts, int32_t n_vars,
                 const int32_t *roots, int32_t n_roots, Compiled *out, std::string *err);

// Reserved result slots (one interval each) sit at the top of the slot file.
constexpr int result_slot_dwords(int n_roots) { return 4 * n_roots; }
constexpr int usable_dwords(int n_roots) { return SLOT_DWORDS - result_slot_dwords(n_roots); }

}  // namespace mvf
