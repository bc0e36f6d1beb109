// mvf_internal.h -- host-side structures of the tape compiler and the library.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "mvf.h"
#include "mvf_isa.h"

namespace mvf {

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
    int64_t ref_fwd = 0, ref_rev = 0, ref_fwd_sparse = 0;
};

// Records the message returned by mvf_last_error() and returns code.
int set_error(int code, const std::string &msg);

// Validates and compiles; returns an MVF_* code and fills err on failure.
int compile_tape(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts, int32_t n_vars,
                 const int32_t *roots, int32_t n_roots, Compiled *out, std::string *err);

// Dwords of the slot file available to a program (root results are kept in LDS).
constexpr int usable_dwords(int /*n_roots*/) { return SLOT_DWORDS; }

}  // namespace mvf
