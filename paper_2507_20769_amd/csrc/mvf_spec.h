// mvf_spec.h -- device helpers of the specialised (run-time-compiled) bounding
// kernel.
//
// The interpreter kernels decode every instruction of a root program at run
// time and move operands through a GPR-indexed slot file.  A specialised
// kernel is generated per tape instead: the same root programs (Sec. 3.2, the
// DAG evaluated node by node) become straight-line code whose operands are
// ordinary variables, so the compiler allocates registers and no instruction
// is decoded or dispatched.  Every operation calls the same interval
// primitives in the same order as the interpreter, so both produce the same
// bits.  The generated functions (namespace spec) are compiled between this
// header and mvf_spec_kernel.h.
#pragma once
#include "mvf_lane.h"

namespace mvf {
namespace dev {

// A lane's subdomain: the breakpoint table in LDS and, per variable, the
// index of the lane's table entry {lo, -hi, c, -c}; the lane's checkpoint
// buffer of the adjoint: each wave owns a contiguous block of the workspace
// laid out [index][lane] (coalesced, 1 KB per index; a wave's checkpoints
// lie within N_CK KB instead of one stretch per index across the whole
// grid's buffer, which took a translation entry per index).
struct SpecLane {
    const double4 *tab;
    int vi[MVF_MAX_VARS];
    double2 *ck;
    int64_t ck_stride;
    Iv *gl;                 // the lane's gradient components kept in LDS (adjoint kernels)
    int gl_stride;
};

// gradient component i of the LDS-resident block of the adjoint's gradient
// (lane-interleaved: entry i of the lane sits i * gl_stride entries after its first)
__device__ __forceinline__ Iv &spec_gl(const SpecLane &L, int i) { return L.gl[i * L.gl_stride]; }

// checkpoint entry i of the lane (stored at a segment boundary, reloaded
// before the segment is recomputed)
__device__ __forceinline__ void spec_ck_st(const SpecLane &L, int i, Iv v) {
    L.ck[(int64_t)i * L.ck_stride] = make_double2(v.lo, v.nh);
}
__device__ __forceinline__ Iv spec_ck_ld(const SpecLane &L, int i) {
    const double2 d = L.ck[(int64_t)i * L.ck_stride];
    return Iv{d.x, d.y};
}

// variable i over the subdomain, [lo, hi]
__device__ __forceinline__ Iv spec_x(const SpecLane &L, int i) {
    const double4 r = L.tab[L.vi[i]];
    return Iv{r.x, r.y};
}
// variable i at the subdomain's centre, [c, c]
__device__ __forceinline__ Iv spec_c(const SpecLane &L, int i) {
    const double4 r = L.tab[L.vi[i]];
    return Iv{r.z, r.w};
}
// X_i - c_i, the factor of G_i in the mean value form
__device__ __forceinline__ Iv spec_dx(const SpecLane &L, int i) {
    const double4 r = L.tab[L.vi[i]];
    return Iv{fadd(r.x, r.w), fadd(r.y, r.z)};
}

}  // namespace dev
}  // namespace mvf
