// mvf_kargs.h -- launch arguments of the bounding kernels, shared by the host
// library, the interpreter kernels and the run-time-compiled specialised
// kernels.
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "mvf_isa.h"

namespace mvf {

constexpr int BLK = 256;            // lanes (subdomains) per workgroup
constexpr int BATCH_TAB_CAP = 256;  // breakpoint-table entries of a batched launch (sum of a node's splits)

// Per-tape arguments (wave-uniform).
struct TapeArgs {
    const Instr *prog;
    int32_t n_instr, n_roots, n, mode;
    int32_t root_base;       // program record index of root 0's {begin, len, result slot, records}
    uint32_t ineq_mask, eq_mask;  // roots that are constraints g <= 0 / h = 0 (bit r for root r)
    int32_t nreg;            // register slots of the launch's tangent chunk; higher slot ids live in LDS
    int32_t spill_slots;     // LDS spill slots per lane (forward tangent passes)
};

// One node box.
struct BoxArgs {
    int32_t splits[MVF_MAX_VARS];
    int32_t tab_off[MVF_MAX_VARS + 1];
    const double *box;       // device [n][2]
    int64_t S;
    double *per_sub;         // [m][2][S] or null
    uint32_t *flags;         // [S] or null
    double *reduced;         // [m][2]
    int64_t *argmin;         // [1] or null
    double *partial;         // [grid][m][2]
    double *partial_lo0;     // [grid]
    int64_t *partial_k;      // [grid]
    double *partial_ext;     // [grid][2]: feasibility-filtered objective bound, upper bound from centres
    double *extra;           // [2] or null
    double2 *rec;            // reverse-mode tape, per wave [rec_lane][64]
    double2 *gacc;           // reverse-mode gradient accumulators, per wave [n][64], when not in LDS
    int64_t rec_lane;        // records (or checkpoint intervals) per lane that rec holds
};

// Many node boxes in one persistent launch.
struct BatchArgs {
    const int32_t *n_nodes_dev;  // device node count (a captured graph changes it between replays) or null
    int32_t n_nodes_val;         // node count when n_nodes_dev is null
    int32_t n;
    int32_t tab_cap;         // breakpoint-table capacity per node (entries)
    int32_t spl;             // subdomains per lane: a work item is spl * BLK subdomains of one node
    const double *boxes;     // [N][n][2]
    const int32_t *splits;   // [N][n]
    double *reduced;         // [N][m][2]
    int64_t *argmin;         // [N] or null
    int32_t *status;         // [N]: 0 ok, 1 invalid node
    int64_t *node_S;         // [N]
    int64_t *item_off;       // [N + 1]
    int64_t *counter;        // work-item counter
    int64_t item_cap;        // capacity of the item partial arrays
    double *partial;         // [items][m][2]
    double *partial_lo0;     // [items]
    int64_t *partial_k;      // [items]
    double *partial_ext;     // [items][2]
    double *extra;           // [N][2] or null
    double2 *rec;            // reverse-mode tape, per wave [rec_lane][64]
    double2 *gacc;           // reverse-mode gradient accumulators, per wave [n][64], when not in LDS
    int64_t rec_lane;        // records (or checkpoint intervals) per lane that rec holds
};

// The bounding kernels take one argument struct each (at kernarg offset 0).
struct BoundKArgs {
    TapeArgs T;
    BoxArgs B;
};
struct BatchKArgs {
    TapeArgs T;
    BatchArgs A;
};

// Point and box entry points (one lane per point or box).
enum : int { PT_EVAL = 0, PT_VJP = 1, PT_GRAD_FWD = 2, PT_GRAD_REV = 3 };
struct PointsArgs {
    const Instr *prog;
    int32_t n_records;       // every program record (all are staged)
    int32_t n_roots, n, root_base, union_base;
    int32_t nreg, spill_slots;   // tangent passes of a forward gradient
    int32_t root;            // the root whose gradient is taken
    int64_t B;
    const double *x;         // points [B][n], or boxes [B][n][2] for gradients
    const double *gout;      // [B][m] cotangents (vector-Jacobian product)
    double *out;             // values [B][m][2], or gradients [B][n][2]
    uint32_t *flags;         // [B] or null: domain violation
    double2 *rec;            // reverse-mode records, per wave [rec_lane][64]
    double2 *gacc;           // gradient accumulators, per wave [n][64], when not in LDS
    int64_t rec_lane;        // records per lane that rec holds
};
struct PointsKArgs {
    PointsArgs P;
};
// Forward-backward bound tightening of many boxes (one lane per box).
struct DagNode {
    int32_t op, a, b, live;  // tape node; live: in some root's cone
};
struct FbbtArgs {
    const DagNode *nodes;
    const double *consts;
    const int32_t *roots;
    int32_t n_nodes, n, m, rounds;
    uint32_t ineq_mask, eq_mask;
    double ub;               // objective upper bound (+inf: none)
    int64_t N;
    const double *boxes;     // [N][n][2]
    double *out;             // [N][n][2]
    int32_t *status;         // [N]: 1 = proven infeasible
    double2 *val;            // scratch [n_nodes][stride]
    int64_t stride;
};

#if defined(__HIPCC__) || defined(__HIPCC_RTC__)
template <typename BA>     // BatchArgs in any address space
__device__ __forceinline__ int node_count(const BA &A) { return A.n_nodes_dev ? *A.n_nodes_dev : A.n_nodes_val; }
#endif

}  // namespace mvf
