// mvf_kernels.h -- launches and LDS sizing of the bounding kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mvf.h"
#include "mvf_internal.h"
#include "mvf_kargs.h"

namespace mvf {

hipError_t launch_points(const PointsArgs &A, int op, int chunk, int grid, size_t lds, hipStream_t stream);

hipError_t launch_bound(const TapeArgs &T, const BoxArgs &B, int chunk, bool rev, int grid, size_t lds,
                        hipStream_t stream,
                        hipEvent_t after = nullptr);
// Step 3 across the workgroups of a single-box launch (per-block partials -> reduced, argmin, extra)
hipError_t launch_finish(const BoxArgs &B, int grid, int m, hipStream_t stream);
// forward-backward bound tightening, one lane per box
hipError_t launch_fbbt(const FbbtArgs &A, hipStream_t stream);
hipError_t launch_batch(const TapeArgs &T, const BatchArgs &A, int chunk, bool rev, int grid, size_t lds,
                        int max_nodes, hipStream_t stream);
// the batched launch's plan kernel and per-node finish kernel (around any persistent bounding kernel)
hipError_t launch_batch_plan(const BatchArgs &A, hipStream_t stream);
hipError_t launch_batch_finish(const BatchArgs &A, int m, int max_nodes, hipStream_t stream);

// This device's copy of the no-allocation entry point's scratch array
// (MVF_NOALLOC_SCRATCH_BYTES), looked up once per device.
hipError_t noalloc_scratch(int device, void **ptr);

constexpr size_t LDS_BUDGET = 160 * 1024;

// LDS bytes of a workgroup (programs, table, gradient accumulators when in
// LDS, spill slots, reduction, ints, vrec).
inline size_t spill_bytes(int spill_slots, int chunk) { return (size_t)spill_slots * (1 + chunk) * 16 * BLK; }
inline size_t lds_bytes(int n_instr, int tab_cap, int n, int m, bool g_in_lds, size_t spill = 0) {
    size_t b = (size_t)n_instr * 16 + (size_t)tab_cap * 32;
    if (g_in_lds) b += (size_t)n * BLK * 16;
    b += spill;
    b += ((size_t)(BLK / 64) * (2 * m + 5) * 8 + 15) & ~(size_t)15;   // per-wave reduction records
    b += (2 * MVF_MAX_VARS + 8) * 4;
    b = (b + 15) & ~(size_t)15;
    b += (size_t)n * BLK * sizeof(uint16_t);
    return b;
}

inline size_t points_lds_bytes(int n_records, int n, bool g_in_lds, size_t spill) {
    return (size_t)n_records * 16 + (g_in_lds ? (size_t)n * BLK * 16 : 0) + spill;
}

// Reverse mode keeps the gradient accumulators in LDS when a workgroup still
// fits; otherwise they live in the workspace (coalesced [dim][lane]).
inline bool grad_in_lds(int n_instr, int tab_cap, int n, int m) {
    // two workgroups per compute unit
    return lds_bytes(n_instr, tab_cap, n, m, true) <= LDS_BUDGET / 2;
}

}  // namespace mvf
