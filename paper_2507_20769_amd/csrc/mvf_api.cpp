// mvf_api.cpp -- the C ABI of libmvf (include/mvf.h): argument checks, workspace
// layout, launches, the batched graph and the autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <string>
#include <vector>

#include "mvf.h"
#include "mvf_internal.h"
#include "mvf_kernels.h"
#include "mvf_spec_internal.h"

using namespace mvf;

struct mvf_tape {
    Compiled C;
    Instr *d_prog = nullptr;
    int device = 0;
    int n_cu = 256;
    uint32_t ineq_mask = 0, eq_mask = 0;   // constraint roots (mvf_tape_set_root_kinds)
    DagNode *d_nodes = nullptr;             // the DAG itself, for bound tightening
    int32_t *d_roots = nullptr;
    double *d_consts = nullptr;
    int32_t n_nodes = 0;
    hipModule_t spec_mod = nullptr;         // specialised kernels (mvf_tape_specialize)
    hipFunction_t spec_fn[2] = {nullptr, nullptr};        // single box: [0] tangent mode, [1] adjoint
    hipFunction_t spec_batch_fn[2] = {nullptr, nullptr};  // batched
    mvf_spec_info spec_info{};
    int32_t spec_ck = 0;                    // checkpoint intervals per lane of the specialised adjoint
    int32_t spec_gl = 0;                    // gradient components per lane its kernels keep in LDS
    uint64_t spec_id = 0;                   // which specialisation (0: none), for the autotuner's cache
};

struct mvf_batch_graph {
    const mvf_tape *tape = nullptr;
    int32_t max_nodes = 0;
    int64_t max_subdomains = 0;
    int32_t mode = 0, grad = 0;
    mvf_tuning tuning{};
    void *d_ws = nullptr;
    size_t ws_bytes = 0;
    double *d_boxes = nullptr;
    int32_t *d_splits = nullptr, *d_count = nullptr, *d_status = nullptr;
    double *d_reduced = nullptr, *d_extra = nullptr;
    int64_t *d_argmin = nullptr;
    double *h_boxes = nullptr, *h_reduced = nullptr, *h_extra = nullptr;
    int32_t *h_splits = nullptr, *h_count = nullptr, *h_status = nullptr;
    int64_t *h_argmin = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;            // recorded after each replay (staging reuse guard)
    bool launched = false;
};

namespace {

thread_local std::string g_err;

int set_err(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_err(hipError_t e, const char *what) { return set_err(MVF_EHIP, std::string(what) + ": " + hipGetErrorString(e)); }

#define HIP_TRY(expr)                                    \
    do {                                                 \
        hipError_t _e = (expr);                          \
        if (_e != hipSuccess) return hip_err(_e, #expr); \
    } while (0)

int check_device(int *n_cu) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_err(MVF_ENOTSUP, std::string("device is ") + prop.gcnArchName + ", need gfx950");
    *n_cu = prop.multiProcessorCount;
    return MVF_OK;
}


// Tangent components per forward pass: the fewest passes over the program
// (then the fewest LDS spill slots, then the smallest chunk) among the chunks
// whose spill slots still let two workgroups share a compute unit (one, for a
// single component, if that is the only way).
void choose_chunk(Compiled &C) {
    const int m = (int)C.roots.size(), n = C.n_vars, ni = C.n_bound;
    const int avail = usable_dwords(m);
    C.chunk = 0;
    C.spill = 0;
    int best_passes = 1 << 30, best_spill = 1 << 30;
    for (int c = 1; c <= std::min(MAX_CHUNK, n); ++c) {
        const int sp = std::max(0, C.max_slots - avail / (4 + 4 * c));
        const size_t lds = lds_bytes(ni, BATCH_TAB_CAP, n, m, false, spill_bytes(sp, c));
        if (!(lds <= LDS_BUDGET / 2 || (c == 1 && lds <= LDS_BUDGET - 1024))) continue;
        const int passes = (n + c - 1) / c;
        if (passes < best_passes || (passes == best_passes && sp < best_spill)) {
            best_passes = passes;
            best_spill = sp;
            C.chunk = c;
            C.spill = sp;
        }
    }
}

int spill_for(const Compiled &C, int chunk) {
    return chunk > 0 ? std::max(0, C.max_slots - usable_dwords((int)C.roots.size()) / (4 + 4 * chunk)) : 0;
}

void fill_stats(const Compiled &C, mvf_tape_stats *st) {
    st->n_vars = C.n_vars;
    st->n_roots = (int32_t)C.roots.size();
    st->n_instr = C.n_prog;
    st->max_slots = C.max_slots;
    st->tangent_chunk = C.chunk;
    st->max_records = C.max_rec;
    st->ref_ops_fwd = C.ref_fwd;
    st->ref_ops_rev = C.ref_rev;
    st->ref_ops_fwd_sparse = C.ref_fwd_sparse;
    spec_ckpt_plan_stats(C, &st->ckpt_segments, &st->ckpt_stored, &st->ckpt_loaded);
}

TapeArgs tape_args(const mvf_tape *t, int mode, int chunk) {
    TapeArgs T;
    std::memset(&T, 0, sizeof T);
    T.prog = t->d_prog;
    T.n_instr = t->C.n_bound;
    T.n_roots = (int32_t)t->C.roots.size();
    T.n = t->C.n_vars;
    T.mode = mode;
    T.root_base = t->C.root_base;
    T.ineq_mask = t->ineq_mask;
    T.eq_mask = t->eq_mask;
    T.nreg = chunk > 0 ? usable_dwords(T.n_roots) / (4 + 4 * chunk) : usable_dwords(T.n_roots) / 4;
    T.spill_slots = spill_for(t->C, chunk);
    return T;
}

// resolve the gradient mode: AUTO takes the cheaper reference cost; forward
// needs at least one tangent component's slots
int resolve_grad(const mvf_tape *t, int mode, int grad, const mvf_tuning *tu, bool *rev, int *chunk) {
    if (tu && tu->grad >= MVF_GRAD_FWD && tu->grad <= MVF_GRAD_REV) grad = tu->grad;
    if (mode == MVF_MODE_NIE) { *rev = false; *chunk = 0; return MVF_OK; }
    if (grad == MVF_GRAD_AUTO) grad = (t->C.chunk == 0 || t->C.ref_rev < t->C.ref_fwd) ? MVF_GRAD_REV : MVF_GRAD_FWD;
    *rev = grad == MVF_GRAD_REV;
    *chunk = *rev ? 0 : t->C.chunk;
    // a tuned chunk may exceed the default one; the launch checks that its spill slots fit in LDS
    if (tu && !*rev && tu->chunk >= 1 && tu->chunk <= std::min(MAX_CHUNK, t->C.n_vars)) *chunk = tu->chunk;
    if (!*rev && *chunk == 0)
        return set_err(MVF_ELIMIT, "a root's live set is too large for tangent passes; use MVF_GRAD_REV");
    return MVF_OK;
}

constexpr int MAX_GRID = 2048;

int single_grid(const mvf_tape *t, int64_t S, bool rev) {
    const int64_t need = (S + BLK - 1) / BLK;
    // reverse mode: as many workgroups as the CUs hold at once (the record tape or
    // the checkpoint buffer scales with the grid): two per CU, or as many waves per
    // SIMD as the specialised adjoint is compiled for
    const int per_cu = t->spec_fn[1] ? std::max(2, t->spec_info.waves) : 2;
    const int cap = rev ? per_cu * t->n_cu : MAX_GRID;
    return (int)std::max<int64_t>(1, std::min<int64_t>(need, cap));
}

int batch_block(const mvf_tuning *tu) { return tu && tu->block > 0 ? tu->block : BLK; }

int batch_grid(const mvf_tape *t, const mvf_tuning *tu) {
    if (tu && tu->grid_blocks > 0) return tu->grid_blocks;
    return 2 * t->n_cu * (BLK / batch_block(tu));      // two 256-lane workgroups' worth per CU
}

int batch_spl(const mvf_tuning *tu) { return tu && tu->sub_per_lane > 0 ? tu->sub_per_lane : 1; }

// the batched forward launch runs the specialised kernel unless told otherwise
int batch_engine(const mvf_tape *t, const mvf_tuning *tu, bool rev, bool *spec) {
    const int e = tu ? tu->engine : MVF_ENGINE_AUTO;
    if (e < MVF_ENGINE_AUTO || e > MVF_ENGINE_SPEC) return set_err(MVF_EINVAL, "bad engine");
    if (tu && (tu->sub_per_lane < 0 || tu->sub_per_lane > 16)) return set_err(MVF_EINVAL, "sub_per_lane outside [0, 16]");
    if (tu && tu->block != 0 && tu->block != 64 && tu->block != 128 && tu->block != BLK)
        return set_err(MVF_EINVAL, "block must be 64, 128 or 256");
    if (e == MVF_ENGINE_SPEC && !t->spec_batch_fn[rev])
        return set_err(MVF_EINVAL, "no specialised kernel for this gradient mode: see mvf_tape_specialize");
    *spec = t->spec_batch_fn[rev] && e != MVF_ENGINE_INTERP;
    if (!*spec && batch_block(tu) != BLK) return set_err(MVF_EINVAL, "the interpreter's workgroup is 256 lanes");
    return MVF_OK;
}

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Reverse-mode intervals per lane in the workspace: the interpreter's record
// tape or the specialised adjoint's checkpoints, whichever the call may use.
size_t rec_per_lane(const mvf_tape *t) { return (size_t)std::max(t->C.max_rec, t->spec_ck); }

struct SingleLayout {
    size_t partial, lo0, k, ext, rec, gacc, total;
    bool g_lds;
};

SingleLayout single_layout(const mvf_tape *t, int grid, bool rev, int tab_total, size_t rec_lane) {
    const size_t m = t->C.roots.size();
    SingleLayout L;
    L.g_lds = grad_in_lds(t->C.n_bound, tab_total, t->C.n_vars, (int)m);
    L.partial = 0;
    L.lo0 = align_up(L.partial + (size_t)grid * m * 2 * 8);
    L.k = align_up(L.lo0 + (size_t)grid * 8);
    L.ext = align_up(L.k + (size_t)grid * 8);
    L.rec = align_up(L.ext + (size_t)grid * 16);
    L.gacc = align_up(L.rec + (rev ? rec_lane * grid * BLK * 16 : 0));
    L.total = L.gacc + (rev && !L.g_lds ? (size_t)t->C.n_vars * grid * BLK * 16 : 0);
    return L;
}

struct BatchLayout {
    size_t node_S, item_off, counter, partial, lo0, k, ext, rec, gacc, total;
    bool g_lds;
};

// grid x block lanes run (the interpreter's block is always 256)
BatchLayout batch_layout(const mvf_tape *t, int max_nodes, int64_t max_sub, int grid, int block, bool rev) {
    const size_t m = t->C.roots.size();
    const size_t items = (size_t)(max_sub / BLK) + (size_t)max_nodes + 1;
    BatchLayout L;
    L.node_S = 0;
    L.item_off = align_up(L.node_S + (size_t)max_nodes * 8);
    L.counter = align_up(L.item_off + ((size_t)max_nodes + 1) * 8);
    L.partial = align_up(L.counter + 8);
    L.lo0 = align_up(L.partial + items * m * 2 * 8);
    L.k = align_up(L.lo0 + items * 8);
    L.ext = align_up(L.k + items * 8);
    L.rec = align_up(L.ext + items * 16);
    L.g_lds = grad_in_lds(t->C.n_bound, BATCH_TAB_CAP, t->C.n_vars, (int)m);
    L.gacc = align_up(L.rec + (rev ? rec_per_lane(t) * grid * block * 16 : 0));
    L.total = L.gacc + (rev && !L.g_lds ? (size_t)t->C.n_vars * grid * BLK * 16 : 0);
    return L;
}

// Point and box entry points: grid, LDS placement of the gradient accumulators,
// workspace (reverse-mode records, then accumulators when not in LDS).
struct PointsLayout {
    int grid = 1, chunk = 0, spill = 0;
    bool g_lds = true;
    size_t rec = 0, gacc = 0, total = 0, lds = 0;
    int64_t recs = 0;        // records per lane
};

int points_layout(const mvf_tape *t, int op, int64_t B, PointsLayout *L) {
    const Compiled &C = t->C;
    const bool rev = op == PT_VJP || op == PT_GRAD_REV;
    if (!C.union_ok) return set_err(MVF_ELIMIT, "the union of the root cones needs more slots than the slot file holds");
    if (op == PT_GRAD_FWD) {
        if (C.chunk == 0) return set_err(MVF_ELIMIT, "a root's live set is too large for tangent passes; use MVF_GRAD_REV");
        L->chunk = C.chunk;
        L->spill = C.spill;
    }
    const int64_t need = std::max<int64_t>(1, (B + BLK - 1) / BLK);
    L->grid = (int)std::min<int64_t>(need, rev ? 2 * t->n_cu : MAX_GRID);
    const size_t spill = spill_bytes(L->spill, L->chunk);
    L->g_lds = points_lds_bytes((int)C.instr.size(), C.n_vars, true, spill) <= LDS_BUDGET / 2;
    L->lds = points_lds_bytes((int)C.instr.size(), C.n_vars, rev && L->g_lds, spill);
    if (L->lds > LDS_BUDGET - 1024) return set_err(MVF_ELIMIT, "programs exceed the LDS budget of the point kernels");
    const int recs = op == PT_VJP ? C.uprog.n_rec : C.max_rec;
    L->recs = recs;
    L->rec = 0;
    L->gacc = align_up(rev ? (size_t)recs * L->grid * BLK * 16 : 0);
    L->total = L->gacc + (rev && !L->g_lds ? (size_t)C.n_vars * L->grid * BLK * 16 : 0);
    return MVF_OK;
}

int launch_points_op(const mvf_tape *t, int op, int64_t B, const double *x, const double *gout, int32_t root,
                     double *out, uint32_t *flags, void *ws, size_t ws_bytes, hipStream_t stream) {
    if (B < 0 || B > (INT64_C(1) << 40)) return set_err(MVF_EINVAL, "point count outside [0, 2^40]");
    if (B == 0) return MVF_OK;
    PointsLayout L;
    int rc = points_layout(t, op, B, &L);
    if (rc != MVF_OK) return rc;
    if (L.total > 0 && (!ws || ws_bytes < L.total)) return set_err(MVF_EINVAL, "workspace too small");
    PointsArgs A;
    std::memset(&A, 0, sizeof A);
    A.prog = t->d_prog;
    A.n_records = (int32_t)t->C.instr.size();
    A.n_roots = (int32_t)t->C.roots.size();
    A.n = t->C.n_vars;
    A.root_base = t->C.root_base;
    A.union_base = t->C.union_base;
    A.nreg = L.chunk > 0 ? usable_dwords(A.n_roots) / (4 + 4 * L.chunk) : usable_dwords(A.n_roots) / 4;
    A.spill_slots = L.spill;
    A.root = root;
    A.B = B;
    A.x = x;
    A.gout = gout;
    A.out = out;
    A.flags = flags;
    uint8_t *w = static_cast<uint8_t *>(ws);
    A.rec = L.total > 0 ? reinterpret_cast<double2 *>(w + L.rec) : nullptr;
    A.rec_lane = L.recs;
    A.gacc = (op == PT_VJP || op == PT_GRAD_REV) && !L.g_lds ? reinterpret_cast<double2 *>(w + L.gacc) : nullptr;
    hipError_t e = launch_points(A, op, L.chunk, L.grid, L.lds, stream);
    if (e != hipSuccess) return hip_err(e, "launch_points");
    return MVF_OK;
}

int check_splits(const mvf_tape *t, const int32_t *splits, int64_t *S, int *tab_total) {
    if (!splits) return set_err(MVF_EINVAL, "splits is null");
    int64_t s = 1;
    int tt = 0;
    for (int i = 0; i < t->C.n_vars; ++i) {
        if (splits[i] < 1 || splits[i] > 65535) return set_err(MVF_EINVAL, "split count outside [1, 65535]");
        tt += splits[i];
        if (s > (INT64_C(1) << 40) / splits[i]) return set_err(MVF_ELIMIT, "more than 2^40 subdomains");
        s *= splits[i];
    }
    if (tt > MVF_MAX_TABLE) return set_err(MVF_ELIMIT, "sum of split counts above MVF_MAX_TABLE");
    *S = s;
    *tab_total = tt;
    return MVF_OK;
}

int fill_batch_args(const mvf_tape *t, int32_t n_nodes, const int32_t *n_nodes_dev, int max_nodes, int64_t max_sub,
                    const double *boxes, const int32_t *splits, double *reduced, int64_t *argmin, int32_t *status,
                    double *extra, void *ws, size_t ws_bytes, int grid, int block, bool rev, int spl,
                    BatchArgs *A) {
    const BatchLayout L = batch_layout(t, max_nodes, max_sub, grid, block, rev);
    if (ws_bytes < L.total) return set_err(MVF_EINVAL, "workspace too small");
    uint8_t *w = static_cast<uint8_t *>(ws);
    std::memset(A, 0, sizeof *A);
    A->n_nodes_dev = n_nodes_dev;
    A->n_nodes_val = n_nodes;
    A->n = t->C.n_vars;
    A->tab_cap = BATCH_TAB_CAP;
    A->spl = spl;
    A->boxes = boxes;
    A->splits = splits;
    A->reduced = reduced;
    A->argmin = argmin;
    A->status = status;
    A->node_S = reinterpret_cast<int64_t *>(w + L.node_S);
    A->item_off = reinterpret_cast<int64_t *>(w + L.item_off);
    A->counter = reinterpret_cast<int64_t *>(w + L.counter);
    A->partial = reinterpret_cast<double *>(w + L.partial);
    A->partial_lo0 = reinterpret_cast<double *>(w + L.lo0);
    A->partial_k = reinterpret_cast<int64_t *>(w + L.k);
    A->partial_ext = reinterpret_cast<double *>(w + L.ext);
    A->extra = extra;
    A->rec = reinterpret_cast<double2 *>(w + L.rec);
    A->rec_lane = (int64_t)rec_per_lane(t);
    A->gacc = rev && !L.g_lds ? reinterpret_cast<double2 *>(w + L.gacc) : nullptr;
    A->item_cap = (int64_t)(max_sub / BLK) + max_nodes + 1;
    return MVF_OK;
}

// plan -> persistent bounding kernel (specialised or interpreter) -> per-node finish
int launch_batched(const mvf_tape *t, int mode, int chunk, bool rev, bool spec, const BatchArgs &A, int grid,
                   int block, int max_nodes, hipStream_t stream) {
    const int m = (int)t->C.roots.size(), n = t->C.n_vars;
    if (spec) {
        // the batched kernels keep their table and gradient in static LDS
        const size_t lds = spec_lds_bytes(0, m);
        HIP_TRY(launch_batch_plan(A, stream));
        BatchKArgs K{tape_args(t, mode, 0), A};
        void *params[] = {&K};
        HIP_TRY(hipModuleLaunchKernel(t->spec_batch_fn[rev], grid, 1, 1, block, 1, 1, (unsigned)lds, stream, params,
                                      nullptr));
        HIP_TRY(launch_batch_finish(A, m, max_nodes, stream));
        return MVF_OK;
    }
    const size_t lds = lds_bytes(t->C.n_bound, BATCH_TAB_CAP, n, m, rev && A.gacc == nullptr,
                                 spill_bytes(spill_for(t->C, chunk), chunk));
    if (lds > LDS_BUDGET - 1024) return set_err(MVF_ELIMIT, "tape and tables exceed the LDS budget");
    hipError_t e = launch_batch(tape_args(t, mode, chunk), A, chunk, rev, grid, lds, max_nodes, stream);
    if (e != hipSuccess) return hip_err(e, "launch_batch");
    return MVF_OK;
}

}  // namespace

int mvf::set_error(int code, const std::string &msg) { return set_err(code, msg); }

extern "C" {

int mvf_tape_set_root_kinds(mvf_tape *t, const int32_t *kinds) {
    if (!t) return set_err(MVF_EINVAL, "null tape");
    uint32_t ineq = 0, eq = 0;
    const int m = (int)t->C.roots.size();
    if (kinds) {
        if (kinds[0] != MVF_ROOT_FREE) return set_err(MVF_EINVAL, "root 0 is the objective (MVF_ROOT_FREE)");
        for (int r = 1; r < m; ++r) {
            if (kinds[r] == MVF_ROOT_INEQ) ineq |= 1u << r;
            else if (kinds[r] == MVF_ROOT_EQ) eq |= 1u << r;
            else if (kinds[r] != MVF_ROOT_FREE) return set_err(MVF_EINVAL, "root kind outside MVF_ROOT_*");
        }
    }
    t->ineq_mask = ineq;
    t->eq_mask = eq;
    return MVF_OK;
}

int mvf_points_workspace(const mvf_tape *t, int32_t op, int64_t B, size_t *bytes) {
    if (!t || !bytes) return set_err(MVF_EINVAL, "null argument");
    if (op < MVF_POINTS_EVAL || op > MVF_BOXES_GRAD_REV) return set_err(MVF_EINVAL, "bad op");
    PointsLayout L;
    const int rc = points_layout(t, op, std::max<int64_t>(B, 1), &L);
    if (rc != MVF_OK) return rc;
    *bytes = L.total;
    return MVF_OK;
}

int mvf_eval_points(const mvf_tape *t, int64_t B, const double *x, double *f, uint32_t *flags, void *workspace,
                    size_t workspace_bytes, hipStream_t stream) {
    if (!t || (B > 0 && (!x || !f))) return set_err(MVF_EINVAL, "null argument");
    return launch_points_op(t, PT_EVAL, B, x, nullptr, 0, f, flags, workspace, workspace_bytes, stream);
}

int mvf_vjp_points(const mvf_tape *t, int64_t B, const double *x, const double *gout, double *gx, uint32_t *flags,
                   void *workspace, size_t workspace_bytes, hipStream_t stream) {
    if (!t || (B > 0 && (!x || !gout || !gx))) return set_err(MVF_EINVAL, "null argument");
    return launch_points_op(t, PT_VJP, B, x, gout, 0, gx, flags, workspace, workspace_bytes, stream);
}

int mvf_gradient_boxes(const mvf_tape *t, int64_t B, const double *boxes, int32_t root, int32_t grad, double *G,
                       uint32_t *flags, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    if (!t || (B > 0 && (!boxes || !G))) return set_err(MVF_EINVAL, "null argument");
    if (root < 0 || root >= (int32_t)t->C.roots.size()) return set_err(MVF_EINVAL, "root out of range");
    if (grad != MVF_GRAD_FWD && grad != MVF_GRAD_REV) return set_err(MVF_EINVAL, "grad must be MVF_GRAD_FWD or MVF_GRAD_REV");
    return launch_points_op(t, grad == MVF_GRAD_FWD ? PT_GRAD_FWD : PT_GRAD_REV, B, boxes, nullptr, root, G, flags,
                            workspace, workspace_bytes, stream);
}

const char *mvf_strerror(int code) {
    switch (code) {
    case MVF_OK: return "ok";
    case MVF_EINVAL: return "invalid argument";
    case MVF_ETAPE: return "malformed tape";
    case MVF_ELIMIT: return "limit exceeded";
    case MVF_ENOMEM: return "out of device memory";
    case MVF_EHIP: return "HIP runtime error";
    case MVF_ENOTSUP: return "unsupported device";
    default: return "unknown error";
    }
}

const char *mvf_last_error(void) { return g_err.c_str(); }

int mvf_tape_check(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts, int32_t n_vars,
                   const int32_t *roots, int32_t n_roots, mvf_tape_stats *stats) {
    Compiled C;
    std::string err;
    int rc = compile_tape(nodes, n_nodes, consts, n_consts, n_vars, roots, n_roots, &C, &err);
    if (rc != MVF_OK) return set_err(rc, err);
    choose_chunk(C);
    if (stats) fill_stats(C, stats);
    return MVF_OK;
}

int mvf_tape_create(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts, int32_t n_vars,
                    const int32_t *roots, int32_t n_roots, mvf_tape **out) {
    if (!out) return set_err(MVF_EINVAL, "out is null");
    *out = nullptr;
    mvf_tape *t = new (std::nothrow) mvf_tape;
    if (!t) return set_err(MVF_ENOMEM, "host allocation failed");
    std::string err;
    int rc = compile_tape(nodes, n_nodes, consts, n_consts, n_vars, roots, n_roots, &t->C, &err);
    if (rc != MVF_OK) { delete t; return set_err(rc, err); }
    choose_chunk(t->C);
    rc = check_device(&t->n_cu);
    if (rc != MVF_OK) { delete t; return rc; }
    hipGetDevice(&t->device);
    if (lds_bytes(t->C.n_bound, BATCH_TAB_CAP, t->C.n_vars, n_roots, false) > LDS_BUDGET - 1024) {
        delete t;
        return set_err(MVF_ELIMIT, "programs and tables exceed the 160 KiB LDS budget");
    }
    const size_t bytes = t->C.instr.size() * sizeof(Instr);
    hipError_t e = hipMalloc(&t->d_prog, bytes);
    if (e != hipSuccess) { delete t; return set_err(MVF_ENOMEM, "hipMalloc of the program failed"); }
    e = hipMemcpy(t->d_prog, t->C.instr.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) { hipFree(t->d_prog); delete t; return hip_err(e, "hipMemcpy program"); }
    // the DAG with its live nodes (in some root's cone), for bound tightening
    std::vector<DagNode> dag(n_nodes);
    std::vector<uint8_t> live(n_nodes, 0);
    for (int r = 0; r < n_roots; ++r) live[roots[r]] = 1;
    for (int i = n_nodes - 1; i >= 0; --i) {
        dag[i] = DagNode{nodes[i].op, nodes[i].a, nodes[i].b, live[i]};
        if (!live[i] || nodes[i].op == MVF_VAR || nodes[i].op == MVF_CONST) continue;
        live[nodes[i].a] = 1;
        if (nodes[i].op <= MVF_DIV) live[nodes[i].b] = 1;
    }
    for (int i = 0; i < n_nodes; ++i) dag[i].live = live[i];
    t->n_nodes = n_nodes;
    const size_t nc = std::max<int32_t>(n_consts, 1);
    if (hipMalloc(&t->d_nodes, (size_t)n_nodes * sizeof(DagNode)) != hipSuccess ||
        hipMalloc(&t->d_roots, (size_t)n_roots * 4) != hipSuccess || hipMalloc(&t->d_consts, nc * 8) != hipSuccess ||
        hipMemcpy(t->d_nodes, dag.data(), (size_t)n_nodes * sizeof(DagNode), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t->d_roots, roots, (size_t)n_roots * 4, hipMemcpyHostToDevice) != hipSuccess ||
        (n_consts > 0 && hipMemcpy(t->d_consts, consts, (size_t)n_consts * 8, hipMemcpyHostToDevice) != hipSuccess)) {
        mvf_tape_destroy(t);
        return set_err(MVF_ENOMEM, "device copy of the DAG failed");
    }
    *out = t;
    return MVF_OK;
}

int mvf_tape_stats_get(const mvf_tape *t, mvf_tape_stats *stats) {
    if (!t || !stats) return set_err(MVF_EINVAL, "null argument");
    fill_stats(t->C, stats);
    return MVF_OK;
}

int mvf_tape_destroy(mvf_tape *t) {
    if (!t) return MVF_OK;
    if (t->spec_mod) hipModuleUnload(t->spec_mod);
    if (t->d_prog) hipFree(t->d_prog);
    hipFree(t->d_nodes);
    hipFree(t->d_roots);
    hipFree(t->d_consts);
    delete t;
    return MVF_OK;
}

int mvf_bound_workspace(const mvf_tape *t, const int32_t *splits, int32_t mode, int32_t grad, size_t *bytes) {
    if (!t || !bytes) return set_err(MVF_EINVAL, "null argument");
    int64_t S;
    int tt;
    int rc = check_splits(t, splits, &S, &tt);
    if (rc != MVF_OK) return rc;
    bool rev;
    int chunk;
    rc = resolve_grad(t, mode, grad, nullptr, &rev, &chunk);
    if (rc != MVF_OK) return rc;
    *bytes = single_layout(t, single_grid(t, S, rev), rev, tt, rec_per_lane(t)).total;
    return MVF_OK;
}

namespace {
// mvf_bound with the workspace given as (ws, ws_bytes); engine_rec: size the
// reverse-mode region for the kernel that runs (else for either, as
// mvf_bound_workspace does)
int bound_impl(const mvf_tape *t, const mvf_bound_args *a, void *ws, size_t ws_bytes, bool engine_rec,
               hipStream_t stream) {
    if (!t || !a) return set_err(MVF_EINVAL, "null argument");
    if (!a->box || !a->reduced || !ws) return set_err(MVF_EINVAL, "box, reduced and workspace are required");
    if (a->mode < MVF_MODE_NIE || a->mode > MVF_MODE_BOTH) return set_err(MVF_EINVAL, "bad mode");
    if (a->grad < MVF_GRAD_FWD || a->grad > MVF_GRAD_AUTO) return set_err(MVF_EINVAL, "bad grad");
    if (a->engine < MVF_ENGINE_AUTO || a->engine > MVF_ENGINE_SPEC) return set_err(MVF_EINVAL, "bad engine");
    int64_t S;
    int tt;
    int rc = check_splits(t, a->splits, &S, &tt);
    if (rc != MVF_OK) return rc;
    bool rev;
    int chunk;
    rc = resolve_grad(t, a->mode, a->grad, a->tuning, &rev, &chunk);
    if (rc != MVF_OK) return rc;
    if (a->engine == MVF_ENGINE_SPEC && !t->spec_fn[rev])
        return set_err(MVF_EINVAL, "no specialised kernel for this gradient mode: see mvf_tape_specialize");
    const int m = (int)t->C.roots.size(), n = t->C.n_vars;
    // the specialised kernel, unless the caller asks for the interpreter, or
    // leaves the choice and the kernel's tables and LDS gradient would not fit
    bool spec = t->spec_fn[rev] && a->engine != MVF_ENGINE_INTERP;
    if (spec && a->engine == MVF_ENGINE_AUTO && spec_lds_bytes(tt, m, rev ? t->spec_gl : 0) > LDS_BUDGET - 1024)
        spec = false;
    const int grid = single_grid(t, S, rev);
    const size_t rec_lane = engine_rec ? (size_t)(spec ? t->spec_ck : t->C.max_rec) : rec_per_lane(t);
    const SingleLayout L = single_layout(t, grid, rev, tt, rec_lane);
    if (ws_bytes < L.total)
        return set_err(engine_rec ? MVF_ELIMIT : MVF_EINVAL,
                       "workspace too small: the call needs " + std::to_string(L.total) + " bytes, " +
                           std::to_string(ws_bytes) + " given");
    const size_t lds = spec ? spec_lds_bytes(tt, m, rev ? t->spec_gl : 0)
                            : lds_bytes(t->C.n_bound, tt, n, m, rev && L.g_lds, spill_bytes(spill_for(t->C, chunk), chunk));
    if (lds > LDS_BUDGET - 1024) return set_err(MVF_ELIMIT, "tape and tables exceed the LDS budget");

    const TapeArgs T = tape_args(t, a->mode, chunk);
    BoxArgs B;
    std::memset(&B, 0, sizeof B);
    B.tab_off[0] = 0;
    for (int i = 0; i < n; ++i) {
        B.splits[i] = a->splits[i];
        B.tab_off[i + 1] = B.tab_off[i] + a->splits[i];
    }
    B.box = a->box;
    B.S = S;
    B.per_sub = a->per_sub;
    B.flags = a->flags;
    B.reduced = a->reduced;
    B.argmin = a->argmin;
    uint8_t *w = static_cast<uint8_t *>(ws);
    B.partial = reinterpret_cast<double *>(w + L.partial);
    B.partial_lo0 = reinterpret_cast<double *>(w + L.lo0);
    B.partial_k = reinterpret_cast<int64_t *>(w + L.k);
    B.partial_ext = reinterpret_cast<double *>(w + L.ext);
    B.extra = a->extra;
    B.rec = reinterpret_cast<double2 *>(w + L.rec);
    B.rec_lane = (int64_t)rec_lane;
    B.gacc = rev && !L.g_lds ? reinterpret_cast<double2 *>(w + L.gacc) : nullptr;
    if (a->kernel_events[0]) HIP_TRY(hipEventRecord(a->kernel_events[0], stream));
    if (spec) {
        BoundKArgs K{T, B};
        void *params[] = {&K};
        hipError_t e =
            hipModuleLaunchKernel(t->spec_fn[rev], grid, 1, 1, BLK, 1, 1, (unsigned)lds, stream, params, nullptr);
        if (e != hipSuccess) return hip_err(e, "hipModuleLaunchKernel (specialised kernel)");
        if (a->kernel_events[1]) HIP_TRY(hipEventRecord(a->kernel_events[1], stream));
        e = launch_finish(B, grid, m, stream);
        if (e != hipSuccess) return hip_err(e, "finish kernel");
        return MVF_OK;
    }
    hipError_t e = launch_bound(T, B, chunk, rev, grid, lds, stream, a->kernel_events[1]);
    if (e != hipSuccess) return hip_err(e, "launch_bound");
    return MVF_OK;
}
}  // namespace

int mvf_bound(const mvf_tape *t, const mvf_bound_args *a, hipStream_t stream) {
    if (!a) return set_err(MVF_EINVAL, "null argument");
    return bound_impl(t, a, a->workspace, a->workspace_bytes, false, stream);
}

int mvf_bound_noalloc(const mvf_tape *t, const mvf_bound_args *a, hipStream_t stream) {
    if (!t || !a) return set_err(MVF_EINVAL, "null argument");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != t->device) return set_err(MVF_EINVAL, "the current device is not the tape's device");
    void *scratch = nullptr;
    HIP_TRY(noalloc_scratch(dev, &scratch));
    return bound_impl(t, a, scratch, MVF_NOALLOC_SCRATCH_BYTES, true, stream);
}

int mvf_fbbt_workspace(const mvf_tape *t, int64_t n_boxes, size_t *bytes) {
    if (!t || !bytes || n_boxes < 0) return set_err(MVF_EINVAL, "bad argument");
    const int64_t stride = (n_boxes + 63) / 64 * 64;
    *bytes = std::max<size_t>((size_t)2 * t->n_nodes * stride * 16, 16);
    return MVF_OK;
}

int mvf_fbbt(const mvf_tape *t, int64_t n_boxes, const double *boxes, double ub, int32_t rounds, double *out,
             int32_t *status, void *workspace, size_t workspace_bytes, hipStream_t stream) {
    if (!t || n_boxes < 0 || (n_boxes > 0 && (!boxes || !out || !status || !workspace)))
        return set_err(MVF_EINVAL, "bad argument");
    if (rounds < 1 || rounds > 64) return set_err(MVF_EINVAL, "rounds outside [1, 64]");
    if (ub != ub) return set_err(MVF_EINVAL, "ub is NaN");
    size_t need = 0;
    mvf_fbbt_workspace(t, n_boxes, &need);
    if (workspace_bytes < need) return set_err(MVF_EINVAL, "workspace too small");
    FbbtArgs A;
    std::memset(&A, 0, sizeof A);
    A.nodes = t->d_nodes;
    A.consts = t->d_consts;
    A.roots = t->d_roots;
    A.n_nodes = t->n_nodes;
    A.n = t->C.n_vars;
    A.m = (int32_t)t->C.roots.size();
    A.rounds = rounds;
    A.ineq_mask = t->ineq_mask;
    A.eq_mask = t->eq_mask;
    A.ub = ub;
    A.N = n_boxes;
    A.boxes = boxes;
    A.out = out;
    A.status = status;
    A.val = static_cast<double2 *>(workspace);
    A.stride = (n_boxes + 63) / 64 * 64;
    hipError_t e = launch_fbbt(A, stream);
    if (e != hipSuccess) return hip_err(e, "fbbt kernel");
    return MVF_OK;
}

int mvf_tape_specialize(mvf_tape *t, const mvf_spec_options *opt, mvf_spec_info *info) {
    if (!t) return set_err(MVF_EINVAL, "null tape");
    if (opt && (opt->waves < 0 || opt->waves > 4)) return set_err(MVF_EINVAL, "waves out of range [0, 4]");
    int chunk;
    int64_t units;
    int rc = spec_plan(t->C, opt, &chunk, &units);
    if (rc != MVF_OK) return rc;
    const int waves = opt && opt->waves > 0 ? opt->waves : 2;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, t->device));
    std::vector<char> code;
    mvf_spec_info in{};
    bool cached = false;
    const auto t0 = std::chrono::steady_clock::now();
    const int grad = opt ? opt->grad : MVF_GRAD_FWD;
    const int budget = spec_ckpt_budget(t->C, opt, waves);
    int ck = 0;
    const int gl = grad == MVF_GRAD_FWD ? 0 : spec_gl_count(t->C, waves);    // the generator's N_GL
    const std::string src =
        spec_source(t->C, chunk, waves, grad, budget, spec_ckpt_min_records(t->C, opt, waves), &ck, &units);
    // the target without its feature suffix (":sramecc+:xnack-"): one code object
    // for either setting, and the same cache key on every gfx950
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    rc = spec_compile(src, arch, opt && opt->use_cache, code, &cached, &in.seconds);
    if (rc != MVF_OK) return rc;
    hipModule_t mod = nullptr;
    HIP_TRY(hipModuleLoadData(&mod, code.data()));
    hipFunction_t fns[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};    // [rev][batched]
    const char *names[2][2] = {{"mvf_spec_bound", "mvf_spec_batch"}, {"mvf_spec_bound_rev", "mvf_spec_batch_rev"}};
    hipError_t e = hipSuccess;
    for (int r = 0; r < 2 && e == hipSuccess; ++r) {
        if ((r == 0 && grad == MVF_GRAD_REV) || (r == 1 && grad == MVF_GRAD_FWD)) continue;
        for (int b = 0; b < 2 && e == hipSuccess; ++b) e = hipModuleGetFunction(&fns[r][b], mod, names[r][b]);
    }
    if (e != hipSuccess) {
        hipModuleUnload(mod);
        return hip_err(e, "hipModuleGetFunction");
    }
    if (t->spec_mod) hipModuleUnload(t->spec_mod);
    t->spec_mod = mod;
    t->spec_ck = grad == MVF_GRAD_FWD ? 0 : ck;
    t->spec_gl = gl;
    {
        static std::atomic<uint64_t> serial{0};
        t->spec_id = ++serial;
    }
    for (int r = 0; r < 2; ++r) {
        t->spec_fn[r] = fns[r][0];
        t->spec_batch_fn[r] = fns[r][1];
    }
    in.chunk = chunk;
    in.waves = waves;
    in.grad = grad;
    in.code_units = units;
    in.code_bytes = (int64_t)code.size();
    in.from_cache = cached ? 1 : 0;
    in.ckpt_budget = budget;
    in.ckpt_intervals = t->spec_ck;
    in.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    t->spec_info = in;
    if (info) *info = in;
    return MVF_OK;
}

namespace {
// compile and plan a tape, then generate its specialised source
int spec_generate(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts, int32_t n_vars,
                  const int32_t *roots, int32_t n_roots, const mvf_spec_options *opt, std::string *src,
                  mvf_spec_info *in) {
    if (opt && (opt->waves < 0 || opt->waves > 4)) return set_err(MVF_EINVAL, "waves out of range [0, 4]");
    Compiled C;
    std::string err;
    int rc = compile_tape(nodes, n_nodes, consts, n_consts, n_vars, roots, n_roots, &C, &err);
    if (rc != MVF_OK) return set_err(rc, err);
    int chunk;
    int64_t units;
    rc = spec_plan(C, opt, &chunk, &units);
    if (rc != MVF_OK) return rc;
    const int waves = opt && opt->waves > 0 ? opt->waves : 2;
    const int grad = opt ? opt->grad : MVF_GRAD_FWD;
    const int budget = spec_ckpt_budget(C, opt, waves);
    int ck = 0;
    *src = spec_source(C, chunk, waves, grad, budget, spec_ckpt_min_records(C, opt, waves), &ck, &units);
    *in = mvf_spec_info{};
    in->ckpt_budget = budget;
    in->ckpt_intervals = grad == MVF_GRAD_FWD ? 0 : ck;
    in->chunk = chunk;
    in->waves = waves;
    in->grad = grad;
    in->code_units = units;
    return MVF_OK;
}
}  // namespace

int mvf_spec_check(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts, int32_t n_vars,
                   const int32_t *roots, int32_t n_roots, const mvf_spec_options *opt, mvf_spec_info *info) {
    std::string src;
    mvf_spec_info in;
    int rc = spec_generate(nodes, n_nodes, consts, n_consts, n_vars, roots, n_roots, opt, &src, &in);
    if (rc != MVF_OK) return rc;
    std::vector<char> code;
    bool cached = false;
    rc = spec_compile(src, "gfx950", opt && opt->use_cache, code, &cached, &in.seconds);
    if (rc != MVF_OK) return rc;
    in.code_bytes = (int64_t)code.size();
    in.from_cache = cached ? 1 : 0;
    if (info) *info = in;
    return MVF_OK;
}

int mvf_spec_source(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts, int32_t n_vars,
                    const int32_t *roots, int32_t n_roots, const mvf_spec_options *opt, char *buf, size_t cap,
                    size_t *len) {
    if (!len) return set_err(MVF_EINVAL, "len is null");
    std::string src;
    mvf_spec_info in;
    int rc = spec_generate(nodes, n_nodes, consts, n_consts, n_vars, roots, n_roots, opt, &src, &in);
    if (rc != MVF_OK) return rc;
    *len = src.size();
    if (buf && cap > 0) {
        const size_t k = std::min(cap - 1, src.size());
        std::memcpy(buf, src.data(), k);
        buf[k] = '\0';
    }
    return MVF_OK;
}

int mvf_batch_workspace(const mvf_tape *t, int32_t max_nodes, int64_t max_subdomains, int32_t mode, int32_t grad,
                        const mvf_tuning *tuning, size_t *bytes) {
    if (!t || !bytes || max_nodes < 1 || max_subdomains < 1) return set_err(MVF_EINVAL, "bad argument");
    bool rev;
    int chunk;
    int rc = resolve_grad(t, mode, grad, tuning, &rev, &chunk);
    if (rc != MVF_OK) return rc;
    *bytes = batch_layout(t, max_nodes, max_subdomains, batch_grid(t, tuning), batch_block(tuning), rev).total;
    return MVF_OK;
}

int mvf_bound_batch(const mvf_tape *t, const mvf_batch_args *a, const mvf_tuning *tuning, hipStream_t stream) {
    if (!t || !a) return set_err(MVF_EINVAL, "null argument");
    if (a->n_nodes < 0 || a->n_nodes > a->max_nodes) return set_err(MVF_EINVAL, "n_nodes outside [0, max_nodes]");
    if (!a->boxes || !a->splits || !a->reduced || !a->status || !a->workspace)
        return set_err(MVF_EINVAL, "boxes, splits, reduced, status and workspace are required");
    if (a->mode < MVF_MODE_NIE || a->mode > MVF_MODE_BOTH) return set_err(MVF_EINVAL, "bad mode");
    bool rev, spec;
    int chunk;
    int rc = resolve_grad(t, a->mode, a->grad, tuning, &rev, &chunk);
    if (rc != MVF_OK) return rc;
    rc = batch_engine(t, tuning, rev, &spec);
    if (rc != MVF_OK) return rc;
    const int grid = batch_grid(t, tuning);
    BatchArgs A;
    rc = fill_batch_args(t, a->n_nodes, nullptr, a->max_nodes, a->max_subdomains, a->boxes, a->splits, a->reduced,
                         a->argmin, a->status, a->extra, a->workspace, a->workspace_bytes, grid, batch_block(tuning),
                         rev, batch_spl(tuning), &A);
    if (rc != MVF_OK) return rc;
    if (a->n_nodes == 0) return MVF_OK;
    return launch_batched(t, a->mode, chunk, rev, spec, A, grid, batch_block(tuning), a->n_nodes, stream);
}

int mvf_batch_graph_create(const mvf_tape *t, int32_t max_nodes, int64_t max_subdomains, int32_t mode, int32_t grad,
                           const mvf_tuning *tuning, hipStream_t stream, mvf_batch_graph **out) {
    if (!t || !out || max_nodes < 1 || max_subdomains < 1) return set_err(MVF_EINVAL, "bad argument");
    *out = nullptr;
    bool rev, spec;
    int chunk;
    int rc = resolve_grad(t, mode, grad, tuning, &rev, &chunk);
    if (rc != MVF_OK) return rc;
    rc = batch_engine(t, tuning, rev, &spec);
    if (rc != MVF_OK) return rc;
    mvf_batch_graph *g = new (std::nothrow) mvf_batch_graph;
    if (!g) return set_err(MVF_ENOMEM, "host allocation failed");
    g->tape = t;
    g->max_nodes = max_nodes;
    g->max_subdomains = max_subdomains;
    g->mode = mode;
    g->grad = rev ? MVF_GRAD_REV : MVF_GRAD_FWD;
    if (tuning) g->tuning = *tuning;
    g->tuning.grad = g->grad;
    g->tuning.chunk = chunk;
    g->tuning.grid_blocks = batch_grid(t, tuning);
    g->tuning.sub_per_lane = batch_spl(tuning);
    g->tuning.engine = spec ? MVF_ENGINE_SPEC : MVF_ENGINE_INTERP;
    g->tuning.block = batch_block(tuning);
    const int n = t->C.n_vars, m = (int)t->C.roots.size();
    const int grid = g->tuning.grid_blocks;
    g->ws_bytes = batch_layout(t, max_nodes, max_subdomains, grid, g->tuning.block, rev).total;
    auto fail = [&](int code, const char *what) {
        mvf_batch_graph_destroy(g);
        return set_err(code, what);
    };
    if (hipMalloc(&g->d_ws, g->ws_bytes) != hipSuccess) return fail(MVF_ENOMEM, "hipMalloc workspace");
    if (hipMalloc(&g->d_boxes, (size_t)max_nodes * n * 2 * 8) != hipSuccess ||
        hipMalloc(&g->d_splits, (size_t)max_nodes * n * 4) != hipSuccess ||
        hipMalloc(&g->d_count, 4) != hipSuccess || hipMalloc(&g->d_status, (size_t)max_nodes * 4) != hipSuccess ||
        hipMalloc(&g->d_reduced, (size_t)max_nodes * m * 2 * 8) != hipSuccess ||
        hipMalloc(&g->d_extra, (size_t)max_nodes * 2 * 8) != hipSuccess ||
        hipMalloc(&g->d_argmin, (size_t)max_nodes * 8) != hipSuccess)
        return fail(MVF_ENOMEM, "hipMalloc node buffers");
    if (hipHostMalloc(reinterpret_cast<void **>(&g->h_boxes), (size_t)max_nodes * n * 2 * 8, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&g->h_splits), (size_t)max_nodes * n * 4, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&g->h_count), 4, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&g->h_status), (size_t)max_nodes * 4, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&g->h_reduced), (size_t)max_nodes * m * 2 * 8,
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&g->h_argmin), (size_t)max_nodes * 8, hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc(reinterpret_cast<void **>(&g->h_extra), (size_t)max_nodes * 2 * 8, hipHostMallocDefault) !=
            hipSuccess)
        return fail(MVF_ENOMEM, "hipHostMalloc staging");
    std::memset(g->h_boxes, 0, (size_t)max_nodes * n * 2 * 8);
    for (size_t i = 0; i < (size_t)max_nodes * n; ++i) g->h_splits[i] = 1;
    *g->h_count = 0;

    BatchArgs A;
    rc = fill_batch_args(t, 0, g->d_count, max_nodes, max_subdomains, g->d_boxes, g->d_splits, g->d_reduced,
                         g->d_argmin, g->d_status, g->d_extra, g->d_ws, g->ws_bytes, grid, g->tuning.block, rev,
                         g->tuning.sub_per_lane, &A);
    if (rc != MVF_OK) { mvf_batch_graph_destroy(g); return rc; }
    if (!spec && lds_bytes(t->C.n_bound, BATCH_TAB_CAP, n, m, rev && A.gacc == nullptr,
                           spill_bytes(spill_for(t->C, chunk), chunk)) > LDS_BUDGET - 1024) {
        mvf_batch_graph_destroy(g);
        return set_err(MVF_ELIMIT, "LDS budget");
    }
    (void)stream;
    hipStream_t cs = nullptr;                    // private capture stream, default priority
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return fail(MVF_EHIP, "hipStreamCreate");
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        hipStreamDestroy(cs);
        return fail(MVF_EHIP, "hipStreamBeginCapture");
    }
    bool ok = hipMemcpyAsync(g->d_count, g->h_count, 4, hipMemcpyHostToDevice, cs) == hipSuccess &&
              hipMemcpyAsync(g->d_boxes, g->h_boxes, (size_t)max_nodes * n * 2 * 8, hipMemcpyHostToDevice, cs) ==
                  hipSuccess &&
              hipMemcpyAsync(g->d_splits, g->h_splits, (size_t)max_nodes * n * 4, hipMemcpyHostToDevice, cs) ==
                  hipSuccess;
    ok = ok && launch_batched(t, mode, chunk, rev, spec, A, grid, g->tuning.block, max_nodes, cs) == MVF_OK;
    ok = ok && hipMemcpyAsync(g->h_reduced, g->d_reduced, (size_t)max_nodes * m * 2 * 8, hipMemcpyDeviceToHost, cs) ==
                   hipSuccess &&
         hipMemcpyAsync(g->h_argmin, g->d_argmin, (size_t)max_nodes * 8, hipMemcpyDeviceToHost, cs) == hipSuccess &&
         hipMemcpyAsync(g->h_status, g->d_status, (size_t)max_nodes * 4, hipMemcpyDeviceToHost, cs) == hipSuccess &&
         hipMemcpyAsync(g->h_extra, g->d_extra, (size_t)max_nodes * 2 * 8, hipMemcpyDeviceToHost, cs) == hipSuccess;
    hipError_t ee = hipStreamEndCapture(cs, &g->graph);
    hipStreamDestroy(cs);
    if (!ok || ee != hipSuccess) return fail(MVF_EHIP, "graph capture failed");
    if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
        return fail(MVF_EHIP, "hipGraphInstantiate");
    if (hipEventCreateWithFlags(&g->done, hipEventDisableTiming) != hipSuccess) return fail(MVF_EHIP, "hipEventCreate");
    *out = g;
    return MVF_OK;
}

int mvf_batch_graph_staging(mvf_batch_graph *g, double **boxes, int32_t **splits) {
    if (!g || !boxes || !splits) return set_err(MVF_EINVAL, "null argument");
    *boxes = g->h_boxes;
    *splits = g->h_splits;
    return MVF_OK;
}

int mvf_batch_graph_launch(mvf_batch_graph *g, int32_t n_nodes, hipStream_t stream) {
    if (!g) return set_err(MVF_EINVAL, "null graph");
    if (n_nodes < 0 || n_nodes > g->max_nodes) return set_err(MVF_EINVAL, "n_nodes outside [0, max_nodes]");
    const int n = g->tape->C.n_vars;
    int64_t total = 0;
    for (int32_t i = 0; i < n_nodes; ++i) {
        int64_t S = 1;
        for (int j = 0; j < n; ++j) {
            const int32_t s = g->h_splits[(size_t)i * n + j];
            if (s < 1 || s > 65535) return set_err(MVF_EINVAL, "split count outside [1, 65535]");
            if (S > (INT64_C(1) << 40) / s) return set_err(MVF_ELIMIT, "node with more than 2^40 subdomains");
            S *= s;
        }
        total += S;
    }
    if (total > g->max_subdomains) return set_err(MVF_ELIMIT, "total subdomains above the graph's capacity");
    // the count sits in pinned memory that the previous replay's first copy reads
    if (g->launched) HIP_TRY(hipEventSynchronize(g->done));
    *g->h_count = n_nodes;
    HIP_TRY(hipGraphLaunch(g->exec, stream));
    HIP_TRY(hipEventRecord(g->done, stream));
    g->launched = true;
    return MVF_OK;
}

int mvf_batch_graph_wait(mvf_batch_graph *g) {
    if (!g) return set_err(MVF_EINVAL, "null graph");
    if (g->launched) HIP_TRY(hipEventSynchronize(g->done));
    return MVF_OK;
}

int mvf_batch_graph_result(mvf_batch_graph *g, const double **reduced, const int64_t **argmin,
                           const int32_t **status, const double **extra) {
    if (!g) return set_err(MVF_EINVAL, "null graph");
    if (reduced) *reduced = g->h_reduced;
    if (argmin) *argmin = g->h_argmin;
    if (status) *status = g->h_status;
    if (extra) *extra = g->h_extra;
    return MVF_OK;
}

int mvf_batch_graph_destroy(mvf_batch_graph *g) {
    if (!g) return MVF_OK;
    if (g->done) hipEventDestroy(g->done);
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    hipFree(g->d_ws);
    hipFree(g->d_boxes);
    hipFree(g->d_splits);
    hipFree(g->d_count);
    hipFree(g->d_status);
    hipFree(g->d_reduced);
    hipFree(g->d_argmin);
    hipFree(g->d_extra);
    hipHostFree(g->h_extra);
    hipHostFree(g->h_boxes);
    hipHostFree(g->h_splits);
    hipHostFree(g->h_count);
    hipHostFree(g->h_status);
    hipHostFree(g->h_reduced);
    hipHostFree(g->h_argmin);
    delete g;
    return MVF_OK;
}

int64_t mvf_adaptive_splits(int32_t n, const double *widths, int64_t budget, int32_t *splits) {
    if (n < 1 || !widths || !splits || budget < 1) return set_err(MVF_EINVAL, "bad argument");
    int64_t N = 1;
    for (;;) {                                   // largest uniform N with N^n <= budget
        int64_t p = 1;
        bool over = false;
        for (int i = 0; i < n && !over; ++i) {
            p *= (N + 1);
            over = p > budget;
        }
        if (over) break;
        ++N;
    }
    int64_t count = 1;
    for (int i = 0; i < n; ++i) { splits[i] = (int32_t)N; count *= N; }
    for (;;) {                                   // +1 on the relatively widest dimension while it fits
        int best = 0;
        for (int i = 1; i < n; ++i)
            if (widths[i] / splits[i] > widths[best] / splits[best]) best = i;
        const int64_t next = count / splits[best] * (splits[best] + 1);
        if (next > budget) break;
        count = next;
        splits[best] += 1;
    }
    return count;
}

int64_t mvf_splits(int32_t rule, int32_t n, const double *widths, int64_t budget, int32_t *splits) {
    if (rule == MVF_SPLITS_ADAPTIVE) return mvf_adaptive_splits(n, widths, budget, splits);
    if (rule != MVF_SPLITS_DOUBLING) return set_err(MVF_EINVAL, "unknown split rule");
    if (n < 1 || !widths || !splits || budget < 1) return set_err(MVF_EINVAL, "bad argument");
    int64_t count = 1;
    for (int i = 0; i < n; ++i) splits[i] = 1;
    while (count * 2 <= budget) {
        int best = -1;                            // a split count stays <= 65535
        for (int i = 0; i < n; ++i)
            if (splits[i] <= 32767 && (best < 0 || widths[i] / splits[i] > widths[best] / splits[best])) best = i;
        if (best < 0) break;
        splits[best] *= 2;
        count *= 2;
    }
    return count;
}

int mvf_autotune_splits(const mvf_tape *t, int32_t n_nodes, const double *boxes, int64_t budget, int32_t mode,
                        int32_t grad, int32_t *rule, int32_t better_nodes[2], hipStream_t stream) {
    if (!t || n_nodes < 1 || !boxes || budget < 1 || !rule) return set_err(MVF_EINVAL, "bad argument");
    const int n = t->C.n_vars, m = (int)t->C.roots.size();
    std::vector<int32_t> sp[2];
    std::vector<double> widths(n);
    int64_t total[2] = {0, 0};
    for (int r = 0; r < 2; ++r) {
        sp[r].resize((size_t)n_nodes * n);
        for (int q = 0; q < n_nodes; ++q) {
            for (int i = 0; i < n; ++i) widths[i] = boxes[((size_t)q * n + i) * 2 + 1] - boxes[((size_t)q * n + i) * 2];
            const int64_t c = mvf_splits(r, n, widths.data(), budget, &sp[r][(size_t)q * n]);
            if (c < 1) return c < 0 ? (int)c : set_err(MVF_EINVAL, "partitioning failed");
            total[r] += c;
        }
    }
    const int64_t cap = std::max(total[0], total[1]);
    size_t ws_bytes = 0;
    int rc = mvf_batch_workspace(t, n_nodes, cap, mode, grad, nullptr, &ws_bytes);
    if (rc != MVF_OK) return rc;
    void *ws = nullptr;
    double *d_boxes = nullptr, *d_red = nullptr, *d_ex = nullptr;
    int32_t *d_splits = nullptr, *d_st = nullptr;
    auto cleanup = [&]() {
        hipFree(ws);
        hipFree(d_boxes);
        hipFree(d_red);
        hipFree(d_ex);
        hipFree(d_splits);
        hipFree(d_st);
    };
    if (hipMalloc(&ws, ws_bytes) != hipSuccess || hipMalloc(&d_boxes, (size_t)n_nodes * n * 16) != hipSuccess ||
        hipMalloc(&d_red, (size_t)n_nodes * m * 16) != hipSuccess || hipMalloc(&d_ex, (size_t)n_nodes * 16) != hipSuccess ||
        hipMalloc(&d_splits, (size_t)n_nodes * n * 4) != hipSuccess || hipMalloc(&d_st, (size_t)n_nodes * 4) != hipSuccess) {
        cleanup();
        return set_err(MVF_ENOMEM, "split tuning buffers");
    }
    std::vector<double> lb[2];
    hipError_t e = hipMemcpyAsync(d_boxes, boxes, (size_t)n_nodes * n * 16, hipMemcpyHostToDevice, stream);
    for (int r = 0; r < 2 && e == hipSuccess && rc == MVF_OK; ++r) {
        e = hipMemcpyAsync(d_splits, sp[r].data(), (size_t)n_nodes * n * 4, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) break;
        mvf_batch_args a{};
        a.n_nodes = n_nodes;
        a.max_nodes = n_nodes;
        a.max_subdomains = cap;
        a.boxes = d_boxes;
        a.splits = d_splits;
        a.mode = mode;
        a.grad = grad;
        a.reduced = d_red;
        a.status = d_st;
        a.workspace = ws;
        a.workspace_bytes = ws_bytes;
        a.extra = d_ex;
        rc = mvf_bound_batch(t, &a, nullptr, stream);
        if (rc != MVF_OK) break;
        std::vector<double> ex((size_t)n_nodes * 2);
        e = hipMemcpyAsync(ex.data(), d_ex, ex.size() * 8, hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        lb[r].resize(n_nodes);
        for (int q = 0; q < n_nodes; ++q) lb[r][q] = ex[2 * (size_t)q];
    }
    cleanup();
    if (rc != MVF_OK) return rc;
    if (e != hipSuccess) return hip_err(e, "split tuning");
    int better[2] = {0, 0};
    for (int q = 0; q < n_nodes; ++q) {
        if (lb[0][q] > lb[1][q]) ++better[0];
        if (lb[1][q] > lb[0][q]) ++better[1];
    }
    *rule = better[1] > better[0] ? MVF_SPLITS_DOUBLING : MVF_SPLITS_ADAPTIVE;
    if (better_nodes) {
        better_nodes[0] = better[0];
        better_nodes[1] = better[1];
    }
    return MVF_OK;
}

namespace {
// results of mvf_autotune, keyed by what determines the timing: the tape's
// programs, the device, the specialised module, the sample's size and the
// bounding mode and gradient mode
struct TuneKey {
    uint64_t tape;
    int device;
    uint64_t module;                    // the tape's specialisation (0: none)
    int32_t n_nodes, mode, grad;
    int64_t n_sub;
    bool operator<(const TuneKey &o) const {
        return std::tie(tape, device, module, n_nodes, mode, grad, n_sub) <
               std::tie(o.tape, o.device, o.module, o.n_nodes, o.mode, o.grad, o.n_sub);
    }
};
std::mutex g_tune_mu;
std::map<TuneKey, mvf_tuning> g_tune_cache;

uint64_t tape_hash(const mvf_tape *t) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    };
    mix(t->C.instr.data(), t->C.instr.size() * sizeof(Instr));
    mix(&t->C.n_vars, sizeof t->C.n_vars);
    mix(&t->ineq_mask, sizeof t->ineq_mask);
    mix(&t->eq_mask, sizeof t->eq_mask);
    return h;
}
}  // namespace

int mvf_autotune(const mvf_tape *t, int32_t n_nodes, const double *boxes, const int32_t *splits, int64_t n_sub,
                 int32_t mode, int32_t grad, mvf_tuning *out, hipStream_t stream) {
    if (!t || !out || n_nodes < 1 || !boxes || !splits || n_sub < 1) return set_err(MVF_EINVAL, "bad argument");
    if (mode < MVF_MODE_NIE || mode > MVF_MODE_BOTH) return set_err(MVF_EINVAL, "bad mode");
    if (grad < MVF_GRAD_FWD || grad > MVF_GRAD_AUTO) return set_err(MVF_EINVAL, "bad grad");
    // the gradient mode is the caller's (it decides the enclosures, hence the
    // bounds); AUTO resolves as in mvf_bound, by the reference op count
    bool rev;
    int chunk0;
    int rc = resolve_grad(t, mode, grad, nullptr, &rev, &chunk0);
    if (rc != MVF_OK) return rc;
    const int g = rev ? MVF_GRAD_REV : MVF_GRAD_FWD;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const TuneKey key{tape_hash(t), dev, t->spec_batch_fn[rev] ? t->spec_id : 0, n_nodes, mode, g, n_sub};
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        const auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *out = it->second;
            return MVF_OK;
        }
    }
    // candidates: kernel (interpreter: each tangent chunk in forward mode;
    // the specialised kernel: each workgroup size) x persistent grid (one,
    // two or four 256-lane workgroups' worth per CU) x subdomains per lane
    std::vector<mvf_tuning> kernels;
    if (!rev)
        for (int chunk = 1; chunk <= t->C.chunk; ++chunk) {
            mvf_tuning c{};
            c.grad = g;
            c.chunk = chunk;
            c.engine = MVF_ENGINE_INTERP;
            c.block = BLK;
            kernels.push_back(c);
        }
    else {
        mvf_tuning c{};
        c.grad = g;
        c.engine = MVF_ENGINE_INTERP;
        c.block = BLK;
        kernels.push_back(c);
    }
    if (t->spec_batch_fn[rev])
        for (int block : {64, 128, BLK}) {
            mvf_tuning c{};
            c.grad = g;
            c.engine = MVF_ENGINE_SPEC;
            c.block = block;
            kernels.push_back(c);
        }
    std::vector<mvf_tuning> cand;
    const int cu = t->n_cu;
    for (const mvf_tuning &kc : kernels)
        for (int mult : {1, 2, 4})
            for (int spl : {1, 2, 4}) {
                mvf_tuning c = kc;
                c.grid_blocks = mult * cu * (BLK / kc.block);
                c.sub_per_lane = spl;
                cand.push_back(c);
            }
    size_t max_ws = 0;
    for (auto &c : cand) {
        size_t b = 0;
        if (mvf_batch_workspace(t, n_nodes, n_sub, mode, c.grad, &c, &b) == MVF_OK) max_ws = std::max(max_ws, b);
    }
    void *ws = nullptr;
    double *red = nullptr;
    int32_t *st = nullptr;
    if (hipMalloc(&ws, max_ws) != hipSuccess || hipMalloc(&red, (size_t)n_nodes * t->C.roots.size() * 16) != hipSuccess ||
        hipMalloc(&st, (size_t)n_nodes * 4) != hipSuccess) {
        hipFree(ws);
        hipFree(red);
        hipFree(st);
        return set_err(MVF_ENOMEM, "autotune workspace");
    }
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    float best = 1e30f;
    int best_i = -1;
    for (size_t i = 0; i < cand.size(); ++i) {
        mvf_batch_args a{};
        a.n_nodes = n_nodes;
        a.max_nodes = n_nodes;
        a.max_subdomains = n_sub;
        a.boxes = boxes;
        a.splits = splits;
        a.mode = mode;
        a.grad = cand[i].grad;
        a.reduced = red;
        a.status = st;
        a.workspace = ws;
        a.workspace_bytes = max_ws;
        if (mvf_bound_batch(t, &a, &cand[i], stream) != MVF_OK) continue;     // warm-up; skips infeasible
        hipEventRecord(e0, stream);
        for (int rep = 0; rep < 2; ++rep) mvf_bound_batch(t, &a, &cand[i], stream);
        hipEventRecord(e1, stream);
        hipEventSynchronize(e1);
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) { best = ms; best_i = (int)i; }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    hipFree(ws);
    hipFree(red);
    hipFree(st);
    if (best_i < 0) return set_err(MVF_ELIMIT, "no feasible tuning");
    *out = cand[best_i];
    out->best_ms = best / 2;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache[key] = *out;
    return MVF_OK;
}

}  // extern "C"
