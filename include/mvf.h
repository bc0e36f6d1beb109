/*
 * mvf.h -- C ABI of the MI355X (gfx950) subdomain Mean-Value-Form bounding library.
 *
 * Method (arXiv 2507.20769): a branch-and-bound node's box is temporarily
 * split into many subdomains (Sec. 3.1 Step 1; Sec. 2.2 "splitting
 * technique", step i; Sec. 3.1.1 uniform partitioning, dimension 1 varying
 * fastest).  On every subdomain X_k each function of the problem (objective
 * first, then constraints; Sec. 3.1 NLP) is bounded in outward-rounded FP64
 * interval arithmetic (Sec. 2.2 "Interval Arithmetic", Sec. 3.2): the Natural
 * Interval Extension NIE(X_k), an interval gradient enclosure G(X_k) and the
 * Mean Value Form  f([c]) + sum_i G_i * (X_{k,i} - c_i)  (Sec. 2.2,
 * Definition "Mean Value Form"), intersected with the NIE.  The bounds are
 * then reduced to their interval hull over the subdomains (Sec. 3.1 Step 3;
 * Sec. 2.2 splitting step iii).
 *
 * Conventions
 *   - Every pointer argument documented as "device" must point to memory on
 *     the current HIP device; "host" pointers are read during the call only.
 *   - The caller owns all buffers and streams.  The library allocates device
 *     memory only inside mvf_tape_create and mvf_batch_graph_create, and frees
 *     it in the matching destroy call.
 *   - Launch entry points are asynchronous on the given stream and return
 *     after enqueueing; results are valid after the caller synchronises.
 *   - No entry point aborts or throws.  Errors are returned as negative
 *     codes; mvf_last_error() gives a thread-local message for the last
 *     failing call.  Asynchronous device faults surface at the caller's next
 *     synchronisation.
 *   - Intervals are stored as (lo, hi) pairs of doubles.
 */
#ifndef MVF_H
#define MVF_H

#ifndef __HIPCC_RTC__   /* the library's run-time-compiled kernels read the constants only */
#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>
#endif

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------- */
#define MVF_OK 0
#define MVF_EINVAL (-1)   /* bad argument (null pointer, size, mode) */
#define MVF_ETAPE (-2)    /* malformed tape */
#define MVF_ELIMIT (-3)   /* tape, dimension or subdomain count beyond a library limit */
#define MVF_ENOMEM (-4)   /* device allocation failed */
#define MVF_EHIP (-5)     /* a HIP runtime call failed (message kept) */
#define MVF_ENOTSUP (-6)  /* current device is not gfx950 */

/* ---- limits --------------------------------------------------------- */
#define MVF_MAX_VARS 64
#define MVF_MAX_ROOTS 16
#define MVF_MAX_NODES 65535
#define MVF_MAX_TABLE 4096      /* sum over dimensions of the split counts */

/* ---- tape ------------------------------------------------------------
 * A factorable function is given as a DAG in SSA order (Sec. 2.2
 * "Factorable function"; Sec. 3.2, Fig. DAG_NIE): node i may only use nodes
 * with smaller indices.  One DAG holds all functions; roots[] names them.
 *   VAR   a = variable index in [0, n_vars)
 *   CONST a = index into consts[] (finite)
 *   ADD SUB MUL DIV  z = node a (op) node b
 *   SQR SQRT EXP LOG z = op(node a)
 *   TANH SIN COS     z = op(node a)  (the activation of the paper's ANN
 *                    workloads and the trigonometric functions of its test
 *                    problems, Sec. 4; intrinsic functions of Sec. 3.2)
 * Interval extensions: + - * / sqrt correctly rounded outward; exp, log,
 * tanh, sin and cos take the library value in round-to-nearest widened
 * outward (2 ulps for exp and log, 4 for tanh, sin and cos; tanh, sin, cos
 * clamped to [-1, 1]); sin and cos reach +-1 where the argument interval may
 * contain an extremum (2 k pi + pi/2 ... tested in outward-rounded interval
 * arithmetic with a two-double enclosure of pi), and are [-1, 1] on
 * intervals of width 6.28 or more.
 */
enum { MVF_VAR = 0, MVF_CONST = 1, MVF_ADD = 2, MVF_SUB = 3, MVF_MUL = 4, MVF_DIV = 5,
       MVF_SQR = 6, MVF_SQRT = 7, MVF_EXP = 8, MVF_LOG = 9, MVF_TANH = 10, MVF_SIN = 11, MVF_COS = 12 };

typedef struct { int32_t op, a, b; } mvf_node;
typedef struct mvf_tape mvf_tape;

/* Bound kind per subdomain: NIE only, MVF only, or MVF intersected with NIE. */
enum { MVF_MODE_NIE = 0, MVF_MODE_MVF = 1, MVF_MODE_BOTH = 2 };
/* Interval gradient: tangent (forward) mode, reverse-mode adjoint, or library choice. */
enum { MVF_GRAD_FWD = 0, MVF_GRAD_REV = 1, MVF_GRAD_AUTO = 2 };

/*
 * Validate the tape (SSA order, opcodes, operand ranges, finite constants,
 * roots), compile one register program per root (its cone in index order,
 * with slots assigned by linear-scan liveness), choose the tangent chunk,
 * plan the adjoint's checkpoints (reported by mvf_tape_stats_get) and upload
 * the programs to the current device.  Host arrays are copied; the library
 * owns *out.
 * Returns MVF_ETAPE for a malformed tape, MVF_ELIMIT when a limit above is
 * exceeded or a root needs more register slots than the slot file holds.
 */
int mvf_tape_create(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts,
                    int32_t n_vars, const int32_t *roots, int32_t n_roots, mvf_tape **out);

/* Same validation and compilation without touching any device (host only). */
typedef struct {
    int32_t n_vars, n_roots;
    int32_t n_instr;          /* total instructions over all root programs */
    int32_t max_slots;        /* largest live set of any root program */
    int32_t tangent_chunk;    /* tangent components carried per forward pass (0: forward mode unavailable) */
    int32_t max_records;      /* reverse-mode tape records per subdomain (largest root program) */
    /* Reference (algorithmic) FP64 op counts per subdomain: values, tangents
     * and the centre pass once per node of the union of the root cones (a
     * node several roots share counts once), an adjoint sweep per root over
     * its own cone, the mean value forms and Step 1. */
    int64_t ref_ops_fwd;      /* forward mode */
    int64_t ref_ops_rev;      /* reverse mode */
    int64_t ref_ops_fwd_sparse;   /* forward mode without the structurally zero tangent components
                                     (what the specialised kernels compute) */
    /* the checkpoint plan of the specialised adjoint (Sec. 3.2's DAG in
     * reverse), at the library's segment budget for two waves per SIMD: */
    int32_t ckpt_segments;    /* segments over all roots (a root kept in one pass counts one) */
    int32_t ckpt_stored;      /* checkpoint intervals the value pass stores per subdomain */
    int32_t ckpt_loaded;      /* checkpoint intervals the reverse sweep loads per subdomain */
} mvf_tape_stats;
int mvf_tape_check(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts,
                   int32_t n_vars, const int32_t *roots, int32_t n_roots, mvf_tape_stats *stats);

int mvf_tape_stats_get(const mvf_tape *tape, mvf_tape_stats *stats);

/*
 * Root kinds of the NLP min f s.t. g_i <= 0, h_j = 0 (Sec. 3.1): root 0 is the
 * objective; every other root is unconstrained (FREE), an inequality g <= 0
 * or an equality h = 0.  kinds [m] host, NULL resets every root to FREE.
 * The kinds feed the two bounds a branch-and-bound needs besides the hulls
 * (the `extra` outputs below); they are read when a call is made (a batch
 * graph keeps the kinds it was created with).
 */
enum { MVF_ROOT_FREE = 0, MVF_ROOT_INEQ = 1, MVF_ROOT_EQ = 2 };
int mvf_tape_set_root_kinds(mvf_tape *tape, const int32_t *kinds);
int mvf_tape_destroy(mvf_tape *tape);

/* ---- bounding one box ----------------------------------------------- */
typedef struct {
    const double *box;        /* device [n][2]: lo_i, hi_i with lo_i <= hi_i */
    const int32_t *splits;    /* host [n]: split count s_i >= 1 per dimension */
    int32_t mode;             /* MVF_MODE_* */
    int32_t grad;             /* MVF_GRAD_* */
    double *reduced;          /* device [m][2]: hull of the subdomain bounds of each root */
    int64_t *argmin;          /* device [1] or NULL: smallest k attaining reduced[0][0] */
    double *per_sub;          /* device [m][2][S] or NULL: bounds of every subdomain */
    uint32_t *flags;          /* device [S] or NULL: 1 where a domain violation or NaN
                                 made every bound of that subdomain [-inf, +inf] */
    void *workspace;          /* device scratch of mvf_bound_workspace() bytes */
    size_t workspace_bytes;
    const struct mvf_tuning *tuning;   /* NULL, or a gradient mode and tangent chunk to use
                                          (grid_blocks is ignored here) */
    double *extra;            /* device [2] or NULL: (0) the objective's lower bound over the
                                 subdomains that no constraint proves infeasible (an inequality
                                 with lower bound > 0, an equality bound without 0), +inf when
                                 every subdomain is infeasible; (1) the least upper bound hi(f(c_k))
                                 over centres whose inequality enclosures are all <= 0 (no
                                 equality roots, MVF modes only), else +inf (Sec. 3.1, the
                                 feasibility check; the centres are rigorously feasible points) */
    int32_t engine;           /* MVF_ENGINE_*: the interpreter or the tape's specialised kernel */
    hipEvent_t kernel_events[2];  /* NULL, or two events that the call records on its stream right
                                     before the bounding kernel and right after it, ahead of the
                                     one-block reduction kernel: the bounding kernel's own duration
                                     (hipEventElapsedTime) for profiling; the caller owns them */
} mvf_bound_args;

/* Kernel choice of mvf_bound: AUTO runs the tape's specialised kernel for the
 * call's gradient mode (NIE calls: the tangent-mode one) when
 * mvf_tape_specialize has built it, else the interpreter; INTERP always the
 * interpreter; SPEC the specialised kernel, or MVF_EINVAL when there is none.
 * Both kernels give the same bits. */
enum { MVF_ENGINE_AUTO = 0, MVF_ENGINE_INTERP = 1, MVF_ENGINE_SPEC = 2 };

/*
 * Subdomain k (0 <= k < S = prod s_i) has indices j_i = (k / prod_{l<i} s_l) mod s_i
 * and box X_{k,i} = [b_{i,j_i}, b_{i,j_i+1}] with breakpoints b_{i,0} = lo_i,
 * b_{i,s_i} = hi_i, b_{i,j} = min(hi_i, RN(lo_i + RN(j * RN(RN(hi_i - lo_i) / s_i))));
 * centre c_i = RN(0.5 * RN(b_lo + b_hi)).
 * Workspace bytes needed by mvf_bound for this tape and these splits.
 */
int mvf_bound_workspace(const mvf_tape *tape, const int32_t *splits, int32_t mode, int32_t grad,
                        size_t *bytes);
/*
 * Bound every subdomain of one box.  grad selects the interval gradient of
 * the MVF: MVF_GRAD_FWD = tangent mode (the paper's choice, Sec. 3.2),
 * MVF_GRAD_REV = reverse-mode interval adjoint (per-lane tape of local
 * partials in the workspace), MVF_GRAD_AUTO = the cheaper of the two by the
 * reference op count.  Returns MVF_ELIMIT when the forward mode is asked for
 * a tape whose live set leaves no room for tangent components.
 */
int mvf_bound(const mvf_tape *tape, const mvf_bound_args *args, hipStream_t stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mvf_bound
 * without a workspace.  The same kernels and the same bits as mvf_bound;
 * args->workspace and args->workspace_bytes are ignored and the call's
 * scratch (per-workgroup partial results; the adjoint's checkpoints or
 * records) lives in a file-scope device array of MVF_NOALLOC_SCRATCH_BYTES
 * that each GPU the library runs on holds until the process ends.  The
 * caller still owns args->box, reduced, argmin, per_sub, flags and extra.
 * Calls that need more scratch than the array holds return MVF_ELIMIT with
 * the size they need (in practice: tangent mode and the NIE at any size, the
 * adjoint only when its checkpoints or records are small).  Nothing is
 * allocated, and no allocating library routine is called; the tape must
 * belong to the current device (else MVF_EINVAL).  Every call on a GPU shares
 * that GPU's array: calls that overlap on one device (two streams, or a call
 * before the previous one's kernels have finished on another stream) race
 * and must not be issued.  Nothing in the array needs clearing between
 * calls: every kernel writes what it later reads.
 */
#define MVF_NOALLOC_SCRATCH_BYTES (8u << 20)
int mvf_bound_noalloc(const mvf_tape *tape, const mvf_bound_args *args, hipStream_t stream);

/* ---- specialised kernels ---------------------------------------------
 * The interpreter kernels evaluate the DAG node by node (the single-kernel
 * evaluation of Sec. 3.2), decoding every instruction at run time.
 * mvf_tape_specialize generates straight-line device code of the tape's root
 * programs instead (per root: the point pass at the centre, the NIE value
 * pass, and tangent passes of `chunk` gradient components, or the value pass
 * with its local partials followed by the reverse-mode adjoint sweep; the MVF
 * combine of Sec. 2.2 and the Step 3 reduction as in the interpreter),
 * single-box and batched, compiles it at
 * run time with hiprtc for the current device and keeps the loaded module in
 * the tape.  Each operation gives the interpreter's result for it, in the
 * same order, so the bounds are bitwise identical (up to the sign of zero
 * endpoints); no instruction is decoded or dispatched at run time.  Where the
 * generator knows more than the interpreter it takes a cheaper form of the
 * same result: one-sided products and quotients where a factor or divisor is
 * known nonnegative (squares, roots, exp, derivative factors of sqrt, exp,
 * log and tanh, sums and products of such values, positive constants) on
 * every subdomain whose bounds are kept, two products per end where a factor
 * is degenerate (a variable at the centre) or straddles zero (X - c in the
 * mean value form).  Tangent components that are structurally zero (a
 * node that does not depend on the component's variable) are neither stored
 * nor computed: with finite enclosures this changes at most the sign of zero
 * endpoints; where a dense product of such a zero with an enclosure unbounded
 * on both sides would give NaN, the exact zero is kept.  The default chunk is
 * the largest whose live values and nonzero components (estimated per pass)
 * stay within about 100 intervals.  Compilation takes seconds to a minute,
 * about linear in the generated size (code_units = sum over roots of program
 * length x passes, the adjoint counting two, plus the recomputed segments of
 * the checkpointed adjoint); MVF_ELIMIT above max_code.  With use_cache the code
 * object is kept under $MVF_SPEC_CACHE (default: _spec_cache/ in the directory
 * of libmvf.so itself; "off" disables) keyed by a hash of the source, options and compiler version;
 * $MVF_SPEC_DUMP names a file that receives a copy of the generated source.
 * Not thread-safe against concurrent calls on the same tape.
 */
typedef struct {
    int32_t chunk;            /* tangent components per pass, 1..n; 0 = library choice */
    int32_t waves;            /* waves per SIMD the kernel is compiled for, 1..4 (2..4 when the
                                 adjoint is built: MVF_EINVAL for 1); 0 = 2 */
    int64_t max_code;         /* size limit in instruction-passes; 0 = default (32000) */
    int32_t use_cache;        /* nonzero: read and write the on-disk code-object cache
                                 (mvf_spec_check: write it, for gfx950, so that a later
                                 mvf_tape_specialize of the same tape and options on any
                                 gfx950 finds the code object) */
    int32_t grad;             /* kernels to build: MVF_GRAD_FWD (tangent mode), MVF_GRAD_REV
                                 (reverse-mode adjoint) or MVF_GRAD_AUTO (both) */
    int32_t ckpt_budget;      /* reverse mode: register budget of one recomputed segment, in
                                 intervals, at most 32 (MVF_EINVAL above); 0 = library choice
                                 (32; 24 at four waves per SIMD or with more than 16 variables,
                                 part of whose gradient stays in registers; the roots are segmented when
                                 the largest one's single-pass adjoint keeps more partials
                                 than twice the register file's intervals), < 0 = none */
} mvf_spec_options;
typedef struct {
    int32_t chunk, waves, grad;
    int64_t code_units;       /* instruction-passes generated (an upper bound for the adjoint) */
    int64_t code_bytes;       /* size of the code object */
    double seconds;           /* generation + compilation (or cache read) */
    int32_t from_cache;
    int32_t ckpt_budget;      /* the segment budget used (<= 0: no checkpointing) */
    int32_t ckpt_intervals;   /* checkpoint intervals per lane (the largest root's); the bounding
                                 workspaces include ckpt_intervals x 16 bytes per launched lane */
} mvf_spec_info;
int mvf_tape_specialize(mvf_tape *tape, const mvf_spec_options *opt, mvf_spec_info *info);
/* Generate and compile for gfx950 without a device or a tape handle (no
 * cache): a check that a tape specialises, and what it costs. */
int mvf_spec_check(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts,
                   int32_t n_vars, const int32_t *roots, int32_t n_roots, const mvf_spec_options *opt,
                   mvf_spec_info *info);
/* The generated device source itself, without compiling it (inspection and
 * host-side checks of the generator): *len receives its length; when buf is
 * not NULL, up to cap - 1 bytes and a terminating NUL are copied into it (the
 * caller's host buffer).  Same options and errors as mvf_spec_check. */
int mvf_spec_source(const mvf_node *nodes, int32_t n_nodes, const double *consts, int32_t n_consts,
                    int32_t n_vars, const int32_t *roots, int32_t n_roots, const mvf_spec_options *opt,
                    char *buf, size_t cap, size_t *len);

/* ---- constraint propagation ------------------------------------------
 * Forward-backward bound tightening (FBBT) of node boxes, the bound
 * tightening the paper reports compatible with its method (constraint
 * propagation, Sec. 3.2; its effect, Sec. 4.3): per
 * box, the interval of every live DAG node (forward; a violated domain gives
 * [-inf, inf] and no narrowing through that node), the roots cut to their
 * feasible ranges (inequality roots <= 0, equality roots = 0, the objective
 * <= ub), then in descending node order each operand intersected with the
 * outward-rounded inverse of its operation (backward: + - * / by the other
 * operand, skipping divisions by intervals that contain 0; +-sqrt for sqr;
 * squares for sqrt; the padded log for exp, exp for log, atanh for tanh;
 * sin and cos only checked against [-1, 1]), and each variable met with its
 * variable nodes.  Rounds repeat this on the tightened box.  One lane per
 * box; the root kinds come from mvf_tape_set_root_kinds.
 *   boxes, out  device [N][n][2]; out receives the tightened boxes
 *   status      device [N]: 0, or 1 where the box is proven infeasible (then
 *               out is undefined)
 *   ub          the objective's upper bound, +inf for none
 *   rounds      1..64
 *   workspace   device scratch of mvf_fbbt_workspace() bytes
 */
int mvf_fbbt_workspace(const mvf_tape *tape, int64_t n_boxes, size_t *bytes);
int mvf_fbbt(const mvf_tape *tape, int64_t n_boxes, const double *boxes, double ub, int32_t rounds, double *out,
             int32_t *status, void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ---- tuning ----------------------------------------------------------- */
typedef struct mvf_tuning {
    int32_t grad;             /* MVF_GRAD_FWD or MVF_GRAD_REV; other values: keep the call's choice */
    int32_t chunk;            /* tangent components per forward pass (1 .. tangent_chunk); 0: default */
    int32_t grid_blocks;      /* persistent workgroups of a batched launch; 0: two per compute unit */
    float best_ms;            /* written by mvf_autotune: time of the chosen configuration */
    int32_t sub_per_lane;     /* batched launches: subdomains per lane of a work item (a work item is
                                 256 * sub_per_lane subdomains of one node), 1..16; 0: 1 */
    int32_t engine;           /* batched launches: MVF_ENGINE_* (AUTO: the tape's specialised kernel
                                 for the gradient mode when mvf_tape_specialize built it, else the
                                 interpreter; SPEC needs it) */
    int32_t block;            /* workgroup lanes of the specialised batched kernel: 64, 128 or 256;
                                 0: 256 (the interpreter's workgroup is always 256) */
} mvf_tuning;

/*
 * Adaptive partitioning (Sec. 3.1.2): the largest uniform split N with
 * N^n <= budget, then +1 on one dimension at a time, the one with the
 * largest relative width w_i / s_i first (ties to the lower index), while
 * the product stays <= budget.  Host only; returns the subdomain count or a
 * negative error code.
 */
int64_t mvf_adaptive_splits(int32_t n, const double *widths, int64_t budget, int32_t *splits);

/*
 * Split rules for a subdomain budget: MVF_SPLITS_ADAPTIVE is the adaptive
 * partitioning above (Sec. 3.1.2); MVF_SPLITS_DOUBLING starts from one
 * subdomain and doubles the split count of the dimension with the largest
 * w_i / s_i (ties to the lower index; counts stay <= 65535) while the
 * product stays <= budget, giving power-of-two counts (bisection-shaped
 * subdomains).  Host only;
 * returns the subdomain count or a negative error code.
 */
enum { MVF_SPLITS_ADAPTIVE = 0, MVF_SPLITS_DOUBLING = 1 };
int64_t mvf_splits(int32_t rule, int32_t n, const double *widths, int64_t budget, int32_t *splits);
/*
 * Split-rule tuning: bounds n_nodes sample node boxes (host [N][n][2]) with
 * each rule at the given budget in one batched launch per rule, and writes
 * to *rule the rule that gives the larger objective lower bound (the
 * feasibility-filtered bound) on more of the nodes; ties go to the adaptive
 * rule.  *better_nodes receives, per rule, the count of nodes where it is
 * strictly tighter.  Allocates temporary device memory.
 */
int mvf_autotune_splits(const mvf_tape *tape, int32_t n_nodes, const double *boxes, int64_t budget, int32_t mode,
                        int32_t grad, int32_t *rule, int32_t better_nodes[2], hipStream_t stream);

/* ---- batched bounding of many nodes ----------------------------------- */
typedef struct {
    int32_t n_nodes;          /* nodes in this call, 0 <= n_nodes <= max_nodes */
    int32_t max_nodes;        /* capacity the workspace was sized for */
    int64_t max_subdomains;   /* capacity: total subdomains over the nodes */
    const double *boxes;      /* device [N][n][2] */
    const int32_t *splits;    /* device [N][n] */
    int32_t mode, grad;
    double *reduced;          /* device [N][m][2]; NaN for an invalid node */
    int64_t *argmin;          /* device [N] or NULL: per node, smallest k attaining reduced[i][0][0] */
    int32_t *status;          /* device [N]: 0; 1 for a node with a split outside [1, 65535],
                                 more than 2^40 subdomains or more than 1024 breakpoints; 2 for
                                 every node when the batch exceeds max_subdomains (nothing runs) */
    void *workspace;          /* device scratch of mvf_batch_workspace() bytes */
    size_t workspace_bytes;
    double *extra;            /* device [N][2] or NULL: per node, as mvf_bound_args.extra */
} mvf_batch_args;

int mvf_batch_workspace(const mvf_tape *tape, int32_t max_nodes, int64_t max_subdomains, int32_t mode,
                        int32_t grad, const mvf_tuning *tuning, size_t *bytes);
/*
 * Bound every node of a batch in one persistent launch: per node the same
 * result as mvf_bound on that node's box and splits, bit for bit.  The node
 * list lives in device memory; work is split into chunks of 256 *
 * sub_per_lane subdomains that persistent workgroups take from an atomic
 * counter.  tuning may be NULL.
 */
int mvf_bound_batch(const mvf_tape *tape, const mvf_batch_args *args, const mvf_tuning *tuning,
                    hipStream_t stream);

/*
 * A batched bound captured once in a HIP graph: {H2D of node count, boxes
 * and splits from pinned staging} -> plan -> persistent kernel -> per-node
 * reduction -> {D2H of reduced, argmin, status to pinned memory}.  Replays
 * take the node count through device memory, so the graph is never
 * re-instantiated.  create allocates all buffers; launch validates the staged
 * splits on the host and enqueues one graph launch (waiting first for the
 * previous replay, whose first copy reads the pinned node count); results are
 * valid after the caller synchronises the stream or calls
 * mvf_batch_graph_wait.
 */
typedef struct mvf_batch_graph mvf_batch_graph;
int mvf_batch_graph_create(const mvf_tape *tape, int32_t max_nodes, int64_t max_subdomains, int32_t mode,
                           int32_t grad, const mvf_tuning *tuning, hipStream_t stream, mvf_batch_graph **out);
int mvf_batch_graph_staging(mvf_batch_graph *g, double **boxes, int32_t **splits);
int mvf_batch_graph_launch(mvf_batch_graph *g, int32_t n_nodes, hipStream_t stream);
/* Blocks until the graph's last replay (its staging H2D copies and its result
 * D2H copies included) has finished.  The staging buffers are read by the
 * replay's copies, so a caller must not write them for the next batch before
 * this returns (or before it has synchronised the replay's stream); the
 * results are valid after it too. */
int mvf_batch_graph_wait(mvf_batch_graph *g);
int mvf_batch_graph_result(mvf_batch_graph *g, const double **reduced, const int64_t **argmin,
                           const int32_t **status, const double **extra);
int mvf_batch_graph_destroy(mvf_batch_graph *g);

/*
 * Autotuner (the batched form's launch configuration; adaptive partitioning
 * matches the subdomain count to the cores, Sec. 3.1.2, and this matches the
 * launch to the machine): times the batched launch on the given sample nodes
 * (device arrays; n_subdomains = their total) for each kernel of the call's
 * gradient mode -- the interpreter (forward mode: each tangent chunk) and the
 * specialised kernel when the tape has one, the latter at workgroups of 64,
 * 128 and 256 lanes -- times the persistent grid (one, two or four 256-lane
 * workgroups' worth per CU) times subdomains per lane (1, 2, 4), and returns
 * the fastest (best_ms its time per launch).  grad is the caller's: the
 * tuner never changes the gradient mode, which decides the enclosures and so
 * the bounds (AUTO resolves as in mvf_bound, by the reference op count, not
 * by timing).  Results are cached per process by (tape programs and root
 * kinds, device, specialised module, sample size in nodes and subdomains,
 * mode, gradient mode): a repeated call returns the cached tuning at once.
 * Allocates temporary device memory.  Split counts are tuned separately
 * (mvf_autotune_splits).
 */
int mvf_autotune(const mvf_tape *tape, int32_t n_nodes, const double *boxes, const int32_t *splits,
                 int64_t n_subdomains, int32_t mode, int32_t grad, mvf_tuning *out, hipStream_t stream);

/* ---- points and boxes (differentiation) -------------------------------
 * One lane per point or box, evaluated with the same register programs and
 * outward-rounded operations as the bounding kernels.  A point x is the
 * degenerate box [x, x] (Sec. 2.2, interval arithmetic: a point interval
 * encloses the real value f(x)).  Every output is an interval [lo, hi]
 * stored as two doubles; where an operation leaves its domain (a divisor
 * containing 0, sqrt of a negative, log of a non-positive value) the row is
 * [-inf, +inf] and flags[b] (nullable) is 1.  Arrays are device memory owned
 * by the caller; the workspace is caller-provided device scratch of
 * mvf_points_workspace() bytes (0 for MVF_POINTS_EVAL and
 * MVF_BOXES_GRAD_FWD; pass NULL then).  Asynchronous on the stream.
 */
enum { MVF_POINTS_EVAL = 0, MVF_POINTS_VJP = 1, MVF_BOXES_GRAD_FWD = 2, MVF_BOXES_GRAD_REV = 3 };
int mvf_points_workspace(const mvf_tape *tape, int32_t op, int64_t n_items, size_t *bytes);

/* f [B][m][2]: enclosure of every root at each point x [B][n] (row major). */
int mvf_eval_points(const mvf_tape *tape, int64_t B, const double *x, double *f, uint32_t *flags,
                    void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * gx [B][n][2]: enclosure of sum_r gout[b][r] * grad f_r(x_b), from one
 * reverse sweep over the union of the root cones seeded with [gout, gout]
 * at the roots (the adjoint of a node collects every root's contribution
 * before it is propagated).  The paper computes gradients in tangent mode
 * (Sec. 3.2, operator overloading); this reverse sweep is the adjoint
 * counterpart of the same local derivative rules.
 */
int mvf_vjp_points(const mvf_tape *tape, int64_t B, const double *x, const double *gout, double *gx,
                   uint32_t *flags, void *workspace, size_t workspace_bytes, hipStream_t stream);

/*
 * G [B][n][2]: interval gradient enclosure of root `root` on each box
 * boxes [B][n][2] (Sec. 2.2, the gradient enclosure in the mean value form),
 * in tangent mode (MVF_GRAD_FWD) or by the reverse-mode adjoint
 * (MVF_GRAD_REV).  flags[b] reports a domain violation anywhere in the
 * union of the root cones.
 */
int mvf_gradient_boxes(const mvf_tape *tape, int64_t B, const double *boxes, int32_t root, int32_t grad,
                       double *G, uint32_t *flags, void *workspace, size_t workspace_bytes, hipStream_t stream);

/* ---- branch and bound -------------------------------------------------
 * Host spatial B&B over the bounding entry points (Sec. 3, Fig. BnB_decompose):
 * best-first on the lower bound (ties to the older node), the node's lower
 * bound = max(parent's, feasibility-filtered objective bound), upper bound =
 * least hi(f(c)) over rigorously feasible subdomain centres (mvf_bound_args.
 * extra; no local solver), pruning when lower >= upper - abs_gap, bisection
 * of the widest variable (ties to the lower index) at RN((lo + hi) / 2).
 * Subdomains per node by the adaptive partitioning (Sec. 3.1.2).  Root kinds
 * come from mvf_tape_set_root_kinds.  Allocates its device buffers (and, for
 * nodes_per_launch > 1, a batched graph whose breakpoint table holds up to
 * 256 split intervals per node) for the duration of the call; synchronous.
 */
typedef struct {
    int32_t max_nodes;            /* bound at most this many nodes (>= 1) */
    int32_t nodes_per_launch;     /* 1: one mvf_bound call per node; K > 1: the K best open nodes
                                     per replay of a batched graph */
    int64_t subdomains_per_node;  /* adaptive-partitioning budget per node (>= 1) */
    double abs_gap;               /* stop when upper - lower <= abs_gap (>= 0) */
    int32_t mode, grad;           /* MVF_MODE_*, MVF_GRAD_* of the bounding calls */
    const struct mvf_tuning *tuning;   /* NULL or the batched launches' tuning */
    int32_t split_rule;           /* MVF_SPLITS_* of each node's partition */
    int32_t fbbt_rounds;          /* 0: off; k >= 1: each taken node's box is first tightened by
                                     mvf_fbbt with k rounds and the objective cut at the current
                                     upper bound; a box proven infeasible is dropped (it holds no
                                     feasible point better than the upper bound) */
} mvf_bnb_options;

typedef struct {
    double lower, upper;          /* certified bounds on the minimum; +inf, +inf when infeasible */
    int64_t nodes;                /* nodes bounded */
    int64_t subdomains;           /* subdomain bounds computed */
    int64_t launches;             /* bounding launches (calls or graph replays) */
    int32_t open;                 /* open nodes left */
    int32_t status;               /* 0: gap reached or tree exhausted, 1: node limit, 2: infeasible */
    double seconds;               /* wall time of the solve */
} mvf_bnb_result;

/* box: host [n][2].  Returns MVF_OK with the result, or an error code. */
int mvf_bnb_solve(mvf_tape *tape, const double *box, const mvf_bnb_options *options, mvf_bnb_result *result,
                  hipStream_t stream);

/* ---- diagnostics ----------------------------------------------------- */
const char *mvf_strerror(int code);
const char *mvf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MVF_H */
