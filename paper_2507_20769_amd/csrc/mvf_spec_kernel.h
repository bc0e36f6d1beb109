// mvf_spec_kernel.h -- the specialised bounding kernels (one node box; many
// nodes), in tangent mode and with the reverse-mode adjoint.
//
// Compiled at run time after the generated namespace spec, which provides
// N_VARS, N_ROOTS and lane<REV>() (every root's bound on one lane's
// subdomain, folded into the wave's reduction record) for the modes it was
// generated for (MVF_SPEC_FWD, MVF_SPEC_REV).  Launch shape, arguments, LDS
// reduction records and partials are those of the interpreter's single-box
// and batched kernels, so their finish kernels complete Step 3.
#pragma once

#ifndef MVF_SPEC_WAVES
#define MVF_SPEC_WAVES 2
#endif

namespace mvf {
namespace dev {

// The workgroup is blockDim.x = 64, 128 or 256 lanes (one to four waves; a
// launch-time choice of the autotuner); LDS is laid out for up to four waves.
// LDS after the breakpoint table, the reduction records and the splits: the
// single-box adjoint's LDS-resident gradient components (spec::N_GL of them
// per lane, for up to BLK lanes), 16-byte aligned
__device__ __forceinline__ size_t spec_gl_offset(int tab_total, int m) {
    size_t b = (size_t)tab_total * 32;
    b += ((size_t)(BLK / 64) * wred_len(m) * 8 + 15) & ~(size_t)15;
    b += (2 * MVF_MAX_VARS + 8) * 4;
    return (b + 15) & ~(size_t)15;
}

template <bool REV>
__device__ __forceinline__ void spec_bound_body() {
    constexpr int n = spec::N_VARS, m = spec::N_ROOTS;
    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, blk = blockDim.x;
    // LDS: breakpoint table, per-wave reduction records, splits and table offsets
    const int tab_total = kargs<BoundKArgs>()->B.tab_off[n];
    double4 *tab = reinterpret_cast<double4 *>(smem);
    double *wred = reinterpret_cast<double *>(smem + (size_t)tab_total * 32);
    int32_t *ints = reinterpret_cast<int32_t *>(smem + (size_t)tab_total * 32 +
                                                (((size_t)(BLK / 64) * wred_len(m) * 8 + 15) & ~(size_t)15));
    {
        const auto K = kargs<BoundKArgs>();
        if (tid <= n) ints[MVF_MAX_VARS + tid] = K->B.tab_off[tid];
        if (tid < n) ints[tid] = K->B.splits[tid];
        __syncthreads();
        build_table(n, K->B.box, ints, ints + MVF_MAX_VARS, tab, tid, blk);
        if (lane == 0) reset_wred(wred + wave * wred_len(m), m);
    }
    __syncthreads();
    // always true, but opaque to the compiler: the generated code is cut into
    // blocks guarded by it, which keeps compile time near linear in its size
    const bool go = kargs<BoundKArgs>()->T.n == n;
    for (int64_t base = (int64_t)blockIdx.x * blk;; base += (int64_t)gridDim.x * blk) {
        const int64_t S = kargs<BoundKArgs>()->B.S;
        if (base >= S) break;
        const int64_t k = base + tid;
        const bool active = k < S;
        SpecLane L;
        L.tab = tab;
        L.ck = kargs<BoundKArgs>()->B.rec + ((int64_t)blockIdx.x * blk + wave * 64) * spec::N_CK + lane;
        L.ck_stride = 64;
        L.gl = reinterpret_cast<Iv *>(smem + spec_gl_offset(tab_total, m)) + tid;
        L.gl_stride = blk;
        int64_t q = active ? k : S - 1;
#pragma unroll
        for (int i = 0; i < n; ++i) {            // dimension 0 fastest (Sec. 3.1.1)
            const int s = ints[i];
            L.vi[i] = ints[MVF_MAX_VARS + i] + (int)(q % s);
            q /= s;
        }
        LaneOut o;
        FeasTrack F;
        uint32_t bad;
        {
            const auto K = kargs<BoundKArgs>();
            o.per_sub = K->B.per_sub;
            o.S = S;
            o.k = k;
            o.w = wred + wave * wred_len(m);
            o.lane = lane;
            o.active = active;
            o.ineq = K->T.ineq_mask;
            o.eq = K->T.eq_mask;
            mode_round_down();
            bad = spec::lane<REV>(L, K->T.mode, go, o, F);
            mode_round_nearest();
        }
        finish_lane(m, bad, F, o, kargs<BoundKArgs>()->B.flags);
    }
    __syncthreads();
    if (tid == 0) {
        const auto K = kargs<BoundKArgs>();
        write_partial(wred, blk / 64, m, K->B.partial + (size_t)blockIdx.x * m * 2, K->B.partial_lo0 + blockIdx.x,
                      K->B.partial_k + blockIdx.x, K->B.partial_ext + 2 * (size_t)blockIdx.x);
    }
}

// The batched form: persistent workgroups take work items (spl * BLK
// subdomains of one node) from the plan kernel's counter, as the
// interpreter's batch kernel does, and leave one partial per item for the
// per-node finish kernel.
template <bool REV>
__device__ __forceinline__ void spec_batch_body() {
    constexpr int n = spec::N_VARS, m = spec::N_ROOTS;
    constexpr int GL = REV ? spec::N_GL : 0;
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ int64_t sh_item;
    __shared__ int sh_node;
    // the table and the adjoint's gradient as static LDS objects, the reduction
    // records and splits in the dynamic LDS
    __shared__ __align__(16) double4 tab[BATCH_TAB_CAP];
    __shared__ __align__(16) Iv gl_lds[GL > 0 ? GL * BLK : 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, blk = blockDim.x;
    double *wred = reinterpret_cast<double *>(smem);
    int32_t *ints = reinterpret_cast<int32_t *>(smem + (((size_t)(BLK / 64) * wred_len(m) * 8 + 15) & ~(size_t)15));
    const bool go = kargs<BatchKArgs>()->T.n == n;        // always true, opaque (see mvf_spec_bound)
    int cur = -1;
    for (;;) {
        {
            const auto K = kargs<BatchKArgs>();
            if (tid == 0) sh_item = atomicAdd(reinterpret_cast<unsigned long long *>(K->A.counter), 1ull);
        }
        __syncthreads();
        const int64_t item = sh_item;
        {
            const auto K = kargs<BatchKArgs>();
            const int N = node_count(K->A);
            if (item >= K->A.item_off[N]) break;           // uniform exit: every wave reaches it
            if (tid == 0) {                                 // node owning the item: last node with item_off <= item
                int lo = 0, hi = N - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (K->A.item_off[mid] <= item) lo = mid; else hi = mid - 1;
                }
                while (lo < N - 1 && K->A.item_off[lo + 1] <= item) ++lo;   // skip nodes without items
                sh_node = lo;
            }
        }
        __syncthreads();
        const int node = sh_node;
        if (node != cur) {                              // new node: splits, offsets, breakpoint table
            const auto K = kargs<BatchKArgs>();
            if (tid < n) ints[tid] = K->A.splits[(int64_t)node * n + tid];
            __syncthreads();
            if (tid == 0) {
                int acc = 0;
                for (int i = 0; i < n; ++i) { ints[MVF_MAX_VARS + i] = acc; acc += ints[i]; }
                ints[MVF_MAX_VARS + n] = acc;
            }
            __syncthreads();
            build_table(n, K->A.boxes + (int64_t)node * n * 2, ints, ints + MVF_MAX_VARS, tab, tid, blk);
            cur = node;
        }
        if (lane == 0) reset_wred(wred + wave * wred_len(m), m);
        __syncthreads();
        int64_t S, base, len;
        {
            const auto K = kargs<BatchKArgs>();
            S = K->A.node_S[node];
            len = (int64_t)K->A.spl * BLK;                  // a work item: spl * 256 subdomains
            base = (item - K->A.item_off[node]) * len;
        }
        for (int64_t off = 0; off < len && base + off < S; off += blk) {      // uniform over the workgroup
            const int64_t k = base + off + tid;
            const bool active = k < S;
            SpecLane L;
            L.tab = tab;
            L.ck = kargs<BatchKArgs>()->A.rec + ((int64_t)blockIdx.x * blk + wave * 64) * spec::N_CK + lane;
            L.ck_stride = 64;
            L.gl = gl_lds + tid;
            L.gl_stride = blk;
            int64_t q = active ? k : S - 1;
#pragma unroll
            for (int i = 0; i < n; ++i) {
                const int s = ints[i];
                L.vi[i] = ints[MVF_MAX_VARS + i] + (int)(q % s);
                q /= s;
            }
            LaneOut o;
            o.per_sub = nullptr;
            o.S = S;
            o.k = k;
            o.w = wred + wave * wred_len(m);
            o.lane = lane;
            o.active = active;
            FeasTrack F;
            uint32_t bad;
            {
                const auto K = kargs<BatchKArgs>();
                o.ineq = K->T.ineq_mask;
                o.eq = K->T.eq_mask;
                mode_round_down();
                bad = spec::lane<REV>(L, K->T.mode, go, o, F);
                mode_round_nearest();
            }
            finish_lane(m, bad, F, o, nullptr);
        }
        __syncthreads();
        if (tid == 0) {
            const auto K = kargs<BatchKArgs>();
            write_partial(wred, blk / 64, m, K->A.partial + (size_t)item * m * 2, K->A.partial_lo0 + item,
                          K->A.partial_k + item, K->A.partial_ext + 2 * (size_t)item);
        }
    }
}

}  // namespace dev
}  // namespace mvf

#define MVF_SPEC_KERNEL(name, KA, body)                                                                     \
    extern "C" __global__ __launch_bounds__(mvf::BLK)                                                       \
        __attribute__((amdgpu_waves_per_eu(MVF_SPEC_WAVES, MVF_SPEC_WAVES))) void name(mvf::KA) {          \
        body;                                                                                               \
    }
#ifdef MVF_SPEC_FWD
MVF_SPEC_KERNEL(mvf_spec_bound, BoundKArgs, mvf::dev::spec_bound_body<false>())
MVF_SPEC_KERNEL(mvf_spec_batch, BatchKArgs, mvf::dev::spec_batch_body<false>())
#endif
#ifdef MVF_SPEC_REV
MVF_SPEC_KERNEL(mvf_spec_bound_rev, BoundKArgs, mvf::dev::spec_bound_body<true>())
MVF_SPEC_KERNEL(mvf_spec_batch_rev, BatchKArgs, mvf::dev::spec_batch_body<true>())
#endif
