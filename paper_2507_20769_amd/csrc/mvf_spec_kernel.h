// mvf_spec_kernel.h -- the specialised bounding kernel (one node box).
//
// Compiled at run time after the generated namespace spec, which provides
// N_VARS, N_ROOTS and lane_bounds() (every root's bound on one lane's
// subdomain, folded into the wave's reduction record).  Launch shape,
// arguments, LDS reduction records and per-block partials are those of the
// interpreter's single-box kernel, so its finish kernel completes Step 3.
#pragma once

#ifndef MVF_SPEC_WAVES
#define MVF_SPEC_WAVES 2
#endif

extern "C" __global__ __launch_bounds__(mvf::BLK) __attribute__((amdgpu_waves_per_eu(MVF_SPEC_WAVES, MVF_SPEC_WAVES)))
void mvf_spec_bound(mvf::BoundKArgs /* read through kargs() */) {
    using namespace mvf;
    using namespace mvf::dev;
    constexpr int n = spec::N_VARS, m = spec::N_ROOTS;
    extern __shared__ __align__(16) uint8_t smem[];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
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
        build_table(n, K->B.box, ints, ints + MVF_MAX_VARS, tab, tid, BLK);
        if (lane == 0) reset_wred(wred + wave * wred_len(m), m);
    }
    __syncthreads();
    // always true, but opaque to the compiler: the generated code is cut into
    // blocks guarded by it, which keeps compile time near linear in its size
    const bool go = kargs<BoundKArgs>()->T.n == n;
    for (int64_t base = (int64_t)blockIdx.x * BLK;; base += (int64_t)gridDim.x * BLK) {
        const int64_t S = kargs<BoundKArgs>()->B.S;
        if (base >= S) break;
        const int64_t k = base + tid;
        const bool active = k < S;
        SpecLane L;
        L.tab = tab;
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
            bad = spec::lane_bounds(L, K->T.mode, go, o, F);
            mode_round_nearest();
        }
        finish_lane(m, bad, F, o, kargs<BoundKArgs>()->B.flags);
    }
    __syncthreads();
    if (tid == 0) {
        const auto K = kargs<BoundKArgs>();
        write_partial(wred, BLK / 64, m, K->B.partial + (size_t)blockIdx.x * m * 2, K->B.partial_lo0 + blockIdx.x,
                      K->B.partial_k + blockIdx.x, K->B.partial_ext + 2 * (size_t)blockIdx.x);
    }
}
