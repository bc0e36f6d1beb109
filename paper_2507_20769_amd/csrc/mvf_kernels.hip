// mvf_kernels.hip -- subdomain MVF bounding kernels for gfx950 and the C ABI.
//
// One lane = one subdomain.  A workgroup stages the register programs (one
// per root) and a per-dimension breakpoint table into LDS; every lane decodes
// its subdomain index, then interprets the programs instruction by
// instruction: the 16-byte instruction is broadcast from LDS to the wave and
// made wave-uniform, operands come from the lane's GPR-indexed slot file, the
// breakpoint table (variables) or the instruction (constants), and the result
// goes back to a slot.  Per root: a point pass at the centre c gives [f(c)],
// tangent passes over X_k give the NIE and C gradient components at a time,
// and the Mean Value Form is accumulated component by component
// (Sec. 2.2 Definition "Mean Value Form"; Sec. 3.1 Step 2), then intersected
// with the NIE.  The subdomain bounds are min-reduced per wave with
// cross-lane shuffles, per workgroup through LDS, and across workgroups by a
// second small kernel (Sec. 3.1 Step 3, the refinement/interval hull).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mvf.h"
#include "mvf_device.h"
#include "mvf_internal.h"

namespace mvf {

constexpr int BLK = 256;
constexpr int WAVES = BLK / 64;

struct BoundParams {
    const Instr *prog;
    int32_t n_instr, n_roots, n, mode;
    int32_t root_begin[MVF_MAX_ROOTS], root_len[MVF_MAX_ROOTS], root_slot[MVF_MAX_ROOTS];
    int32_t splits[MVF_MAX_VARS];
    int32_t tab_off[MVF_MAX_VARS + 1];
    const double *box;
    int64_t S;
    double *per_sub;
    uint32_t *flags;
    double *partial;       // [grid][m][2] (min lo, min nh)
    double *partial_lo0;   // [grid] objective lower bound of the block's argmin
    int64_t *partial_k;    // [grid]
};

namespace dev {

// breakpoint b_j of [lo, hi] split in s (round to nearest; fp-contract off)
__device__ __forceinline__ double breakpoint(double lo, double hi, int s, int j) {
    if (j <= 0) return lo;
    if (j >= s) return hi;
    double w = hi - lo;
    double h = w / (double)s;
    double r = lo + (double)j * h;
    return r < hi ? r : hi;
}

struct Ctx {
    const Instr *prog;       // LDS
    const double4 *tab;      // LDS: {lo, nh, c, -c} per (dim, j)
    const uint16_t *jidx;    // LDS: [dim][BLK]
    const int32_t *tab_off;  // kernel arguments
    int tid;
};

__device__ __forceinline__ double4 var_rec(const Ctx &X, uint32_t i) {
    uint32_t j = X.jidx[i * BLK + X.tid];
    return X.tab[X.tab_off[i] + j];
}

// fetch operand (kind, a): value and C tangent components [c0, c0 + C)
template <int C, bool POINT>
__device__ __forceinline__ void fetch(const Ctx &X, uint32_t kind, uint32_t a, double k, int c0, Iv &val,
                                      Iv (&tan)[C > 0 ? C : 1]) {
    constexpr uint32_t SD = 4 + 4 * C;
    if (kind == K_SLOT) {
        slot_read<C>(a * SD, val, tan);
    } else if (kind == K_VAR) {
        double4 r = var_rec(X, a);
        val = POINT ? Iv{r.z, r.w} : Iv{r.x, r.y};
#pragma unroll
        for (int t = 0; t < C; ++t) {
            const bool hit = (int)a == c0 + t;
            tan[t] = Iv{hit ? 1.0 : 0.0, hit ? -1.0 : 0.0};
        }
    } else {
        val = Iv{k, -k};
#pragma unroll
        for (int t = 0; t < C; ++t) tan[t] = Iv{0.0, 0.0};
    }
}

// Run one root program; returns the root's value interval and (C > 0) its
// tangent components [c0, c0 + C).
template <int C, bool POINT>
__device__ Iv run_program(const Ctx &X, int begin, int len, int res_slot, int c0, Iv (&gout)[C > 0 ? C : 1],
                          uint32_t &bad) {
    constexpr uint32_t SD = 4 + 4 * C;
    const uint4 *P = reinterpret_cast<const uint4 *>(X.prog);
    for (int pc = begin; pc < begin + len; ++pc) {
        uint4 raw = P[pc];
        const uint32_t w0 = __builtin_amdgcn_readfirstlane(raw.x);
        const uint32_t w1 = __builtin_amdgcn_readfirstlane(raw.y);
        const double k = __hiloint2double((int)raw.w, (int)raw.z);
        const uint32_t op = w0 & 0xffu, ak = (w0 >> 8) & 3u, bk = (w0 >> 10) & 3u, a = w0 >> 16;
        const uint32_t b = w1 & 0xffffu, d = w1 >> 16;
        Iv U, V, Z;
        Iv dU[C > 0 ? C : 1], dV[C > 0 ? C : 1], dZ[C > 0 ? C : 1];
        fetch<C, POINT>(X, ak, a, k, c0, U, dU);
        if (op >= I_ADD && op <= I_DIV) fetch<C, POINT>(X, bk, b, k, c0, V, dV);
        switch (op) {
        case I_ADD:
            Z = iadd(U, V);
#pragma unroll
            for (int t = 0; t < C; ++t) dZ[t] = iadd(dU[t], dV[t]);
            break;
        case I_SUB:
            Z = isub(U, V);
#pragma unroll
            for (int t = 0; t < C; ++t) dZ[t] = isub(dU[t], dV[t]);
            break;
        case I_MUL:
            Z = imul(U, V);
#pragma unroll
            for (int t = 0; t < C; ++t) dZ[t] = iadd(imul(V, dU[t]), imul(U, dV[t]));
            break;
        case I_DIV: {
            bad |= (V.lo <= 0.0 && V.nh <= 0.0) ? 1u : 0u;
            Z = idiv(U, V);
            if constexpr (C > 0) {
                Iv R = irecip(V);
#pragma unroll
                for (int t = 0; t < C; ++t) dZ[t] = imul(isub(dU[t], imul(Z, dV[t])), R);
            }
            break;
        }
        case I_SQR: {
            Z = isqr(U);
            if constexpr (C > 0) {
                Iv T = itwice(U);
#pragma unroll
                for (int t = 0; t < C; ++t) dZ[t] = imul(T, dU[t]);
            }
            break;
        }
        case I_SQRT: {
            bad |= U.lo < 0.0 ? 1u : 0u;
            Z = isqrt(U);
            if constexpr (C > 0) {
                Iv R = isqrt_deriv(Z);
#pragma unroll
                for (int t = 0; t < C; ++t) dZ[t] = imul(dU[t], R);
            }
            break;
        }
        case I_EXP:
            Z = iexp(U);
#pragma unroll
            for (int t = 0; t < C; ++t) dZ[t] = imul(Z, dU[t]);
            break;
        case I_LOG: {
            bad |= U.lo <= 0.0 ? 1u : 0u;
            Z = ilog(U);
            if constexpr (C > 0) {
                Iv R = irecip(U);
#pragma unroll
                for (int t = 0; t < C; ++t) dZ[t] = imul(dU[t], R);
            }
            break;
        }
        default:   // I_LOAD
            Z = U;
#pragma unroll
            for (int t = 0; t < C; ++t) dZ[t] = dU[t];
            break;
        }
        slot_write<C>(d * SD, Z, dZ);
    }
    Iv val;
    slot_read<C>((uint32_t)res_slot * SD, val, gout);
    return val;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ void wave_argmin(double &v, int64_t &k) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        double v2 = __shfl_xor(v, o, 64);
        int64_t k2 = __shfl_xor(k, o, 64);
        const bool take = v2 < v || (v2 == v && k2 < k);
        v = take ? v2 : v;
        k = take ? k2 : k;
    }
}

}  // namespace dev

// Bound every subdomain of one box; C tangent components per forward pass
// (C = 0 computes the NIE only).
template <int C>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_num_vgpr(SLOT_BASE))) void bound_kernel(BoundParams P) {
    using namespace dev;
    extern __shared__ __align__(16) uint8_t smem[];
    claim_slot_file();
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = P.n_roots, n = P.n;
    const int tab_total = P.tab_off[n];
    Instr *lprog = reinterpret_cast<Instr *>(smem);
    double4 *tab = reinterpret_cast<double4 *>(smem + (size_t)P.n_instr * sizeof(Instr));
    uint16_t *jidx = reinterpret_cast<uint16_t *>(reinterpret_cast<uint8_t *>(tab) + (size_t)tab_total * sizeof(double4));
    double *wred = reinterpret_cast<double *>(
        reinterpret_cast<uint8_t *>(jidx) + (((size_t)n * BLK * sizeof(uint16_t) + 15) & ~(size_t)15));
    // wred per wave: [m][2] mins, then lo0 and k (as double bits)

    // stage programs and build the breakpoint table (round to nearest)
    {
        const uint4 *src = reinterpret_cast<const uint4 *>(P.prog);
        uint4 *dst = reinterpret_cast<uint4 *>(lprog);
        for (int i = tid; i < P.n_instr; i += BLK) dst[i] = src[i];
        for (int t = tid; t < tab_total; t += BLK) {
            int i = 0;
            while (P.tab_off[i + 1] <= t) ++i;
            const int j = t - P.tab_off[i], s = P.splits[i];
            const double lo = P.box[2 * i], hi = P.box[2 * i + 1];
            const double bl = breakpoint(lo, hi, s, j), bh = breakpoint(lo, hi, s, j + 1);
            const double c = 0.5 * (bl + bh);
            tab[t] = make_double4(bl, -bh, c, -c);
        }
        if (lane == 0) {
            double *w = wred + wave * (2 * m + 2);
            for (int r = 0; r < 2 * m + 1; ++r) w[r] = __builtin_inf();
            reinterpret_cast<int64_t *>(w)[2 * m + 1] = INT64_MAX;
        }
    }
    __syncthreads();

    Ctx X{lprog, tab, jidx, P.tab_off, tid};
    const uint32_t res_base = (uint32_t)usable_dwords(m);
    for (int64_t base = (int64_t)blockIdx.x * BLK; base < P.S; base += (int64_t)gridDim.x * BLK) {
        const int64_t k = base + tid;
        const bool active = k < P.S;
        int64_t q = active ? k : P.S - 1;
        for (int i = 0; i < n; ++i) {          // dimension 0 varies fastest
            const int s = P.splits[i];
            jidx[i * BLK + tid] = (uint16_t)(q % s);
            q /= s;
        }
        mode_round_down();
        uint32_t bad = 0;
        for (int r = 0; r < m; ++r) {
            const int pb = P.root_begin[r], pl = P.root_len[r], rs = P.root_slot[r];
            Iv B;
            if (P.mode == MVF_MODE_NIE || C == 0) {
                Iv g0[1];
                B = run_program<0, false>(X, pb, pl, rs, 0, g0, bad);
            } else {
                Iv g0[1], G[C > 0 ? C : 1];
                const Iv FC = run_program<0, true>(X, pb, pl, rs, 0, g0, bad);
                Iv acc = FC, nie = {0.0, 0.0};
                for (int c0 = 0; c0 < n; c0 += C) {
                    Iv v = run_program<C, false>(X, pb, pl, rs, c0, G, bad);
                    if (c0 == 0) nie = v;
#pragma unroll
                    for (int t = 0; t < C; ++t) {
                        if (c0 + t < n) {
                            const double4 rec = var_rec(X, (uint32_t)(c0 + t));
                            const Iv D = {fadd(rec.x, rec.w), fadd(rec.y, rec.z)};   // X_i - c_i
                            acc = iadd(acc, imul(G[t], D));
                        }
                    }
                }
                if (P.mode == MVF_MODE_MVF) B = acc;
                else B = Iv{fmax_(acc.lo, nie.lo), fmax_(acc.nh, nie.nh)};
            }
            slot_wr(res_base + 4 * r, B);
        }
        mode_round_nearest();
        // domain flag or NaN anywhere: every bound of the subdomain is [-inf, +inf]
        for (int r = 0; r < m; ++r) {
            Iv B = slot_rd(res_base + 4 * r);
            if (B.lo != B.lo || B.nh != B.nh) bad = 1;
        }
        for (int r = 0; r < m; ++r) {
            Iv B = slot_rd(res_base + 4 * r);
            if (bad) B = Iv{-__builtin_inf(), -__builtin_inf()};
            if (active && P.per_sub) {
                P.per_sub[(int64_t)(2 * r) * P.S + k] = B.lo;
                P.per_sub[(int64_t)(2 * r + 1) * P.S + k] = -B.nh;
            }
            const double lo = active ? B.lo : __builtin_inf();
            const double nh = active ? B.nh : __builtin_inf();
            double wl = wave_min(lo), wn = wave_min(nh);
            double *w = wred + wave * (2 * m + 2);
            if (r == 0) {
                double v = lo;
                int64_t kk = active ? k : INT64_MAX;
                wave_argmin(v, kk);
                if (lane == 0) {
                    const double pv = w[2 * m];
                    const int64_t pk = reinterpret_cast<int64_t *>(w)[2 * m + 1];
                    if (v < pv || (v == pv && kk < pk)) {
                        w[2 * m] = v;
                        reinterpret_cast<int64_t *>(w)[2 * m + 1] = kk;
                    }
                }
            }
            if (lane == 0) {
                w[2 * r] = fmin(w[2 * r], wl);
                w[2 * r + 1] = fmin(w[2 * r + 1], wn);
            }
        }
        if (active && P.flags) P.flags[k] = bad;
    }
    __syncthreads();
    if (tid == 0) {
        double best = __builtin_inf();
        int64_t bk = INT64_MAX;
        for (int r = 0; r < m; ++r) {
            double l = __builtin_inf(), h = __builtin_inf();
            for (int w = 0; w < WAVES; ++w) {
                const double *wr = wred + w * (2 * m + 2);
                l = fmin(l, wr[2 * r]);
                h = fmin(h, wr[2 * r + 1]);
            }
            P.partial[((size_t)blockIdx.x * m + r) * 2] = l;
            P.partial[((size_t)blockIdx.x * m + r) * 2 + 1] = h;
        }
        for (int w = 0; w < WAVES; ++w) {
            const double *wr = wred + w * (2 * m + 2);
            const double v = wr[2 * m];
            const int64_t kk = reinterpret_cast<const int64_t *>(wr)[2 * m + 1];
            if (v < best || (v == best && kk < bk)) { best = v; bk = kk; }
        }
        P.partial_lo0[blockIdx.x] = best;
        P.partial_k[blockIdx.x] = bk;
    }
}

// Reduce the per-block partials into reduced[m][2] = (lo, hi) and argmin.
__global__ __launch_bounds__(256) void finish_kernel(const double *partial, const double *plo0, const int64_t *pk,
                                                     int nblocks, int m, double *reduced, int64_t *argmin) {
    __shared__ double sv[256];
    __shared__ int64_t sk[256];
    const int tid = threadIdx.x;
    for (int r = 0; r < m; ++r) {
        for (int c = 0; c < 2; ++c) {
            double v = __builtin_inf();
            for (int b = tid; b < nblocks; b += 256) v = fmin(v, partial[((size_t)b * m + r) * 2 + c]);
            sv[tid] = v;
            __syncthreads();
            for (int s = 128; s > 0; s >>= 1) {
                if (tid < s) sv[tid] = fmin(sv[tid], sv[tid + s]);
                __syncthreads();
            }
            if (tid == 0) reduced[r * 2 + c] = c == 0 ? sv[0] : -sv[0];
            __syncthreads();
        }
    }
    if (argmin) {
        double v = __builtin_inf();
        int64_t k = INT64_MAX;
        for (int b = tid; b < nblocks; b += 256) {
            const double v2 = plo0[b];
            const int64_t k2 = pk[b];
            if (v2 < v || (v2 == v && k2 < k)) { v = v2; k = k2; }
        }
        sv[tid] = v;
        sk[tid] = k;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if (tid < s) {
                const double v2 = sv[tid + s];
                const int64_t k2 = sk[tid + s];
                if (v2 < sv[tid] || (v2 == sv[tid] && k2 < sk[tid])) { sv[tid] = v2; sk[tid] = k2; }
            }
            __syncthreads();
        }
        if (tid == 0) *argmin = sk[0];
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

namespace {
thread_local std::string g_err;

int set_err(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_err(hipError_t e, const char *what) {
    return set_err(MVF_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr)                                  \
    do {                                               \
        hipError_t _e = (expr);                        \
        if (_e != hipSuccess) return hip_err(_e, #expr); \
    } while (0)

int check_device() {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_err(MVF_ENOTSUP, std::string("device is ") + prop.gcnArchName + ", need gfx950");
    return MVF_OK;
}

template <int C>
int launch_bound_c(const BoundParams &P, int grid, size_t lds, hipStream_t stream) {
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(once, [] {
        attr_err = hipFuncSetAttribute(reinterpret_cast<const void *>(&bound_kernel<C>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    });
    if (attr_err != hipSuccess) return hip_err(attr_err, "hipFuncSetAttribute");
    hipLaunchKernelGGL(bound_kernel<C>, dim3(grid), dim3(BLK), lds, stream, P);
    HIP_TRY(hipGetLastError());
    return MVF_OK;
}

}  // namespace

}  // namespace mvf

struct mvf_tape {
    mvf::Compiled C;
    mvf::Instr *d_prog = nullptr;
    int device = 0;
};

using namespace mvf;

namespace {

constexpr int MAX_GRID = 2048;

int grid_for(int64_t S) { return (int)std::min<int64_t>((S + BLK - 1) / BLK, MAX_GRID); }

size_t lds_bytes(const mvf_tape *t, int tab_total) {
    const int m = (int)t->C.roots.size(), n = t->C.n_vars;
    size_t b = (size_t)t->C.instr.size() * sizeof(Instr) + (size_t)tab_total * 32;
    b += ((size_t)n * BLK * sizeof(uint16_t) + 15) & ~(size_t)15;
    b += (size_t)WAVES * (2 * m + 2) * sizeof(double);
    return b;
}

}  // namespace

extern "C" {

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
    if (stats) {
        stats->n_vars = C.n_vars;
        stats->n_roots = (int32_t)C.roots.size();
        stats->n_instr = (int32_t)C.instr.size();
        stats->max_slots = C.max_slots;
        stats->tangent_chunk = C.chunk;
        stats->ref_ops_fwd = C.ref_fwd;
        stats->ref_ops_rev = C.ref_rev;
    }
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
    rc = check_device();
    if (rc != MVF_OK) { delete t; return rc; }
    hipGetDevice(&t->device);
    const size_t bytes = t->C.instr.size() * sizeof(Instr);
    hipError_t e = hipMalloc(&t->d_prog, bytes);
    if (e != hipSuccess) { delete t; return set_err(MVF_ENOMEM, "hipMalloc of the program failed"); }
    e = hipMemcpy(t->d_prog, t->C.instr.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) { hipFree(t->d_prog); delete t; return hip_err(e, "hipMemcpy program"); }
    *out = t;
    return MVF_OK;
}

int mvf_tape_stats_get(const mvf_tape *t, mvf_tape_stats *stats) {
    if (!t || !stats) return set_err(MVF_EINVAL, "null argument");
    stats->n_vars = t->C.n_vars;
    stats->n_roots = (int32_t)t->C.roots.size();
    stats->n_instr = (int32_t)t->C.instr.size();
    stats->max_slots = t->C.max_slots;
    stats->tangent_chunk = t->C.chunk;
    stats->ref_ops_fwd = t->C.ref_fwd;
    stats->ref_ops_rev = t->C.ref_rev;
    return MVF_OK;
}

int mvf_tape_destroy(mvf_tape *t) {
    if (!t) return MVF_OK;
    if (t->d_prog) hipFree(t->d_prog);
    delete t;
    return MVF_OK;
}

static int check_splits(const mvf_tape *t, const int32_t *splits, int64_t *S, int *tab_total) {
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

int mvf_bound_workspace(const mvf_tape *t, const int32_t *splits, int32_t mode, int32_t grad, size_t *bytes) {
    (void)mode; (void)grad;
    if (!t || !bytes) return set_err(MVF_EINVAL, "null argument");
    int64_t S;
    int tt;
    int rc = check_splits(t, splits, &S, &tt);
    if (rc != MVF_OK) return rc;
    const size_t g = (size_t)grid_for(S), m = t->C.roots.size();
    *bytes = g * m * 2 * sizeof(double) + g * sizeof(double) + g * sizeof(int64_t);
    return MVF_OK;
}

int mvf_bound(const mvf_tape *t, const mvf_bound_args *a, hipStream_t stream) {
    if (!t || !a) return set_err(MVF_EINVAL, "null argument");
    if (!a->box || !a->reduced || !a->workspace) return set_err(MVF_EINVAL, "box, reduced and workspace are required");
    if (a->mode < MVF_MODE_NIE || a->mode > MVF_MODE_BOTH) return set_err(MVF_EINVAL, "bad mode");
    if (a->grad < MVF_GRAD_FWD || a->grad > MVF_GRAD_AUTO) return set_err(MVF_EINVAL, "bad grad");
    if (a->grad == MVF_GRAD_REV && a->mode != MVF_MODE_NIE)
        return set_err(MVF_ENOTSUP, "reverse-mode gradients are not available in mvf_bound");
    int64_t S;
    int tt;
    int rc = check_splits(t, a->splits, &S, &tt);
    if (rc != MVF_OK) return rc;
    size_t need = 0;
    mvf_bound_workspace(t, a->splits, a->mode, a->grad, &need);
    if (a->workspace_bytes < need) return set_err(MVF_EINVAL, "workspace too small");
    const int m = (int)t->C.roots.size(), n = t->C.n_vars;
    const int C = a->mode == MVF_MODE_NIE ? 0 : t->C.chunk;
    if (a->mode != MVF_MODE_NIE && C == 0)
        return set_err(MVF_ELIMIT, "live set too large for tangent passes");
    const size_t lds = lds_bytes(t, tt);
    if (lds > 160 * 1024) return set_err(MVF_ELIMIT, "tape and tables exceed the LDS budget");

    BoundParams P;
    std::memset(&P, 0, sizeof P);
    P.prog = t->d_prog;
    P.n_instr = (int32_t)t->C.instr.size();
    P.n_roots = m;
    P.n = n;
    P.mode = a->mode;
    for (int r = 0; r < m; ++r) {
        P.root_begin[r] = t->C.roots[r].begin;
        P.root_len[r] = t->C.roots[r].len;
        P.root_slot[r] = t->C.roots[r].result_slot;
    }
    P.tab_off[0] = 0;
    for (int i = 0; i < n; ++i) {
        P.splits[i] = a->splits[i];
        P.tab_off[i + 1] = P.tab_off[i] + a->splits[i];
    }
    P.box = a->box;
    P.S = S;
    P.per_sub = a->per_sub;
    P.flags = a->flags;
    const int grid = grid_for(S);
    uint8_t *ws = static_cast<uint8_t *>(a->workspace);
    P.partial = reinterpret_cast<double *>(ws);
    P.partial_lo0 = P.partial + (size_t)grid * m * 2;
    P.partial_k = reinterpret_cast<int64_t *>(P.partial_lo0 + grid);

    static_assert(MAX_CHUNK == 2, "one kernel instance per chunk size");
    switch (C) {
    case 0: rc = launch_bound_c<0>(P, grid, lds, stream); break;
    case 1: rc = launch_bound_c<1>(P, grid, lds, stream); break;
    default: rc = launch_bound_c<2>(P, grid, lds, stream); break;
    }
    if (rc != MVF_OK) return rc;
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, stream, P.partial, P.partial_lo0, P.partial_k, grid, m,
                       a->reduced, a->argmin);
    HIP_TRY(hipGetLastError());
    return MVF_OK;
}

}  // extern "C"
