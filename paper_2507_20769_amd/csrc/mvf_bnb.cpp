// mvf_bnb.cpp -- host spatial branch-and-bound driving the GPU lower bounding.
//
// The heterogeneous scheme of Sec. 3 (Fig. BnB_decompose): the host keeps the
// open nodes, selects, prunes and branches; the GPU bounds the selected nodes
// by Subdomain Lower Bounding (Sec. 3.1, Steps 1-3) with the adaptive
// partitioning of Sec. 3.1.2.  Pruning uses the lower-bound test and the
// feasibility check of the constraint bounds (applied per subdomain: the
// feasibility-filtered objective bound).  The paper takes its upper bound from
// a local NLP solver; here it is the least hi(f(c_k)) over subdomain centres
// whose inequality enclosures are all <= 0 -- rigorously feasible points that
// the point pass of the mean value form evaluates anyway.
//
// Two launch forms: one mvf_bound call per node (plain), or the K best open
// nodes per replay of a captured batched graph.  Optionally each taken node's
// box is first tightened by constraint propagation (mvf_fbbt; the constraint
// propagation of Sec. 3.2 and 4.3).  The driver is a client of the public C ABI only.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <queue>
#include <string>
#include <vector>

#include "mvf.h"
#include "mvf_internal.h"

using mvf::set_error;

namespace {

struct Node {
    double lb;
    int64_t id;
    std::vector<double> box;     // [n][2]
};

// least lower bound first, ties to the node created first
struct Later {
    bool operator()(const Node &a, const Node &b) const { return a.lb > b.lb || (a.lb == b.lb && a.id > b.id); }
};

}  // namespace

extern "C" int mvf_bnb_solve(mvf_tape *tape, const double *box, const mvf_bnb_options *opt, mvf_bnb_result *res,
                             hipStream_t stream) {
    if (!tape || !box || !opt || !res) return set_error(MVF_EINVAL, "null argument");
    if (opt->max_nodes < 1 || opt->nodes_per_launch < 1 || opt->subdomains_per_node < 1 || !(opt->abs_gap >= 0) ||
        opt->fbbt_rounds < 0 || opt->fbbt_rounds > 64)
        return set_error(MVF_EINVAL, "options out of range");
    mvf_tape_stats st;
    int rc = mvf_tape_stats_get(tape, &st);
    if (rc != MVF_OK) return rc;
    const int n = st.n_vars, m = st.n_roots;
    const int K = opt->nodes_per_launch;
    const double gap = opt->abs_gap;
    for (int i = 0; i < n; ++i)
        if (!(box[2 * i] <= box[2 * i + 1])) return set_error(MVF_EINVAL, "box with lo > hi or NaN");
    const auto t0 = std::chrono::steady_clock::now();

    // device and pinned buffers of the chosen launch form
    mvf_batch_graph *g = nullptr;
    double *h_boxes = nullptr;
    int32_t *h_splits = nullptr;
    const double *h_ex = nullptr;
    const int32_t *h_status = nullptr;
    double *d_box = nullptr, *d_red = nullptr, *d_ex = nullptr, *p_box = nullptr, *p_ex = nullptr;
    void *d_ws = nullptr;
    size_t ws_bytes = 0;
    // bound tightening of the taken nodes: device boxes in/out, status, scratch, pinned staging
    double *d_fb_in = nullptr, *d_fb_out = nullptr, *p_fb = nullptr;
    int32_t *d_fb_st = nullptr, *p_fb_st = nullptr;
    void *d_fb_ws = nullptr;
    size_t fb_ws = 0;
    auto cleanup = [&]() {
        if (g) mvf_batch_graph_destroy(g);
        hipFree(d_box);
        hipFree(d_red);
        hipFree(d_ex);
        hipFree(d_ws);
        hipHostFree(p_box);
        hipHostFree(p_ex);
        hipFree(d_fb_in);
        hipFree(d_fb_out);
        hipFree(d_fb_st);
        hipFree(d_fb_ws);
        hipHostFree(p_fb);
        hipHostFree(p_fb_st);
    };
    if (opt->fbbt_rounds > 0) {
        mvf_fbbt_workspace(tape, K, &fb_ws);
        if (hipMalloc(&d_fb_in, (size_t)K * n * 16) != hipSuccess ||
            hipMalloc(&d_fb_out, (size_t)K * n * 16) != hipSuccess || hipMalloc(&d_fb_st, (size_t)K * 4) != hipSuccess ||
            hipMalloc(&d_fb_ws, fb_ws) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&p_fb), (size_t)K * n * 16, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&p_fb_st), (size_t)K * 4, hipHostMallocDefault) != hipSuccess) {
            cleanup();
            return set_error(MVF_ENOMEM, "bound tightening buffers");
        }
    }
    if (K > 1) {
        rc = mvf_batch_graph_create(tape, K, (int64_t)K * opt->subdomains_per_node, opt->mode, opt->grad,
                                    opt->tuning, stream, &g);
        if (rc != MVF_OK) return rc;
        mvf_batch_graph_staging(g, &h_boxes, &h_splits);
        mvf_batch_graph_result(g, nullptr, nullptr, &h_status, &h_ex);
    } else {
        if (hipMalloc(&d_box, (size_t)n * 16) != hipSuccess || hipMalloc(&d_red, (size_t)m * 16) != hipSuccess ||
            hipMalloc(&d_ex, 16) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&p_box), (size_t)n * 16, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&p_ex), 16, hipHostMallocDefault) != hipSuccess) {
            cleanup();
            return set_error(MVF_ENOMEM, "device or pinned allocation failed");
        }
    }

    std::priority_queue<Node, std::vector<Node>, Later> open;
    open.push(Node{-INFINITY, 0, std::vector<double>(box, box + 2 * n)});
    int64_t next_id = 1, nodes = 0, subdomains = 0, launches = 0;
    double ub = INFINITY, pruned_lo = INFINITY;
    int status = 1;
    std::vector<Node> take;
    std::vector<int32_t> splits((size_t)K * n);
    std::vector<double> widths(n), filtered(K), centre_ub(K);
    while (!open.empty()) {
        if (ub - open.top().lb <= gap) {
            status = 0;
            break;
        }
        if (nodes >= opt->max_nodes) break;
        take.clear();
        const int64_t room = std::min<int64_t>(K, opt->max_nodes - nodes);
        while (!open.empty() && (int64_t)take.size() < room) {
            Node nd = open.top();
            open.pop();
            if (nd.lb >= ub - gap) {
                pruned_lo = std::min(pruned_lo, nd.lb);
                continue;
            }
            take.push_back(std::move(nd));
        }
        if (take.empty()) continue;
        if (opt->fbbt_rounds > 0) {
            // tighten the taken boxes; drop those proven to hold no feasible point below ub
            const int tc = (int)take.size();
            for (int q = 0; q < tc; ++q) std::memcpy(p_fb + (size_t)q * n * 2, take[q].box.data(), (size_t)n * 16);
            rc = hipMemcpyAsync(d_fb_in, p_fb, (size_t)tc * n * 16, hipMemcpyHostToDevice, stream) == hipSuccess
                     ? MVF_OK : set_error(MVF_EHIP, "hipMemcpyAsync");
            if (rc == MVF_OK)
                rc = mvf_fbbt(tape, tc, d_fb_in, ub, opt->fbbt_rounds, d_fb_out, d_fb_st, d_fb_ws, fb_ws, stream);
            if (rc == MVF_OK &&
                (hipMemcpyAsync(p_fb, d_fb_out, (size_t)tc * n * 16, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                 hipMemcpyAsync(p_fb_st, d_fb_st, (size_t)tc * 4, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                 hipStreamSynchronize(stream) != hipSuccess))
                rc = set_error(MVF_EHIP, "bound tightening copies");
            if (rc != MVF_OK) { cleanup(); return rc; }
            std::vector<Node> kept;
            for (int q = 0; q < tc; ++q) {
                if (p_fb_st[q]) continue;
                std::memcpy(take[q].box.data(), p_fb + (size_t)q * n * 2, (size_t)n * 16);
                kept.push_back(std::move(take[q]));
            }
            nodes += tc - (int64_t)kept.size();
            take.swap(kept);
            if (take.empty()) continue;
        }
        const int cnt = (int)take.size();
        for (int q = 0; q < cnt; ++q) {
            for (int i = 0; i < n; ++i) widths[i] = take[q].box[2 * i + 1] - take[q].box[2 * i];
            const int64_t c = mvf_splits(opt->split_rule, n, widths.data(), opt->subdomains_per_node,
                                         &splits[(size_t)q * n]);
            if (c < 1) { cleanup(); return c < 0 ? (int)c : set_error(MVF_EINVAL, "partitioning failed"); }
            subdomains += c;
        }
        if (K > 1) {
            for (int q = 0; q < cnt; ++q) {
                std::memcpy(h_boxes + (size_t)q * n * 2, take[q].box.data(), (size_t)n * 16);
                std::memcpy(h_splits + (size_t)q * n, &splits[(size_t)q * n], (size_t)n * 4);
            }
            rc = mvf_batch_graph_launch(g, cnt, stream);
            if (rc == MVF_OK && hipStreamSynchronize(stream) != hipSuccess) rc = set_error(MVF_EHIP, "stream sync");
            if (rc != MVF_OK) { cleanup(); return rc; }
            for (int q = 0; q < cnt; ++q) {
                if (h_status[q] != 0) {
                    cleanup();
                    return set_error(MVF_ELIMIT, "a node's partition exceeds the batched breakpoint table");
                }
                filtered[q] = h_ex[2 * q];
                centre_ub[q] = h_ex[2 * q + 1];
            }
            ++launches;
        } else {
            size_t need = 0;
            rc = mvf_bound_workspace(tape, splits.data(), opt->mode, opt->grad, &need);
            if (rc != MVF_OK) { cleanup(); return rc; }
            if (need > ws_bytes) {
                hipFree(d_ws);
                d_ws = nullptr;
                if (hipMalloc(&d_ws, need) != hipSuccess) { cleanup(); return set_error(MVF_ENOMEM, "hipMalloc workspace"); }
                ws_bytes = need;
            }
            std::memcpy(p_box, take[0].box.data(), (size_t)n * 16);
            mvf_bound_args a;
            std::memset(&a, 0, sizeof a);
            a.box = d_box;
            a.splits = splits.data();
            a.mode = opt->mode;
            a.grad = opt->grad;
            a.reduced = d_red;
            a.workspace = d_ws;
            a.workspace_bytes = ws_bytes;
            a.tuning = opt->tuning;
            a.extra = d_ex;
            if (hipMemcpyAsync(d_box, p_box, (size_t)n * 16, hipMemcpyHostToDevice, stream) != hipSuccess)
                rc = set_error(MVF_EHIP, "hipMemcpyAsync");
            if (rc == MVF_OK) rc = mvf_bound(tape, &a, stream);
            if (rc == MVF_OK && (hipMemcpyAsync(p_ex, d_ex, 16, hipMemcpyDeviceToHost, stream) != hipSuccess ||
                                 hipStreamSynchronize(stream) != hipSuccess))
                rc = set_error(MVF_EHIP, "result copy");
            if (rc != MVF_OK) { cleanup(); return rc; }
            filtered[0] = p_ex[0];
            centre_ub[0] = p_ex[1];
            ++launches;
        }
        nodes += cnt;
        for (int q = 0; q < cnt; ++q) ub = std::min(ub, centre_ub[q]);
        for (int q = 0; q < cnt; ++q) {
            const double lo = std::max(take[q].lb, filtered[q]);
            if (lo >= ub - gap) {
                if (std::isfinite(lo)) pruned_lo = std::min(pruned_lo, lo);
                continue;
            }
            const std::vector<double> &b = take[q].box;
            int wi = 0;
            for (int i = 1; i < n; ++i)
                if (b[2 * i + 1] - b[2 * i] > b[2 * wi + 1] - b[2 * wi]) wi = i;
            const double mid = 0.5 * (b[2 * wi] + b[2 * wi + 1]);
            Node left{lo, next_id, b}, right{lo, next_id + 1, b};
            left.box[2 * wi + 1] = mid;
            right.box[2 * wi] = mid;
            next_id += 2;
            open.push(std::move(left));
            open.push(std::move(right));
        }
    }
    if (open.empty() && status == 1) status = std::isfinite(ub) ? 0 : 2;
    const double open_lo = open.empty() ? INFINITY : open.top().lb;
    res->lower = std::min(std::min(open_lo, pruned_lo), ub);
    res->upper = ub;
    res->nodes = nodes;
    res->subdomains = subdomains;
    res->launches = launches;
    res->open = (int32_t)open.size();
    res->status = status;
    res->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    cleanup();
    return MVF_OK;
}
