"""Benchmark: MVF subdomain bounds per second on one MI355X.

Headline step = one call of the whole bounding path on one node box of the
mid workload (6 variables, a 200-op objective and three 80-op constraints,
8^6 = 262,144 subdomains) in the plain form: forward (tangent) mode, one
launch per box -- subdomain generation, point pass, tangent passes, MVF
intersected with the NIE, min/max reduction with argmin.  The tape is
specialised first (straight-line kernel compiled at run time; the compile
time is reported, outside the timed region); --engine interp times the
interpreter kernel instead, which is also reported among the forms.  Inputs
are resident in HBM before the timed region.

The same JSON line carries the comparison of the two forms on the batch
workload (512 B&B-like nodes of [-3,3]^8 with 2^10..2^18 subdomains each,
a 400-op objective and two 150-op constraints):
  * plain    -- forward mode, one launch per node, synchronised per node as a
                branch-and-bound loop would;
  * adjoint+batched -- reverse-mode adjoint, all nodes in one persistent
                launch replayed from a HIP graph (staging H2D and result D2H
                inside the graph),
each with the interpreter and with the specialised kernels; the forward and
adjoint rates of both kernel kinds on mid; the adjoint on the 32-variable
differentiation workload; and the end-to-end branch and bound.  ``value`` is subdomain-bounds/s (one subdomain-bound = the bounds
of the objective and all constraints on one subdomain).  ``roofline`` relates
the bounding kernel to the FP64 VALU issue rate; ``cpu_baseline`` times the
CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 VALU issue rate: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz, one
# non-FMA FP64 op per lane per clock (interval code is FMA-free).  The
# published 78.6 TFLOP/s counts an FMA as two operations.
FP64_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9          # 39.3e12 op/s
FP64_PUBLISHED_PEAK = 78.6e12
# HBM bytes per launch of the headline kernel from rocprofv3 counters (FETCH_SIZE x 2.00 + WRITE_SIZE x 1.00,
# the factors from a 256 MiB copy in the same runs), valid only for the kernel build and tape they were
# taken on: (engine, grad, tape hash) -> bytes
TRAFFIC = {("spec", "fwd", "aa75c5b416e4faea"): (7824.2 * 2.0 + 41133.4) * 1024,
           ("spec", "rev", "aa75c5b416e4faea"): (141888.8 * 2.0 + 278716.2) * 1024}
METRIC = "MVF subdomain bounds/sec (obj+constraints) and % FP64 vector peak; adjoint+batched vs plain"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed steps first: the clocks reach their sustained level under load")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="headline only (used under the profiler)")
    ap.add_argument("--bnb-nodes", type=int, default=1000, help="B&B node limit of the e2e comparison (0: skip)")
    ap.add_argument("--engine", choices=["spec", "interp"], default="spec",
                    help="headline kernel: the tape's specialised kernel or the interpreter")
    ap.add_argument("--grad", choices=["fwd", "rev"], default="fwd",
                    help="gradient mode of the timed step (the headline configuration is forward mode; "
                         "rev times the adjoint, for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device-to-device copy, the reference for HBM counters")
    return ap.parse_args()


def cpu_baseline(w, seconds: float) -> dict:
    """The oracle (untuned) on a contiguous sample of the workload's subdomains."""
    from oracle import oracle as O
    threads = min(os.cpu_count() or 1, 16)
    S = w.n_sub
    done, k0, t0 = 0, 0, time.perf_counter()
    chunk = 64 * threads
    while time.perf_counter() - t0 < seconds and k0 < S:
        k1 = min(S, k0 + chunk)
        O.bound(w.tape, w.box, w.splits, mode=O.MODE_BOTH, grad=O.GRAD_FWD, k_range=(k0, k1), per_sub=False,
                nthreads=threads)
        done += k1 - k0
        k0 = k1
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "subdomain-bounds/s", "cores": threads, "kind": "oracle",
            "sample": f"subdomains 0..{done - 1} of the {w.name} workload ({done} of {S}), "
                      f"forward-mode MVF, {dt:.1f} s"}


def time_calls(launch, steps: int, warmup: int, stream) -> float:
    """Average ms per call between HIP events on ``stream``."""
    import torch
    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        launch()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def ref_ops(st, grad: str, engine: str) -> int:
    """Algorithmic FP64 ops per subdomain of a kernel: the reference count of its
    gradient mode; the specialised forward kernels skip structurally zero
    tangent components, so theirs is the count without them."""
    if grad == "rev":
        return st.ref_ops_rev
    return st.ref_ops_fwd_sparse if engine == "spec" else st.ref_ops_fwd


def forms(seed: int, mid_tape) -> dict:
    """The other kernels and forms.  mid_tape: the headline's tape handle,
    specialised in both gradient modes."""
    import torch

    from paper_2507_20769_amd import inputs as I
    from paper_2507_20769_amd import mvf
    out = {}
    stream = torch.cuda.current_stream()
    # mid: forward and adjoint, interpreter and specialised kernels
    w = I.mid(seed)
    st = mid_tape.stats()
    box = torch.tensor(w.box, device="cuda")
    for grad in ("fwd", "rev"):
        for engine in ("interp", "spec"):
            ref = ref_ops(st, grad, engine)
            call = mvf.BoundCall(mid_tape, box, w.splits, mode="both", grad=grad, engine=engine)
            ms = time_calls(call.launch, 100, 100, stream)
            name = {"fwd": "forward", "rev": "adjoint"}[grad] + {"interp": "_interpreter", "spec": "_specialised"}[engine]
            out[f"mid_{name}"] = {"subdomain_bounds_per_s": w.n_sub / (ms * 1e-3), "ms": ms,
                                  "ref_ops_per_subdomain": ref,
                                  "issue_peak_frac": ref * w.n_sub / (ms * 1e-3) / FP64_ISSUE_PEAK}
    # the 32-variable differentiation workload: adjoint, interpreter (its tape is far above the
    # specialisation size limit)
    w = I.diff(seed)
    h = mvf.Tape(w.tape)
    st = h.stats()
    call = mvf.BoundCall(h, torch.tensor(w.box, device="cuda"), w.splits, mode="both", grad="rev")
    ms = time_calls(call.launch, 4, 1, stream)
    out["diff_adjoint_interpreter"] = {"subdomain_bounds_per_s": w.n_sub / (ms * 1e-3), "ms": ms,
                                       "subdomains": w.n_sub, "ref_ops_per_subdomain": st.ref_ops_rev,
                                       "issue_peak_frac": st.ref_ops_rev * w.n_sub / (ms * 1e-3) / FP64_ISSUE_PEAK}
    h.close()
    # batch workload: plain forward per node vs batched graphs
    bw = I.batch(seed)
    h = mvf.Tape(bw.tape)
    st = h.stats()
    total = int(bw.n_sub.sum())
    boxes = torch.tensor(bw.boxes, device="cuda")
    red_plain = np.empty((len(bw.boxes), bw.tape.n_roots, 2))
    spec_info = h.specialize(grad="auto")
    t_plain = {}
    same_plain = None
    for engine in ("interp", "spec"):
        calls = [mvf.BoundCall(h, boxes[i], bw.splits[i], mode="both", grad="fwd", engine=engine)
                 for i in range(len(bw.boxes))]

        def plain():
            for c in calls:
                c.launch(stream)
                stream.synchronize()               # a B&B loop needs each node's bound before going on
        plain()
        t0 = time.perf_counter()
        plain()
        t_plain[engine] = time.perf_counter() - t0
        red = np.stack([c.reduced.cpu().numpy() for c in calls])
        if engine == "interp":
            red_plain[:] = red
        else:
            same_plain = float(np.mean(red == red_plain))   # the two kernels agree bitwise up to libm
    gs = torch.cuda.Stream()
    t_graph, red_graph = {}, {}
    for grad, engine in (("rev", "interp"), ("rev", "spec"), ("fwd", "spec")):
        tu = mvf.Tuning(grad=0 if grad == "fwd" else 1, chunk=0, grid_blocks=0, best_ms=0.0, sub_per_lane=1,
                        engine=mvf.MVF_ENGINE[engine])
        g = mvf.BatchGraph(h, len(bw.boxes), total, mode="both", grad=grad, tuning=tu)

        def batched():
            g.launch(bw.boxes, bw.splits, stream=gs)
            gs.synchronize()
        batched()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            batched()
        t_graph[(grad, engine)] = (time.perf_counter() - t0) / reps
        red_b, _, status = g.result()
        assert (status == 0).all()
        red_graph[(grad, engine)] = red_b
        g.close()
    # same accuracy: both gradient modes pass parity with their own oracle mode; report how the
    # two gradient enclosures compare on the objective lower bound
    d = red_graph[("rev", "spec")][:, 0, 0] - red_plain[:, 0, 0]
    scale = np.maximum(1.0, np.abs(red_plain[:, 0, :]).max(axis=1))
    best_plain = min(t_plain.values())
    out["batch"] = {
        "nodes": len(bw.boxes), "subdomains": total, "specialisation_compile_s": spec_info["seconds"],
        "plain_forward_per_node_interpreter": {"subdomain_bounds_per_s": total / t_plain["interp"],
                                               "s": t_plain["interp"], "tangent_chunk": st.tangent_chunk},
        "plain_forward_per_node_specialised": {"subdomain_bounds_per_s": total / t_plain["spec"],
                                               "s": t_plain["spec"], "tangent_chunk": spec_info["chunk"],
                                               "hull_endpoints_equal_to_interpreter": same_plain},
        "adjoint_batched_graph_interpreter": {"subdomain_bounds_per_s": total / t_graph[("rev", "interp")],
                                              "s": t_graph[("rev", "interp")]},
        "adjoint_batched_graph_specialised": {"subdomain_bounds_per_s": total / t_graph[("rev", "spec")],
                                              "s": t_graph[("rev", "spec")],
                                              "hull_endpoints_equal_to_interpreter":
                                                  float(np.mean(red_graph[("rev", "spec")] ==
                                                                red_graph[("rev", "interp")]))},
        "forward_batched_graph_specialised": {"subdomain_bounds_per_s": total / t_graph[("fwd", "spec")],
                                              "s": t_graph[("fwd", "spec")]},
        "speedup_adjoint_batched_vs_plain": best_plain / t_graph[("rev", "spec")],
        "speedup_adjoint_batched_vs_plain_same_kernel_kind": {
            "interpreter": t_plain["interp"] / t_graph[("rev", "interp")],
            "specialised": t_plain["spec"] / t_graph[("rev", "spec")]},
        "objective_lb_adjoint_minus_forward": {"tighter_frac": float(np.mean(d > 0)),
                                               "looser_frac": float(np.mean(d < 0)),
                                               "mean_rel": float(np.mean(d / scale))},
    }
    h.close()
    return out


def bnb_forms(seed: int, max_nodes: int) -> dict:
    """NEXT-1: host B&B on the e2e problem (10 variables, an objective and five
    inequality constraints, [-3, 3]^10, 2^16 subdomains per node), plain
    forward mode one node per launch vs reverse mode 16 nodes per graph replay."""
    from paper_2507_20769_amd import inputs as I
    from paper_2507_20769_amd import mvf
    tape = I.e2e_tape(seed)
    h = mvf.Tape(tape)
    h.set_root_kinds([0] + [1] * (tape.n_roots - 1))
    box = np.array([[-3.0, 3.0]] * tape.n_vars)
    out = {"problem": "e2e", "n_vars": tape.n_vars, "roots": tape.n_roots, "subdomains_per_node": 1 << 16,
           "max_nodes": max_nodes, "abs_gap": 1e-4}
    for name, k, grad, fb in (("plain_forward_per_node", 1, "fwd", 0), ("adjoint_batched_graph", 16, "rev", 0),
                              ("adjoint_batched_graph_with_bound_tightening", 16, "rev", 2)):
        r = mvf.bnb_solve(h, box, max_nodes=max_nodes, gap=1e-4, budget=1 << 16, nodes_per_launch=k, grad=grad,
                          fbbt_rounds=fb)
        out[name] = {"nodes_per_s": r["nodes"] / r["seconds"], "subdomain_bounds_per_s": r["subdomains"] / r["seconds"],
                     "seconds": r["seconds"], "nodes": r["nodes"], "lower": r["lower"], "upper": r["upper"],
                     "gap": r["upper"] - r["lower"], "status": r["status"], "launches": r["launches"]}
    out["speedup_adjoint_batched_vs_plain"] = (out["plain_forward_per_node"]["seconds"] /
                                               out["adjoint_batched_graph"]["seconds"])
    h.close()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2507_20769_amd import inputs as I
    from paper_2507_20769_amd import mvf

    torch.cuda.init()
    if args.copy_calibration:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")     # 256 MiB
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = I.mid(args.seed)
    tape = mvf.Tape(w.tape)
    st = tape.stats()
    # both gradient modes: the forms below time the adjoint kernels of the same tape
    spec = tape.specialize(grad="auto") if args.engine == "spec" or not args.no_forms else None
    box = torch.tensor(w.box, dtype=torch.float64, device="cuda")
    call = mvf.BoundCall(tape, box, w.splits, mode="both", grad=args.grad, engine=args.engine)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    ms = time_calls(lambda: call.launch(stream), args.steps, args.warmup, stream)
    wall = time.perf_counter() - t0
    S = w.n_sub
    value = S / (ms * 1e-3)
    ops = ref_ops(st, args.grad, args.engine)
    achieved = ops * S / (ms * 1e-3)                      # algorithmic FP64 ops per second
    reduced = call.reduced.cpu().numpy()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "subdomain-bounds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "mid", "form": "plain: " + ("forward-mode" if args.grad == "fwd" else "adjoint") +
                   " MVF, one launch per node box",
                   "n_vars": w.tape.n_vars, "tape_ops": w.tape.n_ops(), "roots": w.tape.n_roots,
                   "subdomains": S, "splits": [int(s) for s in w.splits], "seed": args.seed,
                   "tape_hash": w.tape.digest(), "engine": args.engine,
                   "tangent_chunk": spec["chunk"] if args.engine == "spec" else st.tangent_chunk},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_ISSUE_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP64_ISSUE_PEAK,
                     "traffic": TRAFFIC.get((args.engine, args.grad, w.tape.digest())),
                     "kernel": {("spec", "fwd"): "mvf_spec_bound", ("spec", "rev"): "mvf_spec_bound_rev",
                                ("interp", "fwd"): f"bound_kernel<{st.tangent_chunk},false>",
                                ("interp", "rev"): "bound_kernel<0,true>"}[(args.engine, args.grad)] +
                               " (+ the 1-block finish kernel inside the timed call)",
                     "ops_per_subdomain": ops,
                     "dense_ops_per_subdomain": st.ref_ops_fwd if args.grad == "fwd" else st.ref_ops_rev,
                     "frac_of_published_78.6": achieved / FP64_PUBLISHED_PEAK},
        "wall_s": wall,
        "objective_lower_bound": float(reduced[0, 0]),
    }
    if spec:
        out["specialisation"] = {"kernels": "tangent mode and adjoint", "compile_s": spec["seconds"],
                                 "from_cache": bool(spec["from_cache"]), "code_units": spec["code_units"],
                                 "code_bytes": spec["code_bytes"], "waves_per_simd": spec["waves"]}
    if not args.no_forms:
        out["forms"] = forms(args.seed, tape)
        if args.bnb_nodes > 0:
            out["forms"]["bnb"] = bnb_forms(args.seed, args.bnb_nodes)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
