"""Benchmark: MVF subdomain bounds per second on one MI355X.

Headline step = one call of the whole bounding path on one node box of the
mid workload (6 variables, a 200-op objective and three 80-op constraints,
8^6 = 262,144 subdomains) in the plain form: forward (tangent) mode, one
launch per box -- subdomain generation, point pass, tangent passes, MVF
intersected with the NIE, min/max reduction with argmin -- in the tape's
specialised kernel (compiled at run time, or read from the code-object cache
that the build fills; outside the timed region).  Inputs are resident in HBM
before the timed region.  Before the W warm-up steps, the step runs for about
one second more, untimed, so that the clocks reach their sustained level.

The same JSON line carries the other forms, each with its own roofline
fraction (algorithmic FP64 ops per second over the FP64 issue rate):
  * mid: forward and adjoint, interpreter and specialised kernels;
  * tiny (2 variables, 4,096 subdomains): forward mode per call (launch-bound);
  * diff (32 variables, 2^20 subdomains): the adjoint, interpreter (record
    tape) and specialised (checkpointed recomputation);
  * batch (512 B&B-like nodes of [-3,3]^8, 2^10..2^18 subdomains each, a
    400-op objective and two 150-op constraints): plain = forward mode, one
    launch per node, synchronised per node as a branch-and-bound loop would;
    adjoint+batched = reverse-mode adjoint, all nodes in one persistent
    launch replayed from a HIP graph in the autotuned configuration (the
    metric's defining comparison); forward+batched likewise;
  * e2e: the host branch and bound (10 variables, a 500-op objective and five
    200-op constraints, 2^16 subdomains per node) to absolute gap 1e-4 or
    10,000 nodes, plain forward per node against the batched adjoint.
``value`` is subdomain-bounds/s (one subdomain-bound = the bounds of the
objective and all constraints on one subdomain).  ``cpu_baseline`` times the
CPU oracle on a bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 VALU issue rate: 256 CUs x 4 SIMDs x 16 FP64 lanes x 2.4 GHz, one
# FP64 operation per lane per clock (interval code is FMA-free, so an FMA
# counted as two operations -- the published 78.6 TFLOP/s -- is out of reach).
FP64_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9          # 39.3e12 op/s
FP64_PUBLISHED_PEAK = 78.6e12
# HBM bytes per launch from rocprofv3 counters (FETCH_SIZE x 2.00 + WRITE_SIZE x
# 1.00, the factors from a 256 MiB copy in the same runs), valid only for the
# kernel build and tape they were taken on: (engine, grad, tape hash, code
# object bytes) -> bytes, with the profile they come from.  A rebuilt kernel
# of another size finds no entry and reports null.
TRAFFIC = {("spec", "fwd", "aa75c5b416e4faea", 944920): (12576.5 * 2.0 + 57174.5) * 1024}
TRAFFIC_SOURCE = {("spec", "fwd", "aa75c5b416e4faea", 944920):
                  "profiles/mvf_spec_bound_mid.md (rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, per dispatch)"}
METRIC = "MVF subdomain bounds/sec (obj+constraints) and % FP64 vector peak; adjoint+batched vs plain"
PEAK_UNIT = "T FP64 op/s (one VALU issue slot per op, FMA = 1)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--prewarm-s", type=float, default=1.0,
                    help="seconds of untimed steps before the warm-up steps (clock ramp)")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=8.0, help="oracle time per CPU-baseline leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="headline only (used under the profiler)")
    ap.add_argument("--forms", default="mid,tiny,diff,batch,bnb", help="comma list of the forms to run")
    ap.add_argument("--bnb-nodes", type=int, default=10000, help="B&B node limit of the e2e comparison (0: skip)")
    ap.add_argument("--engine", choices=["spec", "interp"], default="spec",
                    help="headline kernel: the tape's specialised kernel or the interpreter")
    ap.add_argument("--grad", choices=["fwd", "rev"], default="fwd",
                    help="gradient mode of the timed step (the headline configuration is forward mode; "
                         "rev times the adjoint, for profiling)")
    ap.add_argument("--workload", choices=["mid", "diff", "batch"], default="mid",
                    help="headline workload (mid; diff for profiling the 32-variable adjoint; batch for "
                         "profiling the batched kernels: one step = plan + persistent kernel + per-node "
                         "finish over the 512 nodes, in --grad mode, specialised, default tuning)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 256 MiB device-to-device copy, the reference for HBM counters")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def gpu_clocks() -> dict:
    """The GPU's current clock levels and power cap from the driver's sysfs files
    (sampled right after the timed steps; the clock under load comes from the
    counters: busy cycles over kernel time).  Files only: no child process."""
    import glob
    out = {}
    for dev in sorted(glob.glob("/sys/class/drm/card*/device")):
        for name in ("pp_dpm_sclk", "pp_dpm_mclk", "pp_dpm_fclk"):
            try:
                cur = [ln.split(":", 1)[1].strip().rstrip("*").strip()
                       for ln in open(os.path.join(dev, name)) if ln.rstrip().endswith("*")]
            except OSError:
                continue
            if cur:
                out[name[7:]] = cur[0]
        for cap in glob.glob(os.path.join(dev, "hwmon", "hwmon*", "power1_cap")):
            try:
                out["power_cap_w"] = int(open(cap).read()) / 1e6
            except (OSError, ValueError):
                pass
        if out:
            out["device"] = dev
            return out
    return {"error": "no clock files under /sys/class/drm"}


def _oracle_rate(O, cases, grad: int, threads: int, seconds: float) -> dict:
    """The oracle over (tape, box, splits, ks) cases, 64 subdomains per thread
    at a time, until the cases are done or ``seconds`` have passed."""
    done, t0 = 0, time.perf_counter()
    for tape, box, splits, ks in cases:
        for i in range(0, len(ks), 64 * threads):
            O.bound(tape, box, splits, mode=O.MODE_BOTH, grad=grad, ks=ks[i:i + 64 * threads], per_sub=False,
                    nthreads=threads)
            done += len(ks[i:i + 64 * threads])
            if time.perf_counter() - t0 >= seconds:
                break
        if time.perf_counter() - t0 >= seconds:
            break
    t = time.perf_counter() - t0
    return {"value": done / t, "subdomains": done, "seconds": t}


def other_workload_rates(seed: int, threads: int, seconds: float) -> dict:
    """The oracle's forward and reverse modes on seeded samples of the 32-variable
    and batch workloads (16,384 subdomains each at most, ``seconds`` per leg)."""
    from oracle import oracle as O
    from paper_2507_20769_amd import inputs as I
    rng = np.random.default_rng(seed)
    d = I.diff(seed)
    diff_case = [(d.tape, d.box, d.splits, np.sort(rng.choice(d.n_sub, 16384, replace=False)))]
    bw = I.batch(seed)
    nodes = np.sort(rng.choice(len(bw.boxes), 16, replace=False))
    batch_cases = [(bw.tape, bw.boxes[i], bw.splits[i],
                    np.sort(rng.choice(int(bw.n_sub[i]), min(1024, int(bw.n_sub[i])), replace=False)))
                   for i in nodes]
    out = {}
    for name, cases in (("diff", diff_case), ("batch", batch_cases)):
        for gname, grad in (("adjoint", O.GRAD_REV), ("forward", O.GRAD_FWD)):
            r = _oracle_rate(O, cases, grad, threads, seconds)
            r["unit"] = "subdomain-bounds/s"
            r["sample"] = ("seeded 16,384 of the 1,048,576 subdomains" if name == "diff" else
                           "seeded 1,024 subdomains (or all) of each of 16 seeded nodes of the 512")
            out[f"{name}_{gname}"] = r
    return out


def cpu_baseline(w, seconds: float, other: bool = True) -> dict:
    """The oracle (untuned) on contiguous samples of the workload's subdomains:
    one thread, then every host core the process may use; other: also its rates
    on samples of the 32-variable and batch workloads, every core."""
    from oracle import oracle as O
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    S = w.n_sub

    def leg(threads, k0):
        done, t0 = 0, time.perf_counter()
        chunk = 64 * threads
        while time.perf_counter() - t0 < seconds and k0 + done < S:
            k1 = min(S, k0 + done + chunk)
            O.bound(w.tape, w.box, w.splits, mode=O.MODE_BOTH, grad=O.GRAD_FWD, k_range=(k0 + done, k1),
                    per_sub=False, nthreads=threads)
            done = k1 - k0
        return done, time.perf_counter() - t0

    n1, t1 = leg(1, 0)
    na, ta = leg(cores, n1)
    return {"value": na / ta, "unit": "subdomain-bounds/s", "cores": cores, "kind": "oracle",
            "sample": f"subdomains {n1}..{n1 + na - 1} of the {w.name} workload ({na} of {S}), forward-mode MVF "
                      f"with MVF and NIE, {ta:.1f} s on {cores} threads",
            "cpu_model": cpu_model(),
            "one_thread": {"value": n1 / t1, "sample": f"subdomains 0..{n1 - 1}, {t1:.1f} s"},
            "other_workloads": other_workload_rates(1, cores, min(seconds, 4.0)) if other else None}


def time_calls(launch, steps: int, warmup: int, stream, prewarm_s: float = 0.0, per_step: bool = False):
    """Average ms per call between HIP events on ``stream`` (and, with
    per_step, each call's own events for the median and minimum)."""
    import torch
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < prewarm_s:
        for _ in range(20):
            launch()
        torch.cuda.synchronize()
    for _ in range(warmup):
        launch()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] if per_step else None
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        if per_step:
            ev[i].record(stream)
        launch()
    if per_step:
        ev[steps].record(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    avg = e0.elapsed_time(e1) / steps
    if not per_step:
        return avg
    each = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(steps)])
    return avg, float(np.median(each)), float(each.min())


def kernel_times(call, steps: int, stream) -> dict:
    """Two more passes of K steps of ``call`` (a BoundCall): one with an event before every
    step (each step's own time: median and minimum), one with events around every step's
    bounding kernel alone (recorded by the library on the launch stream).  Each event
    record costs a few microseconds of the step it sits in."""
    import torch
    mk = lambda k: [torch.cuda.Event(enable_timing=True) for _ in range(k)]
    s0 = mk(steps + 1)
    torch.cuda.synchronize()
    for i in range(steps):
        s0[i].record(stream)
        call.launch(stream)
    s0[steps].record(stream)
    torch.cuda.synchronize()
    st = np.array([s0[i].elapsed_time(s0[i + 1]) for i in range(steps)])
    ks, ke = mk(steps), mk(steps)
    for i in range(steps):
        call.time_kernel(ks[i], ke[i])
        call.launch(stream)
    torch.cuda.synchronize()
    call.time_kernel(None, None)
    k = np.array([ks[i].elapsed_time(ke[i]) for i in range(steps)])
    return {"mean_ms": float(k.mean()), "median_ms": float(np.median(k)), "min_ms": float(k.min()),
            "step_median_ms": float(np.median(st)), "step_min_ms": float(st.min())}


def frac(ops: int, n_sub: float, seconds: float) -> float:
    return ops * n_sub / seconds / FP64_ISSUE_PEAK


def ref_ops(st, grad: str, engine: str) -> int:
    """Algorithmic FP64 ops per subdomain of a kernel: the reference count of its
    gradient mode; the specialised forward kernels skip structurally zero
    tangent components, so theirs is the count without them."""
    if grad == "rev":
        return st.ref_ops_rev
    return st.ref_ops_fwd_sparse if engine == "spec" else st.ref_ops_fwd


HBM_PEAK = 8.0e12                               # bytes/s


def checkpoint_bytes(tape, grad: str = "rev") -> int:
    """Bytes per subdomain that the specialised adjoint's checkpoints move by design:
    16 bytes per checkpoint interval stored and per interval loaded (a value several
    segments read is stored once and loaded by each), summed over the roots (counted in
    the generated source at the library's default segment budget)."""
    import re

    from paper_2507_20769_amd import mvf
    src = mvf.spec_source(tape, grad=grad, max_code=10 ** 7)
    return 16 * (len(re.findall(r"spec_ck_st\(L,", src)) + len(re.findall(r"spec_ck_ld\(L,", src)))


def hbm_roofline(bytes_per_sub: int, n_sub: float, seconds: float) -> dict:
    a = bytes_per_sub * n_sub / seconds
    return {"bound": "hbm", "achieved": a / 1e12, "peak": HBM_PEAK / 1e12, "unit": "TB/s",
            "frac": a / HBM_PEAK, "algorithmic_bytes_per_subdomain": bytes_per_sub,
            "what": "checkpoint stores + loads of the checkpointed adjoint"}


def _form(n_sub, seconds, ops, **extra):
    d = {"subdomain_bounds_per_s": n_sub / seconds, "ms": seconds * 1e3, "ref_ops_per_subdomain": ops,
         "issue_peak_frac": frac(ops, n_sub, seconds)}
    d.update(extra)
    return d


def mid_forms(seed: int, mid_tape) -> dict:
    import torch

    from paper_2507_20769_amd import inputs as I
    from paper_2507_20769_amd import mvf
    out = {}
    stream = torch.cuda.current_stream()
    w = I.mid(seed)
    st = mid_tape.stats()
    box = torch.tensor(w.box, device="cuda")
    for grad in ("fwd", "rev"):
        for engine in ("interp", "spec"):
            ref = ref_ops(st, grad, engine)
            call = mvf.BoundCall(mid_tape, box, w.splits, mode="both", grad=grad, engine=engine)
            ms = time_calls(call.launch, 100, 100, stream)
            name = {"fwd": "forward", "rev": "adjoint"}[grad] + {"interp": "_interpreter", "spec": "_specialised"}[engine]
            out[f"mid_{name}"] = _form(w.n_sub, ms * 1e-3, ref)
    return out


def tiny_forms(seed: int) -> dict:
    """The tiny workload (2 variables, 64 x 64 = 4,096 subdomains): one launch is a few
    microseconds of work, so this form measures the per-call latency of the path."""
    import torch

    from paper_2507_20769_amd import inputs as I
    from paper_2507_20769_amd import mvf
    stream = torch.cuda.current_stream()
    w = I.tiny(seed)
    h = mvf.Tape(w.tape)
    st = h.stats()
    info = h.specialize(grad="fwd")
    box = torch.tensor(w.box, device="cuda")
    out = {"subdomains": w.n_sub, "specialisation_compile_s": info["seconds"]}
    for engine in ("interp", "spec"):
        call = mvf.BoundCall(h, box, w.splits, mode="both", grad="fwd", engine=engine)
        ms = time_calls(call.launch, 200, 200, stream)
        out["forward_" + ("interpreter" if engine == "interp" else "specialised")] = _form(
            w.n_sub, ms * 1e-3, ref_ops(st, "fwd", engine), note="launch-bound: bounding + finish kernel per call")
    h.close()
    return out


def diff_forms(seed: int) -> dict:
    """The 32-variable differentiation workload, adjoint: the interpreter's record
    tape against the specialised kernel's checkpointed recomputation."""
    import torch

    from paper_2507_20769_amd import inputs as I
    from paper_2507_20769_amd import mvf
    stream = torch.cuda.current_stream()
    w = I.diff(seed)
    h = mvf.Tape(w.tape)
    st = h.stats()
    box = torch.tensor(w.box, device="cuda")
    info = h.specialize(grad="rev")
    out = {"subdomains": w.n_sub, "n_vars": w.tape.n_vars, "tape_ops": w.tape.n_ops(), "roots": w.tape.n_roots}
    res = {}
    for engine in ("interp", "spec"):
        call = mvf.BoundCall(h, box, w.splits, mode="both", grad="rev", engine=engine)
        ms = time_calls(call.launch, 4, 1, stream)
        res[engine] = call.reduced.cpu().numpy()
        out[f"adjoint_{'interpreter' if engine == 'interp' else 'specialised'}"] = _form(
            w.n_sub, ms * 1e-3, st.ref_ops_rev)
    out["adjoint_specialised"]["hbm_roofline"] = hbm_roofline(checkpoint_bytes(w.tape), w.n_sub,
                                                              out["adjoint_specialised"]["ms"] * 1e-3)
    out["adjoint_specialised"].update({"checkpoint_intervals_per_lane": info["ckpt_intervals"],
                                       "segment_budget": info["ckpt_budget"], "compile_s": info["seconds"],
                                       "from_cache": bool(info["from_cache"])})
    out["adjoint_specialised"]["hull_endpoints_equal_to_interpreter"] = float(np.mean(res["spec"] == res["interp"]))
    h.close()
    return out


def batch_forms(seed: int) -> dict:
    """Plain forward per node vs adjoint+batched (and forward+batched) graphs on
    the batch workload; the batched forms run in the autotuned configuration."""
    import torch

    from paper_2507_20769_amd import inputs as I
    from paper_2507_20769_amd import mvf
    bw = I.batch(seed)
    h = mvf.Tape(bw.tape)
    h.set_root_kinds([0, 1, 1])
    st = h.stats()
    total = int(bw.n_sub.sum())
    boxes = torch.tensor(bw.boxes, device="cuda")
    spec_info = h.specialize(grad="auto")
    stream = torch.cuda.current_stream()
    out = {"nodes": len(bw.boxes), "subdomains": total, "specialisation_compile_s": spec_info["seconds"],
           "specialisation_from_cache": bool(spec_info["from_cache"]),
           "checkpoint_intervals_per_lane": spec_info["ckpt_intervals"]}
    # plain: forward mode, one launch per node, synchronised per node
    t_plain, red_plain = {}, {}
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
        red_plain[engine] = np.stack([c.reduced.cpu().numpy() for c in calls])
        fw = ref_ops(st, "fwd", engine)
        out[f"plain_forward_per_node_{'interpreter' if engine == 'interp' else 'specialised'}"] = _form(
            total, t_plain[engine], fw, tangent_chunk=spec_info["chunk"] if engine == "spec" else st.tangent_chunk)
    out["plain_forward_per_node_specialised"]["hull_endpoints_equal_to_interpreter"] = float(
        np.mean(red_plain["spec"] == red_plain["interp"]))
    # the autotuner on a seeded sample of 64 nodes, per gradient mode (the mode is the caller's)
    rng = np.random.default_rng(seed + 77)
    pick = np.sort(rng.choice(len(bw.boxes), 64, replace=False))
    sb, ss = boxes[pick].contiguous(), torch.tensor(bw.splits[pick], device="cuda")
    tuned = {}
    for grad in ("fwd", "rev"):
        t0 = time.perf_counter()
        tuned[grad] = mvf.autotune(h, sb, ss, mode="both", grad=grad)
        out[f"tuning_{grad}"] = dict(tuned[grad].as_dict(), seconds=time.perf_counter() - t0,
                                     sample="64 seeded nodes of the 512")
    gs = torch.cuda.Stream()
    t_graph, red_graph, t_kernel = {}, {}, {}
    for grad, engine in (("rev", "interp"), ("rev", "spec"), ("fwd", "spec")):
        tu = tuned[grad] if engine == "spec" else mvf.Tuning(grad=1, chunk=0, grid_blocks=0, best_ms=0.0,
                                                             sub_per_lane=1, engine=mvf.MVF_ENGINE["interp"])
        if engine == "spec" and tu.engine != mvf.MVF_ENGINE["spec"]:   # the tuner preferred the interpreter
            tu = mvf.Tuning(**dict(tu.as_dict(), engine=mvf.MVF_ENGINE["spec"], chunk=0))
        g = mvf.BatchGraph(h, len(bw.boxes), total, mode="both", grad=grad, tuning=tu)

        def batched():
            g.launch(bw.boxes, bw.splits, stream=gs)
            gs.synchronize()
        batched()
        reps = 7
        each = []
        for _ in range(reps):                      # each replay on the host clock: the median
            t0 = time.perf_counter()
            batched()
            each.append(time.perf_counter() - t0)
        t_graph[(grad, engine)] = float(np.median(each))
        red_b, _, status = g.result()
        assert (status == 0).all()
        red_graph[(grad, engine)] = red_b
        g.close()
        # the kernel sequence alone (plan, persistent kernel, per-node finish) with HIP events
        call = mvf.BatchCall(h, boxes, torch.tensor(bw.splits, device="cuda"), mode="both", grad=grad, tuning=tu)
        t_kernel[(grad, engine)] = time_calls(lambda: call.launch(stream), 3, 1, stream) * 1e-3
    for (grad, engine), t in t_graph.items():
        name = f"{'adjoint' if grad == 'rev' else 'forward'}_batched_graph_" + \
               ("interpreter" if engine == "interp" else "specialised")
        ops = ref_ops(st, grad, engine)
        out[name] = _form(total, t, ops, kernel_only=_form(total, t_kernel[(grad, engine)], ops),
                          timing="graph replay with staging H2D and result D2H, host clock, median of 7 "
                                 "replays; kernel_only: HIP events around plan + persistent kernel + per-node "
                                 "finish, mean of 3 calls")
    out["adjoint_batched_graph_specialised"]["kernel_only"]["hbm_roofline"] = hbm_roofline(
        checkpoint_bytes(bw.tape), total, t_kernel[("rev", "spec")])
    out["adjoint_batched_graph_specialised"]["hull_endpoints_equal_to_interpreter"] = float(
        np.mean(red_graph[("rev", "spec")] == red_graph[("rev", "interp")]))
    best_plain = min(t_plain.values())
    out["speedup_adjoint_batched_vs_plain"] = best_plain / t_graph[("rev", "spec")]
    out["speedup_adjoint_batched_vs_plain_same_kernel_kind"] = {
        "interpreter": t_plain["interp"] / t_graph[("rev", "interp")],
        "specialised": t_plain["spec"] / t_graph[("rev", "spec")]}
    out["speedup_adjoint_batched_vs_forward_batched"] = t_graph[("fwd", "spec")] / t_graph[("rev", "spec")]
    # same accuracy: both gradient modes pass parity with their own oracle mode; report how the
    # two gradient enclosures compare on the objective lower bound (per node, scaled by the node's bounds)
    d = red_graph[("rev", "spec")][:, 0, 0] - red_plain["spec"][:, 0, 0]
    scale = np.maximum(1.0, np.abs(red_plain["spec"][:, 0, :]).max(axis=1))
    out["objective_lb_adjoint_minus_forward"] = {"tighter_frac": float(np.mean(d > 0)),
                                                 "looser_frac": float(np.mean(d < 0)),
                                                 "mean_rel": float(np.mean(d / scale))}
    h.close()
    return out


def bnb_forms(seed: int, max_nodes: int) -> dict:
    """The host B&B on the e2e problem (10 variables, an objective and five
    inequality constraints, [-3, 3]^10, 2^16 subdomains per node) to gap 1e-4
    or the node limit: plain forward mode one node per launch vs reverse mode
    16 nodes per graph replay (specialised kernels for both)."""
    from paper_2507_20769_amd import inputs as I
    from paper_2507_20769_amd import mvf
    tape = I.e2e_tape(seed)
    h = mvf.Tape(tape)
    h.set_root_kinds([0] + [1] * (tape.n_roots - 1))
    info = h.specialize(grad="auto")
    box = np.array([[-3.0, 3.0]] * tape.n_vars)
    out = {"problem": "e2e", "n_vars": tape.n_vars, "roots": tape.n_roots, "subdomains_per_node": 1 << 16,
           "max_nodes": max_nodes, "abs_gap": 1e-4, "specialisation_compile_s": info["seconds"],
           "specialisation_from_cache": bool(info["from_cache"])}
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


def batch_profile(args) -> dict:
    """The batched kernel sequence alone on the batch workload, for the profiler."""
    import torch

    from paper_2507_20769_amd import inputs as I
    from paper_2507_20769_amd import mvf
    bw = I.batch(args.seed)
    h = mvf.Tape(bw.tape)
    st = h.stats()
    info = h.specialize(grad="auto")
    tu = mvf.Tuning(grad=1 if args.grad == "rev" else 0, chunk=0, grid_blocks=0, best_ms=0.0, sub_per_lane=1,
                    engine=mvf.MVF_ENGINE["spec"], block=256)
    call = mvf.BatchCall(h, torch.tensor(bw.boxes, device="cuda"), torch.tensor(bw.splits, device="cuda"),
                         mode="both", grad=args.grad, tuning=tu)
    stream = torch.cuda.current_stream()
    ms = time_calls(lambda: call.launch(stream), args.steps, args.warmup, stream, args.prewarm_s)
    total = call.total
    ops = ref_ops(st, args.grad, "spec")
    return {"metric": METRIC, "value": total / (ms * 1e-3), "unit": "subdomain-bounds/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "batch", "form": "batched kernel sequence (profiling)", "grad": args.grad,
                       "nodes": len(bw.boxes), "subdomains": total, "tuning": tu.as_dict(),
                       "checkpoint_intervals_per_lane": info["ckpt_intervals"]},
            "roofline": {"bound": "alu", "achieved": ops * total / (ms * 1e-3) / 1e12,
                         "peak": FP64_ISSUE_PEAK / 1e12, "unit": PEAK_UNIT,
                         "frac": ops * total / (ms * 1e-3) / FP64_ISSUE_PEAK, "traffic": None,
                         "ops_per_subdomain": ops}}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU (the path is not sharded across GPUs); --gpus must be 1"}))
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
    if args.workload == "batch":
        print(json.dumps(batch_profile(args)), flush=True)
        return
    w = I.mid(args.seed) if args.workload == "mid" else I.diff(args.seed)
    tape = mvf.Tape(w.tape)
    st = tape.stats()
    spec = None
    if args.engine == "spec":
        spec = tape.specialize(grad="auto" if args.workload == "mid" else "rev")
    box = torch.tensor(w.box, dtype=torch.float64, device="cuda")
    call = mvf.BoundCall(tape, box, w.splits, mode="both", grad=args.grad, engine=args.engine)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    # the timed steps: one event pair around exactly K steps
    ms = time_calls(lambda: call.launch(stream), args.steps, args.warmup, stream, args.prewarm_s)
    wall = time.perf_counter() - t0
    # a second pass of K steps with events around every step and around every step's bounding
    # kernel alone (the events themselves cost a few microseconds per step, so ``value`` comes
    # from the pass above)
    kernel = kernel_times(call, args.steps, stream)
    S = w.n_sub
    value = S / (ms * 1e-3)
    ops = ref_ops(st, args.grad, args.engine)
    achieved = ops * S / (kernel["mean_ms"] * 1e-3)       # algorithmic FP64 ops per second of the kernel
    reduced = call.reduced.cpu().numpy()
    # end to end: the node box from host memory, the bound, the reduced bounds back on the host
    hbox = torch.tensor(w.box, dtype=torch.float64).pin_memory()
    hred = torch.empty_like(call.reduced, device="cpu").pin_memory()

    def e2e():
        box.copy_(hbox, non_blocking=True)
        call.launch(stream)
        hred.copy_(call.reduced, non_blocking=True)
        stream.synchronize()
    e2e()
    t1 = time.perf_counter()
    for _ in range(20):
        e2e()
    e2e_ms = (time.perf_counter() - t1) / 20 * 1e3
    key = (args.engine, args.grad, w.tape.digest(), spec["code_bytes"] if spec else 0)
    kname = {("spec", "fwd"): "mvf_spec_bound", ("spec", "rev"): "mvf_spec_bound_rev",
              ("interp", "fwd"): f"bound_kernel<{st.tangent_chunk},false>",
              ("interp", "rev"): "bound_kernel<0,true>"}[(args.engine, args.grad)]
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
        "config": {"workload": w.name, "form": "plain: " + ("forward-mode" if args.grad == "fwd" else "adjoint") +
                   " MVF, one launch per node box",
                   "n_vars": w.tape.n_vars, "tape_ops": w.tape.n_ops(), "roots": w.tape.n_roots,
                   "subdomains": S, "splits": [int(s) for s in w.splits], "seed": args.seed,
                   "tape_hash": w.tape.digest(), "engine": args.engine,
                   "tangent_chunk": spec["chunk"] if spec else st.tangent_chunk},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_ISSUE_PEAK / 1e12,
                     "unit": PEAK_UNIT, "frac": achieved / FP64_ISSUE_PEAK,
                     "traffic": TRAFFIC.get(key), "traffic_source": TRAFFIC_SOURCE.get(key),
                     "kernel": kname, "duration": "HIP events around the kernel alone, mean over the K steps",
                     "kernel_ms": kernel["mean_ms"],
                     "step_frac": ops * S / (ms * 1e-3) / FP64_ISSUE_PEAK,
                     "ops_per_subdomain": ops, "subdomains_per_launch": S,
                     "dense_ops_per_subdomain": st.ref_ops_fwd if args.grad == "fwd" else st.ref_ops_rev,
                     "frac_of_published_78.6": achieved / FP64_PUBLISHED_PEAK},
        "timing": {"mean_ms": ms, "median_ms": kernel["step_median_ms"], "min_ms": kernel["step_min_ms"],
                   "kernel_mean_ms": kernel["mean_ms"], "kernel_median_ms": kernel["median_ms"],
                   "kernel_min_ms": kernel["min_ms"], "finish_and_gaps_ms": ms - kernel["mean_ms"],
                   "end_to_end_ms": e2e_ms,
                   "end_to_end": "box H2D + bound + reduced D2H + synchronise, host clock, 20 calls",
                   "prewarm_s": args.prewarm_s, "wall_s": wall},
        "objective_lower_bound": float(reduced[0, 0]),
        "gpu_clocks": gpu_clocks(),
    }
    if spec:
        out["specialisation"] = {"kernels": spec["grad"], "compile_s": spec["seconds"],
                                 "from_cache": bool(spec["from_cache"]), "code_units": spec["code_units"],
                                 "code_bytes": spec["code_bytes"], "waves_per_simd": spec["waves"]}
    if not args.no_forms:
        forms = set(args.forms.split(","))
        out["forms"] = {}
        if "mid" in forms and args.workload == "mid":
            out["forms"].update(mid_forms(args.seed, tape))
        if "tiny" in forms:
            out["forms"]["tiny"] = tiny_forms(args.seed)
        if "diff" in forms:
            out["forms"]["diff"] = diff_forms(args.seed)
        if "batch" in forms:
            out["forms"]["batch"] = batch_forms(args.seed)
        if "bnb" in forms and args.bnb_nodes > 0:
            out["forms"]["bnb"] = bnb_forms(args.seed, args.bnb_nodes)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, other=not args.no_forms)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
