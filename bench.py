"""Benchmark: MVF subdomain bounds per second on one MI355X.

One step = one call of the whole bounding path on one node box of the mid
workload (6 variables, a 200-op objective and three 80-op constraints,
8^6 = 262,144 subdomains): subdomain generation, point pass, tangent passes,
MVF intersected with the NIE, and the min/max reduction with argmin.  Inputs
are resident in HBM before the timed region.

Prints one JSON line.  ``value`` is subdomain-bounds/s (one subdomain-bound =
the bounds of the objective and all constraints on one subdomain).
``roofline`` relates the bounding kernel to the FP64 VALU issue peak of the
chip; ``cpu_baseline`` times the CPU oracle on a bounded sample.
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mid", choices=["mid", "tiny"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
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
            "sample": f"subdomains 0..{done - 1} of the {w.name} workload ({done} of {S}), {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2507_20769_amd import inputs as I
    from paper_2507_20769_amd import mvf

    torch.cuda.init()
    w = getattr(I, args.workload)(args.seed)
    tape = mvf.Tape(w.tape)
    st = tape.stats()
    box = torch.tensor(w.box, dtype=torch.float64, device="cuda")
    call = mvf.BoundCall(tape, box, w.splits, mode="both", grad="fwd")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        call.launch(stream)
    torch.cuda.synchronize()

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        call.launch(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    S = w.n_sub
    value = S / (ms * 1e-3)
    ops = st.ref_ops_fwd * S                      # algorithmic FP64 ops per launch
    achieved = ops / (ms * 1e-3)
    reduced = call.reduced.cpu().numpy()

    out = {
        "metric": "MVF subdomain bounds/sec (obj+constraints) and % FP64 vector peak; adjoint+batched vs plain",
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
        "config": {"workload": w.name, "form": "plain forward-mode, one launch per node box",
                   "n_vars": w.tape.n_vars, "tape_ops": w.tape.n_ops(), "roots": w.tape.n_roots,
                   "subdomains": S, "splits": [int(s) for s in w.splits], "seed": args.seed,
                   "tape_hash": w.tape.digest(), "tangent_chunk": st.tangent_chunk},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_ISSUE_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP64_ISSUE_PEAK, "traffic": None,
                     "ops_per_subdomain": st.ref_ops_fwd,
                     "frac_of_published_78.6": achieved / FP64_PUBLISHED_PEAK},
        "wall_s": wall,
        "objective_lower_bound": float(reduced[0, 0]),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
