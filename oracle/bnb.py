"""Reference spatial branch-and-bound over the oracle's subdomain bounds.

TEST INFRASTRUCTURE ONLY (imported by the tests and the benchmark's CPU leg).

The B&B of Sec. 3 with the lower bounding of Sec. 3.1 (Fig. "BnB_decompose"):
the host keeps the open nodes, takes the node(s) with the least lower bound,
bounds them (here: the oracle's Steps 1-3 with the adaptive partitioning of
Sec. 3.1.2), prunes by the lower-bound test and by the feasibility check of
the constraint bounds, and branches the survivors.  Choices the paper leaves
open are fixed as follows (the library's driver makes the same ones):

* node order: least lower bound first, ties to the node created first;
* a node's lower bound: max(parent's, the objective bound over the subdomains
  no constraint proves infeasible) -- +inf when every subdomain is infeasible;
* upper bound: the least hi(f(c_k)) over subdomain centres whose inequality
  enclosures are all <= 0 (no local solver);
* prune when lower >= upper - gap; branch by bisecting the widest variable
  (ties to the lower index) at RN(0.5 * (lo + hi));
* stop when upper - (least open lower bound) <= gap, or after max_nodes
  taken nodes; `batch` nodes are taken per round;
* with fbbt_rounds > 0 the taken boxes are first tightened by the oracle's
  FBBT with the objective cut at the current upper bound; a box proven
  infeasible is dropped and counts as a taken node.
"""
from __future__ import annotations

import heapq

import numpy as np

from oracle import oracle as O


def solve(tape, box, kinds=None, max_nodes: int = 1000, gap: float = 1e-4, budget: int = 4096,
          mode: int = O.MODE_BOTH, grad: int = O.GRAD_FWD, batch: int = 1, nthreads: int = 8,
          fbbt_rounds: int = 0) -> dict:
    box = np.array(box, dtype=np.float64)
    ub = np.inf
    counter = 0
    heap = [(-np.inf, 0, box)]
    counter = 1
    nodes = 0
    subdomains = 0
    pruned_lo = np.inf                 # least lower bound of a node discarded by the bound test
    status = 1
    while heap:
        if ub - heap[0][0] <= gap:
            status = 0
            break
        if nodes >= max_nodes:
            break
        take = []
        while heap and len(take) < min(batch, max_nodes - nodes):
            lb, nid, b = heapq.heappop(heap)
            if lb >= ub - gap:
                pruned_lo = min(pruned_lo, lb)
                continue
            take.append((lb, nid, b))
        if not take:
            continue
        if fbbt_rounds > 0:
            # tighten the taken boxes (objective cut at the current ub); drop those proven to
            # hold no feasible point below ub
            tb, st = O.fbbt(tape, np.stack([b for _, _, b in take]), kinds=kinds, ub=ub, rounds=fbbt_rounds)
            nodes += int(np.count_nonzero(st))
            take = [(lb, nid, tb[q]) for q, (lb, nid, b) in enumerate(take) if st[q] == 0]
            if not take:
                continue
        results = []
        for lb, nid, b in take:
            splits, count = O.adaptive_splits(b[:, 1] - b[:, 0], budget)
            o = O.bound(tape, b, splits, mode=mode, grad=grad, per_sub=False, nthreads=nthreads, kinds=kinds)
            results.append(o)
            subdomains += count
        nodes += len(take)
        for o in results:
            ub = min(ub, o["extra"][1])
        for (lb, nid, b), o in zip(take, results):
            lo = max(lb, o["extra"][0])
            if lo >= ub - gap:
                if np.isfinite(lo):
                    pruned_lo = min(pruned_lo, lo)
                continue
            w = b[:, 1] - b[:, 0]
            i = int(np.argmax(w))                      # first index of the largest width
            mid = 0.5 * (b[i, 0] + b[i, 1])
            left, right = b.copy(), b.copy()
            left[i, 1] = mid
            right[i, 0] = mid
            heapq.heappush(heap, (lo, counter, left))
            heapq.heappush(heap, (lo, counter + 1, right))
            counter += 2
    if not heap and status == 1:
        status = 0 if np.isfinite(ub) else 2
    open_lo = heap[0][0] if heap else np.inf
    lower = min(open_lo, pruned_lo, ub)
    return {"lower": lower, "upper": ub, "nodes": nodes, "subdomains": subdomains, "open": len(heap),
            "status": status}
