"""Seeded synthetic inputs: expression tapes, node boxes and batches of B&B nodes.

This module builds inputs only. It contains no interval arithmetic, no Mean
Value Form and no bounding: both the CPU oracle and the GPU library receive the
arrays produced here and compute everything themselves.

Tape format (shared interface)
------------------------------
A tape is a list of nodes in SSA order (every operand index is smaller than the
node's own index), as in the DAG representation of a factorable function
(paper, Sec. 2.2 "Factorable function" and Sec. 3.2, Fig. "DAG_NIE").  Each node
is three int32 values ``(op, a, b)``:

* ``VAR``   a = variable index (0-based), b = -1
* ``CONST`` a = index into ``consts``, b = -1
* unary ``SQR SQRT EXP LOG``: a = operand node, b = -1
* binary ``ADD SUB MUL DIV``: a, b = operand nodes (z = a op b)

``roots`` lists the function nodes: objective first, then constraints
(paper, Sec. 3.1, the NLP with f, g_i, h_j).

Workload recipe (a reading: the paper's own workloads are trained tanh ANNs
whose weights are not public, Sec. 4.1 and Sec. 4.3)
-----------------------------------------------------------------------------
Random DAG tapes with the op mix add .20, sub .15, mul .25, div .08, sqr .12,
sqrt .07, log .07, exp .06.  Operands come with p=.70 from the last ``window``
arithmetic nodes of the same function (an ANN-like, layer-local live set),
p=.25 from a variable and p=.05 from a constant U[-2,2].  Every result is used:
a result about to leave the window unused is taken first, half of the window
draws go to unused results, and what is left at the end is summed into the
root, so the whole tape lies in the root's cone (no dead code).  Guards keep every
evaluation finite on any sub-box of the root box:

* denominators, sqrt and log arguments are ``sqr(u) + c`` with c ~ U[0.5, 2],
  positive for any interval of u;
* exp arguments are an affine map ``alpha*u + beta`` taking the range of u at
  seeded sample points onto [-5, 5] (the op set has no min/max, so "clamping"
  is read as this squash);
* whenever the sampled range of a node leaves [-1e3, 1e3] (or collapses below
  1e-2 in magnitude), an affine re-normalisation onto [-4, 4] is appended;
* a static bound on |value| over the whole box (triangle inequality) caps
  growth: past 1e6 the node goes through ``4 / (sqr(alpha*z) + 1)``, which lies
  in (0, 4] for any interval, so every enclosure stays finite by construction.

Guard nodes count towards the op budget.  Constraints are shifted by the 80 %
quantile of their sampled values, so each is satisfied on roughly 80 % of the
box.  Sample-point evaluation is plain round-to-nearest float64 evaluation of
the function; it only picks constants.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import List, Sequence, Tuple

import numpy as np

VAR, CONST, ADD, SUB, MUL, DIV, SQR, SQRT, EXP, LOG, TANH, SIN, COS = range(13)
OP_NAMES = ["VAR", "CONST", "ADD", "SUB", "MUL", "DIV", "SQR", "SQRT", "EXP", "LOG", "TANH", "SIN", "COS"]
NODE_DTYPE = np.dtype([("op", "<i4"), ("a", "<i4"), ("b", "<i4")])

_OP_DRAW = [(ADD, .20), (SUB, .15), (MUL, .25), (DIV, .08), (SQR, .12), (SQRT, .07), (LOG, .07), (EXP, .06)]


@dataclasses.dataclass
class Tape:
    nodes: np.ndarray          # NODE_DTYPE [T]
    consts: np.ndarray         # float64 [n_consts]
    roots: np.ndarray          # int32 [m_f]
    n_vars: int

    @property
    def n_nodes(self) -> int:
        return int(self.nodes.shape[0])

    @property
    def n_roots(self) -> int:
        return int(self.roots.shape[0])

    def n_ops(self) -> int:
        """Arithmetic nodes (leaves excluded)."""
        return int(np.count_nonzero(self.nodes["op"] >= ADD))

    def digest(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n_vars).tobytes())
        h.update(np.ascontiguousarray(self.nodes).tobytes())
        h.update(np.ascontiguousarray(self.consts, dtype="<f8").tobytes())
        h.update(np.ascontiguousarray(self.roots, dtype="<i4").tobytes())
        return h.hexdigest()[:16]

    def op_histogram(self) -> dict:
        ops = self.nodes["op"]
        return {OP_NAMES[k]: int(np.count_nonzero(ops == k)) for k in range(len(OP_NAMES))}


def save_tape(tape: Tape, path: str) -> None:
    """Write a tape as an uncompressed .npz: nodes (op, a, b as int32 columns), consts
    (float64), roots (int32) and n_vars; read back with load_tape (no pickled objects)."""
    np.savez(path, op=np.ascontiguousarray(tape.nodes["op"], dtype="<i4"),
             a=np.ascontiguousarray(tape.nodes["a"], dtype="<i4"), b=np.ascontiguousarray(tape.nodes["b"], dtype="<i4"),
             consts=np.ascontiguousarray(tape.consts, dtype="<f8"), roots=np.ascontiguousarray(tape.roots, dtype="<i4"),
             n_vars=np.int64(tape.n_vars))


def load_tape(path: str) -> Tape:
    """A tape written by save_tape (plain arrays only: allow_pickle stays off)."""
    with np.load(path, allow_pickle=False) as z:
        nodes = np.empty(z["op"].shape[0], dtype=NODE_DTYPE)
        nodes["op"], nodes["a"], nodes["b"] = z["op"], z["a"], z["b"]
        return Tape(nodes, np.array(z["consts"], dtype=np.float64), np.array(z["roots"], dtype=np.int32),
                    int(z["n_vars"]))


class TapeBuilder:
    """Append-only SSA tape with hash-consed VAR leaves per function."""

    def __init__(self, n_vars: int):
        self.n_vars = n_vars
        self.nodes: List[Tuple[int, int, int]] = []
        self.consts: List[float] = []
        self.roots: List[int] = []

    def add(self, op: int, a: int = -1, b: int = -1) -> int:
        self.nodes.append((op, a, b))
        return len(self.nodes) - 1

    def var(self, i: int) -> int:
        return self.add(VAR, i)

    def const(self, v: float) -> int:
        self.consts.append(float(v))
        return self.add(CONST, len(self.consts) - 1)

    def pow(self, x: int, k: int) -> int:
        """x**k for an integer k >= 1, expanded by binary powering into sqr and mul nodes
        (the tape has no power node: its interval extension is that of the expansion)."""
        assert k >= 1
        if k == 1:
            return x
        h = self.pow(x, k // 2)
        h2 = self.add(SQR, h)
        return self.add(MUL, h2, x) if k % 2 else h2

    def build(self) -> Tape:
        nodes = np.array(self.nodes, dtype=NODE_DTYPE)
        return Tape(nodes, np.array(self.consts, dtype=np.float64),
                    np.array(self.roots, dtype=np.int32), self.n_vars)


def eval_points_np(tape: Tape, x: np.ndarray) -> np.ndarray:
    """Plain float64 evaluation of every root at points x[B, n] (round to nearest).

    Used by the generator only (constraint shift) and by tests as a sampler of
    true function values; it is point evaluation, not interval bounding.
    """
    x = np.asarray(x, dtype=np.float64)
    vals: List[np.ndarray] = []
    with np.errstate(all="ignore"):
        for op, a, b in tape.nodes.tolist():
            if op == VAR:
                v = x[:, a]
            elif op == CONST:
                v = np.full(x.shape[0], tape.consts[a])
            elif op == ADD:
                v = vals[a] + vals[b]
            elif op == SUB:
                v = vals[a] - vals[b]
            elif op == MUL:
                v = vals[a] * vals[b]
            elif op == DIV:
                v = vals[a] / vals[b]
            elif op == SQR:
                v = vals[a] * vals[a]
            elif op == SQRT:
                v = np.sqrt(vals[a])
            elif op == EXP:
                v = np.exp(vals[a])
            elif op == LOG:
                v = np.log(vals[a])
            elif op == TANH:
                v = np.tanh(vals[a])
            elif op == SIN:
                v = np.sin(vals[a])
            elif op == COS:
                v = np.cos(vals[a])
            else:
                raise ValueError(op)
            vals.append(v)
    return np.stack([vals[r] for r in tape.roots.tolist()], axis=1)


# ----------------------------------------------------------------------------
# random DAG functions
# ----------------------------------------------------------------------------

def _random_function(tb: TapeBuilder, rng: np.random.Generator, n: int, budget: int,
                     window: int, pts: np.ndarray, var_mag: Sequence[float], renorm_hi: float = 1e3,
                     renorm_lo: float = 1e-2, mag_cap: float = 1e6) -> Tuple[int, np.ndarray]:
    """Append one random function to ``tb``; returns (last node, its values at ``pts``).

    ``vals`` are round-to-nearest values at the sample points (they pick the
    affine constants); ``mag`` is a static upper bound on |value| over the whole
    box, valid for any enclosure of the node, which triggers a bounded squash
    ``4 / (sqr(alpha*z) + 1)`` (in (0, 4] for any interval of z) when it passes
    ``mag_cap``.
    """
    vals = {}
    mag = {}
    leaf_var = {}
    recent: List[int] = []
    unused = list(rng.permutation(n))
    used_ops = [0]
    ops_w = np.array([w for _, w in _OP_DRAW])
    ops_w = ops_w / ops_w.sum()

    def vnode(i: int) -> int:
        if i not in leaf_var:
            leaf_var[i] = tb.var(int(i))
            vals[leaf_var[i]] = pts[:, i]
            mag[leaf_var[i]] = float(var_mag[i])
        return leaf_var[i]

    def cnode(v: float) -> int:
        k = tb.const(v)
        vals[k] = np.full(pts.shape[0], v)
        mag[k] = abs(v)
        return k

    def emit(op: int, a: int, b: int, v: np.ndarray, m: float) -> int:
        z = tb.add(op, a, b)
        vals[z] = v
        mag[z] = float(np.float64(m))
        used_ops[0] += 1
        return z

    pending: List[int] = []        # results not yet used as an operand (oldest first)

    def take_recent() -> int:
        lo = max(0, len(recent) - window)
        # a result about to leave the window unused is consumed now; otherwise
        # half of the draws go to a pending result, so every node feeds the root
        if pending and pending[0] <= recent[lo]:
            return pending.pop(0)
        if pending and rng.random() < 0.5:
            return pending.pop(int(rng.integers(0, len(pending))))
        z = recent[int(rng.integers(lo, len(recent)))]
        if z in pending:
            pending.remove(z)
        return z

    def pick(allow_const: bool) -> int:
        if unused:
            return vnode(unused.pop())
        u = rng.random()
        if recent and u < 0.70:
            return take_recent()
        if allow_const and u >= 0.95:
            return cnode(float(rng.uniform(-2.0, 2.0)))
        return vnode(int(rng.integers(0, n)))

    def positive(u: int) -> Tuple[int, float]:
        c = float(rng.uniform(0.5, 2.0))
        s = emit(SQR, u, -1, vals[u] * vals[u], np.float64(mag[u]) ** 2)
        return emit(ADD, s, cnode(c), vals[s] + c, mag[s] + c), c

    def affine(u: int, lo: float, hi: float) -> int:
        m, M = float(vals[u].min()), float(vals[u].max())
        if not (M > m):
            return u
        alpha = (hi - lo) / (M - m)
        beta = lo - alpha * m
        t = emit(MUL, u, cnode(alpha), vals[u] * alpha, abs(alpha) * mag[u])
        return emit(ADD, t, cnode(beta), vals[t] + beta, mag[t] + abs(beta))

    def squash(u: int) -> int:
        amax = float(np.abs(vals[u]).max())
        alpha = 2.0 / amax if amax > 0 else 1.0
        t = emit(MUL, u, cnode(alpha), vals[u] * alpha, alpha * mag[u])
        s = emit(SQR, t, -1, vals[t] * vals[t], np.float64(mag[t]) ** 2)
        d = emit(ADD, s, cnode(1.0), vals[s] + 1.0, mag[s] + 1.0)
        return emit(DIV, cnode(4.0), d, 4.0 / vals[d], 4.0)

    def renorm(z: int) -> int:
        if not (mag[z] <= mag_cap):
            return squash(z)
        amax = float(np.abs(vals[z]).max())
        if amax > renorm_hi or 0.0 < amax < renorm_lo:
            t = affine(z, -4.0, 4.0)
            return squash(t) if not (mag[t] <= mag_cap) else t
        return z

    last = None
    with np.errstate(all="ignore"):
        while used_ops[0] < budget:
            op = _OP_DRAW[int(rng.choice(len(_OP_DRAW), p=ops_w))][0]
            if op in (ADD, SUB, MUL):
                a = pick(True)
                b = pick(tb.nodes[a][0] != CONST)
                if op == MUL:
                    z = emit(op, a, b, vals[a] * vals[b], np.float64(mag[a]) * mag[b])
                else:
                    v = vals[a] + vals[b] if op == ADD else vals[a] - vals[b]
                    z = emit(op, a, b, v, mag[a] + mag[b])
            elif op == DIV:
                a = pick(True)
                den, c = positive(pick(False))
                z = emit(DIV, a, den, vals[a] / vals[den], mag[a] / c)
            elif op == SQR:
                a = pick(False)
                z = emit(SQR, a, -1, vals[a] * vals[a], np.float64(mag[a]) ** 2)
            elif op == SQRT:
                arg, c = positive(pick(False))
                z = emit(SQRT, arg, -1, np.sqrt(vals[arg]), np.sqrt(mag[arg]))
            elif op == LOG:
                arg, c = positive(pick(False))
                z = emit(LOG, arg, -1, np.log(vals[arg]), max(abs(math.log(c)), np.log(mag[arg])))
            else:  # EXP of an argument squashed into [-5, 5] on the sample
                t = affine(pick(False), -5.0, 5.0)
                if not (mag[t] <= 30.0):
                    t = affine(squash(t), -5.0, 5.0)
                z = emit(EXP, t, -1, np.exp(vals[t]), np.exp(mag[t]))
            last = renorm(z)
            recent.append(last)
            pending.append(last)
        pending.remove(last)
        while pending:                                 # every result reaches the root
            a = pending.pop(0)
            last = emit(ADD, last, a, vals[last] + vals[a], mag[last] + mag[a])
        while unused:                                  # every variable appears
            a = vnode(unused.pop())
            last = emit(ADD, last, a, vals[last] + vals[a], mag[last] + mag[a])
    return last, vals[last]


def random_tape(seed: int, n: int, obj_ops: int, con_ops: Sequence[int], lo: np.ndarray, hi: np.ndarray,
                window: int, n_samples: int = 512) -> Tape:
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = lo + (hi - lo) * rng.random((n_samples, n))
    tb = TapeBuilder(n)
    var_mag = np.maximum(np.abs(lo), np.abs(hi))
    tb.roots.append(_random_function(tb, rng, n, obj_ops, window, pts, var_mag)[0])
    for c in con_ops:
        r, v = _random_function(tb, rng, n, c, window, pts, var_mag)
        q = float(np.quantile(v[np.isfinite(v)], 0.8))
        tb.roots.append(tb.add(SUB, r, tb.const(q)))
    return tb.build()


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

def monomial_tape(seed: int, n_terms: int = 8, max_degree: int = 4) -> Tape:
    """Two-variable random polynomial: ``n_terms`` distinct monomials x^a y^b with
    1 <= a+b <= max_degree, coefficients U[-1,1], summed left to right."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pairs = [(a, b) for a in range(max_degree + 1) for b in range(max_degree + 1) if 1 <= a + b <= max_degree]
    chosen = [pairs[i] for i in sorted(rng.choice(len(pairs), size=n_terms, replace=False).tolist())]
    coef = rng.uniform(-1.0, 1.0, size=n_terms)
    tb = TapeBuilder(2)
    xs = [tb.var(0), tb.var(1)]
    powers = [{1: xs[0]}, {1: xs[1]}]

    def power(v: int, e: int) -> int:
        p = powers[v]
        if e in p:
            return p[e]
        if e == 2:
            p[2] = tb.add(SQR, xs[v])
        elif e == 3:
            p[3] = tb.add(MUL, xs[v], power(v, 2))
        elif e == 4:
            p[4] = tb.add(SQR, power(v, 2))
        return p[e]

    acc = None
    for (a, b), c in zip(chosen, coef):
        term = None
        if a:
            term = power(0, a)
        if b:
            yb = power(1, b)
            term = yb if term is None else tb.add(MUL, term, yb)
        term = tb.add(MUL, tb.const(float(c)), term)
        acc = term if acc is None else tb.add(ADD, acc, term)
    tb.roots.append(acc)
    return tb.build()


def cubic_tape() -> Tape:
    """f(x) = 3x^3 + x^2 - 5x - 1, the DAG example of the paper (Sec. 3.2, Fig. DAG_NIE)."""
    tb = TapeBuilder(1)
    x = tb.var(0)
    v1 = tb.add(SQR, x)
    v2 = tb.add(MUL, x, v1)
    v3 = tb.add(MUL, tb.const(3.0), v2)
    v4 = tb.add(ADD, v3, v1)
    v5 = tb.add(MUL, tb.const(5.0), x)
    v6 = tb.add(SUB, v4, v5)
    v7 = tb.add(SUB, v6, tb.const(1.0))
    tb.roots.append(v7)
    return tb.build()


def peaks_tape() -> Tape:
    """The Peaks function of Sec. 4.1 (uses only + - * sqr exp and constants)."""
    tb = TapeBuilder(2)
    x1, x2 = tb.var(0), tb.var(1)
    c = tb.const
    one_m_x1 = tb.add(SUB, c(1.0), x1)
    t1a = tb.add(MUL, c(3.0), tb.add(SQR, one_m_x1))
    x1s = tb.add(SQR, x1)
    e1 = tb.add(EXP, tb.add(SUB, tb.add(SUB, c(0.0), x1s), tb.add(SQR, tb.add(ADD, x2, c(1.0)))))
    t1 = tb.add(MUL, t1a, e1)
    x1c = tb.add(MUL, x1, x1s)
    x2s = tb.add(SQR, x2)
    x2_5 = tb.add(MUL, tb.add(SQR, x2s), x2)
    inner = tb.add(SUB, tb.add(SUB, tb.add(DIV, x1, c(5.0)), x1c), x2_5)
    e2 = tb.add(EXP, tb.add(SUB, tb.add(SUB, c(0.0), x1s), x2s))
    t2 = tb.add(MUL, tb.add(MUL, c(10.0), inner), e2)
    e3 = tb.add(EXP, tb.add(SUB, tb.add(SUB, c(0.0), tb.add(SQR, tb.add(ADD, x1, c(1.0)))), x2s))
    t3 = tb.add(DIV, e3, c(3.0))
    tb.roots.append(tb.add(SUB, tb.add(SUB, t1, t2), t3))
    return tb.build()


def _random_box(rng: np.random.Generator, n: int) -> np.ndarray:
    side = rng.uniform(0.5, 4.0, size=n)
    centre = rng.uniform(-2.0, 2.0, size=n)
    return np.stack([centre - side / 2, centre + side / 2], axis=1)


def widest_bisect_splits(box: np.ndarray, n_dims: int) -> np.ndarray:
    """Split 2 ways on the ``n_dims`` widest dimensions (ties to the lower index)."""
    w = box[:, 1] - box[:, 0]
    order = sorted(range(len(w)), key=lambda i: (-w[i], i))
    s = np.ones(len(w), dtype=np.int32)
    s[order[:n_dims]] = 2
    return s


def doubling_splits(box: np.ndarray, total_log2: int) -> np.ndarray:
    """Reach 2**total_log2 subdomains by repeatedly doubling the split count of
    the dimension with the largest w_i / s_i (ties to the lower index)."""
    w = box[:, 1] - box[:, 0]
    s = np.ones(len(w), dtype=np.int64)
    for _ in range(total_log2):
        i = max(range(len(w)), key=lambda j: (w[j] / s[j], -j))
        s[i] *= 2
    return s.astype(np.int32)


@dataclasses.dataclass
class Workload:
    name: str
    tape: Tape
    box: np.ndarray            # [n, 2] (single-node workloads)
    splits: np.ndarray         # [n] int32
    description: str

    @property
    def n_sub(self) -> int:
        return int(np.prod(self.splits.astype(np.int64)))


@dataclasses.dataclass
class BatchWorkload:
    name: str
    tape: Tape
    boxes: np.ndarray          # [N, n, 2]
    splits: np.ndarray         # [N, n] int32
    description: str

    @property
    def n_sub(self) -> np.ndarray:
        return np.prod(self.splits.astype(np.int64), axis=1)


def tiny(seed: int = 1) -> Workload:
    tape = monomial_tape(seed)
    box = np.array([[-2.0, 2.0], [-2.0, 2.0]])
    return Workload("tiny", tape, box, np.array([64, 64], dtype=np.int32),
                    "2 vars on [-2,2]^2, 8-monomial polynomial, 64x64 = 4,096 subdomains")


def mid(seed: int = 1) -> Workload:
    rng = np.random.Generator(np.random.PCG64(seed + 1000))
    box = _random_box(rng, 6)
    tape = random_tape(seed, 6, 200, [80, 80, 80], box[:, 0], box[:, 1], window=16)
    return Workload("mid", tape, box, np.full(6, 8, dtype=np.int32),
                    "6 vars, 200-op objective + 3x80-op constraints, 8^6 = 262,144 subdomains")


def rational(tape: Tape) -> Tape:
    """The tape with exp replaced by sqr and log by sqrt: a variant of the same
    shape whose bounds every implementation must reproduce bit for bit (the
    remaining operations are correctly rounded)."""
    nodes = tape.nodes.copy()
    nodes["op"][nodes["op"] == EXP] = SQR
    nodes["op"][nodes["op"] == LOG] = SQRT
    return Tape(nodes, tape.consts, tape.roots, tape.n_vars)


def diff(seed: int = 1) -> Workload:
    rng = np.random.Generator(np.random.PCG64(seed + 2000))
    box = _random_box(rng, 32)
    tape = random_tape(seed, 32, 2000, [300, 300, 300, 300], box[:, 0], box[:, 1], window=32)
    return Workload("diff", tape, box, widest_bisect_splits(box, 20),
                    "32 vars, 2,000-op objective + 4x300-op constraints, 2^20 = 1,048,576 subdomains")


def e2e_tape(seed: int = 1) -> Tape:
    lo, hi = np.full(10, -3.0), np.full(10, 3.0)
    return random_tape(seed, 10, 500, [200] * 5, lo, hi, window=32)


def batch(seed: int = 1, n_nodes: int = 512) -> BatchWorkload:
    """512 B&B-like nodes of [-3,3]^8: node i is reached by d_i ~ U{0..16} bisections
    of its widest dimension keeping a random half; it is split into 2^k_i
    subdomains, k_i ~ U{10..18}, by repeated doubling of the widest w_i/s_i."""
    n = 8
    lo, hi = np.full(n, -3.0), np.full(n, 3.0)
    tape = random_tape(seed, n, 400, [150, 150], lo, hi, window=32)
    rng = np.random.Generator(np.random.PCG64(seed + 3000))
    boxes = np.empty((n_nodes, n, 2))
    splits = np.empty((n_nodes, n), dtype=np.int32)
    for i in range(n_nodes):
        b = np.stack([lo, hi], axis=1).copy()
        for _ in range(int(rng.integers(0, 17))):
            w = b[:, 1] - b[:, 0]
            j = int(np.argmax(w))
            mid_ = 0.5 * (b[j, 0] + b[j, 1])
            if rng.random() < 0.5:
                b[j, 1] = mid_
            else:
                b[j, 0] = mid_
        boxes[i] = b
        splits[i] = doubling_splits(b, int(rng.integers(10, 19)))
    return BatchWorkload("batch", tape, boxes, splits,
                         f"{n_nodes} nodes of [-3,3]^8, 400-op objective + 2x150-op constraints, 2^10..2^18 subdomains each")


def small_batch(seed: int, n_nodes: int, k_range=(4, 9)) -> BatchWorkload:
    """A scaled-down batch (same recipe, fewer and smaller nodes) for parity tests."""
    n = 8
    lo, hi = np.full(n, -3.0), np.full(n, 3.0)
    tape = random_tape(seed, n, 60, [25, 25], lo, hi, window=16)
    rng = np.random.Generator(np.random.PCG64(seed + 3000))
    boxes = np.empty((n_nodes, n, 2))
    splits = np.empty((n_nodes, n), dtype=np.int32)
    for i in range(n_nodes):
        b = np.stack([lo, hi], axis=1).copy()
        for _ in range(int(rng.integers(0, 17))):
            w = b[:, 1] - b[:, 0]
            j = int(np.argmax(w))
            m = 0.5 * (b[j, 0] + b[j, 1])
            if rng.random() < 0.5:
                b[j, 1] = m
            else:
                b[j, 0] = m
        boxes[i] = b
        splits[i] = doubling_splits(b, int(rng.integers(k_range[0], k_range[1] + 1)))
    return BatchWorkload("small_batch", tape, boxes, splits, f"{n_nodes} small nodes")


def random_small_tape(seed: int, n: int, ops: int, n_con: int = 1, con_ops: int = 10,
                      window: int = 8, lo: float = -2.0, hi: float = 2.0) -> Tape:
    return random_tape(seed, n, ops, [con_ops] * n_con, np.full(n, lo), np.full(n, hi), window=window)


def shared_roots_tape(seed: int, n: int = 3, ops: int = 60, con_ops: int = 20) -> Tape:
    """Roots that share subexpressions: a random objective, two random
    constraints each plus (minus) a node of the objective's cone, and the
    product of two more of the objective's nodes as a third constraint."""
    base = random_small_tape(seed, n=n, ops=ops, n_con=2, con_ops=con_ops, window=8)
    nodes = [tuple(int(v) for v in nd) for nd in base.nodes.tolist()]
    arith = {ADD, SUB, MUL, DIV, SQR, SQRT, EXP, LOG, TANH, SIN, COS}
    cone, todo = set(), [int(base.roots[0])]
    while todo:
        i = todo.pop()
        if i in cone or nodes[i][0] not in arith:
            continue
        cone.add(i)
        todo.append(nodes[i][1])
        if nodes[i][0] in (ADD, SUB, MUL, DIV):
            todo.append(nodes[i][2])
    rng = np.random.default_rng(seed + 7)
    p = [int(x) for x in rng.choice(sorted(cone - {int(base.roots[0])}), 4, replace=False)]
    nodes += [(ADD, int(base.roots[1]), p[0]), (SUB, int(base.roots[2]), p[1]), (MUL, p[2], p[3])]
    T = len(nodes)
    return Tape(np.array(nodes, dtype=NODE_DTYPE), base.consts.copy(),
                np.array([base.roots[0], T - 3, T - 2, T - 1], dtype=np.int32), n)


def random_points(seed: int, box: np.ndarray, count: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = box[:, 0], box[:, 1]
    return lo + (hi - lo) * rng.random((count, box.shape[0]))


# ----------------------------------------------------------------------------
# ANN-shaped tapes (the paper's tanh-network workloads, Sec. 4.1 and 4.3)
# ----------------------------------------------------------------------------

def _dense_tanh(tb: TapeBuilder, rng: np.random.Generator, inputs: List[int], width: int) -> List[int]:
    """One hidden layer: tanh(W x + b) per neuron, weights U[-1,1]/sqrt(fan-in), biases U[-0.5,0.5]."""
    scale = 1.0 / np.sqrt(len(inputs))
    out = []
    for _ in range(width):
        acc = tb.const(float(rng.uniform(-0.5, 0.5)))
        for x in inputs:
            acc = tb.add(ADD, acc, tb.add(MUL, tb.const(float(rng.uniform(-1.0, 1.0) * scale)), x))
        out.append(tb.add(TANH, acc))
    return out


def ann_tape(seed: int = 1, n_in: int = 4, widths: Sequence[int] = (16, 16)) -> Tape:
    """A seeded feed-forward tanh network (inputs -> hidden tanh layers -> one linear
    output) as the objective, and one trigonometric inequality constraint
    sum_i sin(x_i) cos(x_{i+1}) - 0.5 <= 0.  Weights are drawn, not trained: the
    paper's trained networks are not public."""
    rng = np.random.default_rng(seed)
    tb = TapeBuilder(n_in)
    xs = [tb.var(i) for i in range(n_in)]
    h = xs
    for w in widths:
        h = _dense_tanh(tb, rng, h, w)
    scale = 1.0 / np.sqrt(len(h))
    out = tb.const(float(rng.uniform(-0.5, 0.5)))
    for x in h:
        out = tb.add(ADD, out, tb.add(MUL, tb.const(float(rng.uniform(-1.0, 1.0) * scale)), x))
    tb.roots.append(out)
    xs = [tb.var(i) for i in range(n_in)]
    g = tb.const(-0.5)
    for i in range(n_in):
        g = tb.add(ADD, g, tb.add(MUL, tb.add(SIN, xs[i]), tb.add(COS, xs[(i + 1) % n_in])))
    tb.roots.append(g)
    return tb.build()


def ann(seed: int = 1) -> Workload:
    """4 inputs on [-2, 2]^4, two hidden tanh layers of 16, a sin/cos constraint, 16^4 subdomains."""
    t = ann_tape(seed)
    return Workload("ann", t, np.array([[-2.0, 2.0]] * 4), np.array([16, 16, 16, 16], dtype=np.int32),
                    "tanh network 4-16-16-1 and a sin/cos constraint, [-2,2]^4, 16^4 subdomains")
