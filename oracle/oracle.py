"""ctypes front end of the CPU oracle (``mvf_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the library.  It takes tapes and
boxes as numpy arrays (see ``paper_2507_20769_amd.inputs`` for the format) and
returns numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mvf_oracle.c")
_LIB = os.path.join(_HERE, "libmvf_oracle.so")
_lock = threading.Lock()
_lib = None

GCC_FLAGS = ["-O2", "-std=c11", "-Wall", "-frounding-math", "-ffp-contract=off", "-fno-fast-math",
             "-msse2", "-mfpmath=sse", "-fPIC", "-shared"]

MODE_NIE, MODE_MVF, MODE_BOTH = 0, 1, 2
GRAD_FWD, GRAD_REV = 0, 1
FREE, INEQ, EQ = 0, 1, 2
ADD, SUB, MUL, DIV, SQR, SQRT, EXP, LOG, TANH, SIN, COS = 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, directed rounding via fesetround)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm", "-lpthread"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            L = ctypes.CDLL(build())
            P = ctypes.c_void_p
            i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
            L.orc_round_op.restype = dbl
            L.orc_round_op.argtypes = [ctypes.c_int, ctypes.c_int, dbl, dbl]
            L.orc_interval_op.restype = None
            L.orc_interval_op.argtypes = [ctypes.c_int, P, P, P]
            L.orc_subdomain.restype = None
            L.orc_subdomain.argtypes = [ctypes.c_int, P, P, i64, P, P]
            tape = [P, i32, P, i32, P, i32]
            L.orc_bound.restype = ctypes.c_int
            L.orc_bound.argtypes = tape + [P, P, P, i64, i64, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P,
                                           ctypes.c_int]
            L.orc_nie_boxes.restype = ctypes.c_int
            L.orc_nie_boxes.argtypes = tape + [i64, P, P, P]
            L.orc_gradient_boxes.restype = ctypes.c_int
            L.orc_gradient_boxes.argtypes = tape + [i64, P, i32, ctypes.c_int, P, P]
            L.orc_fbbt.restype = ctypes.c_int
            L.orc_fbbt.argtypes = tape + [P, i64, P, ctypes.c_double, i32, P, P]
            L.orc_eval_points.restype = ctypes.c_int
            L.orc_eval_points.argtypes = tape + [i64, P, P]
            L.orc_vjp_points.restype = ctypes.c_int
            L.orc_vjp_points.argtypes = tape + [i64, P, P, P]
            L.orc_adaptive_splits.restype = i64
            L.orc_adaptive_splits.argtypes = [ctypes.c_int, P, i64, P]
            _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _tape_args(tape):
    nodes = np.ascontiguousarray(tape.nodes)
    consts = np.ascontiguousarray(tape.consts, dtype=np.float64)
    if consts.size == 0:
        consts = np.zeros(1)
    roots = np.ascontiguousarray(tape.roots, dtype=np.int32)
    keep = (nodes, consts, roots)
    return keep, [_p(nodes), len(nodes), _p(consts), int(tape.n_vars), _p(roots), len(roots)]


def round_op(op: int, direction: int, a: float, b: float = 0.0) -> float:
    """One correctly rounded op: direction -1 down, 0 nearest, +1 up."""
    return lib().orc_round_op(op, direction, a, b)


def interval_op(op: int, u, v=None) -> np.ndarray:
    U = np.ascontiguousarray(u, dtype=np.float64)
    V = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
    Z = np.zeros(2)
    lib().orc_interval_op(op, _p(U), None if V is None else _p(V), _p(Z))
    return Z


def subdomain(box: np.ndarray, splits: np.ndarray, k: int):
    box = np.ascontiguousarray(box, dtype=np.float64)
    s = np.ascontiguousarray(splits, dtype=np.int32)
    n = box.shape[0]
    X = np.zeros((n, 2))
    c = np.zeros(n)
    lib().orc_subdomain(n, _p(box), _p(s), int(k), _p(X), _p(c))
    return X, c


def bound(tape, box, splits, mode: int = MODE_BOTH, grad: int = GRAD_FWD, k_range=None, ks=None,
          per_sub: bool = True, nthreads: int = 1, kinds=None):
    """Steps 1-3 on one box.  Returns dict(reduced[m,2], argmin, per_sub[m,2,count], flags[count],
    extra[2]): extra = (objective lower bound over the subdomains no constraint proves
    infeasible, upper bound from rigorously feasible subdomain centres).  kinds[m]: root
    kinds (FREE, INEQ g <= 0, EQ h = 0); None treats every root as unconstrained."""
    keep, targs = _tape_args(tape)
    box = np.ascontiguousarray(box, dtype=np.float64)
    s = np.ascontiguousarray(splits, dtype=np.int32)
    S = int(np.prod(s.astype(np.int64)))
    m = tape.n_roots
    ks_arr = None
    if ks is not None:
        ks_arr = np.ascontiguousarray(ks, dtype=np.int64)
        k0, k1 = 0, len(ks_arr)
    else:
        k0, k1 = (0, S) if k_range is None else k_range
    count = k1 - k0
    ps = np.zeros((m, 2, max(count, 1))) if per_sub else None
    flags = np.zeros(max(count, 1), dtype=np.uint32)
    red = np.zeros((m, 2))
    am = ctypes.c_int64(-1)
    kd = None if kinds is None else np.ascontiguousarray(kinds, dtype=np.int32)
    extra = np.zeros(2)
    lib().orc_bound(*targs, _p(box), _p(s), None if ks_arr is None else _p(ks_arr), k0, k1, mode, grad,
                    None if kd is None else _p(kd), None if ps is None else _p(ps), _p(flags), _p(red),
                    ctypes.byref(am), _p(extra), nthreads)
    out = {"reduced": red, "argmin": am.value, "flags": flags[:count], "extra": extra}
    if per_sub:
        out["per_sub"] = ps[:, :, :count]
    return out


def nie_boxes(tape, boxes):
    keep, targs = _tape_args(tape)
    boxes = np.ascontiguousarray(boxes, dtype=np.float64)
    B = boxes.shape[0]
    out = np.zeros((B, tape.n_roots, 2))
    flags = np.zeros(B, dtype=np.uint32)
    lib().orc_nie_boxes(*targs, B, _p(boxes), _p(out), _p(flags))
    return out, flags


def gradient_boxes(tape, boxes, root: int, grad: int = GRAD_FWD):
    keep, targs = _tape_args(tape)
    boxes = np.ascontiguousarray(boxes, dtype=np.float64)
    B = boxes.shape[0]
    G = np.zeros((B, tape.n_vars, 2))
    flags = np.zeros(B, dtype=np.uint32)
    lib().orc_gradient_boxes(*targs, B, _p(boxes), root, grad, _p(G), _p(flags))
    return G, flags


def fbbt(tape, boxes, kinds=None, ub: float = np.inf, rounds: int = 1):
    """Forward-backward bound tightening of boxes [N, n, 2]: (tightened boxes, status [N],
    1 where a box is proven infeasible)."""
    keep, targs = _tape_args(tape)
    boxes = np.ascontiguousarray(boxes, dtype=np.float64)
    if boxes.ndim == 2:
        boxes = boxes[None]
    N = boxes.shape[0]
    k = None if kinds is None else np.ascontiguousarray(kinds, dtype=np.int32)
    out = np.zeros_like(boxes)
    st = np.zeros(N, dtype=np.int32)
    lib().orc_fbbt(*targs, None if k is None else _p(k), N, _p(boxes), float(ub), int(rounds), _p(out), _p(st))
    return out, st


def eval_points(tape, x):
    keep, targs = _tape_args(tape)
    x = np.ascontiguousarray(x, dtype=np.float64)
    B = x.shape[0]
    f = np.zeros((B, tape.n_roots, 2))
    lib().orc_eval_points(*targs, B, _p(x), _p(f))
    return f


def vjp_points(tape, x, gout):
    keep, targs = _tape_args(tape)
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(gout, dtype=np.float64)
    B = x.shape[0]
    gx = np.zeros((B, tape.n_vars, 2))
    lib().orc_vjp_points(*targs, B, _p(x), _p(g), _p(gx))
    return gx


def adaptive_splits(widths, budget: int):
    w = np.ascontiguousarray(widths, dtype=np.float64)
    s = np.zeros(len(w), dtype=np.int32)
    count = lib().orc_adaptive_splits(len(w), _p(w), int(budget), _p(s))
    return s, count
