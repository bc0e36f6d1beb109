"""Python binding of ``libmvf.so`` (the C ABI in include/mvf.h).

Argument marshalling only: torch supplies device memory (``data_ptr``) and the
current stream; every step of the bounding runs in the library's kernels.
There is no fallback: if the library is not built, importing this module's
functions raises.
"""
from __future__ import annotations

import ctypes
import os
import threading
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmvf.so")

MVF_MODE = {"nie": 0, "mvf": 1, "both": 2}
MVF_GRAD = {"fwd": 0, "rev": 1, "auto": 2}

_lock = threading.Lock()
_lib = None


class MVFError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = lib()
        msg = f"{where}: {L.mvf_strerror(code).decode()} ({code}): {L.mvf_last_error().decode()}"
        super().__init__(msg)
        self.code = code


class _Node(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("a", ctypes.c_int32), ("b", ctypes.c_int32)]


class TapeStats(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_int32), ("n_roots", ctypes.c_int32), ("n_instr", ctypes.c_int32),
                ("max_slots", ctypes.c_int32), ("tangent_chunk", ctypes.c_int32), ("max_records", ctypes.c_int32),
                ("ref_ops_fwd", ctypes.c_int64), ("ref_ops_rev", ctypes.c_int64),
                ("ref_ops_fwd_sparse", ctypes.c_int64), ("ckpt_segments", ctypes.c_int32),
                ("ckpt_stored", ctypes.c_int32), ("ckpt_loaded", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    """mvf_tuning; grad -1 keeps the call's gradient mode."""
    _fields_ = [("grad", ctypes.c_int32), ("chunk", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("best_ms", ctypes.c_float), ("sub_per_lane", ctypes.c_int32), ("engine", ctypes.c_int32),
                ("block", ctypes.c_int32)]

    def __repr__(self):
        return (f"Tuning(grad={self.grad}, chunk={self.chunk}, grid_blocks={self.grid_blocks}, "
                f"sub_per_lane={self.sub_per_lane}, engine={self.engine}, block={self.block}, "
                f"best_ms={self.best_ms:.3f})")

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class BnbOptions(ctypes.Structure):
    _fields_ = [("max_nodes", ctypes.c_int32), ("nodes_per_launch", ctypes.c_int32),
                ("subdomains_per_node", ctypes.c_int64), ("abs_gap", ctypes.c_double), ("mode", ctypes.c_int32),
                ("grad", ctypes.c_int32), ("tuning", ctypes.c_void_p), ("split_rule", ctypes.c_int32),
                ("fbbt_rounds", ctypes.c_int32)]


class BnbResult(ctypes.Structure):
    _fields_ = [("lower", ctypes.c_double), ("upper", ctypes.c_double), ("nodes", ctypes.c_int64),
                ("subdomains", ctypes.c_int64), ("launches", ctypes.c_int64), ("open", ctypes.c_int32),
                ("status", ctypes.c_int32), ("seconds", ctypes.c_double)]


class BatchArgs(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("max_nodes", ctypes.c_int32), ("max_subdomains", ctypes.c_int64),
                ("boxes", ctypes.c_void_p), ("splits", ctypes.c_void_p), ("mode", ctypes.c_int32),
                ("grad", ctypes.c_int32), ("reduced", ctypes.c_void_p), ("argmin", ctypes.c_void_p),
                ("status", ctypes.c_void_p), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("extra", ctypes.c_void_p)]


class BoundArgs(ctypes.Structure):
    _fields_ = [("box", ctypes.c_void_p), ("splits", ctypes.c_void_p), ("mode", ctypes.c_int32),
                ("grad", ctypes.c_int32), ("reduced", ctypes.c_void_p), ("argmin", ctypes.c_void_p),
                ("per_sub", ctypes.c_void_p), ("flags", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("tuning", ctypes.c_void_p), ("extra", ctypes.c_void_p),
                ("engine", ctypes.c_int32), ("kernel_events", ctypes.c_void_p * 2)]


class SpecOptions(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("waves", ctypes.c_int32), ("max_code", ctypes.c_int64),
                ("use_cache", ctypes.c_int32), ("grad", ctypes.c_int32), ("ckpt_budget", ctypes.c_int32)]


class SpecInfo(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_int32), ("waves", ctypes.c_int32), ("grad", ctypes.c_int32),
                ("code_units", ctypes.c_int64),
                ("code_bytes", ctypes.c_int64), ("seconds", ctypes.c_double), ("from_cache", ctypes.c_int32),
                ("ckpt_budget", ctypes.c_int32), ("ckpt_intervals", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


MVF_ENGINE = {"auto": 0, "interp": 1, "spec": 2}
SPLIT_RULES = {"adaptive": 0, "doubling": 1}


EXPORTS = ["mvf_tape_create", "mvf_tape_check", "mvf_tape_stats_get", "mvf_tape_destroy",
           "mvf_bound_workspace", "mvf_bound", "mvf_adaptive_splits", "mvf_batch_workspace", "mvf_bound_batch",
           "mvf_batch_graph_create", "mvf_batch_graph_staging", "mvf_batch_graph_launch", "mvf_batch_graph_result",
           "mvf_batch_graph_destroy", "mvf_autotune", "mvf_strerror", "mvf_last_error",
           "mvf_points_workspace", "mvf_eval_points", "mvf_vjp_points", "mvf_gradient_boxes",
           "mvf_tape_set_root_kinds", "mvf_bnb_solve", "mvf_tape_specialize", "mvf_spec_check", "mvf_splits",
           "mvf_autotune_splits", "mvf_fbbt", "mvf_fbbt_workspace", "mvf_spec_source", "mvf_bound_noalloc", "mvf_batch_graph_wait"]


def lib():
    """Load libmvf.so (raises if it is not built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is not built; run paper_2507_20769_amd/build.py")
            # torch ships its own HIP and HSA runtimes under the same sonames as the
            # system ROCm ones that libmvf links; whichever loads first serves the whole
            # process.  Load torch's first, so that torch and libmvf share one runtime
            # (torch finds no device when it is handed the other one).
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            L = ctypes.CDLL(LIB_PATH)
            P, i32 = ctypes.c_void_p, ctypes.c_int32
            L.mvf_strerror.restype = ctypes.c_char_p
            L.mvf_strerror.argtypes = [ctypes.c_int]
            L.mvf_last_error.restype = ctypes.c_char_p
            L.mvf_last_error.argtypes = []
            tape_args = [P, i32, P, i32, i32, P, i32]
            L.mvf_tape_create.restype = ctypes.c_int
            L.mvf_tape_create.argtypes = tape_args + [ctypes.POINTER(P)]
            L.mvf_tape_check.restype = ctypes.c_int
            L.mvf_tape_check.argtypes = tape_args + [ctypes.POINTER(TapeStats)]
            L.mvf_tape_stats_get.restype = ctypes.c_int
            L.mvf_tape_stats_get.argtypes = [P, ctypes.POINTER(TapeStats)]
            L.mvf_tape_destroy.restype = ctypes.c_int
            L.mvf_tape_destroy.argtypes = [P]
            L.mvf_bound_workspace.restype = ctypes.c_int
            L.mvf_bound_workspace.argtypes = [P, P, i32, i32, ctypes.POINTER(ctypes.c_size_t)]
            L.mvf_bound.restype = ctypes.c_int
            L.mvf_bound.argtypes = [P, ctypes.POINTER(BoundArgs), P]
            L.mvf_bound_noalloc.restype = ctypes.c_int
            L.mvf_bound_noalloc.argtypes = [P, ctypes.POINTER(BoundArgs), P]
            i64 = ctypes.c_int64
            L.mvf_adaptive_splits.restype = i64
            L.mvf_adaptive_splits.argtypes = [i32, P, i64, P]
            L.mvf_fbbt_workspace.restype = ctypes.c_int
            L.mvf_fbbt_workspace.argtypes = [P, i64, ctypes.POINTER(ctypes.c_size_t)]
            L.mvf_fbbt.restype = ctypes.c_int
            L.mvf_fbbt.argtypes = [P, i64, P, ctypes.c_double, i32, P, P, P, ctypes.c_size_t, P]
            L.mvf_splits.restype = i64
            L.mvf_splits.argtypes = [i32, i32, P, i64, P]
            L.mvf_autotune_splits.restype = ctypes.c_int
            L.mvf_autotune_splits.argtypes = [P, i32, P, i64, i32, i32, ctypes.POINTER(ctypes.c_int32), P, P]
            L.mvf_batch_workspace.restype = ctypes.c_int
            L.mvf_batch_workspace.argtypes = [P, i32, i64, i32, i32, ctypes.POINTER(Tuning),
                                              ctypes.POINTER(ctypes.c_size_t)]
            L.mvf_bound_batch.restype = ctypes.c_int
            L.mvf_bound_batch.argtypes = [P, ctypes.POINTER(BatchArgs), ctypes.POINTER(Tuning), P]
            L.mvf_batch_graph_create.restype = ctypes.c_int
            L.mvf_batch_graph_create.argtypes = [P, i32, i64, i32, i32, ctypes.POINTER(Tuning), P, ctypes.POINTER(P)]
            L.mvf_batch_graph_staging.restype = ctypes.c_int
            L.mvf_batch_graph_staging.argtypes = [P, ctypes.POINTER(ctypes.POINTER(ctypes.c_double)),
                                                  ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))]
            L.mvf_batch_graph_launch.restype = ctypes.c_int
            L.mvf_batch_graph_launch.argtypes = [P, i32, P]
            L.mvf_batch_graph_wait.restype = ctypes.c_int
            L.mvf_batch_graph_wait.argtypes = [P]
            L.mvf_batch_graph_result.restype = ctypes.c_int
            L.mvf_batch_graph_result.argtypes = [P, ctypes.POINTER(ctypes.POINTER(ctypes.c_double)),
                                                 ctypes.POINTER(ctypes.POINTER(ctypes.c_int64)),
                                                 ctypes.POINTER(ctypes.POINTER(ctypes.c_int32)),
                                                 ctypes.POINTER(ctypes.POINTER(ctypes.c_double))]
            L.mvf_tape_set_root_kinds.restype = ctypes.c_int
            L.mvf_tape_set_root_kinds.argtypes = [P, P]
            L.mvf_bnb_solve.restype = ctypes.c_int
            L.mvf_bnb_solve.argtypes = [P, P, ctypes.POINTER(BnbOptions), ctypes.POINTER(BnbResult), P]
            L.mvf_batch_graph_destroy.restype = ctypes.c_int
            L.mvf_batch_graph_destroy.argtypes = [P]
            L.mvf_autotune.restype = ctypes.c_int
            L.mvf_autotune.argtypes = [P, i32, P, P, i64, i32, i32, ctypes.POINTER(Tuning), P]
            L.mvf_points_workspace.restype = ctypes.c_int
            L.mvf_points_workspace.argtypes = [P, i32, i64, ctypes.POINTER(ctypes.c_size_t)]
            L.mvf_eval_points.restype = ctypes.c_int
            L.mvf_eval_points.argtypes = [P, i64, P, P, P, P, ctypes.c_size_t, P]
            L.mvf_vjp_points.restype = ctypes.c_int
            L.mvf_vjp_points.argtypes = [P, i64, P, P, P, P, P, ctypes.c_size_t, P]
            L.mvf_gradient_boxes.restype = ctypes.c_int
            L.mvf_gradient_boxes.argtypes = [P, i64, P, i32, i32, P, P, P, ctypes.c_size_t, P]
            L.mvf_tape_specialize.restype = ctypes.c_int
            L.mvf_tape_specialize.argtypes = [P, ctypes.POINTER(SpecOptions), ctypes.POINTER(SpecInfo)]
            L.mvf_spec_check.restype = ctypes.c_int
            L.mvf_spec_check.argtypes = tape_args + [ctypes.POINTER(SpecOptions), ctypes.POINTER(SpecInfo)]
            L.mvf_spec_source.restype = ctypes.c_int
            L.mvf_spec_source.argtypes = tape_args + [ctypes.POINTER(SpecOptions), ctypes.c_char_p, ctypes.c_size_t,
                                                      ctypes.POINTER(ctypes.c_size_t)]
            _lib = L
    return _lib


def _tape_arrays(tape):
    nodes = np.ascontiguousarray(tape.nodes)
    consts = np.ascontiguousarray(tape.consts, dtype=np.float64)
    roots = np.ascontiguousarray(tape.roots, dtype=np.int32)
    keep = (nodes, consts, roots)
    cp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    args = [cp(nodes), len(nodes), cp(consts) if consts.size else None, len(consts), int(tape.n_vars),
            cp(roots), len(roots)]
    return keep, args


def check(tape) -> TapeStats:
    """Validate and compile a tape on the host only (no device needed)."""
    keep, args = _tape_arrays(tape)
    st = TapeStats()
    rc = lib().mvf_tape_check(*args, ctypes.byref(st))
    if rc != 0:
        raise MVFError(rc, "mvf_tape_check")
    return st


def spec_check(tape, chunk: int = 0, waves: int = 0, max_code: int = 0, grad: str = "fwd",
               ckpt_budget: int = 0, cache: bool = False) -> dict:
    """Generate and compile the specialised kernels of a tape for gfx950 on the
    host (no device); cache: write (or read) the code-object cache that
    Tape.specialize with the same options reads; returns the mvf_spec_info fields."""
    keep, args = _tape_arrays(tape)
    info = SpecInfo()
    rc = lib().mvf_spec_check(*args, ctypes.byref(SpecOptions(chunk, waves, max_code, int(cache), MVF_GRAD[grad],
                                                              ckpt_budget)),
                              ctypes.byref(info))
    if rc != 0:
        raise MVFError(rc, "mvf_spec_check")
    return info.as_dict()


def spec_source(tape, chunk: int = 0, waves: int = 0, max_code: int = 0, grad: str = "fwd",
                ckpt_budget: int = 0) -> str:
    """The generated device source of a tape's specialised kernels (mvf_spec_source), not compiled."""
    keep, args = _tape_arrays(tape)
    opt = SpecOptions(chunk, waves, max_code, 0, MVF_GRAD[grad], ckpt_budget)
    n = ctypes.c_size_t()
    rc = lib().mvf_spec_source(*args, ctypes.byref(opt), None, 0, ctypes.byref(n))
    if rc != 0:
        raise MVFError(rc, "mvf_spec_source")
    buf = ctypes.create_string_buffer(n.value + 1)
    rc = lib().mvf_spec_source(*args, ctypes.byref(opt), buf, n.value + 1, ctypes.byref(n))
    if rc != 0:
        raise MVFError(rc, "mvf_spec_source")
    return buf.value.decode()


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Tape:
    """A tape compiled and uploaded to the current device."""

    def __init__(self, tape):
        self.src = tape
        keep, args = _tape_arrays(tape)
        h = ctypes.c_void_p()
        rc = lib().mvf_tape_create(*args, ctypes.byref(h))
        if rc != 0:
            raise MVFError(rc, "mvf_tape_create")
        self.handle = h
        self.n_vars = int(tape.n_vars)
        self.n_roots = int(tape.n_roots)

    @classmethod
    def from_file(cls, path: str) -> "Tape":
        """A tape file written by inputs.save_tape (.npz of plain arrays), compiled and uploaded."""
        from . import inputs
        return cls(inputs.load_tape(path))

    def set_root_kinds(self, kinds):
        """Root kinds: 0 objective/unconstrained, 1 inequality g <= 0, 2 equality h = 0 (root 0: 0)."""
        self._kinds = None if kinds is None else np.ascontiguousarray(kinds, dtype=np.int32)
        rc = lib().mvf_tape_set_root_kinds(self.handle, None if self._kinds is None else
                                           self._kinds.ctypes.data_as(ctypes.c_void_p))
        if rc != 0:
            raise MVFError(rc, "mvf_tape_set_root_kinds")
        return self

    def specialize(self, chunk: int = 0, waves: int = 0, max_code: int = 0, cache: bool = True,
                   grad: str = "fwd", ckpt_budget: int = 0) -> dict:
        """Build the tape's specialised kernels (mvf_tape_specialize); grad "fwd", "rev" or "auto" (both);
        ckpt_budget: segment budget of the checkpointed adjoint (0 library choice, < 0 none)."""
        info = SpecInfo()
        rc = lib().mvf_tape_specialize(self.handle,
                                       ctypes.byref(SpecOptions(chunk, waves, max_code, int(cache), MVF_GRAD[grad],
                                                                ckpt_budget)),
                                       ctypes.byref(info))
        if rc != 0:
            raise MVFError(rc, "mvf_tape_specialize")
        self.spec_info = info.as_dict()
        return self.spec_info

    def stats(self) -> TapeStats:
        st = TapeStats()
        rc = lib().mvf_tape_stats_get(self.handle, ctypes.byref(st))
        if rc != 0:
            raise MVFError(rc, "mvf_tape_stats_get")
        return st

    def close(self):
        if getattr(self, "handle", None):
            lib().mvf_tape_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BoundCall:
    """Pre-marshalled arguments of one mvf_bound call (buffers allocated once,
    so repeated launches only enqueue kernels)."""

    def __init__(self, tape: Tape, box, splits: Sequence[int], mode: str = "both", grad: str = "fwd",
                 per_sub: bool = False, flags: bool = False, tuning: "Tuning | None" = None, engine: str = "auto",
                 noalloc: bool = False):
        """noalloc: launch through mvf_bound_noalloc (no workspace; the library's device scratch)."""
        import torch
        self.tape = tape
        self.tuning = tuning
        self.noalloc = noalloc
        dev = box.device
        assert box.dtype == torch.float64 and box.is_cuda and tuple(box.shape) == (tape.n_vars, 2)
        self.box = box.contiguous()
        self.splits = np.ascontiguousarray(splits, dtype=np.int32)
        assert self.splits.shape == (tape.n_vars,)
        self.S = int(np.prod(self.splits.astype(np.int64)))
        m = tape.n_roots
        self.reduced = torch.empty((m, 2), dtype=torch.float64, device=dev)
        self.argmin = torch.empty(1, dtype=torch.int64, device=dev)
        self.extra = torch.empty(2, dtype=torch.float64, device=dev)
        self.per_sub = torch.empty((m, 2, self.S), dtype=torch.float64, device=dev) if per_sub else None
        self.flags = torch.empty(self.S, dtype=torch.int32, device=dev) if flags else None
        if noalloc:
            self.workspace = None
        else:
            ws = ctypes.c_size_t()
            rc = lib().mvf_bound_workspace(tape.handle, self.splits.ctypes.data_as(ctypes.c_void_p),
                                           MVF_MODE[mode], MVF_GRAD[grad], ctypes.byref(ws))
            if rc != 0:
                raise MVFError(rc, "mvf_bound_workspace")
            self.workspace = torch.empty(max(int(ws.value), 8), dtype=torch.uint8, device=dev)
        self.args = BoundArgs(self.box.data_ptr(), self.splits.ctypes.data, MVF_MODE[mode], MVF_GRAD[grad],
                              self.reduced.data_ptr(), self.argmin.data_ptr(),
                              self.per_sub.data_ptr() if per_sub else None,
                              self.flags.data_ptr() if flags else None,
                              self.workspace.data_ptr() if self.workspace is not None else None,
                              self.workspace.numel() if self.workspace is not None else 0,
                              ctypes.addressof(tuning) if tuning is not None else None, self.extra.data_ptr(),
                              MVF_ENGINE[engine])

    def time_kernel(self, start, end) -> None:
        """Record the torch.cuda.Events ``start`` and ``end`` (or None, None) around the
        bounding kernel alone on later launches."""
        for ev in (start, end):
            if ev is not None and not ev.cuda_event:
                ev.record()            # torch creates its event at the first record
        self.args.kernel_events[0] = start.cuda_event if start is not None else None
        self.args.kernel_events[1] = end.cuda_event if end is not None else None

    def launch(self, stream=None):
        fn = lib().mvf_bound_noalloc if self.noalloc else lib().mvf_bound
        rc = fn(self.tape.handle, ctypes.byref(self.args), _stream_ptr(stream))
        if rc != 0:
            raise MVFError(rc, "mvf_bound_noalloc" if self.noalloc else "mvf_bound")
        return self


def bound(tape: Tape, box, splits: Sequence[int], mode: str = "both", grad: str = "fwd",
          per_sub: bool = False, flags: bool = False, stream=None, engine: str = "auto") -> dict:
    """Bound every subdomain of ``box`` (device float64 [n, 2]).

    Returns device tensors: reduced [m, 2] (lo, hi), argmin [1], and when asked
    per_sub [m, 2, S] and flags [S].  Asynchronous on ``stream``.  ``engine``:
    "auto" (the specialised kernel when the tape has one), "interp" or "spec".
    """
    call = BoundCall(tape, box, splits, mode, grad, per_sub, flags, engine=engine).launch(stream)
    out = {"reduced": call.reduced, "argmin": call.argmin, "extra": call.extra, "workspace": call.workspace}
    if per_sub:
        out["per_sub"] = call.per_sub
    if flags:
        out["flags"] = call.flags
    return out


def adaptive_splits(widths, budget: int):
    """Adaptive partitioning of Sec. 3.1.2 (host computation in the library)."""
    w = np.ascontiguousarray(widths, dtype=np.float64)
    out = np.zeros(len(w), dtype=np.int32)
    count = lib().mvf_adaptive_splits(len(w), w.ctypes.data_as(ctypes.c_void_p), int(budget),
                                      out.ctypes.data_as(ctypes.c_void_p))
    if count < 0:
        raise MVFError(int(count), "mvf_adaptive_splits")
    return out, int(count)


def splits(rule: str, widths, budget: int):
    """Split counts of one box under a split rule ("adaptive", Sec. 3.1.2, or "doubling")."""
    w = np.ascontiguousarray(widths, dtype=np.float64)
    out = np.zeros(len(w), dtype=np.int32)
    count = lib().mvf_splits(SPLIT_RULES[rule], len(w), w.ctypes.data_as(ctypes.c_void_p), int(budget),
                             out.ctypes.data_as(ctypes.c_void_p))
    if count < 0:
        raise MVFError(int(count), "mvf_splits")
    return out, int(count)


def autotune_splits(tape: Tape, boxes, budget: int, mode: str = "both", grad: str = "rev", stream=None):
    """The split rule giving the tighter objective bounds on sample node boxes (host [N, n, 2]).
    Returns (rule name, [nodes where adaptive is tighter, nodes where doubling is tighter])."""
    b = np.ascontiguousarray(boxes, dtype=np.float64)
    assert b.ndim == 3 and b.shape[1:] == (tape.n_vars, 2)
    rule = ctypes.c_int32()
    better = (ctypes.c_int32 * 2)()
    rc = lib().mvf_autotune_splits(tape.handle, b.shape[0], b.ctypes.data_as(ctypes.c_void_p), int(budget),
                                   MVF_MODE[mode], MVF_GRAD[grad], ctypes.byref(rule), better, _stream_ptr(stream))
    if rc != 0:
        raise MVFError(rc, "mvf_autotune_splits")
    return ("adaptive", "doubling")[rule.value], [better[0], better[1]]


def fbbt(tape: Tape, boxes, ub: float = float("inf"), rounds: int = 1, stream=None):
    """Forward-backward bound tightening of boxes (device float64 [N, n, 2]).
    Returns (tightened boxes [N, n, 2], status [N] int32, 1 = proven infeasible)."""
    import torch
    b = boxes.contiguous()
    assert b.dtype == torch.float64 and b.is_cuda and b.dim() == 3 and b.shape[1:] == (tape.n_vars, 2)
    N = int(b.shape[0])
    ws = ctypes.c_size_t()
    rc = lib().mvf_fbbt_workspace(tape.handle, N, ctypes.byref(ws))
    if rc != 0:
        raise MVFError(rc, "mvf_fbbt_workspace")
    work = torch.empty(int(ws.value), dtype=torch.uint8, device=b.device)
    out = torch.empty_like(b)
    st = torch.empty(max(N, 1), dtype=torch.int32, device=b.device)
    rc = lib().mvf_fbbt(tape.handle, N, b.data_ptr(), float(ub), int(rounds), out.data_ptr(), st.data_ptr(),
                        work.data_ptr(), work.numel(), _stream_ptr(stream))
    if rc != 0:
        raise MVFError(rc, "mvf_fbbt")
    return out, st[:N]


def _require_device(where: str, **tensors):
    """The batched entry points hand raw pointers to kernels: every array must be a
    GPU tensor, all on one device (a host pointer would fault the GPU)."""
    devs = set()
    for name, x in tensors.items():
        if not getattr(x, "is_cuda", False):
            raise ValueError(f"{where}: {name} must be a GPU tensor (got {getattr(x, 'device', type(x))})")
        devs.add(x.device)
    if len(devs) > 1:
        raise ValueError(f"{where}: {', '.join(tensors)} must be on one device (got {sorted(map(str, devs))})")


class BatchCall:
    """Pre-marshalled batched bound of many nodes (device boxes [N, n, 2] f64, splits [N, n] i32)."""

    def __init__(self, tape: Tape, boxes, splits, mode: str = "both", grad: str = "rev",
                 tuning: Optional[Tuning] = None, max_subdomains: Optional[int] = None):
        import torch
        _require_device("BatchCall", boxes=boxes, splits=splits)
        self.tape = tape
        self.boxes = boxes.contiguous()
        self.splits = splits.to(torch.int32).contiguous()
        N = int(self.boxes.shape[0])
        assert tuple(self.boxes.shape) == (N, tape.n_vars, 2) and self.boxes.dtype == torch.float64
        assert tuple(self.splits.shape) == (N, tape.n_vars)
        total = int(torch.prod(self.splits.to(torch.int64), dim=1).sum().item()) if N else 0
        self.total = total
        cap = max_subdomains if max_subdomains is not None else total
        dev = self.boxes.device
        m = tape.n_roots
        self.tuning = tuning
        self.empty = N == 0                    # an empty batch: no call, empty results
        if self.empty:
            self.reduced = torch.empty((0, m, 2), dtype=torch.float64, device=dev)
            self.argmin = torch.empty(0, dtype=torch.int64, device=dev)
            self.status = torch.empty(0, dtype=torch.int32, device=dev)
            self.extra = torch.empty((0, 2), dtype=torch.float64, device=dev)
            return
        tp = ctypes.byref(tuning) if tuning is not None else None
        ws = ctypes.c_size_t()
        rc = lib().mvf_batch_workspace(tape.handle, N, max(cap, 1), MVF_MODE[mode], MVF_GRAD[grad], tp,
                                       ctypes.byref(ws))
        if rc != 0:
            raise MVFError(rc, "mvf_batch_workspace")
        self.workspace = torch.empty(max(int(ws.value), 8), dtype=torch.uint8, device=dev)
        self.reduced = torch.empty((N, m, 2), dtype=torch.float64, device=dev)
        self.argmin = torch.empty(N, dtype=torch.int64, device=dev)
        self.status = torch.empty(N, dtype=torch.int32, device=dev)
        self.extra = torch.empty((N, 2), dtype=torch.float64, device=dev)
        self.args = BatchArgs(N, N, max(cap, 1), self.boxes.data_ptr(), self.splits.data_ptr(), MVF_MODE[mode],
                              MVF_GRAD[grad], self.reduced.data_ptr(), self.argmin.data_ptr(), self.status.data_ptr(),
                              self.workspace.data_ptr(), self.workspace.numel(), self.extra.data_ptr())

    def launch(self, stream=None):
        if self.empty:
            return self
        tp = ctypes.byref(self.tuning) if self.tuning is not None else None
        rc = lib().mvf_bound_batch(self.tape.handle, ctypes.byref(self.args), tp, _stream_ptr(stream))
        if rc != 0:
            raise MVFError(rc, "mvf_bound_batch")
        return self


def bound_batch(tape: Tape, boxes, splits, mode: str = "both", grad: str = "rev", tuning=None, stream=None) -> dict:
    call = BatchCall(tape, boxes, splits, mode, grad, tuning).launch(stream)
    return {"reduced": call.reduced, "argmin": call.argmin, "status": call.status, "extra": call.extra}


class BatchGraph:
    """A batched bound captured once in a HIP graph, replayed per call with new node data."""

    def __init__(self, tape: Tape, max_nodes: int, max_subdomains: int, mode: str = "both", grad: str = "rev",
                 tuning: Optional[Tuning] = None):
        self.tape = tape
        self.max_nodes = max_nodes
        h = ctypes.c_void_p()
        tp = ctypes.byref(tuning) if tuning is not None else None
        rc = lib().mvf_batch_graph_create(tape.handle, max_nodes, max_subdomains, MVF_MODE[mode], MVF_GRAD[grad], tp,
                                          None, ctypes.byref(h))
        if rc != 0:
            raise MVFError(rc, "mvf_batch_graph_create")
        self.handle = h
        bp = ctypes.POINTER(ctypes.c_double)()
        sp = ctypes.POINTER(ctypes.c_int32)()
        lib().mvf_batch_graph_staging(h, ctypes.byref(bp), ctypes.byref(sp))
        n = tape.n_vars
        self.h_boxes = np.ctypeslib.as_array(bp, shape=(max_nodes, n, 2))
        self.h_splits = np.ctypeslib.as_array(sp, shape=(max_nodes, n))
        rp = ctypes.POINTER(ctypes.c_double)()
        ap = ctypes.POINTER(ctypes.c_int64)()
        stp = ctypes.POINTER(ctypes.c_int32)()
        ep = ctypes.POINTER(ctypes.c_double)()
        lib().mvf_batch_graph_result(h, ctypes.byref(rp), ctypes.byref(ap), ctypes.byref(stp), ctypes.byref(ep))
        self.h_extra = np.ctypeslib.as_array(ep, shape=(max_nodes, 2))
        self.h_reduced = np.ctypeslib.as_array(rp, shape=(max_nodes, tape.n_roots, 2))
        self.h_argmin = np.ctypeslib.as_array(ap, shape=(max_nodes,))
        self.h_status = np.ctypeslib.as_array(stp, shape=(max_nodes,))

    def launch(self, boxes: np.ndarray, splits: np.ndarray, stream=None):
        """Stage node data (host arrays) into pinned memory and replay the graph.  Waits
        first for the previous replay, whose copies read the staging buffers."""
        N = boxes.shape[0]
        rc = lib().mvf_batch_graph_wait(self.handle)
        if rc != 0:
            raise MVFError(rc, "mvf_batch_graph_wait")
        self.h_boxes[:N] = boxes
        self.h_splits[:N] = splits
        rc = lib().mvf_batch_graph_launch(self.handle, N, _stream_ptr(stream))
        if rc != 0:
            raise MVFError(rc, "mvf_batch_graph_launch")
        self.n = N
        return self

    def result(self):
        """Copies of (reduced [N, m, 2], argmin [N], status [N]); synchronise first."""
        N = self.n
        return self.h_reduced[:N].copy(), self.h_argmin[:N].copy(), self.h_status[:N].copy()

    def extra(self):
        """Copy of the per-node (feasibility-filtered lower bound, centre upper bound) [N, 2]."""
        return self.h_extra[:self.n].copy()

    def close(self):
        if getattr(self, "handle", None):
            lib().mvf_batch_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(tape: Tape, boxes, splits, mode: str = "both", grad: str = "rev", stream=None) -> Tuning:
    """mvf_autotune on sample nodes (device boxes [N, n, 2], splits [N, n]); the
    gradient mode is the caller's (the tuner picks kernel, grid, subdomains per
    lane and workgroup size).  Cached per process."""
    import torch
    _require_device("autotune", boxes=boxes, splits=splits)
    boxes = boxes.contiguous()
    splits = splits.to(torch.int32).contiguous()
    N = int(boxes.shape[0])
    total = int(torch.prod(splits.to(torch.int64), dim=1).sum().item())
    out = Tuning()
    rc = lib().mvf_autotune(tape.handle, N, boxes.data_ptr(), splits.data_ptr(), total, MVF_MODE[mode],
                            MVF_GRAD[grad], ctypes.byref(out), _stream_ptr(stream))
    if rc != 0:
        raise MVFError(rc, "mvf_autotune")
    return out


# ---------------------------------------------------------------------------
# points and boxes
# ---------------------------------------------------------------------------
_PT = {"eval": 0, "vjp": 1, "grad_fwd": 2, "grad_rev": 3}


def _points_ws(tape: Tape, op: str, B: int, device):
    import torch
    nb = ctypes.c_size_t()
    rc = lib().mvf_points_workspace(tape.handle, _PT[op], int(B), ctypes.byref(nb))
    if rc != 0:
        raise MVFError(rc, "mvf_points_workspace")
    return torch.empty(max(int(nb.value), 8), dtype=torch.uint8, device=device), int(nb.value)


def _check_points(tape: Tape, x, width: int):
    import torch
    assert x.dtype == torch.float64 and x.is_cuda, "device float64 tensor expected"
    assert x.dim() == (2 if width == 1 else 3) and x.shape[1] == tape.n_vars
    return x.contiguous()


def eval_points(tape: Tape, x, flags: bool = False, stream=None):
    """Enclosures [B, m, 2] of every root at the points x [B, n] (device float64)."""
    import torch
    x = _check_points(tape, x, 1)
    B = x.shape[0]
    f = torch.empty((B, tape.n_roots, 2), dtype=torch.float64, device=x.device)
    fl = torch.empty(max(B, 1), dtype=torch.int32, device=x.device) if flags else None
    ws, nb = _points_ws(tape, "eval", B, x.device)
    rc = lib().mvf_eval_points(tape.handle, B, x.data_ptr(), f.data_ptr(), fl.data_ptr() if flags else None,
                               ws.data_ptr() if nb else None, nb, _stream_ptr(stream))
    if rc != 0:
        raise MVFError(rc, "mvf_eval_points")
    return (f, fl[:B]) if flags else f


def vjp_points(tape: Tape, x, gout, flags: bool = False, stream=None):
    """Enclosures [B, n, 2] of sum_r gout[:, r] * grad f_r at the points x [B, n]."""
    import torch
    x = _check_points(tape, x, 1)
    B = x.shape[0]
    assert gout.dtype == torch.float64 and tuple(gout.shape) == (B, tape.n_roots)
    gout = gout.contiguous()
    gx = torch.empty((B, tape.n_vars, 2), dtype=torch.float64, device=x.device)
    fl = torch.empty(max(B, 1), dtype=torch.int32, device=x.device) if flags else None
    ws, nb = _points_ws(tape, "vjp", B, x.device)
    rc = lib().mvf_vjp_points(tape.handle, B, x.data_ptr(), gout.data_ptr(), gx.data_ptr(),
                              fl.data_ptr() if flags else None, ws.data_ptr() if nb else None, nb,
                              _stream_ptr(stream))
    if rc != 0:
        raise MVFError(rc, "mvf_vjp_points")
    return (gx, fl[:B]) if flags else gx


def gradient_boxes(tape: Tape, boxes, root: int = 0, grad: str = "rev", flags: bool = False, stream=None):
    """Interval gradient [B, n, 2] of one root on boxes [B, n, 2], tangent or adjoint mode."""
    import torch
    boxes = _check_points(tape, boxes, 2)
    B = boxes.shape[0]
    G = torch.empty((B, tape.n_vars, 2), dtype=torch.float64, device=boxes.device)
    fl = torch.empty(max(B, 1), dtype=torch.int32, device=boxes.device) if flags else None
    op = "grad_fwd" if grad == "fwd" else "grad_rev"
    ws, nb = _points_ws(tape, op, B, boxes.device)
    rc = lib().mvf_gradient_boxes(tape.handle, B, boxes.data_ptr(), int(root), MVF_GRAD[grad], G.data_ptr(),
                                  fl.data_ptr() if flags else None, ws.data_ptr() if nb else None, nb,
                                  _stream_ptr(stream))
    if rc != 0:
        raise MVFError(rc, "mvf_gradient_boxes")
    return (G, fl[:B]) if flags else G


def _midpoint(iv):
    """Midpoint of intervals stored as [..., 2] (lo, hi)."""
    return 0.5 * iv[..., 0] + 0.5 * iv[..., 1]


def _make_point_function():
    import torch

    class MVFPoint(torch.autograd.Function):
        """f(x) for a batch of points, differentiable through the library.

        forward:  x [B, n] (device float64) -> midpoints of the root enclosures [B, m]
        backward: grad [B, m] -> midpoints of the vector-Jacobian enclosures [B, n],
                  one reverse sweep per point (mvf_vjp_points).
        Both enclosures are a few ulps wide at points, so the midpoints carry
        the floating-point values of f and of its gradient.
        """

        @staticmethod
        def forward(ctx, x, tape):
            ctx.tape = tape
            ctx.save_for_backward(x)
            return _midpoint(eval_points(tape, x))

        @staticmethod
        def backward(ctx, grad):
            (x,) = ctx.saved_tensors
            gx = vjp_points(ctx.tape, x.detach(), grad.to(torch.float64).contiguous())
            return _midpoint(gx), None

    return MVFPoint


_MVFPoint = None


def MVFPoint():
    """The torch.autograd.Function class (built on first use so importing this module needs no torch)."""
    global _MVFPoint
    if _MVFPoint is None:
        _MVFPoint = _make_point_function()
    return _MVFPoint


def point_function(tape: Tape, x):
    """Differentiable f(x): MVFPoint().apply(x, tape)."""
    return MVFPoint().apply(x, tape)


# ---------------------------------------------------------------------------
# branch and bound
# ---------------------------------------------------------------------------
def bnb_solve(tape: Tape, box, max_nodes: int = 1000, gap: float = 1e-4, budget: int = 4096,
              nodes_per_launch: int = 1, mode: str = "both", grad: str = "fwd",
              tuning: Optional[Tuning] = None, stream=None, split_rule: str = "adaptive",
              fbbt_rounds: int = 0) -> dict:
    """Spatial B&B with GPU subdomain bounding (synchronous).  box: host [n, 2].

    Root kinds come from Tape.set_root_kinds.  Returns dict(lower, upper,
    nodes, subdomains, launches, open, status, seconds)."""
    b = np.ascontiguousarray(box, dtype=np.float64)
    assert b.shape == (tape.n_vars, 2)
    opt = BnbOptions(int(max_nodes), int(nodes_per_launch), int(budget), float(gap), MVF_MODE[mode], MVF_GRAD[grad],
                     ctypes.addressof(tuning) if tuning is not None else None, SPLIT_RULES[split_rule],
                     int(fbbt_rounds))
    res = BnbResult()
    rc = lib().mvf_bnb_solve(tape.handle, b.ctypes.data_as(ctypes.c_void_p), ctypes.byref(opt), ctypes.byref(res),
                             _stream_ptr(stream))
    if rc != 0:
        raise MVFError(rc, "mvf_bnb_solve")
    return {k: getattr(res, k) for k, _ in BnbResult._fields_}
