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
                ("max_slots", ctypes.c_int32), ("tangent_chunk", ctypes.c_int32),
                ("ref_ops_fwd", ctypes.c_int64), ("ref_ops_rev", ctypes.c_int64)]


class BoundArgs(ctypes.Structure):
    _fields_ = [("box", ctypes.c_void_p), ("splits", ctypes.c_void_p), ("mode", ctypes.c_int32),
                ("grad", ctypes.c_int32), ("reduced", ctypes.c_void_p), ("argmin", ctypes.c_void_p),
                ("per_sub", ctypes.c_void_p), ("flags", ctypes.c_void_p), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t)]


EXPORTS = ["mvf_tape_create", "mvf_tape_check", "mvf_tape_stats_get", "mvf_tape_destroy",
           "mvf_bound_workspace", "mvf_bound", "mvf_strerror", "mvf_last_error"]


def lib():
    """Load libmvf.so (raises if it is not built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is not built; run paper_2507_20769_amd/build.py")
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
                 per_sub: bool = False, flags: bool = False):
        import torch
        self.tape = tape
        dev = box.device
        assert box.dtype == torch.float64 and box.is_cuda and tuple(box.shape) == (tape.n_vars, 2)
        self.box = box.contiguous()
        self.splits = np.ascontiguousarray(splits, dtype=np.int32)
        assert self.splits.shape == (tape.n_vars,)
        self.S = int(np.prod(self.splits.astype(np.int64)))
        m = tape.n_roots
        self.reduced = torch.empty((m, 2), dtype=torch.float64, device=dev)
        self.argmin = torch.empty(1, dtype=torch.int64, device=dev)
        self.per_sub = torch.empty((m, 2, self.S), dtype=torch.float64, device=dev) if per_sub else None
        self.flags = torch.empty(self.S, dtype=torch.int32, device=dev) if flags else None
        ws = ctypes.c_size_t()
        rc = lib().mvf_bound_workspace(tape.handle, self.splits.ctypes.data_as(ctypes.c_void_p), MVF_MODE[mode],
                                       MVF_GRAD[grad], ctypes.byref(ws))
        if rc != 0:
            raise MVFError(rc, "mvf_bound_workspace")
        self.workspace = torch.empty(max(int(ws.value), 8), dtype=torch.uint8, device=dev)
        self.args = BoundArgs(self.box.data_ptr(), self.splits.ctypes.data, MVF_MODE[mode], MVF_GRAD[grad],
                              self.reduced.data_ptr(), self.argmin.data_ptr(),
                              self.per_sub.data_ptr() if per_sub else None,
                              self.flags.data_ptr() if flags else None,
                              self.workspace.data_ptr(), self.workspace.numel())

    def launch(self, stream=None):
        rc = lib().mvf_bound(self.tape.handle, ctypes.byref(self.args), _stream_ptr(stream))
        if rc != 0:
            raise MVFError(rc, "mvf_bound")
        return self


def bound(tape: Tape, box, splits: Sequence[int], mode: str = "both", grad: str = "fwd",
          per_sub: bool = False, flags: bool = False, stream=None) -> dict:
    """Bound every subdomain of ``box`` (device float64 [n, 2]).

    Returns device tensors: reduced [m, 2] (lo, hi), argmin [1], and when asked
    per_sub [m, 2, S] and flags [S].  Asynchronous on ``stream``.
    """
    call = BoundCall(tape, box, splits, mode, grad, per_sub, flags).launch(stream)
    out = {"reduced": call.reduced, "argmin": call.argmin, "workspace": call.workspace}
    if per_sub:
        out["per_sub"] = call.per_sub
    if flags:
        out["flags"] = call.flags
    return out
