"""Symbolic execution of the generated straight-line device code (a test helper).

A generated function is a sequence of assignments ``x = f(a, b)``, multi-result
calls ``imul2(a, b, c, d, r, s)`` and checkpoint stores and loads.  Executing it
over hash-consed expression nodes -- every call becomes the node (f, operand
nodes), shared by every execution that builds the same call on the same operands
-- gives each result a canonical expression graph.  Two functions compute the
same values bit for bit (same operations, same operands, same order inside every
operation) exactly when their results are the same node; this is how the
checkpointed adjoint is compared with the single-pass adjoint without a GPU.
Domain-flag statements (``bad |= ...``) and the guards are ignored."""
from __future__ import annotations

import re
from typing import Dict, List, Tuple

MULTI = {"imul2": 2, "imul_pos2": 2}       # calls whose last k arguments are outputs


class Graph:
    def __init__(self):
        self.ids: Dict[tuple, int] = {}

    def node(self, key: tuple) -> int:
        if key not in self.ids:
            self.ids[key] = len(self.ids)
        return self.ids[key]


def _split_top(text: str, sep: str) -> List[str]:
    out, depth, cur = [], 0, []
    for c in text:
        if c in "({":
            depth += 1
        elif c in ")}":
            depth -= 1
        if c == sep and depth == 0:
            out.append("".join(cur).strip())
            cur = []
        else:
            cur.append(c)
    if "".join(cur).strip():
        out.append("".join(cur).strip())
    return out


def _call(expr: str):
    """(function name, argument texts) of a call expression, or None for a leaf."""
    m = re.match(r"^([A-Za-z_]\w*)\s*\((.*)\)$", expr, flags=re.S)
    if not m:
        return None
    return m.group(1), _split_top(m.group(2), ",")


_GL = re.compile(r"^spec_gl\(L,\s*\d+\)$")


class Machine:
    """One execution: variable bindings and the lane's checkpoint buffer."""

    def __init__(self, g: Graph):
        self.g = g
        self.env: Dict[str, int] = {}
        self.ck: Dict[str, int] = {}
        self.ck_stores = 0
        self.ck_loads = 0
        self.ck_loaded = set()

    def eval(self, expr: str) -> int:
        expr = expr.strip()
        if _GL.match(expr):                 # an LDS-resident gradient component: a variable
            expr = re.sub(r"\s+", "", expr)
            if expr not in self.env:
                raise KeyError(f"read of unassigned variable {expr!r}")
            return self.env[expr]
        c = _call(expr)
        if c is None:
            if expr in self.env:
                return self.env[expr]
            if not re.match(r"^(Iv\{.*\}|[-+0-9a-fA-Fx.p]+|k[A-Z]\w*|L)$", expr, flags=re.S):
                raise KeyError(f"read of unassigned variable {expr!r}")
            return self.g.node(("leaf", re.sub(r"\s+", "", expr)))
        fn, args = c
        return self.g.node((fn,) + tuple(self.eval(a) for a in args))

    def stmt(self, s: str):
        s = s.strip()
        if not s or s.startswith("bad "):
            return
        if s.startswith("spec_ck_st("):
            _, args = _call(s)
            self.ck[args[1]] = self.eval(args[2])
            self.ck_stores += 1
            return
        c = _call(s)
        if c is not None and c[0] in MULTI:
            fn, args = c
            k = MULTI[fn]
            ins = tuple(self.eval(a) for a in args[:-k])
            for j, out in enumerate(args[-k:]):
                self.env[out.strip()] = self.g.node((fn + "#" + str(j),) + ins)
            return
        lhs, rhs = s.split("=", 1)
        lhs, rhs = lhs.strip(), rhs.strip()
        if _GL.match(lhs):
            lhs = re.sub(r"\s+", "", lhs)
        lc = _call(rhs)
        if lc is not None and lc[0] == "spec_ck_ld":
            key = lc[1][1]
            if key not in self.ck:
                raise KeyError(f"checkpoint {key} loaded before it was stored")
            self.env[lhs] = self.ck[key]
            self.ck_loads += 1
            self.ck_loaded.add(key)
            return
        self.env[lhs] = self.eval(rhs)


def functions(src: str) -> Dict[str, str]:
    """Bodies of the generated device functions by name."""
    out = {}
    for m in re.finditer(r"__device__ __forceinline__ \w+ (\w+)\((.*?)\) \{\n(.*?)\n\}\n", src, flags=re.S):
        out[m.group(1)] = m.group(3)
    return out


def run(body: str, g: Graph, n_grad: int) -> Tuple[int, List[int], Machine]:
    """Execute a generated adjoint or pass body; returns the returned node, the
    nodes of G[0..n_grad) and the machine (for checkpoint counts)."""
    M = Machine(g)
    ret = None
    for line in body.split("\n"):
        t = line.strip()
        if (not t or t.startswith("//") or t.startswith("if (go)") or t == "}" or
                re.match(r"^Iv \w+;$", t)):
            continue
        if t.startswith("return "):
            ret = M.eval(t[len("return "):].rstrip(";"))
            continue
        for s in _split_top(t, ";"):
            M.stmt(s)
    grads = [M.env.get(f"G[{i}]", -1) for i in range(n_grad)]
    return ret, grads, M
