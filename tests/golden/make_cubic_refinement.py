"""Writes cubic_refinement_table.txt: the refined lower bounds of the DAG example
of Sec. 3.2 (f = 3x^3 + x^2 - 5x - 1 on X = [-1, 2]) for uniform partitions of
N = 1, 2, 4, ..., 256 subdomains, in the natural interval extension (NIE), the
mean value form (MVF) and MVF intersected with the NIE.

Everything is computed in exact rational arithmetic (fractions.Fraction), with
no floating point and nothing from the oracle or the library: on these
partitions every breakpoint, centre and intermediate bound is a dyadic
rational with few significant bits, so the exact values are also what any
correctly outward-rounded binary64 evaluation must return bit for bit.

The interval operations are the plain definitions (Sec. 2.2, interval
arithmetic): sums endpointwise, a product the hull of the four endpoint
products, the square [min(a^2, b^2), max(a^2, b^2)] or [0, max] when 0 lies
inside.  The gradient enclosure follows the tangent rules of the forward mode
(Sec. 3.2: the DAG evaluated node by node with derivative propagation); the
MVF is f([c]) + G (X - c) with c the midpoint (Sec. 2.2, Definition "Mean
Value Form"); the refinement is the minimum of the subdomain lower bounds
(Sec. 2.2 splitting technique, step iii; Sec. 3.1 Step 3).  Theorem 1
(Sec. 2.2) predicts excess widths of order 1 (NIE) and 2 (MVF) in 1/N, which
the table shows.

Run: python tests/golden/make_cubic_refinement.py  (rewrites the fixture)
"""
from __future__ import annotations

import os
from fractions import Fraction as F

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "cubic_refinement_table.txt")
NS = [1, 2, 4, 8, 16, 32, 64, 128, 256]


def add(u, v):
    return (u[0] + v[0], u[1] + v[1])


def sub(u, v):
    return (u[0] - v[1], u[1] - v[0])


def mul(u, v):
    p = [u[0] * v[0], u[0] * v[1], u[1] * v[0], u[1] * v[1]]
    return (min(p), max(p))


def sqr(u):
    a, b = u
    if a >= 0:
        return (a * a, b * b)
    if b <= 0:
        return (b * b, a * a)
    return (F(0), max(a * a, b * b))


def pt(k):
    return (F(k), F(k))


def cubic(X):
    """Values and tangents of the tape x -> v1 = sqr x, v2 = x v1, v3 = 3 v2,
    v4 = v3 + v1, v5 = 5 x, v6 = v4 - v5, v7 = v6 - 1 (the paper's DAG)."""
    one, zero = pt(1), pt(0)
    x, dx = X, one
    v1 = sqr(x)
    d1 = mul(add(x, x), dx)                               # (2U) dU
    v2 = mul(x, v1)
    d2 = add(mul(v1, dx), mul(x, d1))                     # V dU + U dV
    v3 = mul(pt(3), v2)
    d3 = add(mul(v2, zero), mul(pt(3), d2))
    v4 = add(v3, v1)
    d4 = add(d3, d1)
    v5 = mul(pt(5), x)
    d5 = add(mul(x, zero), mul(pt(5), dx))
    v6 = sub(v4, v5)
    d6 = sub(d4, d5)
    v7 = sub(v6, pt(1))
    return v7, d6


def refined(N: int):
    lo, hi = F(-1), F(2)
    h = (hi - lo) / N
    best = {"nie": None, "mvf": None, "both": None}
    for j in range(N):
        X = (lo + j * h, lo + (j + 1) * h)
        c = (X[0] + X[1]) / 2
        nie, G = cubic(X)
        fc, _ = cubic(pt(c))
        mvf = add(fc, mul(G, sub(X, pt(c))))
        both = (max(mvf[0], nie[0]), min(mvf[1], nie[1]))
        for k, v in (("nie", nie[0]), ("mvf", mvf[0]), ("both", both[0])):
            best[k] = v if best[k] is None else min(best[k], v)
    return best


def table():
    return [(N, refined(N)) for N in NS]


def main():
    lines = ["# Refined lower bounds of the DAG example of Sec. 3.2, f = 3x^3 + x^2 - 5x - 1 on X = [-1, 2],",
             "# uniform partitions into N subdomains: min over the subdomains of the lower bound of the natural",
             "# interval extension (nie), the mean value form (mvf) and mvf intersected with nie (both).",
             "# Exact rational values (written by make_cubic_refinement.py), as exact decimal expansions of",
             "# dyadic rationals.  Theorem 1 (Sec. 2.2): excess width O(1/N) for nie, O(1/N^2) for mvf.",
             "# N nie mvf both"]
    for N, b in table():
        for k in ("nie", "mvf", "both"):
            assert b[k].denominator & (b[k].denominator - 1) == 0      # dyadic
        lines.append(f"lb {N} {float(b['nie'])!r} {float(b['mvf'])!r} {float(b['both'])!r}")
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
