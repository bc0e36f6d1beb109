"""Pins of the oracle against values fixed independently of it.

* The refinement table of the DAG example of Sec. 3.2 (f = 3x^3 + x^2 - 5x - 1
  on [-1, 2], N = 1..256 subdomains, NIE, MVF and MVF with NIE) in
  tests/golden/cubic_refinement_table.txt, written by a script that computes it
  in exact rational arithmetic; every value is a dyadic rational that binary64
  holds exactly, so the oracle's outward-rounded evaluation must return it bit
  for bit.
* Hand-worked reverse-mode adjoints whose expected bits are computed here with
  exact rationals and directed rounding of each operation: a variable read
  through two leaf nodes (where summing the contributions per leaf and summing
  them in sweep order give different bits), and the division and square-root
  adjoint rules.
"""
import math
import os
import sys
from fractions import Fraction as Fr

import numpy as np

from oracle import oracle as O
from paper_2507_20769_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
sys.path.insert(0, GOLDEN)
import make_cubic_refinement as MCR  # noqa: E402


# -- directed rounding of exact rationals --------------------------------
def rd(q: Fr) -> float:
    f = float(q)                                  # round to nearest
    return math.nextafter(f, -math.inf) if Fr(f) > q else f


def ru(q: Fr) -> float:
    f = float(q)
    return math.nextafter(f, math.inf) if Fr(f) < q else f


def iadd(u, v):
    return (rd(Fr(u[0]) + Fr(v[0])), ru(Fr(u[1]) + Fr(v[1])))


def isub(u, v):
    return (rd(Fr(u[0]) - Fr(v[1])), ru(Fr(u[1]) - Fr(v[0])))


def imul(u, v):
    p = [Fr(a) * Fr(b) for a in u for b in v]
    return (min(rd(x) for x in p), max(ru(x) for x in p))


def irecip(v):                                    # 0 not in V
    return (rd(1 / Fr(v[1])), ru(1 / Fr(v[0])))


def idiv(u, v):
    q = [Fr(a) / Fr(b) for a in u for b in v]
    return (min(rd(x) for x in q), max(ru(x) for x in q))


def _tape(nodes, consts, roots, n):
    return I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.array(consts, dtype=np.float64),
                  np.array(roots, dtype=np.int32), n)


# -- the refinement table of the DAG example --------------------------------
def _table():
    rows = []
    for line in open(os.path.join(GOLDEN, "cubic_refinement_table.txt")):
        f = line.split("#")[0].split()
        if f and f[0] == "lb":
            rows.append((int(f[1]), float(f[2]), float(f[3]), float(f[4])))
    return rows


def test_cubic_refinement_fixture_is_the_exact_table():
    # the stored values are the exact rational results (dyadic, so exactly held by the doubles)
    rows = _table()
    exact = MCR.table()
    assert [r[0] for r in rows] == MCR.NS
    for (N, nie, mvf, both), (N2, b) in zip(rows, exact):
        assert N == N2
        assert (Fr(nie), Fr(mvf), Fr(both)) == (b["nie"], b["mvf"], b["both"]), N
    # N = 1 is the hand-worked case: NIE [-23, 32], MVF [-55.375, 49.625]
    assert rows[0][1:] == (-23.0, -55.375, -23.0)


def test_oracle_reproduces_the_refinement_table():
    t = I.cubic_tape()
    box = np.array([[-1.0, 2.0]])
    for N, nie, mvf, both in _table():
        got = [O.bound(t, box, [N], mode=m, per_sub=False)["reduced"][0, 0]
               for m in (O.MODE_NIE, O.MODE_MVF, O.MODE_BOTH)]
        assert got == [nie, mvf, both], (N, got)


def test_refinement_table_theorem1_orders():
    # excess over the true minimum halves (NIE) and quarters (MVF) per doubling of N (Theorem 1)
    true_min = (lambda x: 3 * x ** 3 + x ** 2 - 5 * x - 1)((-1 + math.sqrt(46)) / 9)
    rows = {N: (nie, mvf) for N, nie, mvf, _ in _table()}
    for N in (64, 128):
        r_nie = (true_min - rows[N][0]) / (true_min - rows[2 * N][0])
        r_mvf = (true_min - rows[N][1]) / (true_min - rows[2 * N][1])
        assert 1.9 < r_nie < 2.1 and 3.7 < r_mvf < 4.3, (N, r_nie, r_mvf)


# -- reverse mode by hand -------------------------------------------------------
def test_reverse_mode_variable_read_through_two_leaves():
    # f = x*k1 + x'*k2 + x*k3 with x and x' two leaf nodes of the same variable,
    # k1 = -2^-53, k2 = 2^-53, k3 = 1.  The sweep (descending node index) meets the
    # contributions k3 (through x), k2 (through x'), k1 (through x).  The gradient of a
    # variable is the adjoint of the variable itself -- the paper's DAG (Sec. 3.2) has one
    # input node per variable, which the two leaves merge into -- so the contributions are
    # summed in sweep order: ((0 + k3) + k2) + k1 = [1 - 2^-53, 1 + 2^-52].  Summing per
    # leaf first would give (k3 + k1) + k2 = [1, 1].
    k1, k2, k3 = -2.0 ** -53, 2.0 ** -53, 1.0
    V, C = I.VAR, I.CONST
    nodes = [(V, 0, -1), (V, 0, -1), (C, 0, -1), (C, 1, -1), (C, 2, -1),
             (I.MUL, 0, 2), (I.MUL, 1, 3), (I.ADD, 5, 6), (I.MUL, 0, 4), (I.ADD, 7, 8)]
    t = _tape(nodes, [k1, k2, k3], [9], 1)
    one = (1.0, 1.0)
    g = (0.0, 0.0)
    g = iadd(g, imul(one, (k3, k3)))               # node 8
    g = iadd(g, imul(one, (k2, k2)))               # node 6
    g = iadd(g, imul(one, (k1, k1)))               # node 5
    assert g == (1.0 - 2.0 ** -53, 1.0 + 2.0 ** -52)
    per_leaf = iadd(iadd(imul(one, (k3, k3)), imul(one, (k1, k1))), imul(one, (k2, k2)))
    assert per_leaf == (1.0, 1.0) and per_leaf != g       # the two readings differ here
    box = np.array([[[0.5, 2.0]]])
    G, bad = O.gradient_boxes(t, box, 0, O.GRAD_REV)
    assert not bad.any() and tuple(G[0, 0]) == g
    # the same tape with the two leaves merged into one gives the same bits
    merged = _tape([(V, 0, -1), (V, 0, -1), (C, 0, -1), (C, 1, -1), (C, 2, -1),
                    (I.MUL, 0, 2), (I.MUL, 0, 3), (I.ADD, 5, 6), (I.MUL, 0, 4), (I.ADD, 7, 8)],
                   [k1, k2, k3], [9], 1)
    Gm, _ = O.gradient_boxes(merged, box, 0, O.GRAD_REV)
    assert tuple(Gm[0, 0]) == g


def test_reverse_mode_division_rule():
    # f = 3 (u / v) on U = [1, 3], V = [3, 7] (0 not in V): Z = U/V; the sweep reaches the
    # quotient with the adjoint [3, 3], then t = [3,3] (1/V), u-bar = t, v-bar = -(t Z), each
    # a directed operation on the previous results.  A quotient rule t = [3,3] / V (one
    # rounding instead of two) would give the upper end RU(3/3) = 1 instead of
    # RU(3 RU(1/3)) = 1 + 2^-52.
    U, Vv = (1.0, 3.0), (3.0, 7.0)
    Z = idiv(U, Vv)
    T = imul((3.0, 3.0), irecip(Vv))
    gu = iadd((0.0, 0.0), T)
    gv = isub((0.0, 0.0), imul(T, Z))
    assert gu[1] == 1.0 + 2.0 ** -52 and idiv((3.0, 3.0), Vv)[1] == 1.0
    t = _tape([(I.VAR, 0, -1), (I.VAR, 1, -1), (I.CONST, 0, -1), (I.DIV, 0, 1), (I.MUL, 3, 2)], [3.0], [4], 2)
    G, bad = O.gradient_boxes(t, np.array([[U, Vv]]), 0, O.GRAD_REV)
    assert not bad.any()
    assert tuple(G[0, 0]) == gu and tuple(G[0, 1]) == gv
    # enclosure of the true partial derivatives 3/v and -3u/v^2 on the box
    assert gu[0] <= 3 / 7 and 1 <= gu[1]
    assert gv[0] <= -9 / 9 and -3 / 49 <= gv[1]


def test_reverse_mode_sqrt_and_square_rules():
    # f = sqrt(x) + sqr(y) on X = [4, 9], Y = [-1, 3]: sqrt(X) = [2, 3] exactly,
    # x-bar = [1,1] * 1/(2 Z) = [RD(1/6), RU(1/4)], y-bar = [1,1] * (2Y) = [-2, 6]
    t = _tape([(I.VAR, 0, -1), (I.VAR, 1, -1), (I.SQRT, 0, -1), (I.SQR, 1, -1), (I.ADD, 2, 3)], [], [4], 2)
    G, bad = O.gradient_boxes(t, np.array([[[4.0, 9.0], [-1.0, 3.0]]]), 0, O.GRAD_REV)
    assert not bad.any()
    gx = imul((1.0, 1.0), irecip((4.0, 6.0)))
    assert gx == (rd(Fr(1, 6)), 0.25)
    assert tuple(G[0, 0]) == gx
    assert tuple(G[0, 1]) == (-2.0, 6.0)
