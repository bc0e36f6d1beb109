"""Pins of the reference branch-and-bound (oracle/bnb.py): certified bounds
that bracket minima known in closed form or by dense sampling, infeasibility,
and the node limit."""
import math

import numpy as np

from oracle import bnb
from oracle import oracle as O
from paper_2507_20769_amd import inputs as I


def test_cubic_minimum_closed_form():
    # f = 3x^3 + x^2 - 5x - 1 on [-1, 2]: f' = 9x^2 + 2x - 5 = 0 at x* = (-2 + sqrt(184)) / 18
    xs = (-2.0 + math.sqrt(184.0)) / 18.0
    fs = 3 * xs ** 3 + xs ** 2 - 5 * xs - 1
    r = bnb.solve(I.cubic_tape(), [[-1.0, 2.0]], max_nodes=400, gap=1e-6, budget=64)
    assert r["status"] == 0
    assert r["lower"] <= fs <= r["upper"]
    assert r["upper"] - r["lower"] <= 1e-6


def test_constrained_minimum_on_the_boundary():
    # min -x s.t. x - 0.5 <= 0 on [0, 1]: the minimum -0.5 sits on the constraint
    nodes = [(I.VAR, 0, -1), (I.CONST, 0, -1), (I.CONST, 1, -1), (I.MUL, 0, 1), (I.SUB, 0, 2)]
    t = I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.array([-1.0, 0.5]), np.array([3, 4], dtype=np.int32), 1)
    r = bnb.solve(t, [[0.0, 1.0]], kinds=[O.FREE, O.INEQ], max_nodes=2000, gap=1e-4, budget=16)
    assert r["lower"] <= -0.5 <= r["upper"]
    assert r["status"] == 0 and r["upper"] - r["lower"] <= 1e-4


def test_peaks_against_dense_sampling():
    t = I.peaks_tape()
    box = np.array([[-3.0, 3.0], [-3.0, 3.0]])
    r = bnb.solve(t, box, max_nodes=3000, gap=1e-4, budget=1024)
    g = np.linspace(-3.0, 3.0, 1201)
    X, Y = np.meshgrid(g, g)
    v = I.eval_points_np(t, np.stack([X.ravel(), Y.ravel()], axis=1))[:, 0].min()
    assert r["status"] == 0
    assert r["lower"] <= v + 1e-12
    assert r["upper"] - r["lower"] <= 1e-4
    assert r["upper"] <= v + 1e-4        # the grid minimum is within the grid spacing of the true one


def test_infeasible_problem():
    # min x s.t. x^2 + 1 <= 0
    nodes = [(I.VAR, 0, -1), (I.SQR, 0, -1), (I.CONST, 0, -1), (I.ADD, 1, 2)]
    t = I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.array([1.0]), np.array([0, 3], dtype=np.int32), 1)
    r = bnb.solve(t, [[-2.0, 3.0]], kinds=[O.FREE, O.INEQ], max_nodes=50, budget=8)
    assert r["status"] == 2 and r["nodes"] == 1
    assert r["lower"] == np.inf and r["upper"] == np.inf


def test_node_limit_and_batches():
    t = I.random_small_tape(41, n=3, ops=40, n_con=1, con_ops=12, window=6)
    box = [[-2.0, 2.0]] * 3
    r = bnb.solve(t, box, kinds=[O.FREE, O.INEQ], max_nodes=20, gap=0.0, budget=64)
    assert r["status"] == 1 and r["nodes"] == 20
    rb = bnb.solve(t, box, kinds=[O.FREE, O.INEQ], max_nodes=20, gap=0.0, budget=64, batch=4)
    assert rb["nodes"] == 20 and rb["lower"] <= rb["upper"]


def test_bound_tightening_keeps_the_bracket_and_saves_nodes():
    # min -x s.t. x - 0.5 <= 0 on [0, 1]: tightening cuts the box to [0, 0.5] at the root
    nodes = [(I.VAR, 0, -1), (I.CONST, 0, -1), (I.CONST, 1, -1), (I.MUL, 0, 1), (I.SUB, 0, 2)]
    t = I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.array([-1.0, 0.5]), np.array([3, 4], dtype=np.int32), 1)
    plain = bnb.solve(t, [[0.0, 1.0]], kinds=[O.FREE, O.INEQ], max_nodes=2000, gap=1e-4, budget=16)
    tight = bnb.solve(t, [[0.0, 1.0]], kinds=[O.FREE, O.INEQ], max_nodes=2000, gap=1e-4, budget=16, fbbt_rounds=2)
    for r in (plain, tight):
        assert r["status"] == 0 and r["lower"] <= -0.5 <= r["upper"] and r["upper"] - r["lower"] <= 1e-4
    assert tight["nodes"] <= plain["nodes"]
    # a random constrained problem: the certified bracket holds with tightening too
    t = I.random_small_tape(41, n=3, ops=40, n_con=1, con_ops=12, window=6)
    g = np.linspace(-2.0, 2.0, 41)
    pts = np.stack(np.meshgrid(g, g, g), axis=-1).reshape(-1, 3)
    v = I.eval_points_np(t, pts)
    best = v[v[:, 1] <= 0, 0].min()
    r = bnb.solve(t, [[-2.0, 2.0]] * 3, kinds=[O.FREE, O.INEQ], max_nodes=60, gap=0.0, budget=64, fbbt_rounds=2)
    assert r["lower"] <= best
