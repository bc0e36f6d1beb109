"""Pins of the oracle's forward-backward bound tightening (FBBT): hand-worked
narrowings of each inverse rule, infeasibility proofs, the objective cut,
and soundness on random problems (every sampled feasible point of a box
stays inside its tightened box; a box is declared infeasible only when no
sample is feasible)."""
import math

import numpy as np

from oracle import oracle as O
from paper_2507_20769_amd import inputs as I

V, C = I.VAR, I.CONST


def _tape(nodes, consts, roots, n):
    return I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.array(consts, dtype=np.float64),
                  np.array(roots, dtype=np.int32), n)


def _f(tape, box, kinds=None, ub=np.inf, rounds=1):
    out, st = O.fbbt(tape, np.array(box, dtype=np.float64), kinds=kinds, ub=ub, rounds=rounds)
    return out[0], int(st[0])


def test_linear_inequality_narrows_the_other_variable():
    # objective x, constraint x + y - 1 <= 0 on x in [0.8, 1], y in [0, 1]: y <= 1 - x <= 0.2
    t = _tape([(V, 0, -1), (V, 1, -1), (C, 0, -1), (I.ADD, 0, 1), (I.SUB, 3, 2)], [1.0], [0, 4], 2)
    out, st = _f(t, [[0.8, 1.0], [0.0, 1.0]], kinds=[0, 1])
    assert st == 0
    assert out[0].tolist() == [0.8, 1.0]
    assert out[1][0] == 0.0 and out[1][1] == 1.0 - 0.8                   # RU(1 - 0.8) = RN here
    assert out[1][1] >= 0.2 - 1e-16


def test_square_sqrt_exp_log_tanh_division_inverses():
    # x^2 - 0.25 <= 0 on [-2, 2] -> [-0.5, 0.5]
    t = _tape([(V, 0, -1), (I.SQR, 0, -1), (C, 0, -1), (I.SUB, 1, 2)], [0.25], [0, 3], 1)
    assert _f(t, [[-2.0, 2.0]], [0, 1])[0].tolist() == [[-0.5, 0.5]]
    assert _f(t, [[0.1, 2.0]], [0, 1])[0].tolist() == [[0.1, 0.5]]       # the positive branch only
    # sqrt(x) - 2 <= 0 on [0, 10] -> [0, 4]
    t = _tape([(V, 0, -1), (I.SQRT, 0, -1), (C, 0, -1), (I.SUB, 1, 2)], [2.0], [0, 3], 1)
    assert _f(t, [[0.0, 10.0]], [0, 1])[0].tolist() == [[0.0, 4.0]]
    # exp(x) - 1 <= 0 on [-3, 3] -> x <= log(1) widened by two ulps
    t = _tape([(V, 0, -1), (I.EXP, 0, -1), (C, 0, -1), (I.SUB, 1, 2)], [1.0], [0, 3], 1)
    out = _f(t, [[-3.0, 3.0]], [0, 1])[0]
    assert out[0][0] == -3.0 and 0.0 < out[0][1] < 1e-320
    # log(x) <= 0 on [0.5, 9] -> x <= e^0 = 1 widened
    t = _tape([(V, 0, -1), (I.LOG, 0, -1)], [], [0, 1], 1)
    out = _f(t, [[0.5, 9.0]], [0, 1])[0]
    assert out[0][0] == 0.5 and 1.0 < out[0][1] < 1.0 + 1e-15
    # tanh(x) <= 0 on [-1, 4] -> x <= 0 (atanh(0) widened)
    t = _tape([(V, 0, -1), (I.TANH, 0, -1)], [], [0, 1], 1)
    out = _f(t, [[-1.0, 4.0]], [0, 1])[0]
    assert out[0][0] == -1.0 and 0.0 < out[0][1] < 1e-320
    # 1/x - 0.5 <= 0 on [1, 10] -> x >= 2
    t = _tape([(V, 0, -1), (C, 0, -1), (I.DIV, 1, 0), (C, 1, -1), (I.SUB, 2, 3)], [1.0, 0.5], [0, 4], 1)
    out = _f(t, [[1.0, 10.0]], [0, 1])[0]
    assert out[0].tolist() == [2.0, 10.0]
    # x * y = 6 (equality) with x in [2, 3], y in [0, 10] -> y in [2, 3]
    t = _tape([(V, 0, -1), (V, 1, -1), (I.MUL, 0, 1), (C, 0, -1), (I.SUB, 2, 3)], [6.0], [0, 4], 2)
    out = _f(t, [[2.0, 3.0], [0.0, 10.0]], [0, 2])[0]
    assert out[1].tolist() == [2.0, 3.0]


def test_infeasibility_and_the_objective_cut():
    # x^2 + 1 <= 0 is infeasible everywhere
    t = _tape([(V, 0, -1), (I.SQR, 0, -1), (C, 0, -1), (I.ADD, 1, 2)], [1.0], [0, 3], 1)
    assert _f(t, [[-5.0, 7.0]], [0, 1])[1] == 1
    # sin(x) - 2 >= ... : sin(x) = 2 (equality) is infeasible
    t = _tape([(V, 0, -1), (I.SIN, 0, -1), (C, 0, -1), (I.SUB, 1, 2)], [2.0], [0, 3], 1)
    assert _f(t, [[-5.0, 7.0]], [0, 2])[1] == 1
    # objective x with an upper bound 3 on [0, 10] -> [0, 3]
    t = _tape([(V, 0, -1)], [], [0], 1)
    assert _f(t, [[0.0, 10.0]], None, ub=3.0)[0].tolist() == [[0.0, 3.0]]
    assert _f(t, [[4.0, 10.0]], None, ub=3.0)[1] == 1


def test_soundness_on_random_problems():
    rng = np.random.default_rng(31)
    for seed in range(12):
        t = I.random_small_tape(100 + seed, n=3, ops=40, n_con=2, con_ops=14, window=8)
        kinds = [0, 1, 1]
        lo = rng.uniform(-2.5, 0.5, 3)
        box = np.stack([lo, lo + rng.uniform(0.3, 2.5, 3)], axis=1)
        pts = box[:, 0] + (box[:, 1] - box[:, 0]) * rng.random((4000, 3))
        v = I.eval_points_np(t, pts)
        feas = np.all(v[:, 1:] <= 0, axis=1)
        prev = box
        for rounds in (1, 2, 3):
            out, st = _f(t, box, kinds, rounds=rounds)
            if st:
                assert not feas.any(), seed
                break
            inside = np.all((pts >= out[:, 0]) & (pts <= out[:, 1]), axis=1)
            assert np.all(inside[feas]), (seed, rounds)
            assert np.all(out[:, 0] >= prev[:, 0]) and np.all(out[:, 1] <= prev[:, 1])   # never widens
            prev = out


def test_objective_cut_is_sound():
    t = I.peaks_tape()
    box = np.array([[-3.0, 3.0], [-3.0, 3.0]])
    g = np.linspace(-3, 3, 301)
    X, Y = np.meshgrid(g, g)
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    f = I.eval_points_np(t, pts)[:, 0]
    ub = float(np.quantile(f, 0.05))
    out, st = _f(t, box, None, ub=ub, rounds=3)
    assert st == 0
    keep = f <= ub
    inside = np.all((pts >= out[:, 0]) & (pts <= out[:, 1]), axis=1)
    assert np.all(inside[keep])
    assert math.isfinite(out[0, 0])
