"""Pins of the oracle's feasibility-filtered objective bound and of the upper
bound from rigorously feasible subdomain centres (Sec. 3.1: feasibility check
of the constraint bounds; the B&B upper bound taken at points)."""
import numpy as np

from oracle import oracle as O
from paper_2507_20769_amd import inputs as I


def _neg_x_with_constraint():
    # f = -x (objective), c = x - 0.5 (constraint): node list with a constant 0.5
    nodes = [(I.VAR, 0, -1), (I.CONST, 0, -1), (I.CONST, 1, -1), (I.MUL, 0, 1), (I.SUB, 0, 2)]
    return I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.array([-1.0, 0.5]), np.array([3, 4], dtype=np.int32), 1)


def test_hand_worked_inequality_and_equality():
    # [0, 1] in 4 pieces: f = -x has bounds [-.25,0], [-.5,-.25], [-.75,-.5], [-1,-.75];
    # c = x - .5 has [-.5,-.25], [-.25,0], [0,.25], [.25,.5]; centres .125 .375 .625 .875
    t = _neg_x_with_constraint()
    box = np.array([[0.0, 1.0]])
    for mode in (O.MODE_NIE, O.MODE_MVF, O.MODE_BOTH):
        o = O.bound(t, box, [4], mode=mode, kinds=[O.FREE, O.INEQ])
        assert o["reduced"][0, 0] == -1.0
        assert o["extra"][0] == -0.75                    # piece 4 is proven infeasible (c >= .25 > 0)
        assert o["extra"][1] == (np.inf if mode == O.MODE_NIE else -0.375)   # centres .125, .375 feasible
        e = O.bound(t, box, [4], mode=mode, kinds=[O.FREE, O.EQ])
        assert e["extra"][0] == -0.75                    # pieces 1 and 4 exclude c = 0
        assert e["extra"][1] == np.inf                   # no point can be shown to satisfy c = 0
        f = O.bound(t, box, [4], mode=mode)
        assert f["extra"][0] == -1.0                     # unconstrained: the plain lower bound
        assert f["extra"][1] == (np.inf if mode == O.MODE_NIE else -0.875)


def test_filtered_bound_is_valid_and_tighter_on_random_tapes():
    for seed in (31, 32):
        t = I.random_small_tape(seed, n=3, ops=50, n_con=2, con_ops=20, window=8)
        box = np.array([[-2.0, 2.0]] * 3)
        kinds = [O.FREE, O.INEQ, O.INEQ]
        o = O.bound(t, box, [6, 5, 4], mode=O.MODE_BOTH, kinds=kinds, nthreads=4)
        lb, flb, ub = o["reduced"][0, 0], o["extra"][0], o["extra"][1]
        assert flb >= lb
        # sampled feasible points: every feasible value is >= the filtered bound
        x = I.random_points(seed, box, 20000)
        v = I.eval_points_np(t, x)
        feas = (v[:, 1] <= 0) & (v[:, 2] <= 0)
        assert feas.any()
        assert np.all(v[feas, 0] >= flb - 1e-9 * max(1.0, abs(flb)))
        # the upper bound is attained at a centre whose constraint enclosures are <= 0
        assert ub >= flb
        S = 6 * 5 * 4
        cs = np.array([O.subdomain(box, np.array([6, 5, 4]), k)[1] for k in range(S)])
        fc = O.eval_points(t, cs)
        ok = (fc[:, 1, 1] <= 0) & (fc[:, 2, 1] <= 0)
        assert ub == (fc[ok, 0, 1].min() if ok.any() else np.inf)


def test_filtered_bound_reduces_over_the_per_subdomain_output():
    t = I.random_small_tape(33, n=2, ops=40, n_con=1, con_ops=15, window=6)
    box = np.array([[-1.5, 2.0], [-2.0, 1.0]])
    o = O.bound(t, box, [9, 7], mode=O.MODE_BOTH, kinds=[O.FREE, O.INEQ])
    ps = o["per_sub"]
    infeasible = ps[1, 0, :] > 0
    want = ps[0, 0, ~infeasible].min() if (~infeasible).any() else np.inf
    assert o["extra"][0] == want
