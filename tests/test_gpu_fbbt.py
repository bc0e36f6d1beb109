"""GPU bound tightening (one lane per box) against the oracle's FBBT: the
tightened boxes and the infeasibility status, bitwise for + - * / sqr sqrt
tapes and within 1e-12 of the box scale where library functions appear, for
hand cases, random constrained problems with an objective cut, one to three
rounds, batches with a ragged last wave, and tapes whose node values fill
many lanes', one lane's, or more than the LDS."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_20769_amd import inputs as I

from gpu_util import assert_parity, has_transcendental

pytestmark = pytest.mark.gpu

V, C = I.VAR, I.CONST


def _tape(nodes, consts, roots, n):
    return I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.array(consts, dtype=np.float64),
                  np.array(roots, dtype=np.int32), n)


def _rational(t):
    nodes = t.nodes.copy()
    nodes["op"][nodes["op"] == I.EXP] = I.SQR
    nodes["op"][nodes["op"] == I.LOG] = I.SQRT
    return I.Tape(nodes, t.consts, t.roots, t.n_vars)


def _compare(tape, kinds, boxes, ub=np.inf, rounds=1, what=""):
    import torch
    from paper_2507_20769_amd import mvf
    print(f"[case fbbt] {what} N={len(boxes)} rounds={rounds} ub={ub}", flush=True)
    h = mvf.Tape(tape)
    h.set_root_kinds(kinds)
    out, st = mvf.fbbt(h, torch.tensor(boxes, device="cuda"), ub=ub, rounds=rounds)
    torch.cuda.synchronize()
    out, st = out.cpu().numpy(), st.cpu().numpy()
    oo, ost = O.fbbt(tape, boxes, kinds=kinds, ub=ub, rounds=rounds)
    assert np.array_equal(st, ost), what
    ok = st == 0
    scale = np.maximum(np.abs(boxes).max(), 1.0)
    assert_parity(out[ok], oo[ok], not has_transcendental(tape), scale, what)
    h.close()
    return out, st


def test_hand_cases():
    cases = [
        ("linear", _tape([(V, 0, -1), (V, 1, -1), (C, 0, -1), (I.ADD, 0, 1), (I.SUB, 3, 2)], [1.0], [0, 4], 2),
         [0, 1], [[[0.8, 1.0], [0.0, 1.0]], [[0.0, 2.0], [3.0, 4.0]]]),
        ("square", _tape([(V, 0, -1), (I.SQR, 0, -1), (C, 0, -1), (I.SUB, 1, 2)], [0.25], [0, 3], 1),
         [0, 1], [[[-2.0, 2.0]], [[0.1, 2.0]], [[-3.0, -0.2]], [[1.0, 3.0]]]),
        ("product equality", _tape([(V, 0, -1), (V, 1, -1), (I.MUL, 0, 1), (C, 0, -1), (I.SUB, 2, 3)], [6.0],
                                   [0, 4], 2), [0, 2], [[[2.0, 3.0], [0.0, 10.0]], [[-1.0, 3.0], [0.0, 10.0]]]),
        ("quotient", _tape([(V, 0, -1), (C, 0, -1), (I.DIV, 1, 0), (C, 1, -1), (I.SUB, 2, 3)], [1.0, 0.5], [0, 4], 1),
         [0, 1], [[[1.0, 10.0]], [[-2.0, 10.0]]]),
        ("x*x and x+x", _tape([(V, 0, -1), (I.MUL, 0, 0), (I.ADD, 0, 0), (I.ADD, 1, 2), (C, 0, -1), (I.SUB, 3, 4)],
                              [2.0], [0, 5], 1), [0, 1], [[[-3.0, 3.0]], [[0.5, 4.0]]]),
        ("sqrt/exp/log/tanh", _tape([(V, 0, -1), (V, 1, -1), (I.SQRT, 0, -1), (I.EXP, 1, -1), (I.ADD, 2, 3),
                                     (C, 0, -1), (I.SUB, 4, 5), (I.LOG, 0, -1), (I.TANH, 1, -1), (I.ADD, 7, 8)],
                                    [3.0], [9, 6], 2), [0, 1], [[[0.0, 16.0], [-3.0, 3.0]], [[1.0, 2.0], [0.0, 5.0]]]),
        ("infeasible", _tape([(V, 0, -1), (I.SQR, 0, -1), (C, 0, -1), (I.ADD, 1, 2)], [1.0], [0, 3], 1),
         [0, 1], [[[-5.0, 7.0]]]),
        ("sin equality", _tape([(V, 0, -1), (I.SIN, 0, -1), (C, 0, -1), (I.SUB, 1, 2)], [2.0], [0, 3], 1),
         [0, 2], [[[-5.0, 7.0]]]),
    ]
    for name, t, kinds, boxes in cases:
        for rounds in (1, 2):
            _compare(t, kinds, np.array(boxes), rounds=rounds, what=name)
    t = _tape([(V, 0, -1)], [], [0], 1)
    out, st = _compare(t, [0], np.array([[[0.0, 10.0]], [[4.0, 10.0]]]), ub=3.0, what="objective cut")
    assert st.tolist() == [0, 1] and out[0].tolist() == [[0.0, 3.0]]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_problems_ragged_batches(seed):
    rng = np.random.default_rng(seed)
    t = I.random_small_tape(200 + seed, n=3, ops=50, n_con=2, con_ops=16, window=8)
    for tape in (_rational(t), t):
        N = 70                                         # a full wave and a ragged one
        lo = rng.uniform(-2.5, 0.5, (N, 3))
        boxes = np.stack([lo, lo + rng.uniform(0.2, 2.5, (N, 3))], axis=2)
        f = I.eval_points_np(tape, boxes.mean(axis=2))[:, 0]
        for rounds in (1, 3):
            _compare(tape, [0, 1, 1], boxes, rounds=rounds, what=f"seed {seed}")
            _compare(tape, [0, 1, 2], boxes, ub=float(np.median(f)), rounds=rounds, what=f"seed {seed} eq+ub")


@pytest.mark.parametrize("ops,con_ops", [(1200, 300), (2600, 700)])
def test_large_tapes(ops, con_ops):
    # 2,506 nodes: a lane's values and marks (78 KB) in LDS, one lane per workgroup; 5,542
    # nodes (173 KB): more than the LDS holds, the values in the workspace
    rng = np.random.default_rng(ops)
    t = _rational(I.random_small_tape(301, n=3, ops=ops, n_con=2, con_ops=con_ops, window=8))
    N = 70
    lo = rng.uniform(-2.5, 0.5, (N, 3))
    boxes = np.stack([lo, lo + rng.uniform(0.2, 2.5, (N, 3))], axis=2)
    f = I.eval_points_np(t, boxes.mean(axis=2))[:, 0]
    _compare(t, [0, 1, 1], boxes, ub=float(np.median(f)), rounds=2, what=f"{t.n_nodes} nodes")


def test_bnb_with_tightening_matches_the_reference():
    from oracle import bnb
    from paper_2507_20769_amd import mvf
    t = _rational(I.random_small_tape(57, n=3, ops=50, n_con=2, con_ops=16, window=8))
    kinds = [0, 1, 1]
    for form, K, grad in (("plain", 1, "fwd"), ("batched", 8, "rev")):
        print(f"[case bnb fbbt] {form}", flush=True)
        h = mvf.Tape(t)
        h.set_root_kinds(kinds)
        kw = dict(max_nodes=120, gap=1e-3, budget=256)
        g = mvf.bnb_solve(h, [[-2.0, 2.0]] * 3, nodes_per_launch=K, grad=grad, fbbt_rounds=2, **kw)
        o = bnb.solve(t, [[-2.0, 2.0]] * 3, kinds=kinds, batch=K, grad=O.GRAD_FWD if grad == "fwd" else O.GRAD_REV,
                      fbbt_rounds=2, **kw)
        for key in ("lower", "upper", "nodes", "subdomains", "open", "status"):
            assert g[key] == o[key], (form, key, g[key], o[key])
        h.close()
