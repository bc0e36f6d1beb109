"""GPU parity of the two B&B bounds (feasibility-filtered objective bound,
upper bound from feasible centres) and of the branch-and-bound driver against
the reference branch-and-bound over the oracle."""
import numpy as np
import pytest

from oracle import bnb
from oracle import oracle as O
from paper_2507_20769_amd import inputs as I

from gpu_util import assert_parity, has_transcendental

pytestmark = pytest.mark.gpu

MODES = {"nie": O.MODE_NIE, "mvf": O.MODE_MVF, "both": O.MODE_BOTH}


def _rational(t):
    nodes = t.nodes.copy()
    nodes["op"][nodes["op"] == I.EXP] = I.SQR
    nodes["op"][nodes["op"] == I.LOG] = I.SQRT
    return I.Tape(nodes, t.consts, t.roots, t.n_vars)


def _neg_x_with_constraint():
    nodes = [(I.VAR, 0, -1), (I.CONST, 0, -1), (I.CONST, 1, -1), (I.MUL, 0, 1), (I.SUB, 0, 2)]
    return I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.array([-1.0, 0.5]), np.array([3, 4], dtype=np.int32), 1)


def _extra_gpu(h, box, splits, mode, grad):
    import torch
    from paper_2507_20769_amd import mvf
    out = mvf.bound(h, torch.tensor(box, device="cuda"), splits, mode=mode, grad=grad)
    torch.cuda.synchronize()
    return out["extra"].cpu().numpy(), out["reduced"].cpu().numpy()


@pytest.mark.parametrize("grad", ["fwd", "rev"])
def test_bound_extras_match_oracle(grad):
    from paper_2507_20769_amd import mvf
    cases = [
        ("hand example, inequality", _neg_x_with_constraint(), np.array([[0.0, 1.0]]), [4], [0, 1]),
        ("hand example, equality", _neg_x_with_constraint(), np.array([[0.0, 1.0]]), [4], [0, 2]),
        ("mid, three inequalities", I.mid(1).tape, I.mid(1).box, [4] * 6, [0, 1, 1, 1]),
        ("mid, mixed kinds", I.mid(1).tape, I.mid(1).box, [4] * 6, [0, 1, 2, 0]),
        ("random exp/log", I.random_small_tape(51, n=3, ops=60, n_con=2, con_ops=20, window=8),
         np.array([[-2.0, 2.0]] * 3), [7, 5, 6], [0, 1, 1]),
        ("random rational", _rational(I.random_small_tape(52, n=3, ops=60, n_con=2, con_ops=20, window=8)),
         np.array([[-2.0, 2.0]] * 3), [7, 5, 6], [0, 1, 1]),
    ]
    for name, tape, box, splits, kinds in cases:
        h = mvf.Tape(tape)
        h.set_root_kinds(kinds)
        for mode in ("nie", "mvf", "both"):
            print(f"[case extras] {name} mode={mode} grad={grad}", flush=True)
            ex, red = _extra_gpu(h, box, splits, mode, grad)
            o = O.bound(tape, box, splits, mode=MODES[mode], grad=O.GRAD_FWD if grad == "fwd" else O.GRAD_REV,
                        per_sub=False, nthreads=8, kinds=kinds)
            scale = np.abs(o["reduced"][np.isfinite(o["reduced"])]).max(initial=1.0)
            exact = not has_transcendental(tape)
            assert_parity(ex, o["extra"], exact, scale, f"{name} {mode}")
            assert ex[0] >= red[0, 0]
        h.close()


def test_batched_and_graph_extras_equal_per_node():
    import torch
    from paper_2507_20769_amd import mvf
    bw = I.small_batch(53, 20, k_range=(3, 10))
    h = mvf.Tape(bw.tape)
    kinds = [0] + [1] * (bw.tape.n_roots - 1)
    h.set_root_kinds(kinds)
    for grad in ("fwd", "rev"):
        out = mvf.bound_batch(h, torch.tensor(bw.boxes, device="cuda"), torch.tensor(bw.splits, device="cuda"),
                              mode="both", grad=grad)
        torch.cuda.synchronize()
        ex = out["extra"].cpu().numpy()
        for i in range(len(bw.boxes)):
            e1, _ = _extra_gpu(h, bw.boxes[i], bw.splits[i], "both", grad)
            assert np.array_equal(ex[i], e1), (grad, i)
    total = int(np.prod(bw.splits.astype(np.int64), axis=1).sum())
    g = mvf.BatchGraph(h, len(bw.boxes), total, mode="both", grad="rev")
    s = torch.cuda.Stream()
    g.launch(bw.boxes, bw.splits, stream=s)
    s.synchronize()
    ref = mvf.bound_batch(h, torch.tensor(bw.boxes, device="cuda"), torch.tensor(bw.splits, device="cuda"),
                          mode="both", grad="rev")
    torch.cuda.synchronize()
    assert np.array_equal(g.extra(), ref["extra"].cpu().numpy())
    g.close()
    h.close()


def _bnb_cases():
    yield "cubic", I.cubic_tape(), [[-1.0, 2.0]], None, dict(max_nodes=300, gap=1e-6, budget=64)
    yield "constrained -x", _neg_x_with_constraint(), [[0.0, 1.0]], [0, 1], dict(max_nodes=500, gap=1e-4, budget=16)
    yield ("random rational, two inequalities",
           _rational(I.random_small_tape(54, n=3, ops=50, n_con=2, con_ops=16, window=8)),
           [[-2.0, 2.0]] * 3, [0, 1, 1], dict(max_nodes=150, gap=1e-3, budget=256))


@pytest.mark.parametrize("form", ["plain", "batched"])
def test_bnb_matches_reference(form):
    from paper_2507_20769_amd import mvf
    for name, tape, box, kinds, kw in _bnb_cases():
        print(f"[case bnb] {name} {form}", flush=True)
        h = mvf.Tape(tape)
        h.set_root_kinds(kinds)
        if form == "plain":
            g = mvf.bnb_solve(h, box, grad="fwd", nodes_per_launch=1, **kw)
            o = bnb.solve(tape, box, kinds=kinds, grad=O.GRAD_FWD, batch=1, **kw)
        else:
            g = mvf.bnb_solve(h, box, grad="rev", nodes_per_launch=8, **kw)
            o = bnb.solve(tape, box, kinds=kinds, grad=O.GRAD_REV, batch=8, **kw)
        for key in ("lower", "upper", "nodes", "subdomains", "open", "status"):
            assert g[key] == o[key], (name, form, key, g[key], o[key])
        h.close()


def test_bnb_peaks_brackets_the_minimum():
    from paper_2507_20769_amd import mvf
    t = I.peaks_tape()
    box = [[-3.0, 3.0], [-3.0, 3.0]]
    h = mvf.Tape(t)
    g = np.linspace(-3.0, 3.0, 1201)
    X, Y = np.meshgrid(g, g)
    vmin = I.eval_points_np(t, np.stack([X.ravel(), Y.ravel()], axis=1))[:, 0].min()
    for form, k, grad in (("plain", 1, "fwd"), ("batched", 16, "rev")):
        r = mvf.bnb_solve(h, box, max_nodes=4000, gap=1e-4, budget=4096, nodes_per_launch=k, grad=grad)
        assert r["status"] == 0, (form, r)
        assert r["lower"] <= vmin + 1e-12 and r["upper"] - r["lower"] <= 1e-4, (form, r)
    h.close()
