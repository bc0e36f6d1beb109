"""GPU parity of the reverse-mode (adjoint) gradient and of the batched
persistent launch, through the C ABI, against the oracle and against the
single-box launch."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_20769_amd import inputs as I

from gpu_util import assert_parity, gpu_bound, has_transcendental, scale_of

pytestmark = pytest.mark.gpu


def _rational(t):
    nodes = t.nodes.copy()
    nodes["op"][nodes["op"] == I.EXP] = I.SQR
    nodes["op"][nodes["op"] == I.LOG] = I.SQRT
    return I.Tape(nodes, t.consts, t.roots, t.n_vars)


def _compare_rev(tape, box, splits, mode="both", ks=None):
    print(f"[case rev] n={tape.n_vars} nodes={tape.n_nodes} splits={list(splits)} mode={mode}", flush=True)
    g = gpu_bound(tape, box, splits, mode=mode, grad="rev")
    exact = not has_transcendental(tape)
    MODES = {"nie": O.MODE_NIE, "mvf": O.MODE_MVF, "both": O.MODE_BOTH}
    if ks is None:
        o = O.bound(tape, box, splits, mode=MODES[mode], grad=O.GRAD_REV, nthreads=8)
        sc = scale_of(O.bound(tape, box, splits, mode=O.MODE_NIE, per_sub=False, nthreads=8)["reduced"])
        assert_parity(g["per_sub"], o["per_sub"], exact, sc, "per_sub rev")
        assert_parity(g["reduced"], o["reduced"], exact, sc, "reduced rev")
        assert np.array_equal(g["flags"].astype(np.uint32), o["flags"])
        if exact:
            assert int(g["argmin"][0]) == o["argmin"]
    else:
        o = O.bound(tape, box, splits, mode=MODES[mode], grad=O.GRAD_REV, ks=ks, nthreads=8)
        sc = scale_of(O.bound(tape, box, splits, mode=O.MODE_NIE, ks=ks, per_sub=False, nthreads=8)["reduced"])
        assert_parity(g["per_sub"][:, :, ks], o["per_sub"], exact, sc, "per_sub rev sampled")
    assert np.array_equal(g["reduced"][:, 0], g["per_sub"][:, 0, :].min(axis=1))
    assert np.array_equal(g["reduced"][:, 1], g["per_sub"][:, 1, :].max(axis=1))
    return g


def test_reverse_cubic_and_tiny():
    t = I.cubic_tape()
    for N in (1, 7, 64, 300):
        _compare_rev(t, np.array([[-1.0, 2.0]]), [N], "mvf")
        _compare_rev(t, np.array([[-1.0, 2.0]]), [N], "both")
    w = I.tiny(1)
    _compare_rev(w.tape, w.box, w.splits, "both")
    _compare_rev(w.tape, w.box, w.splits, "mvf")


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_reverse_random_rational_tapes(seed):
    t = _rational(I.random_small_tape(seed, n=3, ops=60, n_con=2, con_ops=20, window=8))
    box = np.array([[-2.0, 2.0], [-1.5, 2.5], [-2.0, 1.0]])
    _compare_rev(t, box, [5, 7, 11], "both")
    _compare_rev(t, box, [5, 7, 11], "mvf")


def test_reverse_exp_log_and_shared_operands():
    t = I.random_small_tape(4, n=4, ops=80, n_con=3, con_ops=25, window=8)
    _compare_rev(t, np.array([[-2.0, 2.0]] * 4), [4, 5, 3, 6], "both")
    # x*x (same operand twice), x/x, leaf roots, a materialised constant pair
    nodes = [(I.VAR, 0, -1), (I.VAR, 1, -1), (I.MUL, 0, 0), (I.ADD, 2, 1), (I.MUL, 3, 3), (I.CONST, 0, -1),
             (I.CONST, 1, -1), (I.ADD, 5, 6), (I.MUL, 4, 7), (I.SUB, 8, 8), (I.ADD, 9, 4)]
    t2 = I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.array([1.5, -0.25]), np.array([10, 0, 5], dtype=np.int32), 2)
    _compare_rev(t2, np.array([[-1.0, 2.0], [0.5, 1.5]]), [9, 4], "both")


def test_reverse_mid_full_size_sampled():
    w = I.mid(1)
    rng = np.random.default_rng(0)
    ks = np.unique(np.concatenate([rng.choice(w.n_sub, 400, replace=False), [0, w.n_sub - 1]]))
    _compare_rev(w.tape, w.box, w.splits, "both", ks=ks)


def test_reverse_diff_workload_sampled():
    # 32 variables, ~3,300 instructions; the full 2^20 partition on the GPU, 96 subdomains by the oracle
    w = I.diff(1)
    rng = np.random.default_rng(1)
    ks = np.unique(np.concatenate([rng.choice(w.n_sub, 94, replace=False), [0, w.n_sub - 1]]))
    _compare_rev(w.tape, w.box, w.splits, "both", ks=ks)


def _per_node_reference(tape, boxes, splits, grad):
    out = []
    for b, s in zip(boxes, splits):
        g = gpu_bound(tape, b, s, mode="both", grad=grad, per_sub=False, flags=False)
        out.append((g["reduced"], int(g["argmin"][0])))
    return out


@pytest.mark.parametrize("grad", ["fwd", "rev"])
def test_batched_equals_per_node(grad):
    import torch
    from paper_2507_20769_amd import mvf
    bw = I.small_batch(11, 24, k_range=(3, 11))
    h = mvf.Tape(bw.tape)
    out = mvf.bound_batch(h, torch.tensor(bw.boxes, device="cuda"), torch.tensor(bw.splits, device="cuda"),
                          mode="both", grad=grad)
    torch.cuda.synchronize()
    red = out["reduced"].cpu().numpy()
    am = out["argmin"].cpu().numpy()
    assert not out["status"].cpu().numpy().any()
    ref = _per_node_reference(bw.tape, bw.boxes, bw.splits, grad)
    for i, (r, a) in enumerate(ref):
        assert np.array_equal(red[i], r), i
        assert am[i] == a, i
    # and against the oracle on a few nodes
    exact = not has_transcendental(bw.tape)
    for i in (0, 5, 17):
        o = O.bound(bw.tape, bw.boxes[i], bw.splits[i], mode=O.MODE_BOTH,
                    grad=O.GRAD_FWD if grad == "fwd" else O.GRAD_REV, per_sub=False, nthreads=8)
        assert_parity(red[i], o["reduced"], exact, scale_of(o["reduced"]), f"node {i}")


def test_batch_invalid_nodes_and_capacity():
    import torch
    from paper_2507_20769_amd import mvf
    bw = I.small_batch(12, 6, k_range=(3, 6))
    splits = bw.splits.copy()
    splits[2, 0] = 0                      # invalid split count
    h = mvf.Tape(bw.tape)
    out = mvf.bound_batch(h, torch.tensor(bw.boxes, device="cuda"), torch.tensor(splits, device="cuda"))
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert st.tolist() == [0, 0, 1, 0, 0, 0]
    assert np.isnan(out["reduced"].cpu().numpy()[2]).all()
    # a batch larger than the workspace's declared capacity runs nothing: capacity is
    # max_subdomains / 256 + nodes + 1 work items, these nodes need 4..16 items each
    big = I.small_batch(12, 6, k_range=(10, 12))
    hb = mvf.Tape(big.tape)
    call = mvf.BatchCall(hb, torch.tensor(big.boxes, device="cuda"), torch.tensor(big.splits, device="cuda"),
                         max_subdomains=16)
    call.launch()
    torch.cuda.synchronize()
    assert (call.status.cpu().numpy() == 2).all()


def test_graph_replay_matches_fresh_launches():
    import torch
    from paper_2507_20769_amd import mvf
    bw = I.small_batch(13, 40, k_range=(3, 10))
    h = mvf.Tape(bw.tape)
    total = int(np.prod(bw.splits.astype(np.int64), axis=1).sum())
    g = mvf.BatchGraph(h, max_nodes=40, max_subdomains=total, mode="both", grad="rev")
    stream = torch.cuda.Stream()
    for rep, sel in enumerate([slice(0, 40), slice(5, 17), slice(0, 40), slice(30, 31), slice(3, 39)]):
        boxes, splits = bw.boxes[sel], bw.splits[sel]
        g.launch(boxes, splits, stream=stream)
        stream.synchronize()
        red, am, st = g.result()
        torch.cuda.synchronize()
        # eager work between replays
        fresh = mvf.bound_batch(h, torch.tensor(boxes, device="cuda"), torch.tensor(splits, device="cuda"),
                                mode="both", grad="rev")
        torch.cuda.synchronize()
        assert not st.any(), rep
        assert np.array_equal(red, fresh["reduced"].cpu().numpy()), rep
        assert np.array_equal(am, fresh["argmin"].cpu().numpy()), rep
    g.close()


def test_empty_batches():
    # no nodes: the batched call is a no-op with empty results, and a graph replay with no
    # nodes between replays with nodes leaves them unaffected
    import torch
    from paper_2507_20769_amd import mvf
    bw = I.small_batch(15, 8, k_range=(3, 8))
    h = mvf.Tape(bw.tape)
    n = bw.tape.n_vars
    out = mvf.bound_batch(h, torch.empty((0, n, 2), dtype=torch.float64, device="cuda"),
                          torch.empty((0, n), dtype=torch.int32, device="cuda"))
    assert out["reduced"].shape == (0, bw.tape.n_roots, 2) and out["status"].numel() == 0
    total = int(np.prod(bw.splits.astype(np.int64), axis=1).sum())
    stream = torch.cuda.Stream()
    for grad in ("fwd", "rev"):
        g = mvf.BatchGraph(h, max_nodes=8, max_subdomains=total, mode="both", grad=grad)
        for rep, sel in enumerate([slice(0, 8), slice(0, 0), slice(2, 5), slice(4, 4), slice(0, 8)]):
            print(f"[case] grad={grad} replay={rep} nodes={sel.stop - sel.start}", flush=True)
            boxes, splits = bw.boxes[sel], bw.splits[sel]
            g.launch(boxes, splits, stream=stream)
            stream.synchronize()
            red, am, st = g.result()
            assert red.shape[0] == sel.stop - sel.start
            if red.shape[0]:
                fresh = mvf.bound_batch(h, torch.tensor(boxes, device="cuda"), torch.tensor(splits, device="cuda"),
                                        mode="both", grad=grad)
                torch.cuda.synchronize()
                assert not st.any(), rep
                assert np.array_equal(red, fresh["reduced"].cpu().numpy()), rep
                assert np.array_equal(am, fresh["argmin"].cpu().numpy()), rep
        g.close()
    h.close()


def test_autotuner_returns_a_feasible_config():
    import torch
    from paper_2507_20769_amd import mvf
    bw = I.small_batch(14, 16, k_range=(6, 10))
    h = mvf.Tape(bw.tape)
    boxes = torch.tensor(bw.boxes, device="cuda")
    splits = torch.tensor(bw.splits, device="cuda")
    tu = mvf.autotune(h, boxes, splits, mode="both", grad="rev")
    assert tu.grad == 1 and tu.grid_blocks > 0 and tu.best_ms > 0 and tu.engine == 1   # no specialised kernel
    out = mvf.bound_batch(h, boxes, splits, mode="both", grad="rev", tuning=tu)
    ref = mvf.bound_batch(h, boxes, splits, mode="both", grad="rev")
    torch.cuda.synchronize()
    assert np.array_equal(out["reduced"].cpu().numpy(), ref["reduced"].cpu().numpy())
