"""GPU parity of the checkpointed reverse-mode adjoint (specialised kernels).

The adjoint's value pass stores, at each segment boundary, the values the
next segment reads; every segment is then recomputed from its checkpoint
just before its reverse sweep.  Recomputation repeats the same operations on
the same operands, so the bounds must equal, bit for bit, those of the
single-pass adjoint (the interpreter's record tape) and the oracle's reverse
mode on rational tapes, at every segment budget; with exp/log the oracle is
met within 1e-12 of the root's scale and the interpreter bit for bit (same
device functions)."""
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


def _spec(tape, kinds=None, **opt):
    from paper_2507_20769_amd import mvf
    h = mvf.Tape(tape)
    if kinds is not None:
        h.set_root_kinds(kinds)
    info = h.specialize(grad="rev", cache=False, **opt)
    print(f"[spec] n={tape.n_vars} budget={info['ckpt_budget']} checkpoints={info['ckpt_intervals']} "
          f"compile={info['seconds']:.2f}s", flush=True)
    return h, info


@pytest.mark.parametrize("seed,budget", [(1, 4), (2, 8), (3, 16), (4, -1)])
def test_checkpointed_adjoint_bitwise(seed, budget):
    # 150-op objective and two 40-op constraints (window 8): several segments per root at
    # small budgets; 5*7*11 = 385 subdomains (a full workgroup and a ragged tail)
    rng = np.random.default_rng(seed)
    t = _rational(I.random_small_tape(seed, n=3, ops=150, n_con=2, con_ops=40, window=8))
    kinds = [0, 1, 2]
    h, info = _spec(t, kinds, ckpt_budget=budget)
    if budget > 0:
        assert info["ckpt_intervals"] > 0, "small budgets must cut the objective into checkpointed segments"
    else:
        assert info["ckpt_intervals"] == 0
    box = np.array([[-2.0, 2.0], [-1.5, 2.5], [-2.0, 1.0]]) + rng.uniform(-0.3, 0.3, (3, 1))
    splits = [5, 7, 11]
    for mode in ("mvf", "both"):
        print(f"[case] seed={seed} budget={budget} mode={mode}", flush=True)
        g = gpu_bound(t, box, splits, mode=mode, grad="rev", handle=h, engine="spec")
        gi = gpu_bound(t, box, splits, mode=mode, grad="rev", handle=h, engine="interp")
        o = O.bound(t, box, splits, mode=O.MODE_MVF if mode == "mvf" else O.MODE_BOTH, grad=O.GRAD_REV,
                    nthreads=8, kinds=kinds)
        for key in ("per_sub", "reduced", "extra"):
            assert_parity(g[key], o[key], True, None, f"{key} vs oracle")
            assert_parity(g[key], gi[key], True, None, f"{key} vs interpreter")
        assert int(g["argmin"][0]) == o["argmin"]
        assert np.array_equal(g["flags"].astype(np.uint32), o["flags"])
    h.close()


def test_checkpointed_adjoint_exp_log_and_batched():
    from paper_2507_20769_amd import mvf
    import torch
    t = I.random_small_tape(7, n=4, ops=120, n_con=2, con_ops=30, window=8)
    assert has_transcendental(t)
    h, info = _spec(t, ckpt_budget=6)
    assert info["ckpt_intervals"] > 0
    box = np.array([[-2.0, 2.0], [-1.0, 2.5], [-2.5, 1.5], [-2.0, 2.0]])
    splits = [4, 5, 3, 6]
    g = gpu_bound(t, box, splits, mode="both", grad="rev", handle=h, engine="spec")
    gi = gpu_bound(t, box, splits, mode="both", grad="rev", handle=h, engine="interp")
    o = O.bound(t, box, splits, mode=O.MODE_BOTH, grad=O.GRAD_REV, nthreads=8)
    sc = scale_of(O.bound(t, box, splits, mode=O.MODE_NIE, per_sub=False, nthreads=8)["reduced"])
    assert_parity(g["per_sub"], o["per_sub"], False, sc, "per_sub vs oracle")
    assert_parity(g["per_sub"], gi["per_sub"], True, None, "per_sub vs interpreter")
    # the batched persistent kernel on a few nodes equals the single-box calls bit for bit
    rng = np.random.default_rng(3)
    n_nodes = 6
    boxes = np.stack([box + rng.uniform(-0.2, 0.2, box.shape) for _ in range(n_nodes)])
    boxes[:, :, 1] = np.maximum(boxes[:, :, 1], boxes[:, :, 0] + 0.5)
    spl = np.array([[2, 3, 4, 5], [1, 1, 1, 1], [8, 2, 2, 2], [3, 3, 3, 3], [16, 1, 4, 1], [5, 5, 2, 3]],
                   dtype=np.int32)
    res = mvf.bound_batch(h, torch.tensor(boxes, device="cuda"), torch.tensor(spl, device="cuda"), mode="both",
                          grad="rev", tuning=mvf.Tuning(grad=1, chunk=0, grid_blocks=0, best_ms=0.0, sub_per_lane=1,
                                                        engine=mvf.MVF_ENGINE["spec"]))
    torch.cuda.synchronize()
    red = res["reduced"].cpu().numpy()
    for i in range(n_nodes):
        one = gpu_bound(t, boxes[i], spl[i], mode="both", grad="rev", handle=h, engine="spec", per_sub=False)
        assert np.array_equal(red[i], one["reduced"]), f"node {i}"
    h.close()


def test_diff_workload_checkpointed_adjoint_sampled():
    # 32 variables, a 2,000-op objective and four 300-op constraints, 2^20 subdomains: the
    # specialised adjoint with checkpointed segments (the library's default budget), sampled
    # against the oracle's reverse mode and bitwise against the interpreter's record-tape adjoint
    from paper_2507_20769_amd import mvf
    w = I.diff(1)
    h = mvf.Tape(w.tape)
    info = h.specialize(grad="rev", max_code=10 ** 6)
    print(f"[spec] diff checkpoints={info['ckpt_intervals']} compile={info['seconds']:.1f}s "
          f"cached={info['from_cache']}", flush=True)
    assert info["ckpt_intervals"] > 0
    g = gpu_bound(w.tape, w.box, w.splits, mode="both", grad="rev", handle=h, engine="spec")
    gi = gpu_bound(w.tape, w.box, w.splits, mode="both", grad="rev", handle=h, engine="interp")
    assert_parity(g["per_sub"], gi["per_sub"], True, None, "diff adjoint vs interpreter")
    assert_parity(g["reduced"], gi["reduced"], True, None, "diff reduced vs interpreter")
    S = w.n_sub
    ks = np.unique(np.concatenate([np.random.default_rng(5).choice(S, 48, replace=False), [0, S - 1]]))
    o = O.bound(w.tape, w.box, w.splits, mode=O.MODE_BOTH, grad=O.GRAD_REV, ks=ks, nthreads=8)
    sc = scale_of(O.bound(w.tape, w.box, w.splits, mode=O.MODE_NIE, ks=ks, per_sub=False, nthreads=8)["reduced"])
    assert_parity(g["per_sub"][:, :, ks], o["per_sub"], not has_transcendental(w.tape), sc,
                  "diff adjoint sampled vs oracle")
    h.close()


def test_automatic_engine_takes_the_interpreter_when_the_lds_gradient_leaves_no_room():
    # 13 variables: the specialised adjoint keeps the 13 gradient components in LDS (52 KB per
    # workgroup); beside a 3,500-entry breakpoint table (112 KB) they no longer fit, so the
    # automatic choice runs the interpreter and an explicit request for the specialised kernel
    # is refused; with a small table the automatic choice is the specialised kernel, bitwise
    # the interpreter's bounds either way
    from paper_2507_20769_amd import mvf
    t = _rational(I.random_small_tape(21, n=13, ops=300, n_con=1, con_ops=20, window=8))
    h, info = _spec(t)
    assert info["ckpt_intervals"] > 0
    box = np.array([[-2.0, 2.0]] * 13)
    for splits in ([3500] + [1] * 12, [5, 3] + [1] * 11):
        print(f"[case] splits={splits[:2]}...", flush=True)
        ga = gpu_bound(t, box, splits, mode="both", grad="rev", handle=h, engine="auto")
        gi = gpu_bound(t, box, splits, mode="both", grad="rev", handle=h, engine="interp")
        for key in ("per_sub", "reduced", "argmin", "flags", "extra"):
            assert_parity(ga[key], gi[key], True, None, f"{key}: automatic engine vs interpreter")
    with pytest.raises(mvf.MVFError):
        gpu_bound(t, box, [3500] + [1] * 12, mode="both", grad="rev", handle=h, engine="spec")
    gs = gpu_bound(t, box, [5, 3] + [1] * 11, mode="both", grad="rev", handle=h, engine="spec")
    assert_parity(gs["per_sub"], gi["per_sub"], True, None, "specialised vs interpreter")
    h.close()
