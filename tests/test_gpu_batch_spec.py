"""GPU tests of the batched launch configurations: subdomains per lane and the
specialised batch kernel give per node exactly the single-box result, inside
and outside a captured graph, and the autotuner's choice among them is
feasible and exact."""
import numpy as np
import pytest

from paper_2507_20769_amd import inputs as I

pytestmark = pytest.mark.gpu


def _rational(t):
    nodes = t.nodes.copy()
    nodes["op"][nodes["op"] == I.EXP] = I.SQR
    nodes["op"][nodes["op"] == I.LOG] = I.SQRT
    return I.Tape(nodes, t.consts, t.roots, t.n_vars)


def _per_node(h, bw, grad):
    import torch
    from paper_2507_20769_amd import mvf
    red, am, ex = [], [], []
    for i in range(len(bw.boxes)):
        out = mvf.bound(h, torch.tensor(bw.boxes[i], device="cuda"), bw.splits[i], mode="both", grad=grad,
                        engine="interp")
        torch.cuda.synchronize()
        red.append(out["reduced"].cpu().numpy())
        am.append(int(out["argmin"].item()))
        ex.append(out["extra"].cpu().numpy())
    return np.stack(red), np.array(am), np.stack(ex)


def _tuning(grad, spl, engine, grid=0, block=0):
    from paper_2507_20769_amd import mvf
    return mvf.Tuning(grad=grad, chunk=0, grid_blocks=grid, best_ms=0.0, sub_per_lane=spl,
                      engine=mvf.MVF_ENGINE[engine], block=block)


@pytest.mark.parametrize("grad,spl,engine,block", [
    ("fwd", 2, "interp", 0), ("fwd", 4, "interp", 0), ("rev", 2, "interp", 0), ("rev", 4, "interp", 0),
    ("fwd", 1, "spec", 0), ("fwd", 2, "spec", 128), ("fwd", 4, "spec", 64), ("rev", 1, "spec", 64),
    ("rev", 4, "spec", 0), ("rev", 2, "spec", 128)])
def test_batched_configurations_equal_per_node(grad, spl, engine, block):
    import torch
    from paper_2507_20769_amd import mvf
    bw = I.small_batch(21, 20, k_range=(3, 12))           # 8 .. 4096 subdomains: ragged items
    tape = _rational(bw.tape)
    h = mvf.Tape(tape)
    h.set_root_kinds([0] + [1] * (tape.n_roots - 1))
    if engine == "spec":
        h.specialize(grad="auto")
    print(f"[case] grad={grad} spl={spl} engine={engine} block={block}", flush=True)
    tu = _tuning(0 if grad == "fwd" else 1, spl, engine, grid=37, block=block)   # an odd grid: items wrap unevenly
    out = mvf.bound_batch(h, torch.tensor(bw.boxes, device="cuda"), torch.tensor(bw.splits, device="cuda"),
                          mode="both", grad=grad, tuning=tu)
    torch.cuda.synchronize()
    assert not out["status"].cpu().numpy().any()
    red, am, ex = _per_node(h, bw, grad)
    assert np.array_equal(out["reduced"].cpu().numpy(), red)
    assert np.array_equal(out["argmin"].cpu().numpy(), am)
    assert np.array_equal(out["extra"].cpu().numpy(), ex)
    h.close()


def test_spec_batch_graph_replays_match_fresh_launches():
    import torch
    from paper_2507_20769_amd import mvf
    bw = I.small_batch(22, 24, k_range=(4, 10))
    h = mvf.Tape(_rational(bw.tape))
    h.specialize()
    total = int(np.prod(bw.splits.astype(np.int64), axis=1).sum())
    g = mvf.BatchGraph(h, len(bw.boxes), total, mode="both", grad="fwd", tuning=_tuning(0, 2, "spec"))
    s = torch.cuda.Stream()
    ref = mvf.bound_batch(h, torch.tensor(bw.boxes, device="cuda"), torch.tensor(bw.splits, device="cuda"),
                          mode="both", grad="fwd", tuning=_tuning(0, 1, "interp"))
    torch.cuda.synchronize()
    want = ref["reduced"].cpu().numpy()
    for rep in range(3):                                # several replays, eager work in between
        n = len(bw.boxes) - 4 * rep
        g.launch(bw.boxes[:n], bw.splits[:n], stream=s)
        s.synchronize()
        red, am, st = g.result()
        assert not st.any()
        assert np.array_equal(red, want[:n]), rep
        torch.cuda.synchronize()
    g.close()
    h.close()


@pytest.mark.parametrize("grad", ["fwd", "rev"])
def test_autotuner_considers_the_specialised_kernel(grad):
    # the tuner keeps the caller's gradient mode, picks among interpreter and specialised kernels
    # (the latter at three workgroup sizes), grids and subdomains per lane, and caches its answer;
    # whatever it picks gives the bits of the interpreter's plain configuration
    import time
    import torch
    from paper_2507_20769_amd import mvf
    bw = I.small_batch(23, 16, k_range=(6, 11))
    h = mvf.Tape(bw.tape)
    h.specialize(grad="auto")
    boxes = torch.tensor(bw.boxes, device="cuda")
    splits = torch.tensor(bw.splits, device="cuda")
    t0 = time.perf_counter()
    tu = mvf.autotune(h, boxes, splits, mode="both", grad=grad)
    t1 = time.perf_counter()
    print(f"[autotune] {tu} in {t1 - t0:.2f} s", flush=True)
    g = 0 if grad == "fwd" else 1
    assert tu.grad == g and tu.grid_blocks > 0 and tu.best_ms > 0 and tu.sub_per_lane in (1, 2, 4)
    assert tu.engine in (1, 2) and tu.block in (64, 128, 256)
    again = mvf.autotune(h, boxes, splits, mode="both", grad=grad)          # cached
    assert time.perf_counter() - t1 < 0.1 * (t1 - t0) and again.as_dict() == tu.as_dict()
    out = mvf.bound_batch(h, boxes, splits, mode="both", grad=grad, tuning=tu)
    ref = mvf.bound_batch(h, boxes, splits, mode="both", grad=grad, tuning=_tuning(g, 1, "interp"))
    torch.cuda.synchronize()
    assert np.array_equal(out["reduced"].cpu().numpy(), ref["reduced"].cpu().numpy())
    assert np.array_equal(out["argmin"].cpu().numpy(), ref["argmin"].cpu().numpy())
    h.close()


def test_batched_engine_errors():
    import torch
    from paper_2507_20769_amd import mvf
    bw = I.small_batch(24, 4, k_range=(3, 5))
    h = mvf.Tape(bw.tape)
    boxes = torch.tensor(bw.boxes, device="cuda")
    splits = torch.tensor(bw.splits, device="cuda")
    for tu, grad in ((_tuning(0, 1, "spec"), "fwd"),      # not specialised
                     (_tuning(0, 17, "interp"), "fwd"),   # sub_per_lane out of range
                     (_tuning(0, 1, "interp", block=128), "fwd"),   # the interpreter's workgroup is 256
                     (_tuning(0, 1, "auto", block=96), "fwd")):     # not 64, 128 or 256
        with pytest.raises(mvf.MVFError) as e:
            mvf.bound_batch(h, boxes, splits, grad=grad, tuning=tu)
        assert e.value.code == -1
    h.specialize()                                         # tangent mode only
    with pytest.raises(mvf.MVFError) as e:
        mvf.bound_batch(h, boxes, splits, grad="rev", tuning=_tuning(1, 1, "spec"))
    assert e.value.code == -1
    h.specialize(grad="rev")                               # adjoint only
    with pytest.raises(mvf.MVFError) as e:
        mvf.bound_batch(h, boxes, splits, grad="fwd", tuning=_tuning(0, 1, "spec"))
    assert e.value.code == -1
    h.close()


def test_split_rule_tuning_and_bnb_under_both_rules():
    import torch
    from paper_2507_20769_amd import mvf
    bw = I.small_batch(25, 12, k_range=(3, 6))
    h = mvf.Tape(bw.tape)
    rule, better = mvf.autotune_splits(h, bw.boxes, 512, mode="both", grad="rev")
    print(f"[splits] rule={rule} better={better}", flush=True)
    # the same comparison by hand
    lbs = []
    for r in ("adaptive", "doubling"):
        sp = np.stack([mvf.splits(r, b[:, 1] - b[:, 0], 512)[0] for b in bw.boxes])
        out = mvf.bound_batch(h, torch.tensor(bw.boxes, device="cuda"), torch.tensor(sp, device="cuda"),
                              mode="both", grad="rev")
        torch.cuda.synchronize()
        lbs.append(out["extra"].cpu().numpy()[:, 0])
    assert better == [int(np.sum(lbs[0] > lbs[1])), int(np.sum(lbs[1] > lbs[0]))]
    assert rule == ("doubling" if better[1] > better[0] else "adaptive")
    # the B&B driver under both rules brackets the cubic's minimum
    t = I.cubic_tape()
    hc = mvf.Tape(t)
    xs = (-2.0 + np.sqrt(184.0)) / 18.0
    fs = 3 * xs ** 3 + xs ** 2 - 5 * xs - 1
    for r in ("adaptive", "doubling"):
        res = mvf.bnb_solve(hc, [[-1.0, 2.0]], max_nodes=300, gap=1e-6, budget=64, split_rule=r)
        assert res["status"] == 0 and res["lower"] <= fs <= res["upper"] and res["upper"] - res["lower"] <= 1e-6, r
    hc.close()
    h.close()
