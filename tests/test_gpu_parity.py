"""GPU parity: libmvf (through the C ABI) against the CPU oracle, element by element.

Bit-exact (==) where the tape uses only + - * / sqr sqrt; within 1e-12 of the
root's scale where exp or log appear (the two sides call different libms).
Every case also checks that the GPU's own bounds enclose sampled values.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_20769_amd import inputs as I

from gpu_util import assert_parity, gpu_bound, has_transcendental, scale_of

pytestmark = pytest.mark.gpu

MODES = {"nie": O.MODE_NIE, "mvf": O.MODE_MVF, "both": O.MODE_BOTH}


def _check_enclosure(tape, box, splits, per_sub, sc, n_sub=16, n_pts=8):
    # the GPU's bounds of seeded subdomains contain the function at points drawn in them
    # (round-to-nearest point evaluation: a slack of 1e-9 of the root's scale)
    rng = np.random.default_rng(123)
    S = per_sub.shape[2]
    for k in rng.choice(S, min(S, n_sub), replace=False):
        X, _ = O.subdomain(box, np.asarray(splits), int(k))
        pts = X[:, 0] + (X[:, 1] - X[:, 0]) * rng.random((n_pts, X.shape[0]))
        f = I.eval_points_np(tape, pts)                          # [n_pts, m]
        for r in range(per_sub.shape[0]):
            lo, hi = per_sub[r, 0, k], per_sub[r, 1, k]
            tol = 1e-9 * sc[r]
            v = f[:, r][~np.isnan(f[:, r])]          # points outside the function's domain bound nothing
            assert np.all(v >= lo - tol) and np.all(v <= hi + tol), f"subdomain {k} root {r}"


def _compare(tape, box, splits, mode="both", per_sub=True):
    print(f"[case] n={tape.n_vars} nodes={tape.n_nodes} splits={list(splits)} mode={mode}", flush=True)
    g = gpu_bound(tape, box, splits, mode=mode, per_sub=per_sub)
    o = O.bound(tape, box, splits, mode=MODES[mode], per_sub=per_sub, nthreads=8)
    exact = not has_transcendental(tape)
    sc = scale_of(O.bound(tape, box, splits, mode=O.MODE_NIE, per_sub=False, nthreads=8)["reduced"])
    if per_sub:
        assert_parity(g["per_sub"], o["per_sub"], exact, sc, "per_sub")
        assert np.array_equal(g["flags"].astype(np.uint32), o["flags"])
        # the reduction is the hull of the GPU's own per-subdomain output, bitwise
        assert np.array_equal(g["reduced"][:, 0], g["per_sub"][:, 0, :].min(axis=1))
        assert np.array_equal(g["reduced"][:, 1], g["per_sub"][:, 1, :].max(axis=1))
        lo0 = g["per_sub"][0, 0, :]
        assert int(g["argmin"][0]) == int(np.argmax(lo0 == lo0.min()))
        _check_enclosure(tape, box, splits, g["per_sub"], sc)
    assert_parity(g["reduced"], o["reduced"], exact, sc, "reduced")
    if exact:
        assert int(g["argmin"][0]) == o["argmin"]
    return g, o


def test_cubic_refinement_table():
    # the DAG example of Sec. 3.2 on [-1, 2]: N = 1 gives NIE [-23, 32], MVF [-55.375, 49.625]
    t = I.cubic_tape()
    box = np.array([[-1.0, 2.0]])
    g = gpu_bound(t, box, [1], mode="nie")
    assert g["reduced"][0].tolist() == [-23.0, 32.0]
    g = gpu_bound(t, box, [1], mode="mvf")
    assert g["reduced"][0].tolist() == [-55.375, 49.625]
    for N in (1, 2, 3, 8, 64, 255, 256, 1000):
        for mode in MODES:
            _compare(t, box, [N], mode)


def test_tiny_workload_full():
    w = I.tiny(1)
    for mode in MODES:
        _compare(w.tape, w.box, w.splits, mode)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_rational_tapes_ragged(seed):
    # + - * / sqr sqrt only; 5*7*11 = 385 subdomains: a full 256-lane block plus a ragged tail
    rng = np.random.default_rng(seed)
    t = I.random_small_tape(seed, n=3, ops=60, n_con=2, con_ops=20, window=8)
    nodes = t.nodes.copy()
    nodes["op"][nodes["op"] == I.EXP] = I.SQR      # exp -> sqr, log (positive argument) -> sqrt
    nodes["op"][nodes["op"] == I.LOG] = I.SQRT
    t = I.Tape(nodes, t.consts, t.roots, t.n_vars)
    box = np.array([[-2.0, 2.0], [-1.5, 2.5], [-2.0, 1.0]]) + rng.uniform(-0.3, 0.3, (3, 1))
    for mode in MODES:
        _compare(t, box, [5, 7, 11], mode)


@pytest.mark.parametrize("seed", [4, 5])
def test_random_tapes_with_exp_log(seed):
    t = I.random_small_tape(seed, n=4, ops=80, n_con=3, con_ops=25, window=8)
    assert has_transcendental(t)
    box = np.array([[-2.0, 2.0]] * 4)
    _compare(t, box, [4, 5, 3, 6], "both")


def test_peaks_function():
    t = I.peaks_tape()
    _compare(t, np.array([[-3.0, 3.0], [-3.0, 3.0]]), [40, 37], "both")


def test_single_subdomain_and_degenerate_box():
    t = I.random_small_tape(9, n=2, ops=30, n_con=1, con_ops=10)
    _compare(t, np.array([[-1.0, 1.0], [0.5, 0.5]]), [1, 1], "both")      # zero-width dimension
    _compare(t, np.array([[-1.0, 1.0], [0.5, 0.5]]), [3, 1], "both")


def test_domain_violations_flag_subdomains():
    # 1/x on [-1, 1]: the subdomains touching 0 are flagged and bounded by [-inf, inf]
    nodes = np.array([(I.CONST, 0, -1), (I.VAR, 0, -1), (I.DIV, 0, 1), (I.VAR, 1, -1), (I.SQRT, 3, -1),
                      (I.ADD, 2, 4)], dtype=I.NODE_DTYPE)
    t = I.Tape(nodes, np.array([1.0]), np.array([5, 4], dtype=np.int32), 2)
    g, o = _compare(t, np.array([[-1.0, 1.0], [-0.5, 1.0]]), [4, 3], "both")
    assert g["flags"].sum() > 0


def test_mid_workload_full_size_sampled():
    # the 262,144-subdomain mid workload in the benchmark's launch; 512 sampled subdomains
    # are recomputed by the oracle one by one
    w = I.mid(1)
    g = gpu_bound(w.tape, w.box, w.splits, mode="both")
    S = w.n_sub
    rng = np.random.default_rng(0)
    ks = np.unique(np.concatenate([rng.choice(S, 500, replace=False), [0, S - 1, 255, 256]]))
    o = O.bound(w.tape, w.box, w.splits, mode=O.MODE_BOTH, ks=ks, nthreads=8)
    sc = scale_of(O.bound(w.tape, w.box, w.splits, mode=O.MODE_NIE, ks=ks, per_sub=False, nthreads=8)["reduced"])
    assert_parity(g["per_sub"][:, :, ks], o["per_sub"], not has_transcendental(w.tape), sc, "mid sampled")
    assert np.array_equal(g["reduced"][:, 0], g["per_sub"][:, 0, :].min(axis=1))
    assert np.array_equal(g["reduced"][:, 1], g["per_sub"][:, 1, :].max(axis=1))
    assert not g["flags"].any()


def test_gpu_bounds_enclose_samples():
    t = I.random_small_tape(7, n=3, ops=50, n_con=2, con_ops=15)
    box = np.array([[-2.0, 2.0]] * 3)
    splits = np.array([4, 4, 4])
    g = gpu_bound(t, box, splits, mode="both")
    rng = np.random.default_rng(1)
    for k in range(0, 64, 5):
        X, c = O.subdomain(box, splits, k)
        pts = X[:, 0] + (X[:, 1] - X[:, 0]) * rng.random((300, 3))
        v = I.eval_points_np(t, pts)
        sl = 1e-12 * np.maximum(1, np.abs(v).max(axis=0))
        assert np.all(g["per_sub"][:, 0, k] - sl <= v.min(axis=0))
        assert np.all(v.max(axis=0) <= g["per_sub"][:, 1, k] + sl)


@pytest.mark.parametrize("name", ["batch", "e2e"])
def test_forward_with_lds_spill_slots(name):
    # tapes whose live set exceeds the register slots at one tangent component: the
    # highest slot ids live in LDS during tangent passes
    from paper_2507_20769_amd import mvf
    if name == "batch":
        bw = I.batch(1, n_nodes=4)
        tape, box, splits = bw.tape, bw.boxes[1], bw.splits[1]
    else:
        tape = I.e2e_tape(1)
        box = np.array([[-3.0, 3.0]] * 10)
        splits = np.array([2, 2, 2, 2, 2, 2, 2, 2, 1, 1])
    st = mvf.check(tape)
    assert st.tangent_chunk >= 1 and st.max_slots * (4 + 4 * st.tangent_chunk) > 160 - 4 * tape.n_roots
    g = gpu_bound(tape, box, splits, mode="both", grad="fwd")
    S = int(np.prod(splits))
    ks = np.unique(np.concatenate([np.random.default_rng(2).choice(S, min(S, 120), replace=False), [0, S - 1]]))
    o = O.bound(tape, box, splits, mode=O.MODE_BOTH, ks=ks, nthreads=8)
    sc = scale_of(O.bound(tape, box, splits, mode=O.MODE_NIE, ks=ks, per_sub=False, nthreads=8)["reduced"])
    assert_parity(g["per_sub"][:, :, ks], o["per_sub"], not has_transcendental(tape), sc, f"{name} fwd spill")


@pytest.mark.parametrize("engine", ["interp", "spec"])
def test_repeated_launches_reuse_the_workspace(engine):
    # back-to-back launches on one workspace with changing boxes each give the oracle's
    # result (the partials of one launch never leak into the next)
    import torch
    from paper_2507_20769_amd import mvf
    t = I.random_small_tape(7, n=3, ops=40, n_con=1, con_ops=12)
    nodes = t.nodes.copy()                             # rational: results bit for bit
    nodes["op"][nodes["op"] == I.EXP] = I.SQR
    nodes["op"][nodes["op"] == I.LOG] = I.SQRT
    t = I.Tape(nodes, t.consts, t.roots, t.n_vars)
    h = mvf.Tape(t)
    if engine == "spec":
        h.specialize()
    rng = np.random.default_rng(8)
    boxes = []
    for _ in range(5):
        lo = rng.uniform(-2, 1, 3)
        boxes.append(np.stack([lo, lo + rng.uniform(0.1, 2.0, 3)], axis=1))
    dbox = torch.tensor(boxes[0], device="cuda")
    call = mvf.BoundCall(h, dbox, [37, 9, 5], mode="both", grad="fwd", engine=engine)    # 1,665 subdomains
    for i, b in enumerate(boxes):
        dbox.copy_(torch.tensor(b, device="cuda"))
        call.launch()
        torch.cuda.synchronize()
        o = O.bound(t, b, [37, 9, 5], mode=O.MODE_BOTH, nthreads=8)
        assert np.array_equal(call.reduced.cpu().numpy(), o["reduced"]), i
        assert int(call.argmin.item()) == o["argmin"], i
    h.close()


@pytest.mark.parametrize("engine", ["interp", "spec"])
def test_largest_partition_table(engine):
    # the breakpoint table at its capacity (2,048 + 2,048 = MVF_MAX_TABLE entries, 4,194,304
    # subdomains): 400 sampled subdomains recomputed by the oracle one by one, the hull equal to
    # the per-subdomain extremes, and one more split refused with MVF_ELIMIT
    import torch
    from paper_2507_20769_amd import mvf
    t = I.random_small_tape(12, n=2, ops=30, n_con=1, con_ops=10)
    nodes = t.nodes.copy()
    nodes["op"][nodes["op"] == I.EXP] = I.SQR
    nodes["op"][nodes["op"] == I.LOG] = I.SQRT
    t = I.Tape(nodes, t.consts, t.roots, t.n_vars)
    h = mvf.Tape(t)
    if engine == "spec":
        h.specialize()
    box = np.array([[-1.5, 2.0], [-0.5, 1.0]])
    splits = [2048, 2048]
    print(f"[case] table capacity engine={engine}", flush=True)
    g = gpu_bound(t, box, splits, mode="both", handle=h, engine=engine)
    S = 2048 * 2048
    ks = np.unique(np.concatenate([np.random.default_rng(13).choice(S, 400, replace=False), [0, 2047, 2048, S - 1]]))
    o = O.bound(t, box, splits, mode=O.MODE_BOTH, ks=ks, nthreads=8)
    assert_parity(g["per_sub"][:, :, ks], o["per_sub"], True, None, "sampled")
    assert np.array_equal(g["reduced"][:, 0], g["per_sub"][:, 0, :].min(axis=1))
    assert np.array_equal(g["reduced"][:, 1], g["per_sub"][:, 1, :].max(axis=1))
    with pytest.raises(mvf.MVFError) as e:
        mvf.bound(h, torch.tensor(box, device="cuda"), [2049, 2048], engine=engine)
    assert e.value.code == -3
    h.close()


def test_tape_from_file_bounds_like_the_oracle(tmp_path):
    # mvf.Tape.from_file reads what inputs.save_tape wrote; the bounds are the oracle's, bitwise
    import torch
    from paper_2507_20769_amd import mvf
    w = I.tiny(2)
    path = str(tmp_path / "tiny.npz")
    I.save_tape(w.tape, path)
    h = mvf.Tape.from_file(path)
    out = mvf.bound(h, torch.tensor(w.box, device="cuda"), w.splits, mode="both")
    torch.cuda.synchronize()
    o = O.bound(w.tape, w.box, w.splits, mode=O.MODE_BOTH, per_sub=False, nthreads=8)
    assert_parity(out["reduced"].cpu().numpy(), o["reduced"], not has_transcendental(w.tape), None, "reduced")
    h.close()
