"""GPU parity of the specialised (run-time-compiled) forward kernel.

Each case runs the specialised kernel through the C ABI and compares it with
the oracle element by element (bit-exact for + - * / sqr sqrt tapes, 1e-12 of
the root's scale with exp/log), and with the interpreter kernel on the same
device: the two evaluate the same instructions with the same primitives, so
rational tapes must agree bitwise in every output (per-subdomain bounds,
flags, hulls, argmin and the two branch-and-bound bounds)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_20769_amd import inputs as I

from gpu_util import assert_parity, gpu_bound, has_transcendental, scale_of

pytestmark = pytest.mark.gpu

MODES = {"nie": O.MODE_NIE, "mvf": O.MODE_MVF, "both": O.MODE_BOTH}


def _handle(tape, kinds=None, **spec):
    from paper_2507_20769_amd import mvf
    h = mvf.Tape(tape)
    if kinds is not None:
        h.set_root_kinds(kinds)
    info = h.specialize(**spec)
    print(f"[spec] n={tape.n_vars} chunk={info['chunk']} units={info['code_units']} "
          f"compile={info['seconds']:.2f}s cached={info['from_cache']}", flush=True)
    return h


def _compare(h, tape, box, splits, mode="both", kinds=None, grad="fwd"):
    print(f"[case] n={tape.n_vars} nodes={tape.n_nodes} splits={list(splits)} mode={mode} grad={grad}", flush=True)
    g = gpu_bound(tape, box, splits, mode=mode, grad=grad, handle=h, engine="spec")
    gi = gpu_bound(tape, box, splits, mode=mode, grad=grad, handle=h, engine="interp")
    o = O.bound(tape, box, splits, mode=MODES[mode], grad=O.GRAD_FWD if grad == "fwd" else O.GRAD_REV, nthreads=8,
                kinds=kinds)
    exact = not has_transcendental(tape)
    sc = scale_of(O.bound(tape, box, splits, mode=O.MODE_NIE, per_sub=False, nthreads=8)["reduced"])
    assert_parity(g["per_sub"], o["per_sub"], exact, sc, "per_sub vs oracle")
    assert_parity(g["reduced"], o["reduced"], exact, sc, "reduced vs oracle")
    assert np.array_equal(g["flags"].astype(np.uint32), o["flags"])
    if exact:
        assert int(g["argmin"][0]) == o["argmin"]
        assert_parity(g["extra"], o["extra"], True, None, "extra vs oracle")
        for key in ("per_sub", "reduced", "argmin", "flags", "extra"):
            assert_parity(g[key], gi[key], True, None, f"{key} vs interpreter")
    else:
        assert_parity(g["per_sub"], gi["per_sub"], False, sc, "per_sub vs interpreter")
    return g


def test_cubic_table_and_modes():
    t = I.cubic_tape()
    h = _handle(t)
    box = np.array([[-1.0, 2.0]])
    g = gpu_bound(t, box, [1], mode="nie", handle=h, engine="spec")
    assert g["reduced"][0].tolist() == [-23.0, 32.0]
    g = gpu_bound(t, box, [1], mode="mvf", handle=h, engine="spec")
    assert g["reduced"][0].tolist() == [-55.375, 49.625]
    for N in (1, 2, 255, 256, 1000):
        for mode in MODES:
            _compare(h, t, box, [N], mode)
    h.close()


def test_tiny_full():
    w = I.tiny(1)
    h = _handle(w.tape)
    for mode in MODES:
        _compare(h, w.tape, w.box, w.splits, mode)
    h.close()


def _rational(t):
    nodes = t.nodes.copy()
    nodes["op"][nodes["op"] == I.EXP] = I.SQR
    nodes["op"][nodes["op"] == I.LOG] = I.SQRT
    return I.Tape(nodes, t.consts, t.roots, t.n_vars)


@pytest.mark.parametrize("seed,chunk", [(1, 0), (2, 1), (3, 2)])
def test_random_rational_tapes_ragged(seed, chunk):
    # 5*7*11 = 385 subdomains: a full workgroup and a ragged tail; three chunkings
    rng = np.random.default_rng(seed)
    t = _rational(I.random_small_tape(seed, n=3, ops=60, n_con=2, con_ops=20, window=8))
    kinds = [0, 1, 2]
    h = _handle(t, kinds, chunk=chunk)
    box = np.array([[-2.0, 2.0], [-1.5, 2.5], [-2.0, 1.0]]) + rng.uniform(-0.3, 0.3, (3, 1))
    for mode in MODES:
        _compare(h, t, box, [5, 7, 11], mode, kinds)
    h.close()


@pytest.mark.parametrize("seed", [4, 5])
def test_random_tapes_with_exp_log(seed):
    t = I.random_small_tape(seed, n=4, ops=80, n_con=3, con_ops=25, window=8)
    assert has_transcendental(t)
    h = _handle(t)
    _compare(h, t, np.array([[-2.0, 2.0]] * 4), [4, 5, 3, 6], "both")
    h.close()


def test_peaks_degenerate_and_domain_violations():
    t = I.peaks_tape()
    h = _handle(t)
    _compare(h, t, np.array([[-3.0, 3.0], [-3.0, 3.0]]), [40, 37], "both")
    h.close()
    t = I.random_small_tape(9, n=2, ops=30, n_con=1, con_ops=10)
    h = _handle(t)
    _compare(h, t, np.array([[-1.0, 1.0], [0.5, 0.5]]), [1, 1], "both")      # one subdomain, zero width
    _compare(h, t, np.array([[-1.0, 1.0], [0.5, 0.5]]), [3, 1], "both")
    h.close()
    # 1/x on [-1, 1] and sqrt(y) on [-0.5, 1]: flagged subdomains are [-inf, inf]
    nodes = np.array([(I.CONST, 0, -1), (I.VAR, 0, -1), (I.DIV, 0, 1), (I.VAR, 1, -1), (I.SQRT, 3, -1),
                      (I.ADD, 2, 4)], dtype=I.NODE_DTYPE)
    t = I.Tape(nodes, np.array([1.0]), np.array([5, 4], dtype=np.int32), 2)
    h = _handle(t)
    g = _compare(h, t, np.array([[-1.0, 1.0], [-0.5, 1.0]]), [4, 3], "both")
    assert g["flags"].sum() > 0
    h.close()


def test_mid_full_size_sampled():
    # the 262,144-subdomain mid workload in the benchmark's launch; 512 sampled
    # subdomains recomputed by the oracle one by one, the rest against the interpreter
    w = I.mid(1)
    kinds = [0, 1, 1, 1]
    h = _handle(w.tape, kinds)
    g = gpu_bound(w.tape, w.box, w.splits, mode="both", handle=h, engine="spec")
    gi = gpu_bound(w.tape, w.box, w.splits, mode="both", handle=h, engine="interp")
    S = w.n_sub
    rng = np.random.default_rng(0)
    ks = np.unique(np.concatenate([rng.choice(S, 508, replace=False), [0, S - 1, 255, 256]]))
    o = O.bound(w.tape, w.box, w.splits, mode=O.MODE_BOTH, ks=ks, nthreads=8, kinds=kinds)
    sc = scale_of(O.bound(w.tape, w.box, w.splits, mode=O.MODE_NIE, ks=ks, per_sub=False, nthreads=8)["reduced"])
    exact = not has_transcendental(w.tape)
    assert_parity(g["per_sub"][:, :, ks], o["per_sub"], exact, sc, "mid sampled vs oracle")
    assert_parity(g["per_sub"], gi["per_sub"], exact, sc, "mid vs interpreter")
    assert np.array_equal(g["reduced"][:, 0], g["per_sub"][:, 0, :].min(axis=1))
    assert np.array_equal(g["reduced"][:, 1], g["per_sub"][:, 1, :].max(axis=1))
    assert not g["flags"].any()
    same = np.mean(g["per_sub"] == gi["per_sub"])
    print(f"[mid] fraction of per-subdomain endpoints bitwise equal to the interpreter: {same:.6f}", flush=True)
    h.close()


@pytest.mark.parametrize("grad", ["fwd", "rev"])
@pytest.mark.parametrize("rational", [True, False])
def test_roots_sharing_subexpressions(grad, rational):
    # every node of the union of the root cones is computed once per pass and
    # each root's bound is taken where its value is computed: bitwise the
    # interpreter's (which computes each root's cone on its own) and the oracle's
    t = I.shared_roots_tape(11)
    if rational:
        t = I.rational(t)
    kinds = [0, 1, 2, 1]
    h = _handle(t, kinds, grad="auto")
    box = np.array([[-2.0, 2.0], [-1.5, 2.5], [-2.0, 1.0]])
    for mode in MODES:
        _compare(h, t, box, [5, 7, 11], mode, kinds, grad=grad)
    h.close()


def test_largest_variable_count():
    # 64 variables (MVF_MAX_VARS): many tangent passes in forward mode, a gradient partly in
    # LDS and partly in registers in the adjoint; ragged and power-of-two partitions
    rng = np.random.default_rng(64)
    tb = I.TapeBuilder(64)
    xs = [tb.var(i) for i in range(64)]
    f = tb.const(0.5)
    for i in range(64):                    # f = 0.5 + sum_i (x_i - k_i)^2 / (1 + x_{i+1}^2) in a running sum
        d = tb.add(I.SUB, xs[i], tb.const(float(rng.uniform(-1, 1))))
        q = tb.add(I.DIV, tb.add(I.SQR, d), tb.add(I.ADD, tb.const(1.0), tb.add(I.SQR, xs[(i + 1) % 64])))
        f = tb.add(I.ADD, f, q)
    tb.roots.append(f)
    g = tb.const(-1.0)
    for i in range(0, 64, 2):              # g = sum_i x_{2i} x_{2i+1} - 1 <= 0
        g = tb.add(I.ADD, g, tb.add(I.MUL, xs[i], xs[i + 1]))
    tb.roots.append(g)
    t = tb.build()
    kinds = [0, 1]
    h = _handle(t, kinds, grad="auto")
    box = np.array([[-2.0, 2.0]] * 64) + rng.uniform(-0.3, 0.3, (64, 1))
    for splits in ([3, 5] + [1] * 62, [2] * 8 + [1] * 56):
        for grad in ("fwd", "rev"):
            _compare(h, t, box, splits, "both", kinds, grad=grad)
    h.close()


@pytest.mark.parametrize("grad", ["fwd", "rev"])
def test_mid_rational_full_size_bitwise(grad):
    # the mid workload's shape with exp -> sqr and log -> sqrt, at full size in the
    # benchmark's launch: every per-subdomain endpoint, flag, hull, argmin and both
    # branch-and-bound bounds bitwise equal to the interpreter's, and 1,024 sampled
    # subdomains (the grid's first and last among them) bitwise equal to the oracle's
    w = I.mid(1)
    t = I.rational(w.tape)
    assert not has_transcendental(t)
    kinds = [0, 1, 1, 1]
    h = _handle(t, kinds, grad="auto")   # both gradient modes' kernels (the precompiled object)
    g = gpu_bound(t, w.box, w.splits, mode="both", grad=grad, handle=h, engine="spec")
    gi = gpu_bound(t, w.box, w.splits, mode="both", grad=grad, handle=h, engine="interp")
    for key in ("per_sub", "reduced", "argmin", "flags", "extra"):
        assert_parity(g[key], gi[key], True, None, f"mid rational {grad}: {key} vs interpreter")
    assert not g["flags"].any()
    S = w.n_sub
    rng = np.random.default_rng(2)
    ks = np.unique(np.concatenate([rng.choice(S, 1020, replace=False), [0, 255, 256, S - 1]]))
    o = O.bound(t, w.box, w.splits, mode=O.MODE_BOTH, grad=O.GRAD_FWD if grad == "fwd" else O.GRAD_REV,
                ks=ks, nthreads=8, kinds=kinds)
    assert_parity(g["per_sub"][:, :, ks], o["per_sub"], True, None, f"mid rational {grad}: sampled vs oracle")
    assert np.array_equal(g["reduced"][:, 0], g["per_sub"][:, 0, :].min(axis=1))
    assert np.array_equal(g["reduced"][:, 1], g["per_sub"][:, 1, :].max(axis=1))
    h.close()


def test_engine_selection_errors():
    import torch
    from paper_2507_20769_amd import mvf
    t = I.cubic_tape()
    h = mvf.Tape(t)
    box = torch.tensor([[-1.0, 2.0]], dtype=torch.float64, device="cuda")
    with pytest.raises(mvf.MVFError) as e:
        mvf.bound(h, box, [8], engine="spec")             # not specialised yet
    assert e.value.code == -1
    h.specialize()
    with pytest.raises(mvf.MVFError) as e:
        mvf.bound(h, box, [8], grad="rev", engine="spec")  # built for tangent mode only
    assert e.value.code == -1
    mvf.bound(h, box, [8], grad="rev")                     # auto: reverse mode interprets
    a = mvf.bound(h, box, [8], grad="fwd")                 # auto: the specialised kernel
    b = mvf.bound(h, box, [8], grad="fwd", engine="interp")
    torch.cuda.synchronize()
    assert torch.equal(a["reduced"], b["reduced"]) and torch.equal(a["argmin"], b["argmin"])
    h.close()


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_reverse_specialised_rational_and_small_cases(seed):
    # the adjoint kernels (grad "rev"/"auto") against the oracle's reverse mode and bitwise
    # against the interpreter's adjoint
    rng = np.random.default_rng(seed)
    t = _rational(I.random_small_tape(seed, n=3, ops=60, n_con=2, con_ops=20, window=8))
    kinds = [0, 1, 2]
    h = _handle(t, kinds, grad="auto")
    box = np.array([[-2.0, 2.0], [-1.5, 2.5], [-2.0, 1.0]]) + rng.uniform(-0.3, 0.3, (3, 1))
    for mode in MODES:
        _compare(h, t, box, [5, 7, 11], mode, kinds, grad="rev")
    h.close()
    if seed == 1:
        for tape, box, splits in ((I.cubic_tape(), np.array([[-1.0, 2.0]]), [256]),
                                  (I.tiny(1).tape, I.tiny(1).box, I.tiny(1).splits),
                                  (I.peaks_tape(), np.array([[-3.0, 3.0], [-3.0, 3.0]]), [40, 37])):
            h = _handle(tape, grad="rev")
            _compare(h, tape, box, splits, "both", grad="rev")
            h.close()


def test_reverse_specialised_exp_log_and_mid():
    t = I.random_small_tape(4, n=4, ops=80, n_con=3, con_ops=25, window=8)
    h = _handle(t, grad="rev")
    _compare(h, t, np.array([[-2.0, 2.0]] * 4), [4, 5, 3, 6], "both", grad="rev")
    h.close()
    w = I.mid(1)
    kinds = [0, 1, 1, 1]
    h = _handle(w.tape, kinds, grad="rev")
    g = gpu_bound(w.tape, w.box, w.splits, mode="both", grad="rev", handle=h, engine="spec")
    gi = gpu_bound(w.tape, w.box, w.splits, mode="both", grad="rev", handle=h, engine="interp")
    S = w.n_sub
    ks = np.unique(np.concatenate([np.random.default_rng(1).choice(S, 300, replace=False), [0, S - 1]]))
    o = O.bound(w.tape, w.box, w.splits, mode=O.MODE_BOTH, grad=O.GRAD_REV, ks=ks, nthreads=8, kinds=kinds)
    sc = scale_of(O.bound(w.tape, w.box, w.splits, mode=O.MODE_NIE, ks=ks, per_sub=False, nthreads=8)["reduced"])
    exact = not has_transcendental(w.tape)
    assert_parity(g["per_sub"][:, :, ks], o["per_sub"], exact, sc, "mid adjoint sampled vs oracle")
    assert_parity(g["per_sub"], gi["per_sub"], exact, sc, "mid adjoint vs interpreter")
    assert not g["flags"].any()
    h.close()


def test_division_by_constants_at_the_extremes():
    # x / k with constant k: endpoints rounded outward bit for bit as the oracle's, through
    # overflow, the subnormal range and exact quotients (a quotient estimate corrected with a
    # residual that falls below the normal range would be several ulps off there)
    import torch
    from paper_2507_20769_amd import mvf
    big = np.finfo(np.float64).max
    boxes = [[-big, big], [-big, -1e300], [1e-310, 3e-308], [-5.0, 7.0], [-3e-320, 1e-320], [0.0, 0.0],
             [-1e308, 1e308], [1.0, 3.0], [-6.0, -2.0]]
    for k in (0.5, 3.0, 0.1, 7.0, 1e-300, 1e300, 0.3, 2.0):
        tape = I.Tape(np.array([(I.VAR, 0, -1), (I.CONST, 0, -1), (I.DIV, 0, 1)], dtype=I.NODE_DTYPE),
                      np.array([k]), np.array([2], dtype=np.int32), 1)
        h = mvf.Tape(tape)
        h.specialize()
        for b in boxes:
            box = np.array([b])
            o = O.bound(tape, box, [1], mode=O.MODE_NIE, nthreads=1)
            for engine in ("spec", "interp"):
                g = gpu_bound(tape, box, [1], mode="nie", handle=h, engine=engine)
                assert np.array_equal(g["per_sub"], o["per_sub"]), (k, b, engine, g["per_sub"], o["per_sub"])
        h.close()


@pytest.mark.parametrize("engine", ["interp", "spec"])
def test_square_at_sign_boundaries(engine):
    # x^2 (the interval square) and x*x (the general product) on one-subdomain boxes whose ends
    # are zeros of either sign, tiny, huge or on both sides of 0: bitwise the oracle's, and the
    # square is [0, max(a^2, b^2)] when a <= 0 <= b, [min^2, max^2] otherwise
    from fractions import Fraction
    V = I.VAR
    nodes = np.array([(V, 0, -1), (I.SQR, 0, -1), (I.MUL, 0, 0)], dtype=I.NODE_DTYPE)
    tape = I.Tape(nodes, np.zeros(0), np.array([1, 2], dtype=np.int32), 1)
    ends = [(-2.0, 3.0), (-3.0, 2.0), (2.0, 5.0), (-5.0, -2.0), (-0.0, 0.0), (0.0, 0.0), (-0.0, 4.0),
            (-4.0, -0.0), (1e-200, 2e-200), (-1e-200, 1e-200), (-3e-160, -1e-160), (1e200, 1e300),
            (-1e300, 1e250), (0.1, 0.3), (-0.7, 0.2), (5e-324, 1e-323)]
    h = _handle(tape, grad="auto") if engine == "spec" else None
    for a, b in ends:
        box = np.array([[a, b]])
        print(f"[case] square of [{a!r}, {b!r}] engine={engine}", flush=True)
        for grad in ("fwd", "rev"):
            g = gpu_bound(tape, box, [1], mode="nie", grad=grad, handle=h, engine=engine)
            o = O.bound(tape, box, [1], mode=O.MODE_NIE, grad=O.GRAD_FWD if grad == "fwd" else O.GRAD_REV)
            assert_parity(g["per_sub"], o["per_sub"], True, what=f"[{a}, {b}] {grad}")
        lo, hi = g["per_sub"][0, :, 0]
        fa, fb = Fraction(a), Fraction(b)
        sq_hi = max(fa * fa, fb * fb)
        sq_lo = Fraction(0) if a <= 0.0 <= b else min(fa * fa, fb * fb)
        assert (lo == 0.0 or Fraction(lo) <= sq_lo) and (hi == np.inf or sq_hi <= Fraction(hi)), (a, b, lo, hi)
        if a <= 0.0 <= b:
            assert lo == 0.0 and not np.signbit(lo), (a, b, lo)
    if h is not None:
        h.close()
