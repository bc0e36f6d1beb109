"""The specialised-kernel generator on the host: generated sources compile
with hiprtc for gfx950 (no device needed), the tangent chunk and the size
accounting follow the documented rule, and bad options are rejected."""
import numpy as np
import pytest

from paper_2507_20769_amd import inputs as I
from paper_2507_20769_amd import mvf


def _tape(nodes, consts, roots, n):
    return I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.array(consts, dtype=np.float64),
                  np.array(roots, dtype=np.int32), n)


def _every_form():
    # every opcode and the constant-operand forms (x + k, k - x, x * k, x * -k, x / k, x / -k,
    # k / x), a leaf root, a constant root and a variable used twice by one product
    V = I.VAR
    nodes = [(V, 0, -1), (V, 1, -1), (I.CONST, 0, -1), (I.CONST, 1, -1), (I.CONST, 2, -1),
             (I.ADD, 0, 2), (I.SUB, 3, 1), (I.MUL, 5, 3), (I.MUL, 4, 6), (I.DIV, 7, 3),
             (I.DIV, 8, 4), (I.DIV, 2, 1), (I.MUL, 0, 0), (I.SQR, 9, -1), (I.ADD, 13, 2),
             (I.SQRT, 14, -1), (I.LOG, 14, -1), (I.EXP, 10, -1), (I.SUB, 15, 16), (I.ADD, 18, 17),
             (I.MUL, 19, 11), (I.ADD, 20, 12)]
    return _tape(nodes, [1.5, -0.75, 2.0], [21, 1, 3], 2)


def _trig():
    V = I.VAR
    nodes = [(V, 0, -1), (V, 1, -1), (I.CONST, 0, -1), (I.MUL, 0, 1), (I.TANH, 3, -1), (I.MUL, 2, 0),
             (I.SIN, 5, -1), (I.COS, 1, -1), (I.MUL, 6, 7), (I.ADD, 4, 8), (I.COS, 0, -1), (I.SUB, 10, 1)]
    return _tape(nodes, [3.0], [9, 11], 2)


def _deps(tape):
    """Variables each node depends on, as bit masks."""
    dep = []
    for op, a, b in zip(tape.nodes["op"], tape.nodes["a"], tape.nodes["b"]):
        if op == I.VAR:
            dep.append(1 << int(a))
        elif op == I.CONST:
            dep.append(0)
        else:
            dep.append(dep[a] | (dep[b] if op in (I.ADD, I.SUB, I.MUL, I.DIV) else 0))
    return dep


def _peak_live(tape, cmask, dep):
    """Intervals a tangent pass over the union of the root cones keeps live: each
    operation's value from its node to its last reader (a root is consumed where it is
    computed) with its structurally nonzero components in cmask."""
    ops, A, B = tape.nodes["op"], tape.nodes["a"], tape.nodes["b"]
    cone, stack = set(), [int(r) for r in tape.roots]
    while stack:
        x = stack.pop()
        if x not in cone:
            cone.add(x)
            if ops[x] >= I.ADD:
                stack.append(int(A[x]))
            if ops[x] in (I.ADD, I.SUB, I.MUL, I.DIV):
                stack.append(int(B[x]))
    order = sorted(x for x in cone if ops[x] not in (I.VAR, I.CONST))
    last = {}
    for x in order:
        for y in ([A[x], B[x]] if ops[x] in (I.ADD, I.SUB, I.MUL, I.DIV) else [A[x]]):
            last[int(y)] = max(last.get(int(y), -1), x)
    return max((sum(1 + bin(dep[y] & cmask).count("1") for y in order if y <= x and last.get(y, y) >= x)
                for x in order), default=1)


def _default_chunk(tape, limit=100):
    """The fewest tangent passes whose live intervals stay within the limit."""
    n, dep = tape.n_vars, _deps(tape)
    for passes in range(1, n + 1):
        c = -(-n // passes)
        peak = max(_peak_live(tape, ((1 << min(c, n - c0)) - 1) << c0, dep) for c0 in range(0, n, c))
        if peak <= limit:
            return c
    return 1


@pytest.mark.parametrize("name", ["cubic", "every form", "tiny", "random", "trig"])
def test_generated_source_compiles(name):
    tape = {"cubic": I.cubic_tape, "every form": _every_form, "tiny": lambda: I.tiny(1).tape,
            "random": lambda: I.random_small_tape(5, n=4, ops=60, n_con=2, con_ops=20, window=8),
            "trig": _trig}[name]()
    st = mvf.check(tape)
    info = mvf.spec_check(tape)
    n = tape.n_vars
    assert info["chunk"] == _default_chunk(tape) == n        # small live sets: one pass
    assert info["code_units"] == st.n_instr * (2 + -(-n // info["chunk"]))
    assert info["code_bytes"] > 0 and info["from_cache"] == 0 and info["waves"] == 2


def test_default_chunk_follows_the_live_set():
    # mid's live set fits one pass of all six components; the tanh network's dense layers
    # keep 16 values with 4 components each live, so it takes two passes of two.  The plan
    # (chunk and size) is made before the size limit refuses the tape.
    for tape, want in ((I.mid(1).tape, 6), (I.ann(1).tape, 2)):
        assert _default_chunk(tape) == want
        with pytest.raises(mvf.MVFError):
            mvf.spec_check(tape, grad="fwd", max_code=10)
        units = mvf.check(tape).n_instr * (2 + -(-tape.n_vars // want))
        assert f"{units} instruction-passes" in mvf.lib().mvf_last_error().decode()


def test_structurally_zero_components_are_not_computed(tmp_path, monkeypatch):
    # f = x0 x1 + sqr(x2) depends on every variable, g = exp(x0) only on x0: g's tangent pass
    # hands back exact zeros for x1 and x2 and the MVF combine of g skips them
    V = I.VAR
    t = _tape([(V, 0, -1), (V, 1, -1), (V, 2, -1), (I.MUL, 0, 1), (I.SQR, 2, -1), (I.ADD, 3, 4),
               (I.EXP, 0, -1)], [], [5, 6], 3)
    dump = tmp_path / "g.hip"
    monkeypatch.setenv("MVF_SPEC_DUMP", str(dump))
    info = mvf.spec_check(t, grad="fwd")
    assert info["chunk"] == 3
    src = dump.read_text()
    funcs = {f.split("(")[0].split()[-1]: f for f in src.split("__device__")[1:]}
    g_pass = funcs["tangent_1_0"]
    assert "G[1] = kZero;" in g_pass and "G[2] = kZero;" in g_pass and "G[0] = kZero;" not in g_pass
    lane = funcs["lane<false>"]
    root1 = lane[lane.index("tangent_1_0"):]
    assert "spec_dx(L, 0)" in root1 and "spec_dx(L, 1)" not in root1 and "spec_dx(L, 2)" not in root1
    f_pass = funcs["tangent_0_0"]
    assert "kZero;" not in f_pass.split("return")[0].split("G[0]")[-1]       # f: no zero component
    assert "utangent_0" not in funcs                                        # disjoint cones: a pass per root


def test_roots_sharing_nodes_take_passes_over_the_union(tmp_path, monkeypatch):
    # the product x0 x1 feeds f = x0 x1 + sqr(x2) and g = exp(x0) + x0 x1: one centre pass and
    # one tangent pass over both cones compute it once, and g's terms skip component 2
    V = I.VAR
    t = _tape([(V, 0, -1), (V, 1, -1), (V, 2, -1), (I.MUL, 0, 1), (I.SQR, 2, -1), (I.ADD, 3, 4),
               (I.EXP, 0, -1), (I.ADD, 6, 3)], [], [5, 7], 3)
    dump = tmp_path / "u.hip"
    monkeypatch.setenv("MVF_SPEC_DUMP", str(dump))
    info = mvf.spec_check(t, grad="fwd")
    st = mvf.check(t)
    assert info["code_units"] < st.n_instr * (2 + 1)                          # the shared product once per pass
    src = dump.read_text()
    funcs = {f.split("(")[0].split()[-1]: f for f in src.split("__device__")[1:]}
    assert "tangent_0_0" not in funcs and "point_0" not in funcs
    u = funcs["utangent_0"]
    g_terms = u[u.index("nie[1] ="):].split("}")[0]
    assert "spec_dx(L, 0)" in g_terms and "spec_dx(L, 1)" in g_terms and "spec_dx(L, 2)" not in g_terms
    f_terms = u[u.index("nie[0] ="):].split("}")[0]
    assert all(f"spec_dx(L, {i})" in f_terms for i in range(3)) and f_terms.count("acc[0] = iadd(") == 3


def test_chunk_and_waves_options():
    t = I.random_small_tape(6, n=5, ops=30, n_con=1, con_ops=10, window=8)
    st = mvf.check(t)
    for chunk in (1, 2, 5):
        info = mvf.spec_check(t, chunk=chunk, waves=1)
        assert info["chunk"] == chunk and info["waves"] == 1
        assert info["code_units"] == st.n_instr * (2 + -(-5 // chunk))


def test_bad_options_and_size_limit():
    t = I.random_small_tape(6, n=5, ops=30, n_con=1, con_ops=10, window=8)
    for kw in ({"chunk": 6}, {"waves": 5}):
        with pytest.raises(mvf.MVFError) as e:
            mvf.spec_check(t, **kw)
        assert e.value.code == -1
    with pytest.raises(mvf.MVFError) as e:
        mvf.spec_check(t, max_code=10)
    assert e.value.code == -3 and "instruction-passes" in mvf.lib().mvf_last_error().decode()
    # the plan (and the size limit) is checked before anything is generated: the 32-variable
    # workload's tangent mode (3,286 instructions, 32 components) is far above the default limit
    with pytest.raises(mvf.MVFError) as e:
        mvf.spec_check(I.diff(1).tape, grad="fwd")
    assert e.value.code == -3


def test_both_gradient_modes_compile_and_are_counted():
    t = _trig()
    st = mvf.check(t)
    for grad, extra in (("fwd", None), ("rev", 2), ("auto", None)):
        info = mvf.spec_check(t, grad=grad, ckpt_budget=-1)
        passes = -(-t.n_vars // info["chunk"])
        # a centre and a value pass per root; forward: the tangent passes; reverse: the
        # adjoint's value pass and its sweep
        want = st.n_instr * (2 + (passes if grad != "rev" else 0) + (2 if grad != "fwd" else 0))
        assert info["code_units"] == want and info["grad"] == {"fwd": 0, "rev": 1, "auto": 2}[grad]
        assert info["ckpt_intervals"] == 0


def test_checkpointed_adjoint_plan_and_size():
    # a 150-op objective cut into segments: the adjoint recomputes all but the last segment
    # (at most one extra pass), stores checkpoints only for segments 1 .. K-2, and a larger
    # budget never needs more segments
    t = I.random_small_tape(3, n=3, ops=150, n_con=1, con_ops=20, window=8)
    st = mvf.check(t)
    one = mvf.spec_check(t, grad="rev", ckpt_budget=-1)
    assert one["code_units"] == 4 * st.n_instr and one["ckpt_intervals"] == 0
    prev = None
    for budget in (4, 8, 16, 32):
        info = mvf.spec_check(t, grad="rev", ckpt_budget=budget)
        assert info["ckpt_budget"] == budget
        assert 4 * st.n_instr < info["code_units"] <= 5 * st.n_instr
        assert info["ckpt_intervals"] > 0
        if prev is not None:
            assert info["code_units"] <= prev["code_units"] + st.n_instr
        prev = info


def test_adjoint_settings_outside_the_verified_range_are_refused():
    # segment budgets above 32 (40 and 58 on the 32-variable workload) and the adjoint at one
    # wave per SIMD failed on the GPU without a cause found (wrong bounds, a memory fault): the
    # library refuses them
    t = I.random_small_tape(6, n=5, ops=30, n_con=1, con_ops=10, window=8)
    for kw in ({"grad": "rev", "ckpt_budget": 33}, {"grad": "rev", "waves": 1}, {"grad": "auto", "waves": 1}):
        with pytest.raises(mvf.MVFError) as e:
            mvf.spec_source(t, **kw)
        assert e.value.code == -1, kw
    assert mvf.spec_source(t, grad="fwd", waves=1)                 # tangent mode alone is built at one wave
    assert mvf.spec_source(t, grad="rev", ckpt_budget=32)


@pytest.mark.parametrize("name", ["mid", "batch", "diff"])
def test_tape_stats_report_the_generated_checkpoint_plan(name):
    # the plan that mvf_tape_check / mvf_tape_stats_get report at load is the one the
    # generator writes: segments, intervals stored by the value pass and loaded by the sweep
    import re
    t = {"mid": lambda: I.mid(1).tape, "batch": lambda: I.batch(1).tape, "diff": lambda: I.diff(1).tape}[name]()
    st = mvf.check(t)
    src = mvf.spec_source(t, grad="rev", max_code=10 ** 7)
    segs = sum(int(k) for k, _ in re.findall(r"// (\d+) segment\(s\), (\d+) checkpoint intervals", src))
    assert (st.ckpt_segments, st.ckpt_stored, st.ckpt_loaded) == (
        segs, len(re.findall(r"spec_ck_st\(L,", src)), len(re.findall(r"spec_ck_ld\(L,", src)))
    if name == "mid":
        assert st.ckpt_stored == 0 and st.ckpt_segments == t.n_roots      # short roots: one pass each
    else:
        assert st.ckpt_loaded >= st.ckpt_stored > 0
