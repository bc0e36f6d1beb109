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


@pytest.mark.parametrize("name", ["cubic", "every form", "tiny", "random", "trig"])
def test_generated_source_compiles(name):
    tape = {"cubic": I.cubic_tape, "every form": _every_form, "tiny": lambda: I.tiny(1).tape,
            "random": lambda: I.random_small_tape(5, n=4, ops=60, n_con=2, con_ops=20, window=8),
            "trig": _trig}[name]()
    st = mvf.check(tape)
    info = mvf.spec_check(tape)
    n = tape.n_vars
    passes = (n + 2) // 3
    assert info["chunk"] == (n + passes - 1) // passes
    assert info["code_units"] == st.n_instr * (2 + -(-n // info["chunk"]))
    assert info["code_bytes"] > 0 and info["from_cache"] == 0 and info["waves"] == 2


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
    # the e2e tape is above the default size limit
    with pytest.raises(mvf.MVFError) as e:
        mvf.spec_check(I.e2e_tape(1))
    assert e.value.code == -3


def test_both_gradient_modes_compile_and_are_counted():
    t = _trig()
    st = mvf.check(t)
    for grad, extra in (("fwd", None), ("rev", 2), ("auto", None)):
        info = mvf.spec_check(t, grad=grad)
        passes = -(-t.n_vars // info["chunk"])
        want = st.n_instr * (2 + (passes if grad != "rev" else 0) + (2 if grad != "fwd" else 0))
        assert info["code_units"] == want and info["grad"] == {"fwd": 0, "rev": 1, "auto": 2}[grad]
