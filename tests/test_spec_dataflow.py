"""The checkpointed adjoint computes what the single-pass adjoint computes.

Both are generated as straight-line device code; executing them symbolically
(tests/spec_dataflow.py: every operation a hash-consed node over its operand
nodes) must give every root's returned value and every gradient component the
same expression node -- the same operations on the same operands in the same
order, hence the same bits on any device -- while the checkpointed form
stores each checkpoint index once, before it is loaded, and loads each one it
stores.
Host only (the generator's source through mvf_spec_source, nothing compiled)."""
import pytest

from paper_2507_20769_amd import inputs as I
from paper_2507_20769_amd import mvf

import spec_dataflow as D


def _check(tape, budget, waves=2):
    one = D.functions(mvf.spec_source(tape, grad="rev", ckpt_budget=-1, waves=waves, max_code=10 ** 7))
    ck = D.functions(mvf.spec_source(tape, grad="rev", ckpt_budget=budget, waves=waves, max_code=10 ** 7))
    g = D.Graph()
    stores = 0
    for r in range(tape.n_roots):
        ra, ga, Ma = D.run(one[f"adjoint_{r}"], g, tape.n_vars)
        rb, gb, Mb = D.run(ck[f"adjoint_{r}"], g, tape.n_vars)
        assert Ma.ck_stores == 0 and Ma.ck_loads == 0
        assert ra == rb, f"root {r}: value differs"
        assert ga == gb, f"root {r}: gradient components {[i for i in range(tape.n_vars) if ga[i] != gb[i]]} differ"
        assert all(x >= 0 for x in gb), f"root {r}: a gradient component is never written"
        # every checkpoint index is stored once (no value overwrites another) and read at least
        # once; a value several segments read is stored once and loaded by each of them
        assert Mb.ck_stores == len(Mb.ck) == len(Mb.ck_loaded) <= Mb.ck_loads
        stores += Mb.ck_stores
    return stores


@pytest.mark.parametrize("seed,budget", [(1, 3), (2, 6), (3, 12), (4, 24)])
def test_random_tapes(seed, budget):
    t = I.random_small_tape(seed, n=4, ops=150, n_con=2, con_ops=40, window=8)
    assert _check(t, budget) > 0


def test_reloads_recompute_cheap_values_and_share_stores():
    # the checked plans do exercise both economies: some reloaded inputs are recomputed from
    # variables and constants instead of loaded, and some stored value is loaded by more than
    # one segment (one store, several loads)
    import re
    t = I.random_small_tape(2, n=4, ops=150, n_con=2, con_ops=40, window=8)
    src = mvf.spec_source(t, grad="rev", ckpt_budget=6)
    reload_lines = [ln for ln in src.splitlines() if "spec_ck_ld" in ln]
    assert sum(len(re.findall(r"v\d+ = (?!spec_ck_ld)\w+\(", ln)) for ln in reload_lines) > 0
    assert len(re.findall(r"spec_ck_ld\(L,", src)) > len(re.findall(r"spec_ck_st\(L,", src))


@pytest.mark.parametrize("name,budget", [("mid", 32), ("batch", 0), ("e2e", 0), ("diff", 0), ("diff", 12)])
def test_workload_tapes(name, budget):
    # budget 0: the library's choice (mid's roots are short enough to stay single-pass there)
    t = {"mid": lambda: I.mid(1).tape, "batch": lambda: I.batch(1).tape, "e2e": lambda: I.e2e_tape(1),
         "diff": lambda: I.diff(1).tape}[name]()
    assert _check(t, budget) > 0


def test_the_check_sees_a_wrong_adjoint():
    # the symbolic comparison is not vacuous: dropping one contribution to the gradient
    # (its update assigned to a variable nobody reads) changes a gradient node
    import re
    t = I.random_small_tape(5, n=3, ops=60, n_con=1, con_ops=10, window=8)
    body = D.functions(mvf.spec_source(t, grad="rev", ckpt_budget=-1))["adjoint_0"]
    m = re.search(r"G\[(\d+)\] = i(add|sub)\(G\[\1\], ", body)
    assert m is not None
    broken = body[:m.start()] + "dropped" + body[m.start() + len(f"G[{m.group(1)}]"):]
    g = D.Graph()
    _, ga, _ = D.run(body, g, t.n_vars)
    _, gb, _ = D.run(broken, g, t.n_vars)
    assert ga != gb
