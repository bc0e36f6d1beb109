"""mvf_bound_noalloc, the entry point for callers that cannot allocate device
memory, against mvf_bound: same kernels, same bits, on two calls in a row
(the second on a smaller input, so the shared device scratch holds the first
call's contents), through the C ABI."""
import numpy as np
import pytest

from paper_2507_20769_amd import inputs as I

pytestmark = pytest.mark.gpu


def _run(h, box, splits, grad, engine, noalloc):
    import torch
    from paper_2507_20769_amd import mvf
    c = mvf.BoundCall(h, box, splits, mode="both", grad=grad, per_sub=True, flags=True, engine=engine,
                      noalloc=noalloc)
    c.launch()
    torch.cuda.synchronize()
    return {k: getattr(c, k).cpu().numpy() for k in ("reduced", "argmin", "per_sub", "flags", "extra")}


@pytest.mark.parametrize("grad,engine", [("fwd", "spec"), ("fwd", "interp"), ("rev", "spec")])
def test_noalloc_equals_bound_on_two_calls(grad, engine):
    import torch
    from paper_2507_20769_amd import mvf
    w = I.mid(1)
    h = mvf.Tape(w.tape)
    if engine == "spec":
        h.specialize(grad=grad)
    box = torch.tensor(w.box, device="cuda")
    for splits in (w.splits, [4, 3, 5, 2, 3, 1]):             # 262,144 then 360 subdomains
        print(f"[case] grad={grad} engine={engine} splits={list(splits)}", flush=True)
        a = _run(h, box, splits, grad, engine, noalloc=False)
        b = _run(h, box, splits, grad, engine, noalloc=True)
        for k in a:
            assert np.array_equal(a[k], b[k], equal_nan=True), k
    h.close()


def test_noalloc_rejects_calls_beyond_its_scratch():
    # the interpreter's reverse-mode record tape of mid needs far more than the 8 MiB array
    import torch
    from paper_2507_20769_amd import mvf
    w = I.mid(1)
    h = mvf.Tape(w.tape)
    box = torch.tensor(w.box, device="cuda")
    with pytest.raises(mvf.MVFError) as e:
        mvf.BoundCall(h, box, w.splits, mode="both", grad="rev", engine="interp", noalloc=True).launch()
    assert e.value.code == -3 and "bytes" in mvf.lib().mvf_last_error().decode()
    h.close()
