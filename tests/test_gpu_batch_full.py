"""The batch workload at full size (512 nodes of [-3,3]^8 from random bisections,
2^10..2^18 subdomains each, 24.7 M subdomains; a 400-op objective and two
150-op constraints) through the batched graph in the autotuned configuration,
in both gradient modes, against the oracle.

Every node's reduced bounds must equal the single-box call's bit for bit;
single-box calls on sampled nodes are compared with the oracle: every
subdomain of the small nodes (2^10 subdomains: full hulls, argmin and the two
branch-and-bound bounds) and sampled subdomains of the largest node.  The tape
has exp and log, so the oracle is met within 1e-12 of the root's scale."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_20769_amd import inputs as I

from gpu_util import assert_parity, gpu_bound, scale_of

pytestmark = pytest.mark.gpu

KINDS = [0, 1, 1]


@pytest.fixture(scope="module")
def batch_setup():
    import torch
    from paper_2507_20769_amd import mvf
    bw = I.batch(1)
    h = mvf.Tape(bw.tape)
    h.set_root_kinds(KINDS)
    info = h.specialize(grad="auto")
    print(f"[spec] batch compile={info['seconds']:.1f}s cached={info['from_cache']}", flush=True)
    yield bw, h
    h.close()


@pytest.mark.parametrize("grad", ["fwd", "rev"])
def test_full_batch_tuned_graph_against_oracle(batch_setup, grad):
    import torch
    from paper_2507_20769_amd import mvf
    bw, h = batch_setup
    total = int(bw.n_sub.sum())
    # tune on a seeded sample of 64 nodes, then run all 512 nodes in one graph replay
    rng = np.random.default_rng(11)
    pick = np.sort(rng.choice(len(bw.boxes), 64, replace=False))
    tu = mvf.autotune(h, torch.tensor(bw.boxes[pick], device="cuda"), torch.tensor(bw.splits[pick], device="cuda"),
                      mode="both", grad=grad)
    print(f"[case] grad={grad} tuning={tu}", flush=True)
    g = mvf.BatchGraph(h, len(bw.boxes), total, mode="both", grad=grad, tuning=tu)
    g.launch(bw.boxes, bw.splits)
    torch.cuda.synchronize()
    red, am, st = g.result()
    ex = g.extra()
    g.close()
    assert not st.any()
    S = bw.n_sub
    small = [int(i) for i in np.flatnonzero(S == S.min())[:4]]
    big = int(np.argmax(S))
    nie = O.MODE_NIE
    for i in small + [big]:
        one = gpu_bound(bw.tape, bw.boxes[i], bw.splits[i], mode="both", grad=grad, handle=h,
                        per_sub=(i == big))
        assert np.array_equal(red[i], one["reduced"]) and am[i] == int(one["argmin"][0]), f"node {i}"
        assert np.array_equal(ex[i], one["extra"]), f"node {i}"
        og = O.GRAD_FWD if grad == "fwd" else O.GRAD_REV
        if i == big:
            ks = np.unique(np.concatenate([rng.choice(int(S[i]), 64, replace=False), [0, int(S[i]) - 1]]))
            o = O.bound(bw.tape, bw.boxes[i], bw.splits[i], mode=O.MODE_BOTH, grad=og, ks=ks, nthreads=8,
                        kinds=KINDS)
            sc = scale_of(O.bound(bw.tape, bw.boxes[i], bw.splits[i], mode=nie, ks=ks, per_sub=False,
                                  nthreads=8)["reduced"])
            assert_parity(one["per_sub"][:, :, ks], o["per_sub"], False, sc, f"node {i} sampled vs oracle")
        else:
            o = O.bound(bw.tape, bw.boxes[i], bw.splits[i], mode=O.MODE_BOTH, grad=og, per_sub=False,
                        nthreads=8, kinds=KINDS)
            sc = scale_of(O.bound(bw.tape, bw.boxes[i], bw.splits[i], mode=nie, per_sub=False,
                                  nthreads=8)["reduced"])
            assert_parity(red[i], o["reduced"], False, sc, f"node {i} hull vs oracle")
            assert_parity(ex[i], o["extra"], False, sc[0], f"node {i} extras vs oracle")
            if am[i] != o["argmin"]:
                # exp and log come from different libraries: the GPU's argmin must then be a near-tie,
                # its subdomain's lower bound (by the oracle) within the tolerance of the node's minimum
                at = O.bound(bw.tape, bw.boxes[i], bw.splits[i], mode=O.MODE_BOTH, grad=og, ks=[int(am[i])],
                             nthreads=1, kinds=KINDS)["per_sub"][0, 0, 0]
                assert abs(at - o["reduced"][0, 0]) <= 1e-12 * sc[0], f"node {i} argmin"
