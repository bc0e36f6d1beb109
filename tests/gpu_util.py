"""Shared helpers of the GPU parity tests (device runs through the C ABI, comparison with the oracle)."""
import numpy as np

from oracle import oracle as O
from paper_2507_20769_amd import inputs as I


def has_transcendental(tape) -> bool:
    """Whether the tape calls a library function (exp log tanh sin cos): parity is then
    within 1e-12 of the root's scale, the two sides calling different libms."""
    ops = tape.nodes["op"]
    return bool(np.any(np.isin(ops, [I.EXP, I.LOG, I.TANH, I.SIN, I.COS])))


def gpu_bound(tape, box, splits, mode="both", grad="fwd", per_sub=True, flags=True, handle=None, engine="auto"):
    import torch
    from paper_2507_20769_amd import mvf
    t = handle if handle is not None else mvf.Tape(tape)
    dbox = torch.tensor(np.asarray(box, dtype=np.float64), device="cuda")
    out = mvf.bound(t, dbox, splits, mode=mode, grad=grad, per_sub=per_sub, flags=flags, engine=engine)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items() if k != "workspace"}
    if handle is None:
        t.close()
    return res


def scale_of(oracle_reduced: np.ndarray) -> np.ndarray:
    """S_r: the magnitude of root r's bounds on the node box (floor of the relative test)."""
    a = np.abs(oracle_reduced)
    a = np.where(np.isfinite(a), a, 0.0)
    return np.maximum(a.max(axis=1), 1e-300)


def assert_parity(gpu: np.ndarray, ref: np.ndarray, exact: bool, scale=None, what=""):
    """Bit-exact (==, so -0 == +0) for rational tapes; otherwise
    |a - b| <= 1e-12 * max(|a|, |b|, S_r) with S_r the root's scale."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    assert gpu.shape == ref.shape, (what, gpu.shape, ref.shape)
    same_inf = (gpu == ref) | (np.isnan(gpu) & np.isnan(ref))
    if exact:
        bad = ~same_inf
        assert not bad.any(), f"{what}: {bad.sum()} mismatches, first at {np.argwhere(bad)[0]}: " \
                              f"gpu {gpu[tuple(np.argwhere(bad)[0])]!r} ref {ref[tuple(np.argwhere(bad)[0])]!r}"
        return
    s = np.broadcast_to(np.asarray(scale)[(...,) + (None,) * (gpu.ndim - 1)], gpu.shape) if scale is not None else 0.0
    tol = 1e-12 * np.maximum(np.maximum(np.abs(gpu), np.abs(ref)), s)
    with np.errstate(invalid="ignore"):
        ok = same_inf | (np.abs(gpu - ref) <= tol)
    bad = ~ok
    assert not bad.any(), f"{what}: {bad.sum()} outside tolerance, first at {np.argwhere(bad)[0]}"
