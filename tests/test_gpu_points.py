"""GPU parity of the point and box entry points (values and vector-Jacobian
products at points, interval gradients on boxes) against the oracle, and the
torch.autograd.Function built on them against finite differences and an
independent reference gradient (plain torch autograd on the CPU)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_20769_amd import inputs as I

from gpu_util import assert_parity, has_transcendental

pytestmark = pytest.mark.gpu


def _rational(t):
    nodes = t.nodes.copy()
    nodes["op"][nodes["op"] == I.EXP] = I.SQR
    nodes["op"][nodes["op"] == I.LOG] = I.SQRT
    return I.Tape(nodes, t.consts, t.roots, t.n_vars)


def _shared_tape():
    # x*x (same operand twice), x/x, a variable root, a constant root, a root that
    # another root uses, a repeated root
    nodes = [(I.VAR, 0, -1), (I.VAR, 1, -1), (I.MUL, 0, 0), (I.ADD, 2, 1), (I.MUL, 3, 3), (I.CONST, 0, -1),
             (I.CONST, 1, -1), (I.ADD, 5, 6), (I.MUL, 4, 7), (I.SUB, 8, 8), (I.ADD, 9, 4), (I.DIV, 10, 1),
             (I.SQRT, 11, -1), (I.MUL, 12, 4)]
    return I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.array([1.5, -0.25]),
                  np.array([10, 0, 5, 13, 4, 4], dtype=np.int32), 2)


def _tapes():
    yield "random rational", _rational(I.random_small_tape(21, n=4, ops=90, n_con=2, con_ops=30, window=8))
    yield "random exp/log", I.random_small_tape(22, n=3, ops=70, n_con=2, con_ops=25, window=8)
    yield "shared operands and leaf roots", _shared_tape()


def _scale(a, b):
    m = np.concatenate([np.abs(a[np.isfinite(a)]), np.abs(b[np.isfinite(b)]), [1.0]])
    return float(m.max())


@pytest.mark.parametrize("B", [1, 257, 1000])
def test_eval_and_vjp_points_match_oracle(B):
    import torch
    from paper_2507_20769_amd import mvf
    for name, tape in _tapes():
        print(f"[case points] {name} B={B}", flush=True)
        box = np.array([[0.5, 2.0]] * tape.n_vars)
        x = I.random_points(B, box, B)
        g = np.random.default_rng(B).uniform(-1, 1, (B, tape.n_roots))
        h = mvf.Tape(tape)
        f, fl = mvf.eval_points(h, torch.tensor(x, device="cuda"), flags=True)
        gx, gfl = mvf.vjp_points(h, torch.tensor(x, device="cuda"), torch.tensor(g, device="cuda"), flags=True)
        torch.cuda.synchronize()
        f, gx = f.cpu().numpy(), gx.cpu().numpy()
        fo = O.eval_points(tape, x)
        go = O.vjp_points(tape, x, g)
        exact = not has_transcendental(tape)
        assert_parity(f, fo, exact, _scale(f, fo), f"{name} eval")
        assert_parity(gx, go, exact, _scale(gx, go), f"{name} vjp")
        assert np.array_equal(fl.cpu().numpy(), gfl.cpu().numpy())
        h.close()


def test_points_domain_violation_and_empty_batch():
    import torch
    from paper_2507_20769_amd import mvf
    # f = log(x0) + sqrt(x1): points with x0 <= 0 or x1 < 0 are flagged
    nodes = [(I.VAR, 0, -1), (I.VAR, 1, -1), (I.LOG, 0, -1), (I.SQRT, 1, -1), (I.ADD, 2, 3)]
    tape = I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.zeros(0), np.array([4], dtype=np.int32), 2)
    x = np.array([[1.0, 1.0], [-1.0, 1.0], [1.0, -1.0], [2.0, 4.0]])
    h = mvf.Tape(tape)
    f, fl = mvf.eval_points(h, torch.tensor(x, device="cuda"), flags=True)
    gx = mvf.vjp_points(h, torch.tensor(x, device="cuda"), torch.ones((4, 1), dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert fl.cpu().numpy().tolist() == [0, 1, 1, 0]
    f, gx = f.cpu().numpy(), gx.cpu().numpy()
    assert np.isneginf(f[1:3, 0, 0]).all() and np.isposinf(f[1:3, 0, 1]).all()
    assert np.isneginf(gx[1:3, :, 0]).all() and np.isposinf(gx[1:3, :, 1]).all()
    fo = O.eval_points(tape, x)
    assert_parity(f, fo, False, _scale(f, fo), "domain eval")
    # an empty batch is a no-op
    e = mvf.eval_points(h, torch.zeros((0, 2), dtype=torch.float64, device="cuda"))
    assert tuple(e.shape) == (0, 1, 2)
    h.close()


@pytest.mark.parametrize("grad", ["fwd", "rev"])
def test_gradient_boxes_match_oracle(grad):
    import torch
    from paper_2507_20769_amd import mvf
    for name, tape in _tapes():
        rng = np.random.default_rng(5)
        B = 300
        lo = rng.uniform(0.3, 1.5, (B, tape.n_vars))
        boxes = np.stack([lo, lo + rng.uniform(0.0, 0.5, (B, tape.n_vars))], axis=2)
        boxes[0, :, 1] = boxes[0, :, 0]                      # a degenerate box
        h = mvf.Tape(tape)
        exact = not has_transcendental(tape)
        for r in range(tape.n_roots):
            print(f"[case grad] {name} root={r} grad={grad}", flush=True)
            G = mvf.gradient_boxes(h, torch.tensor(boxes, device="cuda"), root=r, grad=grad)
            torch.cuda.synchronize()
            G = G.cpu().numpy()
            Go, _ = O.gradient_boxes(tape, boxes, r, O.GRAD_FWD if grad == "fwd" else O.GRAD_REV)
            assert_parity(G, Go, exact, _scale(G, Go), f"{name} root {r} {grad}")
            # forward and reverse enclosures of the same gradient set intersect
            Gf, _ = O.gradient_boxes(tape, boxes, r, O.GRAD_FWD)
            fin = np.isfinite(G).all(axis=2) & np.isfinite(Gf).all(axis=2)
            assert (np.maximum(G[..., 0], Gf[..., 0]) <= np.minimum(G[..., 1], Gf[..., 1]))[fin].all()
        h.close()


def _torch_reference(tape, x):
    """f_r(x) for every root with plain torch float64 ops (a reference
    evaluation independent of the library and the oracle)."""
    import torch
    vals = []
    for (op, a, b) in tape.nodes.tolist():
        if op == I.VAR:
            v = x[:, a]
        elif op == I.CONST:
            v = torch.full((x.shape[0],), float(tape.consts[a]), dtype=torch.float64)
        elif op == I.ADD:
            v = vals[a] + vals[b]
        elif op == I.SUB:
            v = vals[a] - vals[b]
        elif op == I.MUL:
            v = vals[a] * vals[b]
        elif op == I.DIV:
            v = vals[a] / vals[b]
        elif op == I.SQR:
            v = vals[a] * vals[a]
        elif op == I.SQRT:
            v = torch.sqrt(vals[a])
        elif op == I.EXP:
            v = torch.exp(vals[a])
        else:
            v = torch.log(vals[a])
        vals.append(v)
    return torch.stack([vals[r] for r in tape.roots.tolist()], dim=1)


def test_autograd_function_on_the_differentiation_workload():
    """32 variables, five roots, 1,024 seeded points: the backward pass of the
    autograd Function against central differences (h = 1e-6) and against
    torch autograd of a plain float64 evaluation."""
    import torch
    from paper_2507_20769_amd import mvf
    w = I.diff(1)
    tape = w.tape
    n, m, P = tape.n_vars, tape.n_roots, 1024
    x = I.random_points(7, w.box, P)
    wts = np.random.default_rng(8).uniform(-1.0, 1.0, m)
    h = mvf.Tape(tape)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    y = mvf.point_function(h, xt)
    assert tuple(y.shape) == (P, m)
    (y * torch.tensor(wts, device="cuda")).sum().backward()
    g = xt.grad.cpu().numpy()

    # values against the float64 reference
    xr = torch.tensor(x, requires_grad=True)
    yr = _torch_reference(tape, xr)
    S = np.abs(yr.detach().numpy()).max(axis=0)
    assert np.all(np.abs(y.detach().cpu().numpy() - yr.detach().numpy()) <= 1e-9 * np.maximum(1.0, S))
    # gradient against torch autograd of the reference
    (yr * torch.tensor(wts)).sum().backward()
    gr = xr.grad.numpy()
    Sg = np.abs(gr).max()
    assert np.all(np.abs(g - gr) <= 1e-9 * max(1.0, Sg)), np.abs(g - gr).max()

    # central differences of the library's own values, h = 1e-6
    hstep = 1e-6
    xp = np.repeat(x[:, None, :], n, axis=1)
    xm = xp.copy()
    idx = np.arange(n)
    xp[:, idx, idx] += hstep
    xm[:, idx, idx] -= hstep
    fp = mvf.eval_points(h, torch.tensor(xp.reshape(-1, n), device="cuda")).cpu().numpy()
    fm = mvf.eval_points(h, torch.tensor(xm.reshape(-1, n), device="cuda")).cpu().numpy()
    mid = lambda a: 0.5 * a[..., 0] + 0.5 * a[..., 1]
    fd = ((mid(fp) - mid(fm)).reshape(P, n, m) @ wts) / (2 * hstep)
    S_r = np.abs(mid(fp)).max()
    assert np.all(np.abs(fd - g) <= 1e-6 * np.maximum(1.0, np.abs(g)) + 1e-6 * S_r), np.abs(fd - g).max()
    h.close()


def test_autograd_gradcheck_small_tape():
    import torch
    from paper_2507_20769_amd import mvf
    h = mvf.Tape(_rational(I.random_small_tape(23, n=3, ops=40, n_con=1, con_ops=12, window=6)))
    x = torch.tensor(I.random_points(3, np.array([[0.5, 1.5]] * 3), 6), device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda z: mvf.point_function(h, z), (x,), eps=1e-6, atol=1e-6, rtol=1e-4)
    h.close()
