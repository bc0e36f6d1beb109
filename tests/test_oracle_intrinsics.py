"""Pins of the oracle's tanh, sin and cos (the intrinsics of the paper's ANN
workloads and trigonometric test problems): the padded library values
enclose 60-digit decimal values, the extremum rule of sin and cos matches
the places where the functions reach +-1, enclosures contain densely sampled
values, and interval gradients through these functions enclose finite
differences."""
import decimal
import functools
import math

import numpy as np

from oracle import oracle as O
from paper_2507_20769_amd import inputs as I

TANH, SIN, COS = 10, 11, 12
D = decimal.Decimal


@functools.lru_cache(maxsize=None)
def _pi():
    """pi to the context precision (Machin's formula)."""
    def arctan_inv(x):
        x = D(x)
        s, term, k, x2 = D(0), D(1) / x, 0, x * x
        while True:
            t = term / (2 * k + 1)
            if t == 0:
                return s
            s += t if k % 2 == 0 else -t
            term /= x2
            k += 1
    return 16 * arctan_inv(5) - 4 * arctan_inv(239)


def _sin_cos(x):
    """(sin x, cos x) of a double by range reduction with the decimal pi and Taylor series."""
    pi = _pi()
    y = D(float(x))
    k = (y / (2 * pi)).to_integral_value()
    y -= k * 2 * pi
    s, c, term = D(0), D(0), D(1)
    for n in range(90):                           # term = y^n / n!, |y| <= pi: 90 terms reach 1e-70
        if n % 4 == 0:
            c += term
        elif n % 4 == 1:
            s += term
        elif n % 4 == 2:
            c -= term
        else:
            s -= term
        term = term * y / (n + 1)
    return s, c


def _encloses(z, t):
    return D(float(z[0])) <= t <= D(float(z[1]))


def _tanh(a):
    y = D(float(a))
    if abs(y) < D("1e-8"):                        # the series: no cancellation near 0
        return y - y ** 3 / 3 + 2 * y ** 5 / 15
    e2 = (2 * y).exp()
    return (e2 - 1) / (e2 + 1)


def test_tanh_sin_cos_pad_enclose_high_precision_values():
    decimal.getcontext().prec = 60
    rng = np.random.default_rng(21)
    pts = np.concatenate([rng.uniform(-10, 10, 60), rng.uniform(-1e4, 1e4, 20), [0.0, 1e-300, -1e-300, 0.5, 40.0, -40.0]])
    for a in pts:
        assert _encloses(O.interval_op(TANH, [a, a]), _tanh(a)), a
        s, c = _sin_cos(a)
        assert _encloses(O.interval_op(SIN, [a, a]), s), a
        assert _encloses(O.interval_op(COS, [a, a]), c), a


def test_tanh_is_clamped_and_monotone():
    assert O.interval_op(TANH, [20.0, 30.0]).tolist()[1] == 1.0
    assert O.interval_op(TANH, [-30.0, -20.0]).tolist()[0] == -1.0
    z = O.interval_op(TANH, [-0.5, 0.25])
    assert z[0] <= math.tanh(-0.5) <= z[1] and z[0] <= math.tanh(0.25) <= z[1]
    assert z[1] < math.tanh(0.26) and z[0] > math.tanh(-0.51)      # no wider than the endpoint values need


def test_sin_cos_extrema():
    pi = math.pi
    # an interior maximum or minimum reaches exactly +-1
    assert O.interval_op(SIN, [1.0, 2.0])[1] == 1.0                 # pi/2 inside
    assert O.interval_op(SIN, [4.0, 5.0])[0] == -1.0                # 3 pi/2 inside
    assert O.interval_op(COS, [-0.1, 0.1])[1] == 1.0                # 0 inside
    assert O.interval_op(COS, [3.0, 3.3])[0] == -1.0                # pi inside
    assert O.interval_op(SIN, [1.0 + 200 * pi, 2.0 + 200 * pi])[1] == 1.0
    # none inside: both ends come from the endpoint values
    z = O.interval_op(SIN, [-0.5, 0.5])
    assert -1 < z[0] < -0.47 and 0.47 < z[1] < 1
    z = O.interval_op(COS, [0.5, 2.5])
    assert -1 < z[0] < math.cos(2.5) + 1e-12 and math.cos(0.5) - 1e-12 < z[1] < 1
    # a full period or more
    assert O.interval_op(SIN, [0.0, 6.3]).tolist() == [-1.0, 1.0]
    assert O.interval_op(COS, [-100.0, 100.0]).tolist() == [-1.0, 1.0]
    # an interval that just misses pi/2 is not widened to 1
    z = O.interval_op(SIN, [0.0, 1.5])
    assert z[1] < 1.0 and z[1] >= math.sin(1.5)


def test_sin_cos_tanh_enclose_dense_samples():
    rng = np.random.default_rng(22)
    for _ in range(300):
        a = rng.uniform(-20, 20)
        w = 10 ** rng.uniform(-6, 0.9)
        xs = np.linspace(a, a + w, 2001)
        for op, f in ((TANH, np.tanh), (SIN, np.sin), (COS, np.cos)):
            z = O.interval_op(op, [a, a + w])
            v = f(xs)
            assert z[0] <= v.min() + 1e-15 and v.max() - 1e-15 <= z[1], (op, a, w)


def _trig_tape():
    # f = tanh(x0 * x1) + sin(3 x0) * cos(x1),  g = cos(x0) - x1
    V, C = I.VAR, I.CONST
    nodes = [(V, 0, -1), (V, 1, -1), (C, 0, -1), (I.MUL, 0, 1), (I.TANH, 3, -1), (I.MUL, 2, 0), (I.SIN, 5, -1),
             (I.COS, 1, -1), (I.MUL, 6, 7), (I.ADD, 4, 8), (I.COS, 0, -1), (I.SUB, 10, 1)]
    return I.Tape(np.array(nodes, dtype=I.NODE_DTYPE), np.array([3.0]), np.array([9, 11], dtype=np.int32), 2)


def test_bounds_on_trig_and_ann_tapes_enclose_samples():
    rng = np.random.default_rng(23)
    for tape, box, splits in ((_trig_tape(), np.array([[-1.0, 2.0], [-2.0, 1.5]]), np.array([7, 5])),
                              (I.ann_tape(2, n_in=3, widths=(6, 5)), np.array([[-2.0, 2.0]] * 3), np.array([3, 4, 2]))):
        for grad in (O.GRAD_FWD, O.GRAD_REV):
            o = O.bound(tape, box, splits, mode=O.MODE_BOTH, grad=grad, nthreads=4)
            assert not o["flags"].any()
            S = int(np.prod(splits))
            for k in range(S):
                X, c = O.subdomain(box, splits, k)
                pts = X[:, 0] + (X[:, 1] - X[:, 0]) * rng.random((64, X.shape[0]))
                v = I.eval_points_np(tape, pts)
                assert np.all(o["per_sub"][:, 0, k] <= v.min(axis=0) + 1e-12)
                assert np.all(v.max(axis=0) - 1e-12 <= o["per_sub"][:, 1, k])


def test_gradients_through_trig_and_tanh_enclose_finite_differences():
    tape = _trig_tape()
    rng = np.random.default_rng(24)
    for _ in range(20):
        lo = rng.uniform(-2, 1, 2)
        box = np.stack([lo, lo + rng.uniform(0.01, 0.5, 2)], axis=1)
        for grad in (O.GRAD_FWD, O.GRAD_REV):
            Gs, fl = O.gradient_boxes(tape, box[None], 0, grad=grad)
            assert not fl.any()
            G = Gs[0]
            for _ in range(5):
                x = box[:, 0] + (box[:, 1] - box[:, 0]) * rng.random(2)
                for j in range(2):
                    h = 1e-6
                    xp, xm = x.copy(), x.copy()
                    xp[j] += h
                    xm[j] -= h
                    fd = (I.eval_points_np(tape, xp[None])[0, 0] - I.eval_points_np(tape, xm[None])[0, 0]) / (2 * h)
                    assert G[j, 0] - 1e-6 <= fd <= G[j, 1] + 1e-6, (grad, j)


def test_pow_expansion_matches_power():
    tb = I.TapeBuilder(1)
    x = tb.var(0)
    for k in (1, 2, 3, 5, 8, 13):
        tb.roots.append(tb.pow(x, k))
    t = tb.build()
    xs = np.linspace(-1.7, 1.9, 11)[:, None]
    v = I.eval_points_np(t, xs)
    assert np.allclose(v, xs ** np.array([1, 2, 3, 5, 8, 13]), rtol=1e-14)
    o = O.bound(t, np.array([[-1.7, 1.9]]), np.array([5]), mode=O.MODE_NIE, per_sub=False)
    assert np.all(o["reduced"][:, 0] <= v.min(axis=0)) and np.all(v.max(axis=0) <= o["reduced"][:, 1])
