"""Host logic of the split rules: the adaptive rule agrees with the oracle's
independent implementation (Sec. 3.1.2), and the doubling rule keeps its
invariants (power-of-two counts, within budget, maximal, widest relative
width first)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2507_20769_amd import mvf


def test_adaptive_rule_matches_the_oracle():
    rng = np.random.default_rng(3)
    for _ in range(200):
        n = int(rng.integers(1, 9))
        w = rng.uniform(0.01, 10.0, n)
        budget = int(rng.integers(1, 5000))
        s, c = mvf.splits("adaptive", w, budget)
        so, co = O.adaptive_splits(w, budget)
        assert c == co and s.tolist() == list(so)


def test_doubling_rule_invariants():
    rng = np.random.default_rng(4)
    for _ in range(200):
        n = int(rng.integers(1, 9))
        w = rng.uniform(0.01, 10.0, n)
        budget = int(rng.integers(1, 1 << 20))
        s, c = mvf.splits("doubling", w, budget)
        assert c == int(np.prod(s.astype(np.int64))) and c <= budget
        assert budget < 2 * c or (s > 32767).all()                  # maximal, up to the 65535 split cap
        assert all(int(x) & (int(x) - 1) == 0 for x in s)           # powers of two
        # replay: each step doubles the first dimension of largest w_i / s_i among those below the cap
        cur = np.ones(n, dtype=np.int64)
        while cur.prod() * 2 <= budget:
            r = np.where(cur <= 32767, w / cur, -np.inf)
            if not np.isfinite(r.max()):
                break
            cur[int(np.argmax(r))] *= 2
        assert s.tolist() == cur.tolist()


def test_split_rule_errors():
    out = np.zeros(2, dtype=np.int32)
    w = np.ones(2)
    assert mvf.lib().mvf_splits(7, 2, w.ctypes.data, 16, out.ctypes.data) == -1      # unknown rule
    assert mvf.lib().mvf_splits(1, 2, w.ctypes.data, 0, out.ctypes.data) == -1       # empty budget
