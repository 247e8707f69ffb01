"""The seeded input generator: range, determinism, edge injection."""

import numpy as np

import gfp_inputs as gi
from oracle.field import GFPField, P8, P16


def test_digits_in_range_and_deterministic():
    for params in (P8, P16):
        k, r = params["k"], params["r"]
        a = gi.uniform_digits(k, r, 5000, seed=1, stream=0)
        b = gi.uniform_digits(k, r, 5000, seed=1, stream=0)
        c = gi.uniform_digits(k, r, 5000, seed=1, stream=1)
        assert a.shape == (k, 5000) and a.dtype == np.uint64
        assert (a < np.uint64(r)).all()
        assert np.array_equal(a, b) and not np.array_equal(a, c)
        # top bit is used: digits are not confined to a smaller range
        assert int(a.max()) > r // 2


def test_edge_patterns_are_canonical_and_distinct():
    for params in (P8, P16, dict(k=4, r=4)):
        F = GFPField(**params)
        pats = gi.edge_patterns(F.k, F.r)
        vals = [F.to_int(p) for p in pats]
        assert all(F.is_canonical(p) for p in pats)
        assert len(set(vals)) == len(vals)
        assert F.p - 1 in vals and 0 in vals and 1 in vals


def test_inject_edges():
    k, r = P8["k"], P8["r"]
    x = gi.operand(k, r, 1000, seed=3, stream=0, edge_frac=0.02)
    F = GFPField(**P8)
    cols = [F.to_int([int(x[d, i]) for d in range(k)]) for i in range(1000)]
    assert F.p - 1 in cols and 0 in cols
    assert all(F.is_canonical([int(x[d, i]) for d in range(k)]) for i in range(1000))
