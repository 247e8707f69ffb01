"""The multithreaded C++ CPU transform (the timed CPU baseline) against the
Python oracle: forward and inverse against the pinned radix-2 transform
(which is pinned against the DFT's definition), products against the
schoolbook product, on the workload primes, with edge values, at several
thread counts."""

import numpy as np
import pytest

import gfp_inputs as gi
from oracle import cpu_ntt
from oracle import transform as T
from oracle.field import GFPField, P8, P16, P32
from tests.helpers import canonical_mask, to_ints


@pytest.mark.parametrize("params,N", [(P8, 16), (P8, 256), (P8, 4096), (P16, 32), (P16, 1024), (P32, 64)])
@pytest.mark.parametrize("threads", [1, 3])
def test_transform_matches_oracle(params, N, threads):
    F = GFPField(**params)
    x = gi.operand(F.k, F.r, N, gi.BASE_SEED + 60 + N, 0, edge_frac=0.05)
    xi = to_ints(x, F.r)
    w = F.paper_root_of_unity(N)
    y = cpu_ntt.transform(F.k, F.r, x, w, threads=threads)
    assert canonical_mask(y, F.r).all()
    assert to_ints(y, F.r) == T.ntt(xi, w, F.p)
    winv = pow(w, F.p - 2, F.p)
    z = cpu_ntt.transform(F.k, F.r, x, winv, inverse=True, threads=threads)
    assert to_ints(z, F.r) == T.intt(xi, w, F.p)


@pytest.mark.parametrize("params", [P8, P16])
@pytest.mark.parametrize("la,lb", [(1, 1), (5, 3), (100, 157), (2048, 2048)])
def test_polymul_matches_schoolbook(params, la, lb):
    F = GFPField(**params)
    if F.k == 16 and la == 2048:
        la = lb = 300
    a = gi.operand(F.k, F.r, la, gi.BASE_SEED + 70 + la, 0, edge_frac=0.1)
    b = gi.operand(F.k, F.r, lb, gi.BASE_SEED + 70 + la, 1, edge_frac=0.1)
    n = 1
    while n < max(la + lb - 1, 2):
        n *= 2
    w = F.paper_root_of_unity(max(n, 2 * F.k))
    n = max(n, 2 * F.k)
    c = cpu_ntt.polymul(F.k, F.r, a, b, n, w, pow(w, F.p - 2, F.p), threads=4)
    assert canonical_mask(c, F.r).all()
    assert to_ints(c, F.r) == T.polymul(to_ints(a, F.r), to_ints(b, F.r), F.p)


def test_every_coefficient_p_minus_one():
    """Constant p - 1: transform (N (p - 1), 0, ..., 0), and p - 1 comes back
    in its (0, ..., 0, r) encoding."""
    F = GFPField(**P8)
    N = 64
    x = np.zeros((F.k, N), dtype=np.uint64)
    x[F.k - 1, :] = np.uint64(F.r)
    w = F.paper_root_of_unity(N)
    y = cpu_ntt.transform(F.k, F.r, x, w)
    got = to_ints(y, F.r)
    assert got[0] == (-N) % F.p and all(v == 0 for v in got[1:])
    back = cpu_ntt.transform(F.k, F.r, y, pow(w, F.p - 2, F.p), inverse=True)
    assert np.array_equal(back, x)


def test_bad_arguments_rejected():
    F = GFPField(**P8)
    with pytest.raises(ValueError):
        cpu_ntt.transform(F.k, F.r, np.zeros((F.k, 12), dtype=np.uint64), 1)


def _golden():
    import json
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sampled_fullsize.json")
    with open(path) as fh:
        return json.load(fh)


@pytest.mark.parametrize("key", ["k8-1048576", "k8-524288", "k16-1048576", "k32-262144"])
def test_fullsize_golden_agrees_with_cpu_transform(key):
    """The stored full-size expected values (Python oracle, Y_i = X(w^i) by
    blocked evaluation) agree with the whole transform computed by the C++
    oracle: two independent computations of the same definition."""
    g = _golden()["fft"][key]
    k, r, n = g["k"], g["r"], g["n"]
    F = GFPField(k, r)
    x = gi.operand(k, r, n, g["seed"], g["stream"], edge_frac=g["edge_frac"])
    y = cpu_ntt.transform(k, r, x, F.paper_root_of_unity(n))
    idx = g["indices"]
    assert to_ints(y[:, idx], r) == [int(v, 16) for v in g["values"]]


@pytest.mark.parametrize("name", ["k8", "k16"])
def test_fullsize_product_golden_agrees_with_cpu_product(name):
    g = _golden()["polymul"][name]
    k, r = g["k"], g["r"]
    F = GFPField(k, r)
    a = gi.operand(k, r, g["la"], g["seed"], 0, edge_frac=g["edge_frac"])
    b = gi.operand(k, r, g["lb"], g["seed"], 1, edge_frac=g["edge_frac"])
    n = 2 * g["la"]
    w = F.paper_root_of_unity(n)
    c = cpu_ntt.polymul(k, r, a, b, n, w, pow(w, F.p - 2, F.p))
    cols = g["coeff_indices"]
    assert to_ints(c[:, cols], r) == [int(v, 16) for v in g["coeff_values"]]
    ci = to_ints(c, r)
    for z, want in zip(g["points"], g["point_values"]):
        assert T.poly_eval(ci, int(z, 16), F.p) == int(want, 16)
