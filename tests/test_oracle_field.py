"""Pins for oracle.field: encoding, the paper's element algorithms and the
root of unity, checked against plain modular arithmetic, exhaustive runs on
tiny generalized Fermat primes and the facts the paper states."""

import itertools
import json
import os
import random

import pytest

from oracle.field import GFPField, P8, P16, P32, P64, v2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# Tiny generalized Fermat primes: 257 = 2^8+1 = 4^4+1 = 16^2+1,
# 65537 = 2^16+1 = 4^8+1 = 16^4+1 = 256^2+1, and 37 = 6^2+1, 1297 = 6^4+1.
TINY = [(2, 8), (4, 4), (16, 2), (6, 2), (6, 4), (4, 8), (2, 16), (16, 4), (256, 2)]


@pytest.mark.parametrize("r,k", TINY)
def test_tiny_fields_are_prime(r, k):
    assert GFPField(k, r).is_prime()


@pytest.mark.parametrize("r,k", [(2, 8), (4, 4), (16, 2), (6, 2), (6, 4)])
def test_encoding_roundtrip_exhaustive(r, k):
    F = GFPField(k, r)
    seen = set()
    for v in range(F.p):
        d = F.from_int(v)
        assert F.is_canonical(d)
        assert F.to_int(d) == v
        seen.add(tuple(d))
    assert len(seen) == F.p
    # p - 1 is the only value with a digit equal to r
    assert F.from_int(F.p - 1) == [0] * (k - 1) + [r]


def test_noncanonical_rejected():
    F = GFPField(4, 4)
    assert not F.is_canonical([4, 0, 0, 0])
    assert not F.is_canonical([0, 0, 1, 4])
    assert not F.is_canonical([0, 0, 0, 5])
    assert F.is_canonical([0, 0, 0, 4])


@pytest.mark.parametrize("r,k", [(2, 8), (4, 4), (16, 2), (6, 2), (6, 4)])
def test_paper_add_sub_exhaustive(r, k):
    F = GFPField(k, r)
    enc = [F.from_int(v) for v in range(F.p)]
    step = 1 if F.p < 300 else 7
    for a in range(0, F.p, step):
        for b in range(F.p):
            s = F.paper_add(enc[a], enc[b])
            assert s == enc[(a + b) % F.p], (a, b)
            d = F.paper_sub(enc[a], enc[b])
            assert d == enc[(a - b) % F.p], (a, b)


@pytest.mark.parametrize("r,k", [(2, 8), (4, 4), (16, 2), (6, 4)])
def test_paper_mul_pow_r_exhaustive(r, k):
    F = GFPField(k, r)
    for a in range(F.p):
        x = F.from_int(a)
        for s in range(0, 2 * k + 3):
            assert F.paper_mul_pow_r(x, s) == F.from_int(a * r ** s), (a, s)


@pytest.mark.parametrize("r,k", [(2, 8), (4, 4), (16, 2), (6, 2)])
def test_paper_mul_exhaustive(r, k):
    F = GFPField(k, r)
    enc = [F.from_int(v) for v in range(F.p)]
    for a in range(F.p):
        for b in range(a, F.p):
            assert F.paper_mul(enc[a], enc[b]) == enc[a * b % F.p], (a, b)


@pytest.mark.parametrize("params", [P8, P16, P32, P64, dict(k=8, r=2 ** 59 + 2 ** 16), dict(k=16, r=2 ** 58 + 2 ** 10)])
def test_paper_algorithms_random_large(params):
    F = GFPField(**params)
    g = random.Random(7)
    vals = [0, 1, 2, F.p - 1, F.p - 2, F.r ** (F.k - 1), F.r ** F.k - 1, F.r - 1]
    vals += [g.randrange(F.p) for _ in range(60)]
    for a, b in itertools.product(vals[:12], vals):
        x, y = F.from_int(a), F.from_int(b)
        assert F.paper_add(x, y) == F.from_int(a + b)
        assert F.paper_sub(x, y) == F.from_int(a - b)
        assert F.paper_mul(x, y) == F.from_int(a * b)
    for a in vals:
        for s in (1, F.k - 1, F.k, F.k + 1, 2 * F.k - 1):
            assert F.paper_mul_pow_r(F.from_int(a), s) == F.from_int(a * F.r ** s)


def test_worked_example_double_p_minus_one():
    """Section 2.2: r^k + r^k has every digit r - 1, i.e. -2 mod p."""
    ex = json.load(open(os.path.join(GOLDEN, "worked_examples.json")))["double_p_minus_one"]
    for params in (P8, P16, dict(k=4, r=4)):
        F = GFPField(**params)
        pm1 = [0] * (F.k - 1) + [F.r]
        out = F.paper_add(pm1, pm1)
        assert out == [F.r + ex["result_digit_offset_from_r"]] * F.k
        assert F.to_int(out) == ex["value_mod_p"] % F.p


def test_negacyclic_column_bound():
    """|u_m| < k r^2 (section 3.1.1) with the extreme inputs."""
    for params in (P8, P16, P32):
        F = GFPField(**params)
        top = [F.r - 1] * F.k
        cols = F.paper_negacyclic_columns(top, top)
        assert all(abs(u) < F.k * F.r ** 2 for u in cols)
        assert cols[F.k - 1] == F.k * (F.r - 1) ** 2  # the all-positive column


@pytest.mark.parametrize("params", [P8, P16, P32, P64, dict(k=8, r=2 ** 59 + 2 ** 16),
                                    dict(k=16, r=2 ** 58 + 2 ** 10), dict(k=8, r=4), dict(k=4, r=4)])
def test_field_structure(params):
    """r^k = -1, r^(2k) = 1 and r has order exactly 2k (section 2)."""
    F = GFPField(**params)
    assert F.is_prime()
    assert pow(F.r, F.k, F.p) == F.p - 1
    assert pow(F.r, 2 * F.k, F.p) == 1
    for d in range(1, 2 * F.k):
        if (2 * F.k) % d == 0:
            assert pow(F.r, d, F.p) != 1
    assert F.max_log2_n == F.k * v2(F.r)


def test_workload_valuations():
    assert GFPField(**P8).max_log2_n == 272
    assert GFPField(**P16).max_log2_n == 576
    assert GFPField(**P32).max_log2_n == 1792
    assert GFPField(**P64).max_log2_n == 2560


@pytest.mark.parametrize("params,N", [(P8, 16), (P8, 256), (P8, 4096), (P8, 2 ** 20), (P16, 32), (P16, 1024), (P16, 2 ** 20),
                                      (P32, 64), (P32, 4096), (P32, 2 ** 18), (P64, 128), (P64, 2 ** 14),
                                      (dict(k=8, r=4), 16), (dict(k=8, r=4), 256), (dict(k=4, r=4), 8)])
def test_root_of_unity(params, N):
    """Alg. 1: w^(N/2k) = r, w^(N/2) = -1, w^N = 1 (w primitive)."""
    F = GFPField(**params)
    w = F.paper_root_of_unity(N)
    assert pow(w, N // (2 * F.k), F.p) == F.r
    assert pow(w, N // 2, F.p) == F.p - 1
    assert pow(w, N, F.p) == 1


def test_roots_are_nested():
    """With g = h^((p-1)/N), a = g^(N/2k) = h^((p-1)/2k) does not depend on
    N, so Alg. 1 finds the same j and w_N = w_M^(M/N)."""
    for params, sizes in ((P8, [16, 256, 4096, 65536, 2 ** 20]), (P16, [32, 1024, 32768, 2 ** 20])):
        F = GFPField(**params)
        M = sizes[-1]
        wM = F.paper_root_of_unity(M)
        for N in sizes:
            assert F.paper_root_of_unity(N) == pow(wM, M // N, F.p)


def test_smallest_nonresidue_is_nonresidue():
    for params in (P8, P16):
        F = GFPField(**params)
        h = F.smallest_nonresidue()
        assert pow(h, (F.p - 1) // 2, F.p) == F.p - 1
        for t in range(2, h):
            assert pow(t, (F.p - 1) // 2, F.p) == 1
