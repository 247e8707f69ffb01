"""Pins for the oracle's BPSW test against facts outside the oracle."""

import json
import os

import pytest

from oracle.primality import is_probable_prime, jacobi, strong_fermat, strong_lucas

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _trial_division_prime(n):
    if n < 2:
        return False
    i = 2
    while i * i <= n:
        if n % i == 0:
            return False
        i += 1
    return True


def test_matches_trial_division_below_20000():
    for n in range(20000):
        assert is_probable_prime(n) == _trial_division_prime(n), n


def test_matches_sympy_on_random_large():
    sympy = pytest.importorskip("sympy")
    import random

    g = random.Random(1811)
    for _ in range(300):
        n = g.getrandbits(g.choice([64, 128, 256, 512])) | 1
        assert is_probable_prime(n) == sympy.isprime(n), n


def test_jacobi_against_euler_criterion():
    # For an odd prime q, (a/q) = a^((q-1)/2) mod q.
    for q in (3, 5, 7, 11, 13, 101, 257, 65537):
        for a in range(0, 50):
            e = pow(a, (q - 1) // 2, q)
            expect = 0 if a % q == 0 else (1 if e == 1 else -1)
            assert jacobi(a, q) == expect


def test_each_half_catches_the_others_pseudoprimes():
    # Strong pseudoprimes to base 2 (pass the Fermat half, fail Lucas).
    for n in (2047, 3277, 4033, 4681, 8321, 15841, 29341, 42799, 49141, 52633, 65281, 74665, 80581, 85489):
        assert strong_fermat(n, 2) and not _trial_division_prime(n)
        assert not is_probable_prime(n)
    # Strong Lucas pseudoprimes (Selfridge parameters): pass Lucas, fail base 2.
    for n in (5459, 5777, 10877, 16109, 18971, 22499, 24569, 25199, 40309, 58519):
        assert strong_lucas(n) and not _trial_division_prime(n)
        assert not is_probable_prime(n)
    # Carmichael numbers.
    for n in (561, 1105, 1729, 2465, 2821, 6601, 8911, 41041, 825265):
        assert not is_probable_prime(n)


def test_table1_primes_and_valuations():
    rows = json.load(open(os.path.join(GOLDEN, "table1_srgfn.json")))["rows"]
    for row in rows:
        if row["k"] > 64:
            continue  # 8192-bit; covered by the slow test below
        r = 2 ** row["w"] + row["sign"] * 2 ** row["u"]
        p = r ** row["k"] + 1
        assert is_probable_prime(p), row
        assert ((p - 1) & -(p - 1)).bit_length() - 1 == row["log2_max_n"], row


@pytest.mark.slow
def test_table1_largest_prime():
    row = json.load(open(os.path.join(GOLDEN, "table1_srgfn.json")))["rows"][-1]
    r = 2 ** row["w"] + row["sign"] * 2 ** row["u"]
    assert is_probable_prime(r ** row["k"] + 1)


def test_testprimes_table():
    rows = json.load(open(os.path.join(GOLDEN, "table_testprimes.json")))["rows"]
    for row in rows:
        assert row["K"] == 2 * row["k"]
        r = 2 ** row["w"] + 2 ** row["u"]
        assert is_probable_prime(r ** row["k"] + 1), row


def test_workload_prime_search():
    """The smallest s >= 30 making (2^63 + 2^s)^8 + 1 prime is 34, and for
    (2^62 + 2^s)^16 + 1 it is 36: the Table 1 rows 3 and 4 primes."""
    found8 = next(s for s in range(30, 63) if is_probable_prime((2 ** 63 + 2 ** s) ** 8 + 1))
    found16 = next(s for s in range(30, 62) if is_probable_prime((2 ** 62 + 2 ** s) ** 16 + 1))
    assert (found8, found16) == (34, 36)
