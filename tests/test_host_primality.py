"""The library's host-side probable-prime test (Baillie-PSW in csrc/bigint.hpp,
used by gfp_field_create) pinned without a GPU: a tiny C++ driver compiled
with g++ against the header answers for a list of numbers, and the answers
are checked against trial division, sympy, pseudoprimes that fool exactly
one half of the test, and the primes of Table 1."""

import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLDEN = os.path.join(ROOT, "tests", "golden")

DRIVER = r'''
#include "bigint.hpp"
#include <cstdio>
#include <iostream>
#include <string>
// one decimal number per line; prints "<bpsw> <strong base 2> <strong Lucas>"
static gfp::Big parse(const std::string& s) {
  gfp::Big v;
  for (char c : s) v = gfp::add(gfp::mul_small(v, 10), gfp::Big((uint64_t)(c - '0')));
  return v;
}
int main() {
  std::string line;
  while (std::getline(std::cin, line)) {
    if (line.empty()) continue;
    const gfp::Big n = parse(line);
    const gfp::Mont M(n);
    std::printf("%d %d %d\n", (int)gfp::bpsw(n), (int)gfp::strong_probable_prime_base2(n, M),
                (int)gfp::strong_lucas_probable_prime(n, M));
  }
  return 0;
}
'''


@pytest.fixture(scope="module")
def host_test(tmp_path_factory):
    cxx = shutil.which("g++")
    if not cxx:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("bpsw")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "paper_1811_01490_amd", "csrc"), str(src),
                    "-o", str(exe)], check=True)

    def run(nums):
        out = subprocess.run([str(exe)], input="\n".join(str(n) for n in nums) + "\n", capture_output=True,
                             text=True, check=True).stdout.split("\n")
        return [tuple(int(v) for v in line.split()) for line in out if line]
    return run


def _prime(n):
    if n < 2:
        return False
    i = 2
    while i * i <= n:
        if n % i == 0:
            return False
        i += 1
    return True


def test_matches_trial_division(host_test):
    nums = list(range(5, 30001, 2))
    for n, (b, _, _) in zip(nums, host_test(nums)):
        assert b == int(_prime(n)), n


def test_each_half_is_fooled_by_its_own_pseudoprimes(host_test):
    # strong pseudoprimes to base 2 (OEIS A001262): pass the first half only
    sp2 = [2047, 3277, 4033, 4681, 8321, 15841, 29341, 42799, 49141, 52633, 65281, 74665, 80581, 85489]
    for n, (b, f, l) in zip(sp2, host_test(sp2)):
        assert (b, f, l) == (0, 1, 0), n
    # strong Lucas pseudoprimes with Selfridge's parameters (OEIS A217255): pass the second half only
    slp = [5459, 5777, 10877, 16109, 18971, 22499, 24569, 25199, 40309, 58519, 75077, 97439]
    for n, (b, f, l) in zip(slp, host_test(slp)):
        assert (b, f, l) == (0, 0, 1), n


def test_matches_sympy_on_random_large(host_test):
    sympy = pytest.importorskip("sympy")
    import random

    g = random.Random(18110149)
    nums = [g.getrandbits(g.choice([64, 130, 300, 600])) | 1 for _ in range(200)]
    nums += [sympy.nextprime(g.getrandbits(200)) for _ in range(20)]  # some primes for sure
    for n, (b, _, _) in zip(nums, host_test(nums)):
        assert b == int(sympy.isprime(n)), n


def test_table1_primes_and_the_workload_prime_search(host_test):
    rows = json.load(open(os.path.join(GOLDEN, "table1_srgfn.json")))["rows"]
    nums = [(2 ** r["w"] + r["sign"] * 2 ** r["u"]) ** r["k"] + 1 for r in rows if r["k"] <= 64]
    assert all(b == 1 for b, _, _ in host_test(nums))
    # r = 2^63 + 2^s, k = 8: composite for s = 30..33, prime at 34
    cand = [(2 ** 63 + 2 ** s) ** 8 + 1 for s in range(30, 35)]
    assert [b for b, _, _ in host_test(cand)] == [0, 0, 0, 0, 1]
