"""Field arithmetic kernels (section 2) against the oracle, bit-exact:
addition, subtraction, multiplication by r^s and multiplication (schoolbook
and FFT-based), on the seven compiled radix shapes, with random operands and
injected edge values."""

import numpy as np
import pytest

import gfp_inputs as gi
from oracle.field import GFPField
from tests.helpers import canonical_mask, to_ints

pytestmark = pytest.mark.gpu

SHAPES = [dict(k=8, r=2 ** 63 + 2 ** 34), dict(k=16, r=2 ** 62 + 2 ** 36),
          dict(k=8, r=2 ** 59 + 2 ** 16), dict(k=16, r=2 ** 58 + 2 ** 10), dict(k=32, r=2 ** 62 + 2 ** 56),
          dict(k=32, r=2 ** 56 + 2 ** 21), dict(k=64, r=2 ** 63 - 2 ** 40)]


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _operands(params, n, seed):
    k, r = params["k"], params["r"]
    x = gi.operand(k, r, n, seed, 0, edge_frac=0.02)
    y = gi.operand(k, r, n, seed, 1, edge_frac=0.02)
    # every pair of edge patterns appears once at the front
    pats = gi.edge_patterns(k, r)
    cnt = len(pats)
    for i in range(cnt):
        for j in range(cnt):
            x[:, i * cnt + j] = pats[i]
            y[:, i * cnt + j] = pats[j]
    return x, y


@pytest.mark.parametrize("params", SHAPES, ids=lambda p: "k%d" % p["k"] + ("r%x" % p["r"])[:6])
def test_add_sub_mul(torch_mod, params):
    from paper_1811_01490_amd import Field, to_device, to_host
    from paper_1811_01490_amd.gfp import OP_ADD, OP_MUL, OP_SUB

    k, r = params["k"], params["r"]
    F = GFPField(k, r)
    n = 3001  # ragged: not a multiple of the 4-wavefront block
    x, y = _operands(params, n, gi.BASE_SEED + 77)
    f = Field(k, r)
    dx, dy = to_device(x), to_device(y)
    xi, yi = to_ints(x, r), to_ints(y, r)
    for op, fn in ((OP_ADD, lambda a, b: (a + b) % F.p), (OP_SUB, lambda a, b: (a - b) % F.p),
                   (OP_MUL, lambda a, b: a * b % F.p)):
        z = to_host(f.elementwise(op, dx, dy))
        assert canonical_mask(z, r).all(), op
        got = to_ints(z, r)
        want = [fn(a, b) for a, b in zip(xi, yi)]
        bad = [i for i in range(n) if got[i] != want[i]]
        assert not bad, (op, bad[:5], len(bad))


@pytest.mark.parametrize("params", SHAPES[:2] + SHAPES[4:], ids=["k8", "k16", "k32", "k32t", "k64"])
def test_mul_pow_r_and_const(torch_mod, params):
    from paper_1811_01490_amd import Field, to_device, to_host
    from paper_1811_01490_amd.gfp import OP_MUL_CONST, OP_MUL_POW_R

    k, r = params["k"], params["r"]
    F = GFPField(k, r)
    n = 777
    x, _ = _operands(params, n, gi.BASE_SEED + 78)
    f = Field(k, r)
    dx = to_device(x)
    xi = to_ints(x, r)
    for s in (0, 1, k - 1, k, k + 1, 2 * k - 1, 2 * k, -1, 5 * k + 3):
        z = to_host(f.elementwise(OP_MUL_POW_R, dx, s=s))
        assert canonical_mask(z, r).all()
        assert to_ints(z, r) == [v * pow(F.r, s % (2 * k), F.p) % F.p for v in xi], s
    c = F.paper_root_of_unity(4096)
    for s in (0, 3, k + 2):
        z = to_host(f.elementwise(OP_MUL_CONST, dx, s=s, c=F.from_int(c)))
        assert to_ints(z, r) == [v * c * pow(F.r, s, F.p) % F.p for v in xi], s
    # p - 1 as the constant
    z = to_host(f.elementwise(OP_MUL_CONST, dx, s=0, c=F.from_int(F.p - 1)))
    assert to_ints(z, r) == [(-v) % F.p for v in xi]


@pytest.mark.parametrize("params", [SHAPES[0], SHAPES[4], SHAPES[6]], ids=["k8", "k32", "k64"])
def test_mul_large_random(torch_mod, params):
    """200k random products on the k = 8, 32 and 64 workload primes."""
    from paper_1811_01490_amd import Field, to_device, to_host
    from paper_1811_01490_amd.gfp import OP_MUL

    k, r = params["k"], params["r"]
    F = GFPField(k, r)
    n = 200_003
    x = gi.uniform_digits(k, r, n, gi.BASE_SEED + 79, 0)
    y = gi.uniform_digits(k, r, n, gi.BASE_SEED + 79, 1)
    f = Field(k, r)
    z = to_host(f.elementwise(OP_MUL, to_device(x), to_device(y)))
    xi, yi, zi = to_ints(x, r), to_ints(y, r), to_ints(z, r)
    assert canonical_mask(z, r).all()
    bad = [i for i in range(n) if zi[i] != xi[i] * yi[i] % F.p]
    assert not bad, bad[:5]


@pytest.mark.parametrize("params", SHAPES, ids=lambda p: "k%d" % p["k"] + ("r%x" % p["r"])[:6])
def test_mul_ntt(torch_mod, params):
    """The FFT-based product (section 3.3: negacyclic convolutions modulo word
    primes, CRT) gives x y mod p, the same as the schoolbook product, on
    random operands and every pair of edge values."""
    from paper_1811_01490_amd import Field, to_device, to_host
    from paper_1811_01490_amd.gfp import OP_MUL, OP_MUL_NTT

    k, r = params["k"], params["r"]
    F = GFPField(k, r)
    n = 3001
    x, y = _operands(params, n, gi.BASE_SEED + 81)
    f = Field(k, r)
    dx, dy = to_device(x), to_device(y)
    z = to_host(f.elementwise(OP_MUL_NTT, dx, dy))
    assert canonical_mask(z, r).all()
    xi, yi = to_ints(x, r), to_ints(y, r)
    assert to_ints(z, r) == [a * b % F.p for a, b in zip(xi, yi)]
    assert np.array_equal(z, to_host(f.elementwise(OP_MUL, dx, dy)))


def test_check_canonical(torch_mod):
    """gfp_check_canonical counts exactly the elements outside the section 2
    encoding: a digit >= r, or a top digit r with a nonzero lower digit."""
    from paper_1811_01490_amd import Field, to_device

    for params in SHAPES[:2] + SHAPES[4:]:
        k, r = params["k"], params["r"]
        f = Field(k, r)
        x = gi.operand(k, r, 5000, gi.BASE_SEED + 900, 0, edge_frac=0.05)  # includes p - 1 = (0, ..., 0, r)
        assert f.check_canonical(to_device(x)) == 0
        bad = x.copy()
        bad[0, 10] = np.uint64(r)           # digit 0 equal to r
        bad[k - 1, 20] = np.uint64(r + 1)   # top digit above r
        bad[k - 1, 30] = np.uint64(r)       # top digit r with a nonzero lower digit
        bad[3, 30] = np.uint64(1)
        bad[2, 4999] = np.uint64(2 ** 64 - 1)
        assert f.check_canonical(to_device(bad)) == 4
        assert f.check_canonical(to_device(bad), n=4999) == 3
