"""Integer products through the polynomial product over Z/pZ: c = a * b must
equal the product of the same integers as Python integers (the plain
definition), for random, all-ones (longest carry chains), zero and
power-of-two operands, ragged lengths, on every compiled radix shape."""

import numpy as np
import pytest

import gfp_inputs as gi

pytestmark = pytest.mark.gpu

SHAPES = {"k8": (8, 2 ** 63 + 2 ** 34), "k16": (16, 2 ** 62 + 2 ** 36),
          "k8t": (8, 2 ** 59 + 2 ** 16), "k16t": (16, 2 ** 58 + 2 ** 10), "k32": (32, 2 ** 62 + 2 ** 56),
          "k32t": (32, 2 ** 56 + 2 ** 21), "k64": (64, 2 ** 63 - 2 ** 40)}


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def words_to_int(w: np.ndarray) -> int:
    return int.from_bytes(np.ascontiguousarray(w, dtype="<u8").tobytes(), "little")


def int_to_words(v: int, n: int) -> np.ndarray:
    return np.frombuffer(v.to_bytes(8 * n, "little"), dtype="<u8").copy()


def _mul(f, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    import torch

    da = torch.from_numpy(a.view(np.int64)).cuda()
    db = torch.from_numpy(b.view(np.int64)).cuda()
    c = f.bigint_mul(da, db)
    torch.cuda.synchronize()
    return c.cpu().numpy().view(np.uint64)


@pytest.mark.parametrize("name", list(SHAPES))
def test_random_products(torch_mod, name):
    from paper_1811_01490_amd import Field

    k, r = SHAPES[name]
    f = Field(k, r)
    g = gi.rng(gi.BASE_SEED + 800, k)
    for na, nb in [(1, 1), (1, 17), (5, 3), (100, 257), (1000, 1000), (4096, 3000), (3, 2 ** 14)]:
        a = g.integers(0, 2 ** 64, size=na, dtype=np.uint64)
        b = g.integers(0, 2 ** 64, size=nb, dtype=np.uint64)
        got = _mul(f, a, b)
        assert got.shape == (na + nb,)
        assert words_to_int(got) == words_to_int(a) * words_to_int(b), (na, nb)


def test_carry_chains_and_special_values(torch_mod):
    """(2^(64n) - 1)^2 = 2^(128n) - 2^(64n+1) + 1 has the longest carry
    chains the evaluation can meet; zero, one and powers of two."""
    from paper_1811_01490_amd import Field

    f = Field(*SHAPES["k8"])
    for n in (1, 2, 63, 64, 1025, 5000):
        ones = np.full(n, 2 ** 64 - 1, dtype=np.uint64)
        got = words_to_int(_mul(f, ones, ones))
        assert got == (2 ** (64 * n) - 1) ** 2, n
    z = np.zeros(300, dtype=np.uint64)
    x = gi.rng(gi.BASE_SEED + 801, 0).integers(0, 2 ** 64, size=200, dtype=np.uint64)
    assert words_to_int(_mul(f, z, x)) == 0
    one = np.zeros(7, dtype=np.uint64)
    one[0] = 1
    assert words_to_int(_mul(f, one, x)) == words_to_int(x)
    for e1, e2 in [(0, 0), (63, 64), (4095, 1), (64 * 700 + 5, 64 * 300 + 61)]:
        a = int_to_words(1 << e1, e1 // 64 + 1)
        b = int_to_words(1 << e2, e2 // 64 + 1)
        assert words_to_int(_mul(f, a, b)) == 1 << (e1 + e2)


def test_large_product(torch_mod):
    """2^16 x 2^16 words (4 Mbit each): transform size 2^18 for k = 8."""
    from paper_1811_01490_amd import Field

    f = Field(*SHAPES["k8"])
    g = gi.rng(gi.BASE_SEED + 802, 0)
    a = g.integers(0, 2 ** 64, size=2 ** 16, dtype=np.uint64)
    b = g.integers(0, 2 ** 64, size=2 ** 16, dtype=np.uint64)
    assert words_to_int(_mul(f, a, b)) == words_to_int(a) * words_to_int(b)
