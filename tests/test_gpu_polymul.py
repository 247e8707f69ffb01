"""Polynomial product (section 3.3, Alg. Fast Convolution) against the
schoolbook product, bit-exact; at the full workload size (two degree < 2^19
factors) by Schwartz-Zippel evaluation and sampled coefficients."""

import numpy as np
import pytest

import gfp_inputs as gi
from oracle import transform as T
from oracle.field import GFPField, P8, P16, P32, P64
from tests.helpers import canonical_mask, to_ints

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(params, la, lb, seed, edge=0.02):
    from paper_1811_01490_amd import Field, to_device, to_host

    F = GFPField(**params)
    f = Field(params["k"], params["r"])
    a = gi.operand(F.k, F.r, la, seed, 0, edge_frac=edge)
    b = gi.operand(F.k, F.r, lb, seed, 1, edge_frac=edge)
    c = to_host(f.polymul(to_device(a), to_device(b)))
    assert c.shape == (F.k, la + lb - 1)
    assert canonical_mask(c, F.r).all()
    return F, a, b, c


def test_degree_2048_schoolbook(torch_mod):
    """k = 8, la = lb = 2048 (transform size 16^3 = 4096), every coefficient
    against the schoolbook product."""
    F, a, b, c = _run(P8, 2048, 2048, gi.BASE_SEED + 0)
    want = T.polymul(to_ints(a, F.r), to_ints(b, F.r), F.p)
    got = to_ints(c, F.r)
    bad = [m for m in range(len(want)) if got[m] != want[m]]
    assert not bad, (bad[:8], len(bad))


@pytest.mark.parametrize("params", [P8, P16, P32, P64], ids=["k8", "k16", "k32", "k64"])
@pytest.mark.parametrize("la,lb", [(1, 1), (1, 17), (3, 5), (9, 8), (8, 9), (16, 1), (100, 157), (300, 1), (513, 512)])
def test_ragged_schoolbook(torch_mod, params, la, lb):
    F, a, b, c = _run(params, la, lb, gi.BASE_SEED + la * 1000 + lb, edge=0.2)
    assert to_ints(c, F.r) == T.polymul(to_ints(a, F.r), to_ints(b, F.r), F.p)


@pytest.mark.parametrize("name,params", [("k8", P8), ("k16", P16)])
def test_full_size_sampled(torch_mod, name, params):
    """la = lb = 2^19 (transform size 2^20): 13 sampled coefficients (the
    ends, the middle and 8 seeded ones) against their schoolbook sums, and
    Schwartz-Zippel at 8 random points z: c(z) = a(z) b(z).  The expected
    values were written by the oracle into tests/golden/sampled_fullsize.json
    from the same seeded operands; c(z) is evaluated here from the GPU
    output."""
    import json
    import os

    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sampled_fullsize.json")
    with open(path) as fh:
        g = json.load(fh)["polymul"][name]
    assert (g["k"], g["r"]) == (params["k"], params["r"])
    F, a, b, c = _run(params, g["la"], g["lb"], g["seed"], edge=g["edge_frac"])
    cols = g["coeff_indices"]
    assert len(cols) >= 13
    for m, got, want in zip(cols, to_ints(c[:, cols], F.r), g["coeff_values"]):
        assert got == int(want, 16), m
    ci = to_ints(c, F.r)
    assert len(g["points"]) >= 8
    for z, want in zip(g["points"], g["point_values"]):
        assert T.poly_eval(ci, int(z, 16), F.p) == int(want, 16), z
