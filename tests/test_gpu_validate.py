"""GFP_VALIDATE: a field created with the variable set rejects non-canonical
inputs of transforms, products and elementwise operations with GFP_EINVAL
before any work; canonical inputs (p - 1 included) pass."""

import os

import pytest

import gfp_inputs as gi
from oracle.field import P8

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_validate_rejects_non_canonical_inputs(torch_mod):
    from paper_1811_01490_amd import Field, GFPError, to_device
    from paper_1811_01490_amd.gfp import GFP_EINVAL, OP_ADD

    k, r = P8["k"], P8["r"]
    os.environ["GFP_VALIDATE"] = "1"
    try:
        f = Field(k, r)
    finally:
        del os.environ["GFP_VALIDATE"]
    n = 4096
    x = gi.operand(k, r, n, gi.BASE_SEED + 90, 0, edge_frac=0.05)  # includes p - 1 = (0, ..., 0, r)
    good = to_device(x)
    f.fft_forward(good)
    f.fft_inverse(good)
    f.polymul(good[:, :100], good[:, 100:300])
    f.elementwise(OP_ADD, good, good)
    bad = good.clone()
    bad[3, 17] = r - (1 << 64)  # digit 3 equal to r (int64 bit pattern): not canonical
    for call in (lambda: f.fft_forward(bad), lambda: f.fft_inverse(bad), lambda: f.polymul(bad, good),
                 lambda: f.polymul(good, bad), lambda: f.elementwise(OP_ADD, good, bad)):
        with pytest.raises(GFPError) as e:
            call()
        assert e.value.code == GFP_EINVAL
    torch_mod.cuda.synchronize()
    f.close()
