"""Twiddle tables built on the device (k <= 16) against the host-built ones
(GFP_HOST_TABLES): both are canonical digits of the same powers of the root,
so every transform must come out bit-identical, forward and inverse, from
the smallest size (one pass) to 2^20."""

import os

import numpy as np
import pytest

import gfp_inputs as gi
from oracle.field import P8, P16

pytestmark = pytest.mark.gpu

K8B = dict(k=8, r=2 ** 59 + 2 ** 16)
K16B = dict(k=16, r=2 ** 58 + 2 ** 10)


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _host_field(params):
    from paper_1811_01490_amd import Field

    os.environ["GFP_HOST_TABLES"] = "1"
    try:
        return Field(params["k"], params["r"])
    finally:
        del os.environ["GFP_HOST_TABLES"]


@pytest.mark.parametrize("params", [P8, P16, K8B, K16B], ids=["k8", "k16", "k8-59-16", "k16-58-10"])
def test_device_tables_equal_host_tables(torch_mod, params):
    import torch

    from paper_1811_01490_amd import Field, to_device

    k, r = params["k"], params["r"]
    fd = Field(k, r)
    fh = _host_field(params)
    K = 2 * k
    sizes = [K, 2 * K, K * K, 2 * K * K, 2 ** 15, 2 ** 20]
    for i, n in enumerate(sizes):
        print("tables", k, r, n, flush=True)
        x = to_device(gi.uniform_digits(k, r, n, gi.BASE_SEED + 330, i))
        yd, yh = fd.fft_forward(x), fh.fft_forward(x)
        torch.cuda.synchronize()
        assert torch.equal(yd, yh), ("forward", n)
        zd, zh = fd.fft_inverse(yd), fh.fft_inverse(yh)
        torch.cuda.synchronize()
        assert torch.equal(zd, zh), ("inverse", n)
        assert torch.equal(zd, x), ("round trip", n)
