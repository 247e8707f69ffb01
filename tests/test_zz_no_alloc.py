"""gfp_fft_noalloc (the transform with the library's static device scratch,
no allocation inside the call) against gfp_fft_forward / gfp_fft_inverse of
the same inputs: bit-identical, on two calls in a row with the second one
smaller, for both transform directions and two fields; plus its error
returns (tables not built yet, size above the scratch limit)."""

import numpy as np
import pytest

import gfp_inputs as gi
from oracle.field import P8, P16

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


# (field, [n of the first call, n of the second, smaller call])
CASES = [(P8, [1 << 16, 1 << 12]), (P16, [1 << 15, 1 << 10]), (P8, [1 << 18, 16])]


@pytest.mark.parametrize("params,sizes", CASES)
@pytest.mark.parametrize("inverse", [False, True])
def test_noalloc_equals_workspace_entry_point(torch_mod, params, sizes, inverse):
    from paper_1811_01490_amd import Field, to_device, to_host

    k, r = params["k"], params["r"]
    f = Field(k, r)
    for i, n in enumerate(sizes):
        print("noalloc case k=%d n=%d inverse=%d call=%d" % (k, n, inverse, i), flush=True)
        x = to_device(gi.operand(k, r, n, gi.BASE_SEED + 70 + i, 0, edge_frac=0.02))
        # the existing entry point first: it also builds the size's tables
        want = f.fft_inverse(x) if inverse else f.fft_forward(x)
        y = torch_mod.full((k, n), -1, dtype=torch_mod.int64, device=x.device)
        f.fft_noalloc(x, y=y, inverse=inverse)
        torch_mod.cuda.synchronize()
        assert np.array_equal(to_host(y), to_host(want)), "k=%d n=%d call %d" % (k, n, i)
        # in place (x == y) gives the same
        xin = x.clone()
        f.fft_noalloc(xin, y=xin, inverse=inverse)
        torch_mod.cuda.synchronize()
        assert np.array_equal(to_host(xin), to_host(want))
    f.close()


def test_noalloc_errors(torch_mod):
    from paper_1811_01490_amd import Field, GFPError, to_device
    from paper_1811_01490_amd.gfp import GFP_EINVAL, GFP_ENOTREADY

    k, r = 8, 2 ** 59 + 2 ** 16  # a field no other test of this file builds tables for
    f = Field(k, r)
    x = to_device(gi.operand(k, r, 4096, gi.BASE_SEED + 80, 0))
    y = torch_mod.empty_like(x)
    with pytest.raises(GFPError) as e:
        f.fft_noalloc(x, y=y)
    assert e.value.code == GFP_ENOTREADY
    f.fft_forward(x)  # builds the tables of size 4096
    f.fft_noalloc(x, y=y)
    torch_mod.cuda.synchronize()
    # 2 n k 8 bytes above the 32 MiB scratch
    big = torch_mod.zeros((k, 1 << 19), dtype=torch_mod.int64, device=x.device)
    with pytest.raises(GFPError) as e:
        f.fft_noalloc(big, y=big)
    assert e.value.code == GFP_EINVAL
    f.close()
