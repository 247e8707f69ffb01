"""The FFT-based multiplication of section 3.3 as the twiddle multiplier of
the k = 32 and k = 64 passes (plan character 'n'): transforms under every
plan that selects it equal the oracle element by element where the oracle is
fast, and equal the schoolbook plans bit for bit at larger sizes."""

import numpy as np
import pytest

import gfp_inputs as gi
from oracle import transform as T
from oracle.field import GFPField, P32, P64
from tests.helpers import canonical_mask, to_ints

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _plans(e):
    out = [""]
    for _ in range(e):
        out = [p + c for p in out for c in "1n"]
    return out


# (field, N): one pass, radix-2 + one pass, two passes, radix-2 + two passes
@pytest.mark.parametrize("params,N", [(P64, 128), (P64, 256), (P64, 16384), (P32, 64), (P32, 4096), (P32, 8192)])
def test_ntt_twiddle_plans_match_oracle(torch_mod, params, N):
    from paper_1811_01490_amd import Field, to_device, to_host

    F = GFPField(**params)
    f = Field(**params)
    lk = 6 if F.k == 32 else 7
    e = (N.bit_length() - 1) // lk
    x = gi.operand(F.k, F.r, N, gi.BASE_SEED + 900 + N, 0, edge_frac=0.03)
    y = gi.operand(F.k, F.r, N, gi.BASE_SEED + 900 + N, 1, edge_frac=0.03)
    w = F.paper_root_of_unity(N)
    want_f = T.ntt(to_ints(x, F.r), w, F.p)
    want_i = T.intt(to_ints(y, F.r), w, F.p)
    for plan in _plans(e):
        print("ntt twiddle case k=%d N=%d plan=%s" % (F.k, N, plan), flush=True)
        f.set_plan(N, plan)
        got = to_host(f.fft_forward(to_device(x)))
        assert canonical_mask(got, F.r).all(), plan
        assert to_ints(got, F.r) == want_f, plan
        assert to_ints(to_host(f.fft_inverse(to_device(y))), F.r) == want_i, plan
    f.close()


@pytest.mark.parametrize("params,N", [(P64, 2 ** 17), (P32, 2 ** 18), (P64, 2 ** 20)])
def test_ntt_twiddle_plans_equal_schoolbook(torch_mod, params, N):
    from paper_1811_01490_amd import Field, to_device, to_host

    k = params["k"]
    f = Field(**params)
    lk = 6 if k == 32 else 7
    e = (N.bit_length() - 1) // lk
    x = to_device(gi.operand(k, params["r"], N, gi.BASE_SEED + 910, 0, edge_frac=0.005))
    ref_f, ref_i = to_host(f.fft_forward(x)), to_host(f.fft_inverse(x))
    for plan in _plans(e)[1:]:
        print("ntt twiddle case k=%d N=%d plan=%s" % (k, N, plan), flush=True)
        f.set_plan(N, plan)
        assert np.array_equal(to_host(f.fft_forward(x)), ref_f), plan
        assert np.array_equal(to_host(f.fft_inverse(x)), ref_i), plan
    f.close()
