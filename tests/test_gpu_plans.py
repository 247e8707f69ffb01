"""Stage groupings: every plan (passes per launch, with two passes fused
through LDS) must give bit-identical transforms -- equal to the oracle where
it is fast -- and the autotuner must pick a valid plan without changing any
result."""

import numpy as np
import pytest

import gfp_inputs as gi
from oracle import transform as T
from oracle.field import GFPField, P8, P16
from tests.helpers import canonical_mask, to_ints

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def compositions(e, log2n=None, s=0, lk=4):
    """Every plan: '1' one pass, '2' a fused pair, and for k = 8 (lk = 4)
    'w' a wide fused pair (needs log2n - 8 - 4 s >= 3 at its first pass s)."""
    if s == e:
        return [""]
    out = []
    for c, passes in (("1", 1), ("2", 2), ("w", 2)):
        if s + passes > e or (c == "w" and (lk != 4 or log2n is None or log2n - 8 - 4 * s < 3)):
            continue
        out += [c + rest for rest in compositions(e, log2n, s + passes, lk)]
    return out


def compositions_n(N, lk=4):
    """Plans for size N = R K^e (K = 2^lk): the radix-R pass is implicit, the
    plan covers the e radix-K passes starting at Ns = R."""
    lg = N.bit_length() - 1
    return compositions(lg // lk, lg - (lg % lk), 0, lk) if lg % lk == 0 else \
        [p for p in compositions(lg // lk, lg - (lg % lk), 0, lk) if _wide_ok(p, lg, lg % lk)]


def _wide_ok(plan, lg, lr):
    s = 0
    for c in plan:
        if c == "w" and lg - 8 - lr - 4 * s < 3:
            return False
        s += 1 if c == "1" else 2
    return True


@pytest.mark.parametrize("params,N", [(P8, 256), (P8, 4096), (P8, 512), (P8, 8192),
                                      (P16, 1024), (P16, 2048), (P16, 32768), (P16, 65536)])
def test_every_plan_matches_oracle(torch_mod, params, N):
    from paper_1811_01490_amd import Field, to_device, to_host

    F = GFPField(**params)
    f = Field(**params)
    lk = 4 if F.k == 8 else 5
    x = gi.operand(F.k, F.r, N, gi.BASE_SEED + 700 + N, 0, edge_frac=0.03)
    y = gi.operand(F.k, F.r, N, gi.BASE_SEED + 700 + N, 1, edge_frac=0.03)
    w = F.paper_root_of_unity(N)
    want_f = T.dft(to_ints(x, F.r), w, F.p) if N <= 256 else T.ntt(to_ints(x, F.r), w, F.p)
    want_i = T.idft(to_ints(y, F.r), w, F.p) if N <= 256 else T.intt(to_ints(y, F.r), w, F.p)
    for plan in compositions_n(N, lk):
        print("plan case k=%d N=%d plan=%s" % (F.k, N, plan), flush=True)
        f.set_plan(N, plan)
        assert f.plan(N) == plan
        got = to_host(f.fft_forward(to_device(x)))
        assert canonical_mask(got, F.r).all(), plan
        assert to_ints(got, F.r) == want_f, plan
        got = to_host(f.fft_inverse(to_device(y)))
        assert to_ints(got, F.r) == want_i, plan
        buf = to_device(x)  # in place (a one-launch plan goes through the workspace)
        f.fft_forward(buf, y=buf)
        assert to_ints(to_host(buf), F.r) == want_f, plan
    f.set_plan(N, None)


@pytest.mark.parametrize("params,N", [(P8, 65536), (P8, 2 ** 20), (P8, 2 ** 19), (P16, 2 ** 20), (P16, 2 ** 16)])
def test_every_plan_agrees(torch_mod, params, N):
    """All plans give the output of the all-single-pass plan (pinned to the
    oracle by the transform tests), forward and inverse, digit-major with a
    padded row stride."""
    import torch

    from paper_1811_01490_amd import Field, to_device, to_host

    k = params["k"]
    f = Field(**params)
    x = gi.operand(k, params["r"], N, gi.BASE_SEED + 710, 0, edge_frac=0.005)
    dx = to_device(x)
    ref_f = ref_i = None
    for plan in compositions_n(N, 4 if k == 8 else 5):
        print("plan case k=%d N=%d plan=%s" % (k, N, plan), flush=True)
        f.set_plan(N, plan)
        yf = torch.full((k, N + 8), 3, dtype=torch.int64, device="cuda")
        f.fft_forward(dx, y=yf, n=N)
        yi = f.fft_inverse(dx)
        hf, hi = to_host(yf), to_host(yi)
        assert (hf[:, N:] == 3).all(), plan
        if ref_f is None:
            ref_f, ref_i = hf[:, :N], hi
        else:
            assert np.array_equal(hf[:, :N], ref_f), plan
            assert np.array_equal(hi, ref_i), plan
    assert np.array_equal(to_host(f.fft_inverse(to_device(ref_f))), x)
    f.set_plan(N, None)


def test_plans_in_batched_products(torch_mod):
    """Batched products under different plans for their batch classes give
    the same results as single products under the default plans."""
    import torch

    from paper_1811_01490_amd import Field, to_device, to_host
    from paper_1811_01490_amd.gfp import LAYOUT_ELEMENT_MAJOR

    f = Field(**P8)
    sizes = [(100, 100)] * 9 + [(1500, 1000)] * 3 + [(20000, 20000)] * 2
    ops = [(to_device(gi.operand(8, P8["r"], la, gi.BASE_SEED + 720, 2 * i)),
            to_device(gi.operand(8, P8["r"], lb, gi.BASE_SEED + 720, 2 * i + 1))) for i, (la, lb) in enumerate(sizes)]
    ref = [to_host(f.polymul(a, b)) for a, b in ops]
    em = LAYOUT_ELEMENT_MAJOR
    for plans in ({256: "11", 4096: "111", 65536: "1111"}, {256: "2", 4096: "12", 65536: "211"},
                  {256: "2", 4096: "21", 65536: "22"}, {256: "2", 4096: "w1", 65536: "w2"},
                  {256: "11", 4096: "w1", 65536: "1w1"}):
        for n, plan in plans.items():
            for nvec in (2, 8, 64):  # every batch class the chunks can use
                f.set_plan(n, plan, nvec=nvec, layout=em)
        outs = [torch.empty((8, a.shape[1] + b.shape[1] - 1), dtype=torch.int64, device="cuda") for a, b in ops]
        f.polymul_batched(f.batch_descs([(a, b, c) for (a, b), c in zip(ops, outs)]))
        torch.cuda.synchronize()
        for i, (c, r) in enumerate(zip(outs, ref)):
            assert np.array_equal(to_host(c), r), (plans, i)


def test_plans_in_batched_products_k16(torch_mod):
    """The same for k = 16, whose fused pairs take one 1024-element block per
    workgroup."""
    import torch

    from paper_1811_01490_amd import Field, to_device, to_host
    from paper_1811_01490_amd.gfp import LAYOUT_ELEMENT_MAJOR

    f = Field(**P16)
    sizes = [(600, 400)] * 5 + [(10000, 9000)] * 2  # transform sizes 1024 = K^2 and 32768 = K^3
    ops = [(to_device(gi.operand(16, P16["r"], la, gi.BASE_SEED + 725, 2 * i)),
            to_device(gi.operand(16, P16["r"], lb, gi.BASE_SEED + 725, 2 * i + 1))) for i, (la, lb) in enumerate(sizes)]
    ref = [to_host(f.polymul(a, b)) for a, b in ops]
    em = LAYOUT_ELEMENT_MAJOR
    for plans in ({1024: "11", 32768: "111"}, {1024: "2", 32768: "21"}, {1024: "2", 32768: "12"}):
        for n, plan in plans.items():
            for nvec in (2, 8):
                f.set_plan(n, plan, nvec=nvec, layout=em)
        outs = [torch.empty((16, a.shape[1] + b.shape[1] - 1), dtype=torch.int64, device="cuda") for a, b in ops]
        f.polymul_batched(f.batch_descs([(a, b, c) for (a, b), c in zip(ops, outs)]))
        torch.cuda.synchronize()
        for i, (c, r) in enumerate(zip(outs, ref)):
            assert np.array_equal(to_host(c), r), (plans, i)


def test_tuner_picks_a_valid_plan(torch_mod):
    from paper_1811_01490_amd import Field, to_device, to_host

    f = Field(**P8)
    N = 65536
    x = to_device(gi.operand(8, P8["r"], N, gi.BASE_SEED + 730, 0))
    before = to_host(f.fft_forward(x))
    plan, us = f.tune(N)
    assert plan in compositions(4, 16) and us > 0
    assert f.plan(N) == plan
    assert np.array_equal(to_host(f.fft_forward(x)), before)
    plan_em, _ = f.tune(N, nvec=2, layout=1)
    assert plan_em in compositions(4, 16) and f.plan(N, nvec=2, layout=1) == plan_em
    plan16, _ = Field(**P16).tune(32768, nvec=2, layout=1)
    assert plan16 in compositions(3, 15, 0, 5)  # fused pairs, no wide pair for k = 16
    plan32, _ = Field(k=32, r=2 ** 62 + 2 ** 56).tune(2 ** 18)
    assert len(plan32) == 3 and set(plan32) <= {"1", "n"}  # one pass per launch for k = 32, either multiplier
