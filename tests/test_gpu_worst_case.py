"""Worst-case digit magnitudes through the transforms, against closed forms.

Lazy digits in the kernels are bounded by arguments about their largest
inputs: a pass after the first accepts any digit in [0, 2^64), and the
last pass must bring the largest lazy values back to the canonical encoding.
Uniform inputs almost never reach those bounds, so these tests feed the
extremes and compare every output with a value the definition fixes:

* a constant input c (every coefficient p - 1, or every digit r - 1, i.e.
  c = -2) has forward transform N c at index 0 and 0 elsewhere, and inverse
  transform c at index 0 and 0 elsewhere (the DFT of section 1.1; the inverse
  includes 1/N, section 3.3), through the default plan and every fused plan;
* the product of two constant polynomials of length L has coefficient
  c_m = (min(m, 2L - 2 - m) + 1) a b (the schoolbook sum);
* one pass s >= 1 run alone (gfp_fft_pass) on an element-major input whose
  every digit is 2^64 - 1: every slot holds the same value c, so output t of
  group j is c sum_u w_L^((a + t Ns) u) (a = j mod Ns, L = K Ns, section 4.1:
  the twiddle w_L^(a u) times the base-case root r = w_L^Ns); the fused pairs
  must equal the two single passes.
"""

import numpy as np
import pytest

from oracle.field import GFPField, P8, P16, P32, P64
from tests.helpers import canonical_mask, to_ints
from tests.test_gpu_plans import compositions_n

pytestmark = pytest.mark.gpu

SHAPES = {"k8": P8, "k16": P16, "k32": P32, "k64": P64}


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _fields(name):
    from paper_1811_01490_amd import Field

    prm = SHAPES[name]
    return GFPField(**prm), Field(prm["k"], prm["r"])


def _constant(torch, F, digits, n):
    col = torch.tensor(np.array(digits, dtype=np.uint64).view(np.int64), device="cuda")
    return col[:, None].expand(F.k, n).contiguous()


def _check_delta0(torch, F, y, value):
    """y (k, n) on the device: canonical digits of value at index 0, zero
    elsewhere."""
    assert int(torch.count_nonzero(y[:, 1:])) == 0
    got = y[:, 0].cpu().numpy().view(np.uint64)
    assert [int(v) for v in got] == F.from_int(value)


def _plans(name, n):
    if name == "k8":
        return [None] + compositions_n(n)
    return [None]


@pytest.mark.parametrize("name,N", [("k8", 2 ** 20), ("k16", 2 ** 20), ("k32", 2 ** 17), ("k64", 2 ** 17)])
def test_constant_inputs_every_plan(torch_mod, name, N):
    torch = torch_mod
    F, f = _fields(name)
    k, r, p = F.k, F.r, F.p
    consts = {"p-1": [0] * (k - 1) + [r], "all r-1": [r - 1] * k}
    for plan in _plans(name, N):
        f.set_plan(N, plan)
        for label, digits in consts.items():
            c = F.to_int(digits)
            x = _constant(torch, F, digits, N)
            _check_delta0(torch, F, f.fft_forward(x), N * c % p)
            _check_delta0(torch, F, f.fft_inverse(x), c % p)
            torch.cuda.synchronize()
    f.set_plan(N, None)


@pytest.mark.parametrize("name", ["k8", "k16"])
def test_constant_polymul_full_size(torch_mod, name):
    """la = lb = 2^19 (transform size 2^20), both factors constant at the
    largest digits; every output coefficient against its closed form."""
    torch = torch_mod
    F, f = _fields(name)
    k, r, p = F.k, F.r, F.p
    L = 2 ** 19
    for da, db in (([0] * (k - 1) + [r], [r - 1] * k), ([r - 1] * k, [r - 1] * k)):
        a = _constant(torch, F, da, L)
        b = _constant(torch, F, db, L)
        c = f.polymul(a, b)
        torch.cuda.synchronize()
        ch = c.cpu().numpy().view(np.uint64)
        assert canonical_mask(ch, r).all()
        ab = F.to_int(da) * F.to_int(db) % p
        got = to_ints(ch, r)
        want = [(min(m, 2 * L - 2 - m) + 1) * ab % p for m in range(2 * L - 1)]
        bad = [m for m in range(2 * L - 1) if got[m] != want[m]]
        assert not bad, (bad[:8], len(bad))


def _stages(F, n):
    K = 2 * F.k
    e, t = 0, 1
    while t * K <= n:
        t *= K
        e += 1
    R = n // t
    return R, e + (1 if R > 1 else 0)


def _pass_closed_form(F, n, s, inverse, c):
    """Values of stage s >= 1 run on an input whose every element is c:
    position o holds c sum_u z^u, z = w_L^(a + t Ns) = w_L^(o mod L).  For
    k >= 32 and n > K the inverse's stage 1 also carries the 1/n factor."""
    p, K = F.p, 2 * F.k
    R, S = _stages(F, n)
    ns = R * K ** (s - (1 if R > 1 else 0))
    L = K * ns
    w = F.paper_root_of_unity(n)
    if inverse:
        w = pow(w, p - 2, p)
    wl = pow(w, n // L, p)
    scale = pow(n, p - 2, p) if (inverse and F.k >= 32 and s == 1 and n > K) else 1
    cls = {}
    for e in range(L):  # e = a + t Ns runs over every class once
        z = pow(wl, e, p)
        acc, zu = 0, 1
        for _ in range(K):
            acc += zu
            zu = zu * z % p
        cls[e] = c * acc % p * scale % p
    # o = (j - a) K + a + t Ns with j - a a multiple of Ns: o mod L = a + t Ns
    return [cls[o % L] for o in range(n)], S


PASS_CASES = [("k8", 4096, 1), ("k8", 4096, 2), ("k8", 65536, 1), ("k8", 65536, 2), ("k8", 65536, 3),
              ("k16", 32768, 1), ("k16", 32768, 2), ("k32", 4096, 1), ("k32", 2 * 64 * 64, 1),
              ("k32", 2 * 64 * 64, 2), ("k64", 128 * 128, 1), ("k64", 2 * 128 * 128, 1)]


@pytest.mark.parametrize("name,N,s", PASS_CASES)
def test_pass_all_ones_digits(torch_mod, name, N, s):
    torch = torch_mod
    F, f = _fields(name)
    k, r = F.k, F.r
    c = F.to_int([2 ** 64 - 1] * k) % F.p
    for inverse in (False, True):
        want, S = _pass_closed_form(F, N, s, inverse, c)
        last = s == S - 1
        x = torch.full((N * k,), -1, dtype=torch.int64, device="cuda")
        y = torch.empty((k, N) if last else (N * k,), dtype=torch.int64, device="cuda")
        f.fft_pass(s, x, y, N, inverse=inverse, in_element_major=True, out_element_major=not last)
        torch.cuda.synchronize()
        yh = y.cpu().numpy().view(np.uint64)
        if last:
            assert canonical_mask(yh, r).all()
        else:
            yh = yh.reshape(N, k).T
        got = to_ints(np.ascontiguousarray(yh), r)
        bad = [i for i in range(N) if got[i] % F.p != want[i]]
        assert not bad, (inverse, bad[:8], len(bad))


@pytest.mark.parametrize("N,s,code", [(4096, 1, "2"), (65536, 1, "w"), (65536, 1, "2"), (65536, 2, "2"),
                                      (2 ** 20, 2, "2"), (2 ** 20, 1, "w")])
def test_fused_pair_all_ones_equals_single_passes(torch_mod, N, s, code):
    """k = 8: a fused launch (code '2' or 'w') on all-ones digits gives
    exactly the two single passes it fuses (pinned above by the closed form)."""
    torch = torch_mod
    F, f = _fields("k8")
    k = F.k
    _, S = _stages(F, N)
    last = s + 1 == S - 1
    for inverse in (False, True):
        x = torch.full((N * k,), -1, dtype=torch.int64, device="cuda")
        mid = torch.empty((N * k,), dtype=torch.int64, device="cuda")
        shape = (k, N) if last else (N * k,)
        y1 = torch.empty(shape, dtype=torch.int64, device="cuda")
        y2 = torch.empty(shape, dtype=torch.int64, device="cuda")
        f.fft_pass(s, x, mid, N, inverse=inverse, in_element_major=True, out_element_major=True)
        f.fft_pass(s + 1, mid, y1, N, inverse=inverse, in_element_major=True, out_element_major=not last)
        f.fft_pass(s, x, y2, N, inverse=inverse, in_element_major=True, out_element_major=not last, code=code)
        torch.cuda.synchronize()
        assert torch.equal(y1, y2), (N, s, code, inverse)
