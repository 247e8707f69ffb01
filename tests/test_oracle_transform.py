"""Pins for oracle.transform: the DFT definition, the radix-2 NTT, the
paper's DFT_general schedule, the tensor identities of sections 1.1 and 4.1
and the polynomial product, against closed forms, the paper's worked
examples, independent machine-integer arithmetic and brute force."""

import json
import os
import random

import pytest

from oracle import transform as T
from oracle.field import GFPField, P8, P16

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _field_and_root(params, N):
    F = GFPField(**params)
    return F, F.paper_root_of_unity(N)


# ---- worked examples of section 4.1 ------------------------------------------------

def test_kronecker_worked_example():
    ex = json.load(open(os.path.join(GOLDEN, "worked_examples.json")))["kronecker"]
    assert T.kron(ex["A"], ex["B"]) == ex["A_kron_B"]


def test_stride_permutation_worked_example():
    ex = json.load(open(os.path.join(GOLDEN, "worked_examples.json")))["stride_permutation"]
    assert T.stride_permutation(ex["input"], ex["m"], ex["n"]) == ex["output"]
    # and the matrix form agrees with the vector form
    M = T.L_matrix(ex["m"], ex["n"])
    assert T.matvec(M, ex["input"], 10 ** 9) == ex["output"]


def test_direct_sum_shape():
    A = [[1, 2], [3, 4]]
    B = [[5]]
    assert T.direct_sum([A, B]) == [[1, 2, 0], [3, 4, 0], [0, 0, 5]]


# ---- DFT definition: closed forms ---------------------------------------------------

@pytest.mark.parametrize("params,N", [(P8, 16), (P8, 64), (P16, 32), (dict(k=8, r=4), 256)])
def test_dft_closed_forms(params, N):
    F, w = _field_and_root(params, N)
    p = F.p
    # delta at s -> column of powers w^(s i)
    for s in (0, 1, N // 2, N - 1):
        x = [0] * N
        x[s] = 1
        assert T.dft(x, w, p) == [pow(w, s * i, p) for i in range(N)]
    # constant 1 -> N at 0, zero elsewhere (geometric sums of roots of unity)
    assert T.dft([1] * N, w, p) == [N % p] + [0] * (N - 1)
    # alternating signs -> N at N/2
    assert T.dft([(-1) ** j % p for j in range(N)], w, p) == [0] * (N // 2) + [N % p] + [0] * (N // 2 - 1)


@pytest.mark.parametrize("params,N", [(P8, 16), (P16, 32), (dict(k=8, r=4), 64)])
def test_dft_inverse_and_linearity(params, N):
    F, w = _field_and_root(params, N)
    p = F.p
    g = random.Random(N)
    x = [g.randrange(p) for _ in range(N)]
    y = [g.randrange(p) for _ in range(N)]
    c = g.randrange(p)
    X, Y = T.dft(x, w, p), T.dft(y, w, p)
    assert T.idft(X, w, p) == x
    assert T.dft([(a + c * b) % p for a, b in zip(x, y)], w, p) == [(a + c * b) % p for a, b in zip(X, Y)]


def test_dft_machine_integers_mod_257():
    """Independent check with machine-size ints on GF(257): w = 3 is a
    primitive root mod 257, so w^(256/N) has order N."""
    p = 257
    for N in (2, 4, 8, 16, 32, 64, 128, 256):
        w = pow(3, 256 // N, p)
        g = random.Random(N)
        x = [g.randrange(p) for _ in range(N)]
        expect = []
        for i in range(N):
            s = 0
            for j in range(N):
                s = (s + x[j] * pow(w, (i * j) % N, p)) % p
            expect.append(s)
        assert T.dft(x, w, p) == expect
        assert T.ntt(x, w, p) == expect


# ---- radix-2 NTT vs definition ------------------------------------------------------

@pytest.mark.parametrize("params,N", [(P8, 16), (P8, 256), (P8, 4096), (P16, 32), (P16, 1024)])
def test_ntt_matches_definition(params, N):
    F, w = _field_and_root(params, N)
    p = F.p
    g = random.Random(N + 1)
    x = [g.randrange(p) for _ in range(N)]
    if N == 4096:  # the O(N^2) definition at N = 4096 on sampled outputs
        X = T.ntt(x, w, p)
        for i in (0, 1, 2, 17, 1000, 2048, 4095):
            assert X[i] == T.horner(x, pow(w, i, p), p)
    else:
        assert T.ntt(x, w, p) == T.dft(x, w, p)
    assert T.intt(T.ntt(x, w, p), w, p) == x


# ---- the paper's DFT_general -------------------------------------------------------

@pytest.mark.parametrize("params,K,e", [(dict(k=8, r=4), 16, 2), (dict(k=4, r=4), 8, 2), (dict(k=2, r=16), 4, 3),
                                        (dict(k=2, r=16), 4, 4), (P8, 16, 2), (P16, 32, 2)])
def test_dft_general_is_natural_order_dft(params, K, e):
    F = GFPField(**params)
    N = K ** e
    w = F.paper_root_of_unity(N) if K == 2 * F.k else None
    if w is None:
        pytest.skip("needs K = 2k")
    assert pow(w, N // K, F.p) == F.r  # the base case runs at w_a = r
    g = random.Random(N)
    x = [g.randrange(F.p) for _ in range(N)]
    assert T.dft_general(x, K, e, w, F.p) == T.dft(x, w, F.p)


# ---- tensor identities (section 1.1 eq. CTCT, section 4.1 eq. sixstepfft) -----------

@pytest.mark.parametrize("J,K", [(2, 4), (4, 2), (4, 4), (2, 8), (8, 2)])
def test_cooley_tukey_identities(J, K):
    p = 257
    N = J * K
    w = pow(3, 256 // N, p)
    DFT_N = T.dft_matrix(N, w, p)
    DFT_J = T.dft_matrix(J, pow(w, K, p), p)
    DFT_K = T.dft_matrix(K, pow(w, J, p), p)
    # eq. (CTCT): DFT_{JK} = (DFT_J (x) I_K) D_{J,K} (I_J (x) DFT_K) L_J^{JK}
    rhs = T.matmul(T.matmul(T.matmul(T.kron(DFT_J, T.identity(K)), T.D_matrix(J, K, w, p), p),
                            T.kron(T.identity(J), DFT_K), p), T.L_matrix(J, K), p)
    assert rhs == DFT_N
    # eq. (sixstepfft): DFT_N = L_K^N (I_J (x) DFT_K) L_J^N D_{K,J} (I_K (x) DFT_J) L_K^N
    six = T.matmul(T.L_matrix(K, J), T.kron(T.identity(J), DFT_K), p)
    six = T.matmul(six, T.L_matrix(J, K), p)
    six = T.matmul(six, T.D_matrix(K, J, w, p), p)
    six = T.matmul(six, T.kron(T.identity(K), DFT_J), p)
    six = T.matmul(six, T.L_matrix(K, J), p)
    assert six == DFT_N


def test_identity_fails_with_planted_transpose():
    """A plausible slip (L_J^{JK} replaced by its inverse L_K^{JK}) breaks
    eq. (CTCT) -- the identity test above can tell the two apart."""
    p, J, K = 257, 2, 4
    N = J * K
    w = pow(3, 256 // N, p)
    DFT_J = T.dft_matrix(J, pow(w, K, p), p)
    DFT_K = T.dft_matrix(K, pow(w, J, p), p)
    wrong = T.matmul(T.matmul(T.matmul(T.kron(DFT_J, T.identity(K)), T.D_matrix(J, K, w, p), p),
                              T.kron(T.identity(J), DFT_K), p), T.L_matrix(K, J), p)
    assert wrong != T.dft_matrix(N, w, p)


# ---- polynomial product --------------------------------------------------------------

def test_polymul_small_closed_form():
    p = 10 ** 9 + 7
    # (1 + x)^2 = 1 + 2x + x^2 ; (1 + x + x^2)(1 - x) = 1 - x^3
    assert T.polymul([1, 1], [1, 1], p) == [1, 2, 1]
    assert T.polymul([1, 1, 1], [1, p - 1], p) == [1, 0, 0, p - 1]
    assert T.polymul([], [1], p) == []


@pytest.mark.parametrize("params", [P8, P16])
def test_polymul_convolution_theorem(params):
    F = GFPField(**params)
    p = F.p
    g = random.Random(3)
    for la, lb in ((1, 1), (3, 5), (8, 8), (17, 9)):
        a = [g.randrange(p) for _ in range(la)]
        b = [g.randrange(p) for _ in range(lb)]
        c = T.polymul(a, b, p)
        N = 2 * F.k
        while N < la + lb - 1:
            N *= 2
        w = F.paper_root_of_unity(N)
        A = T.ntt(a + [0] * (N - la), w, p)
        B = T.ntt(b + [0] * (N - lb), w, p)
        C = T.intt([x * y % p for x, y in zip(A, B)], w, p)
        assert C[:la + lb - 1] == c and all(v == 0 for v in C[la + lb - 1:])
        for m in range(la + lb - 1):
            assert T.polymul_coeff(a, b, m, p) == c[m]
        z = g.randrange(p)
        assert T.horner(c, z, p) == T.horner(a, z, p) * T.horner(b, z, p) % p


def test_horner_matches_power_sum():
    p = 2 ** 61 - 1
    g = random.Random(5)
    coeffs = [g.randrange(p) for _ in range(20)]
    z = g.randrange(p)
    assert T.horner(coeffs, z, p) == sum(c * pow(z, i, p) for i, c in enumerate(coeffs)) % p


@pytest.mark.parametrize("n", [0, 1, 2, 7, 8, 9, 63, 64, 65, 200])
def test_poly_eval_matches_horner_and_power_sum(n):
    """Blocked evaluation (block 8 here, so the lengths cross block
    boundaries) equals Horner and the power sum, for random coefficients on
    the k = 8 workload prime, and for coefficients of every size class."""
    import random

    F = GFPField(**P8)
    p = F.p
    g = random.Random(n)
    coeffs = [g.randrange(p) for _ in range(n)]
    for z in (0, 1, p - 1, g.randrange(p)):
        want = sum(c * pow(z, i, p) for i, c in enumerate(coeffs)) % p
        assert T.poly_eval(coeffs, z, p, block=8) == want
        assert T.poly_eval(coeffs, z, p) == want
        assert T.horner(coeffs, z, p) == want
