"""Baillie-PSW probable-prime test (oracle; test infrastructure only).

The paper takes its primes p = r^k + 1 from Table 1 (section 2, "SRGFNs of
practical interest") and Table testprimes (section 5.3) without saying how
primality was established.  The oracle checks them with BPSW: a strong
Fermat test to base 2 followed by a strong Lucas test with Selfridge's
parameter choice (method A).  No composite passing BPSW is known.

Written from the textbook definitions (Baillie & Wagstaff 1980; Crandall &
Pomerance, "Prime Numbers", sections 3.5-3.6); plain Python integers.
"""

_SMALL_PRIMES = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61, 67, 71, 73, 79, 83, 89, 97]


def jacobi(a: int, n: int) -> int:
    """Jacobi symbol (a/n) for odd n > 0, by quadratic reciprocity."""
    if n <= 0 or n % 2 == 0:
        raise ValueError("n must be odd and positive")
    a %= n
    result = 1
    while a != 0:
        while a % 2 == 0:
            a //= 2
            if n % 8 in (3, 5):
                result = -result
        a, n = n, a
        if a % 4 == 3 and n % 4 == 3:
            result = -result
        a %= n
    return result if n == 1 else 0


def is_square(n: int) -> bool:
    if n < 0:
        return False
    s = _isqrt(n)
    return s * s == n


def _isqrt(n: int) -> int:
    if n < 2:
        return n
    x = 1 << ((n.bit_length() + 1) // 2)
    while True:
        y = (x + n // x) // 2
        if y >= x:
            return x
        x = y


def strong_fermat(n: int, base: int) -> bool:
    """Strong probable-prime test: n - 1 = d * 2^s with d odd; n passes if
    base^d = 1 or base^(d 2^j) = -1 (mod n) for some 0 <= j < s."""
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    x = pow(base, d, n)
    if x == 1 or x == n - 1:
        return True
    for _ in range(s - 1):
        x = x * x % n
        if x == n - 1:
            return True
    return False


def _selfridge(n: int):
    """First D in 5, -7, 9, -11, ... with (D/n) = -1; P = 1, Q = (1 - D)/4."""
    d = 5
    while True:
        j = jacobi(d, n)
        if j == -1:
            return d, 1, (1 - d) // 4
        if j == 0 and abs(d) != n:
            return None  # nontrivial common factor: composite
        d = -d - 2 if d > 0 else -d + 2


def strong_lucas(n: int) -> bool:
    """Strong Lucas probable-prime test with Selfridge parameters.

    n + 1 = d * 2^s with d odd; n passes if U_d = 0 or V_(d 2^j) = 0 (mod n)
    for some 0 <= j < s, where U, V are the Lucas sequences of (P, Q)."""
    if is_square(n):
        return False
    params = _selfridge(n)
    if params is None:
        return False
    D, P, Q = params
    d, s = n + 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1

    def half(x):  # x / 2 mod n
        return (x + n) // 2 % n if x % 2 else x // 2 % n

    # Left-to-right binary evaluation of (U_d, V_d, Q^d).
    U, V, Qk = 1, P % n, Q % n  # index 1
    for bit in bin(d)[3:]:
        # doubling: U_2m = U_m V_m, V_2m = V_m^2 - 2 Q^m
        U, V = U * V % n, (V * V - 2 * Qk) % n
        Qk = Qk * Qk % n
        if bit == "1":
            # increment: U_(m+1) = (P U_m + V_m)/2, V_(m+1) = (D U_m + P V_m)/2
            U, V = half(P * U + V), half(D * U + P * V)
            Qk = Qk * Q % n
    if U == 0 or V == 0:
        return True
    for _ in range(s - 1):
        V = (V * V - 2 * Qk) % n
        Qk = Qk * Qk % n
        if V == 0:
            return True
    return False


def is_probable_prime(n: int) -> bool:
    """Baillie-PSW: trial division, strong Fermat base 2, strong Lucas."""
    if n < 2:
        return False
    for q in _SMALL_PRIMES:
        if n == q:
            return True
        if n % q == 0:
            return False
    return strong_fermat(n, 2) and strong_lucas(n)
