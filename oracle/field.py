"""The prime field Z/pZ, p = r^k + 1 (oracle; test infrastructure only).

Section 2 of the paper ("Generalized Fermat prime fields").  Elements are
written in radix r with k digits (the element-representation equation of
section 2): x = x_{k-1} r^{k-1} + ... + x_1 r + x_0 with every digit in
[0, r), except that p - 1 = r^k is written with x_{k-1} = r and all other
digits 0.  That makes the representation unique, so comparing canonical
digit vectors is comparing field elements.

Two kinds of code live here:

* plain definitions (``add``, ``sub``, ``mul``, ``pow``, ``inv`` on Python
  integers modulo p, ``to_int``/``from_int`` for the encoding) -- these are
  what the parity tests compare against;
* the paper's own element algorithms, taken step by step from the text
  (``paper_add`` = Alg. 2 of section 2.2, ``paper_sub`` = the subtraction
  the text names but never prints, ``paper_mul_pow_r`` = the signed
  cyclic shift of section 2.3, ``paper_mul`` = Alg. 3 of section 2.4 with
  the column formula and (l, h, c) split of section 3.1.1,
  ``paper_root_of_unity`` = Alg. 1 of section 2.1).  They work on digit vectors with unbounded Python integers,
  so the 64-bit overflow the printed C would hit for r > 2^63 cannot occur
  here.  Tests pin them to the plain definitions.
"""

from __future__ import annotations

from dataclasses import dataclass, field as dc_field

from .primality import is_probable_prime


def v2(n: int) -> int:
    """2-adic valuation of n > 0."""
    if n <= 0:
        raise ValueError("n must be positive")
    return (n & -n).bit_length() - 1


@dataclass(frozen=True)
class GFPField:
    """Z/pZ with p = r^k + 1, k a power of two, p prime (section 2)."""

    k: int
    r: int
    p: int = dc_field(init=False)

    def __post_init__(self):
        if self.k < 1 or self.k & (self.k - 1):
            raise ValueError("k must be a power of two")
        if self.r < 2 or self.r % 2:
            raise ValueError("r must be even and >= 2 so that p = r^k + 1 is odd")
        object.__setattr__(self, "p", self.r ** self.k + 1)

    # -- structure -----------------------------------------------------------------
    def is_prime(self) -> bool:
        return is_probable_prime(self.p)

    @property
    def max_log2_n(self) -> int:
        """Largest e with 2^e | p - 1: the longest power-of-two FFT
        (Table 1, second column).  p - 1 = r^k, so it is k * v2(r)."""
        return v2(self.p - 1)

    @property
    def K(self) -> int:
        """Base-case size 2k: r is a primitive 2k-th root of unity."""
        return 2 * self.k

    # -- encoding (section 2, element representation) ----------------------------
    def to_int(self, digits) -> int:
        """Value of a digit vector, least significant digit first."""
        if len(digits) != self.k:
            raise ValueError("expected %d digits" % self.k)
        v = 0
        for d in reversed(digits):
            v = v * self.r + int(d)
        return v

    def is_canonical(self, digits) -> bool:
        ds = [int(d) for d in digits]
        if len(ds) != self.k or any(d < 0 for d in ds):
            return False
        if ds[-1] == self.r and all(d == 0 for d in ds[:-1]):
            return True  # the encoding of p - 1
        return all(d < self.r for d in ds)

    def from_int(self, v: int) -> list:
        """Canonical digits of v mod p."""
        v %= self.p
        if v == self.p - 1:
            return [0] * (self.k - 1) + [self.r]
        out = []
        for _ in range(self.k):
            v, d = divmod(v, self.r)
            out.append(d)
        assert v == 0
        return out

    # -- plain arithmetic (definitions) ------------------------------------------
    def add(self, a: int, b: int) -> int:
        return (a + b) % self.p

    def sub(self, a: int, b: int) -> int:
        return (a - b) % self.p

    def mul(self, a: int, b: int) -> int:
        return a * b % self.p

    def pow(self, a: int, e: int) -> int:
        return pow(a, e, self.p)

    def inv(self, a: int) -> int:
        if a % self.p == 0:
            raise ZeroDivisionError("0 has no inverse")
        return pow(a, self.p - 2, self.p)

    # -- the paper's element algorithms on digit vectors -----------------------
    def paper_add(self, x, y) -> list:
        """Alg. 2 (section 2.2, BigPrimeFieldAddition).

        Digit-wise sums with carry in radix r; a carry out of the top digit
        stands for r^k = -1, so it is taken away again: the lowest nonzero
        digit is decremented and the digits below it become r - 1; if every
        digit is zero the result is r^k = p - 1, written (r, 0, ..., 0).
        The digit sums are integers (reading: 'in Z/pZ' in step 1 of the
        printed algorithm means the plain integer sum).  Reading: with the
        Euclidean division of step 4 the top carry z_k is 2 when a top digit
        r meets a top digit sum of r (e.g. (p-1) + (p-1)); the 'subtract one'
        of steps 6-7 is then applied z_k times, the second time starting from
        the (r, 0, ..., 0) encoding, which gives the worked example's
        r^k + r^k = (r-1, ..., r-1)."""
        k, r = self.k, self.r
        z = [int(a) + int(b) for a, b in zip(x, y)] + [0]
        for i in range(k):
            q, s = divmod(z[i], r)
            z[i], z[i + 1] = s, z[i + 1] + q
        out = z[:k]
        assert z[k] in (0, 1, 2)
        for _ in range(z[k]):
            if all(d == 0 for d in out):
                out = [0] * (k - 1) + [r]  # 0 - 1 = r^k = p - 1
                continue
            i0 = next(i for i in range(k) if out[i] != 0)
            out[i0] -= 1
            for i in range(i0):
                out[i] = r - 1
        return out

    def paper_neg(self, x) -> list:
        """-x from digits: r^k - X = (r - 1 - x_i) digits + 1, i.e. p - 1 - X
        in radix r with the p - 1 encoding handled first."""
        k, r = self.k, self.r
        xs = [int(d) for d in x]
        if all(d == 0 for d in xs):
            return [0] * k
        if xs[-1] == r:  # x = p - 1, -x = 1
            return [1] + [0] * (k - 1)
        # p - x = r^k + 1 - X; r^k - 1 - X has digits r - 1 - x_i (no borrow),
        # then add 2 with carry (cannot reach r^k + 1 since X >= 1).
        z = [r - 1 - d for d in xs]
        return self.paper_add(z, [2] + [0] * (k - 1)) if k > 1 else self.from_int(self.to_int(z) + 2)

    def paper_sub(self, x, y) -> list:
        """x - y (section 2.2 names BigPrimeFieldSubtraction without printing
        it; reading: x + (-y) with the digit negation above)."""
        return self.paper_add(x, self.paper_neg(y))

    def paper_mul_pow_r(self, x, s: int) -> list:
        """x * r^s (section 2.3: multiplying by a power of r is a cyclic shift
        of the digits in which every digit that passes r^(k-1) changes sign,
        because r^k = -1).

        Written from that identity: r has order 2k, so only s mod 2k
        matters; r^s = (-1)^e r^t with s = e k + t, 0 <= t < k.  Digit i of x
        then lands at position (i + t) mod k, with sign -1 when i + t >= k,
        and the whole vector takes the sign (-1)^e.  The signed digits are
        summed as an integer and brought back to the canonical encoding by
        from_int, so the p - 1 encoding (top digit r) needs no special case:
        its digit r simply moves like any other digit."""
        k, r = self.k, self.r
        e, t = divmod(s % (2 * k), k)
        signed = [0] * k
        for i, d in enumerate(int(v) for v in x):
            pos = i + t
            signed[pos % k] += -d if pos >= k else d
        value = sum(d * r ** j for j, d in enumerate(signed))
        return self.from_int(-value if e else value)

    def paper_negacyclic_columns(self, x, y) -> list:
        """u_m = sum_{i+j=m} x_i y_j - sum_{i+j=k+m} x_i y_j, 0 <= m < k:
        f_x f_y mod (R^k + 1) over Z (section 3.1.1, general column formula;
        the expanded rows printed above it repeat R^(k-2) and mis-index one
        negative term -- reading: the general formula is authoritative)."""
        k = self.k
        u = [0] * k
        for i in range(k):
            for j in range(k):
                if i + j < k:
                    u[i + j] += int(x[i]) * int(y[j])
                else:
                    u[i + j - k] -= int(x[i]) * int(y[j])
        return u

    def paper_lhc(self, u: int):
        """(l, h, c) with u = c r^2 + h r + l, 0 <= h, l < r (section 3.1.1).
        For negative u the paper asks c u >= 0; floor division gives
        0 <= l, h < r with c possibly negative, which is that split."""
        r = self.r
        c, rest = divmod(u, r * r)
        h, l = divmod(rest, r)
        return l, h, c

    def paper_mul(self, x, y) -> list:
        """Alg. 3 (section 2.4) with the refinements of section 3.1.1.

        1. u = f_x f_y mod (R^k + 1) over Z (negacyclic columns).
        2. each u_i = c_i r^2 + h_i r + l_i.
        3. l, h r, c r^2 as three field elements: h shifted up one digit and c
           two digits, the digits pushed past r^(k-1) wrapping with a minus
           sign (reading: the printed shifted vectors omit that sign, the
           cyclic shift of section 2.3 supplies it).
        4. u = l + h + c by the field addition."""
        k = self.k
        cols = self.paper_negacyclic_columns(x, y)
        lhc = [self.paper_lhc(u) for u in cols]
        # Each (l_i, h_i, c_i) contributes (l_i + h_i r + c_i r^2) r^i.  Build
        # l, h, c as field elements from their digit vectors, using the plain
        # encoding for the (possibly negative) c_i, then shift by r, r^2.
        l_vec = [t[0] for t in lhc]
        h_vec = [t[1] for t in lhc]
        c_val = 0
        for i, (_, _, c) in enumerate(lhc):
            c_val += c * self.r ** i
        l_el = self.from_int(self.to_int(l_vec))
        h_el = self.paper_mul_pow_r(self.from_int(self.to_int(h_vec)), 1)
        c_el = self.paper_mul_pow_r(self.from_int(c_val), 2)
        return self.paper_add(self.paper_add(l_el, h_el), c_el)

    # -- roots of unity (section 2.1) --------------------------------------------
    def smallest_nonresidue(self) -> int:
        """Smallest h >= 2 with h^((p-1)/2) = -1 (Euler's criterion).

        Alg. 1 takes a primitive N-th root g as input and the paper does not
        say where g comes from; reading: g = h^((p-1)/N) for this h.  Then g
        has order exactly N because N is a power of two dividing p - 1 and h
        generates the full 2-Sylow subgroup of (Z/pZ)^*."""
        h = 2
        while pow(h, (self.p - 1) // 2, self.p) != self.p - 1:
            h += 1
        return h

    def paper_root_of_unity(self, N: int) -> int:
        """Alg. 1 (section 2.1): a primitive N-th root w with w^(N/2k) = r.

        a = g^(N/2k) is a primitive 2k-th root, hence a power of r; step j
        until a^j = r and return w = g^j."""
        k = self.k
        if N < 2 * k or N & (N - 1) or (self.p - 1) % N:
            raise ValueError("N must be a power of two, 2k <= N, N | p - 1")
        g = pow(self.smallest_nonresidue(), (self.p - 1) // N, self.p)
        a = pow(g, N // (2 * k), self.p)
        b, j = a, 1
        while b != self.r:
            b = b * a % self.p
            j += 1
        return pow(g, j, self.p)


# Primes of the workloads (Table 1 rows 3 to 6).
P8 = dict(k=8, r=2 ** 63 + 2 ** 34)
P16 = dict(k=16, r=2 ** 62 + 2 ** 36)
P32 = dict(k=32, r=2 ** 62 + 2 ** 56)
P64 = dict(k=64, r=2 ** 63 - 2 ** 40)
