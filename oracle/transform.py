"""DFTs and polynomial products over Z/pZ (oracle; test infrastructure only).

Plain definitions first:

* ``dft``      Y_i = sum_j X_j w^(ij) mod p, i = 0..N-1, natural order: the
               values f(w^0), ..., f(w^(N-1)) of section 1.1.
* ``idft``     X_j = N^-1 sum_i Y_i w^(-ij): the inverse of Alg. Fast
               Convolution (section 3.3), (1/n) DFT at w^-1.
* ``polymul``  c_m = sum_{i+j=m} a_i b_j mod p (schoolbook).
* ``horner``   f(z) mod p.
* ``poly_eval`` the same value as a sum of blocks of B coefficients,
               f(z) = sum_b (z^B)^b sum_{i<B} c_{bB+i} z^i, one reduction
               per block (faster for long vectors; pinned against horner).

Then, for sizes where the O(N^2) definition is too slow:

* ``ntt``      a textbook iterative radix-2 Cooley-Tukey transform (bit
               reversal, then log2 N butterfly levels).  Same output as
               ``dft``; pinned against it by tests.

And the paper's own schedule, kept to check that reading of the paper:

* ``stride_permutation``, ``twiddle``, ``dft_general``: Alg. DFT_general of
  section 4.3 with the stride permutation L_m^{mn} and twiddle D of
  section 4.1, base case DFT_K at w^(N/K).
* ``kron``, ``direct_sum``, ``L_matrix``, ``D_matrix``, ``dft_matrix``:
  the tensor-algebra operators of section 4.1 as explicit matrices, used by
  tests to check eq. (CTCT) of section 1.1 and eq. (sixstepfft) of
  section 4.1 on small sizes.
"""

from __future__ import annotations


def dft(x, w: int, p: int) -> list:
    """Definition of the DFT at w (natural order)."""
    n = len(x)
    out = []
    for i in range(n):
        wi = pow(w, i, p)
        acc, t = 0, 1
        for j in range(n):
            acc += x[j] * t
            t = t * wi % p
        out.append(acc % p)
    return out


def idft(y, w: int, p: int) -> list:
    """Inverse DFT: N^-1 times the DFT at w^-1 (section 3.3)."""
    n = len(y)
    winv = pow(w, p - 2, p)
    ninv = pow(n, p - 2, p)
    return [v * ninv % p for v in dft(y, winv, p)]


def _bit_reverse(i: int, bits: int) -> int:
    return int(format(i, "0%db" % bits)[::-1], 2) if bits else 0


def ntt(x, w: int, p: int) -> list:
    """Textbook radix-2 decimation-in-time transform, natural order in and
    out.  Requires len(x) a power of two and w of that exact order."""
    n = len(x)
    bits = n.bit_length() - 1
    if 1 << bits != n:
        raise ValueError("length must be a power of two")
    a = [x[_bit_reverse(i, bits)] % p for i in range(n)]
    size = 2
    while size <= n:
        wm = pow(w, n // size, p)  # primitive size-th root
        half = size // 2
        for start in range(0, n, size):
            t = 1
            for j in range(half):
                u = a[start + j]
                v = a[start + j + half] * t % p
                a[start + j] = (u + v) % p
                a[start + j + half] = (u - v) % p
                t = t * wm % p
        size *= 2
    return a


def intt(y, w: int, p: int) -> list:
    n = len(y)
    winv = pow(w, p - 2, p)
    ninv = pow(n, p - 2, p)
    return [v * ninv % p for v in ntt(y, winv, p)]


def polymul(a, b, p: int) -> list:
    """Schoolbook product; len(a) + len(b) - 1 coefficients."""
    if not a or not b:
        return []
    c = [0] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        if ai:
            for j, bj in enumerate(b):
                c[i + j] += ai * bj
    return [v % p for v in c]


def polymul_coeff(a, b, m: int, p: int) -> int:
    """One coefficient c_m of the product, O(min(len a, len b))."""
    lo = max(0, m - (len(b) - 1))
    hi = min(m, len(a) - 1)
    acc = 0
    for i in range(lo, hi + 1):
        acc += a[i] * b[m - i]
    return acc % p


def horner(coeffs, z: int, p: int) -> int:
    acc = 0
    for c in reversed(coeffs):
        acc = (acc * z + c) % p
    return acc


def poly_eval(coeffs, z: int, p: int, block: int = 1024) -> int:
    """f(z) mod p for f = sum_i c_i z^i, by blocks: the powers z^0 .. z^(B-1)
    are formed once, each block of B coefficients is a plain sum of products
    (reduced once), and the blocks are combined from the top with z^B."""
    n = len(coeffs)
    if n == 0:
        return 0
    width = min(block, n)
    powers = [1] * width
    for i in range(1, width):
        powers[i] = powers[i - 1] * z % p
    z_block = powers[-1] * z % p
    acc = 0
    for start in range(((n - 1) // block) * block, -1, -block):
        part = sum(c * w for c, w in zip(coeffs[start:start + block], powers))
        acc = (acc * z_block + part) % p
    return acc


# ---------------------------------------------------------------------------
# Section 4.1 operators as explicit matrices (lists of lists mod p)
# ---------------------------------------------------------------------------

def kron(A, B):
    """Tensor (Kronecker) product: block (i, j) is a_ij B (eq. TensorProduct)."""
    m, n = len(A), len(A[0])
    q, s = len(B), len(B[0])
    out = [[0] * (n * s) for _ in range(m * q)]
    for i in range(m):
        for j in range(n):
            for u in range(q):
                for v in range(s):
                    out[i * q + u][j * s + v] = A[i][j] * B[u][v]
    return out


def direct_sum(mats):
    """Block-diagonal matrix A_0 (+) A_1 (+) ... (eq. DirectSum2)."""
    rows = sum(len(M) for M in mats)
    cols = sum(len(M[0]) for M in mats)
    out = [[0] * cols for _ in range(rows)]
    r0 = c0 = 0
    for M in mats:
        for i, row in enumerate(M):
            for j, v in enumerate(row):
                out[r0 + i][c0 + j] = v
        r0 += len(M)
        c0 += len(M[0])
    return out


def identity(n):
    return [[1 if i == j else 0 for j in range(n)] for i in range(n)]


def matmul(A, B, p):
    n, m, q = len(A), len(B), len(B[0])
    out = [[0] * q for _ in range(n)]
    for i in range(n):
        for t in range(m):
            a = A[i][t]
            if a:
                row = B[t]
                for j in range(q):
                    out[i][j] += a * row[j]
    return [[v % p for v in row] for row in out]


def matvec(A, x, p):
    return [sum(a * b for a, b in zip(row, x)) % p for row in A]


def stride_permutation(x, m: int, n: int) -> list:
    """L_m^{mn} applied to a vector (section 4.1): the vector is an n x m
    row-major matrix and the result its transpose, i.e. output position
    i*n + j takes input position j*m + i (0 <= i < m, 0 <= j < n)."""
    if len(x) != m * n:
        raise ValueError("length must be m*n")
    return [x[j * m + i] for i in range(m) for j in range(n)]


def L_matrix(m: int, n: int):
    """Matrix of L_m^{mn}: row i*n + j has its 1 in column j*m + i."""
    N = m * n
    M = [[0] * N for _ in range(N)]
    for i in range(m):
        for j in range(n):
            M[i * n + j][j * m + i] = 1
    return M


def D_matrix(K: int, J: int, w: int, p: int):
    """Twiddle D_{K,J} = (+)_{j<K} diag(1, w^j, ..., w^(j(J-1))) with w a
    primitive KJ-th root (eq. twiddle of section 4.1)."""
    blocks = []
    for j in range(K):
        blocks.append([[pow(w, j * i, p) if i == t else 0 for t in range(J)] for i in range(J)])
    return direct_sum(blocks)


def dft_matrix(n: int, w: int, p: int):
    return [[pow(w, i * j, p) for j in range(n)] for i in range(n)]


def twiddle(v, m: int, n: int, w: int, p: int) -> list:
    """Section 4.3's twiddle step on a block of n*m entries: entry j*m + i
    is multiplied by w^(i j), 0 <= i < m, 0 <= j < n."""
    out = list(v)
    for j in range(n):
        for i in range(m):
            out[j * m + i] = out[j * m + i] * pow(w, i * j, p) % p
    return out


def dft_general(x, K: int, e: int, w: int, p: int) -> list:
    """Alg. DFT_general (section 4.3): DFT of size N = K^e at w.

    Step 1 permutes nested blocks into place; step 2 runs DFT_K at
    w_a = w^(K^(e-1)) on consecutive blocks of K; then for i = e-2 down to 0
    each block of size K^(e-i) is twiddled at w_i = w^(K^i) and permuted, the
    DFT_K pass runs again, and the blocks are permuted back.  DFT_K here is
    the definition (``dft``) at w_a; for p = r^k + 1 and K = 2k, w_a = r."""
    N = K ** e
    if len(x) != N:
        raise ValueError("length must be K^e")
    a = [v % p for v in x]

    def on_block(start, size, fn):
        a[start:start + size] = fn(a[start:start + size])

    for i in range(e - 1):  # step 1
        size = K ** (e - i)
        for j in range(K ** i):
            on_block(j * size, size, lambda b: stride_permutation(b, K, K ** (e - i - 1)))
    wa = pow(w, K ** (e - 1), p)
    for j in range(K ** (e - 1)):  # step 2
        on_block(j * K, K, lambda b: dft(b, wa, p))
    for i in range(e - 2, -1, -1):
        wi = pow(w, K ** i, p)
        size = K ** (e - i)
        for j in range(K ** i):  # steps 3 and 4
            on_block(j * size, size, lambda b: twiddle(b, K ** (e - i - 1), K, wi, p))
            on_block(j * size, size, lambda b: stride_permutation(b, K ** (e - i - 1), K))
        for j in range(K ** (e - 1)):  # step 5
            on_block(j * K, K, lambda b: dft(b, wa, p))
        for j in range(K ** i):  # step 6
            on_block(j * size, size, lambda b: stride_permutation(b, K, K ** (e - i - 1)))
    return a
