"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds no field arithmetic: it only draws digits.  An element of
Z/pZ, p = r^k + 1, is k radix-r digits (least significant first); a uniform
draw of k independent digits in [0, r) is a uniform draw from [0, r^k) =
[0, p - 1), which differs from uniform on [0, p) only by missing the single
value p - 1 (probability 1/p, below 2^-500 for the primes used here).  That
value, and the other edge patterns below, are injected explicitly.

Arrays are structure-of-arrays: shape (k, n), dtype uint64, row d holding
digit d of every element -- the layout the library takes.

Seeds: workload c uses base seed 1811014900 + c; operand a is stream 0,
operand b stream 1, request i of a batch or request stream is stream 2 + i.
"""

from __future__ import annotations

import numpy as np

BASE_SEED = 1811014900


def rng(seed: int, stream: int = 0) -> np.random.Generator:
    """PCG64 generator for (seed, stream)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(stream,))))


def uniform_digits(k: int, r: int, n: int, seed: int, stream: int = 0) -> np.ndarray:
    """(k, n) uint64 array of independent uniform digits in [0, r).

    Rejection sampling on words masked to bit_length(r) bits, drawn in
    chunks so the result depends only on (k, r, n, seed, stream)."""
    if not (2 <= r < 2 ** 64):
        raise ValueError("r must fit in 64 bits")
    g = rng(seed, stream)
    bits = int(r).bit_length()
    mask = np.uint64((1 << bits) - 1) if bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    rr = np.uint64(r)
    need = k * n
    out = np.empty(need, dtype=np.uint64)
    filled = 0
    while filled < need:
        chunk = max(1024, int((need - filled) * 2.2))
        w = g.integers(0, 2 ** 64, size=chunk, dtype=np.uint64, endpoint=False) & mask
        w = w[w < rr]
        take = min(len(w), need - filled)
        out[filled:filled + take] = w[:take]
        filled += take
    return out.reshape(k, n)


def edge_patterns(k: int, r: int) -> list:
    """Digit vectors (least significant first) of values that uniform
    sampling essentially never produces: 0, 1, p - 1 (written with top digit
    r), r^(k-1), r^k - 1 (every digit r - 1), r - 1, (r-1) r^(k-1), 2,
    r^(k-1) + 1, and one with alternating 0 / r-1 digits."""
    pats = [
        [0] * k,
        [1] + [0] * (k - 1),
        [0] * (k - 1) + [r],
        [0] * (k - 1) + [1],
        [r - 1] * k,
        [r - 1] + [0] * (k - 1),
        [0] * (k - 1) + [r - 1],
        [2] + [0] * (k - 1),
        [1] + [0] * (k - 2) + [1],
        [(r - 1) if i % 2 else 0 for i in range(k)],
    ]
    return pats


def inject_edges(x: np.ndarray, r: int, frac: float, seed: int, stream: int = 0) -> np.ndarray:
    """Overwrite about ``frac`` of the columns of x (shape (k, n)) with edge
    patterns at seeded positions; the first few positions are always hit.
    Returns x (modified in place)."""
    k, n = x.shape
    if n == 0:
        return x
    pats = edge_patterns(k, r)
    g = rng(seed, 1000 + stream)
    count = max(len(pats), int(round(frac * n)))
    count = min(count, n)
    pos = g.choice(n, size=count, replace=False)
    pos[: min(len(pats), count)] = np.arange(min(len(pats), count))  # always include the head
    for t, c in enumerate(pos):
        x[:, c] = np.array(pats[t % len(pats)], dtype=np.uint64)
    return x


def operand(k: int, r: int, n: int, seed: int, stream: int, edge_frac: float = 0.0) -> np.ndarray:
    """Uniform operand of n elements, optionally with injected edge values."""
    x = uniform_digits(k, r, n, seed, stream)
    if edge_frac > 0:
        inject_edges(x, r, edge_frac, seed, stream)
    return x


def sample_indices(n: int, count: int, seed: int, stream: int = 0, must=()) -> list:
    """Seeded distinct indices in [0, n) for spot checks, plus ``must``."""
    g = rng(seed, 2000 + stream)
    count = min(count, n)
    idx = set(int(i) for i in g.choice(n, size=count, replace=False)) if n else set()
    idx.update(int(m) % n for m in must if n)
    return sorted(idx)
