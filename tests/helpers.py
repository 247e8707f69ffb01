"""Test-side conversions between SoA digit arrays and oracle integers."""

import numpy as np


def to_ints(x: np.ndarray, r: int) -> list:
    """(k, n) uint64 digits -> list of Python ints sum_d x_d r^d."""
    k = x.shape[0]
    obj = x.astype(object)
    val = obj[k - 1].copy()
    for d in range(k - 2, -1, -1):
        val = val * r + obj[d]
    return [int(v) for v in val]


def canonical_mask(x: np.ndarray, r: int) -> np.ndarray:
    """Columns that are in the canonical encoding of section 2."""
    k = x.shape[0]
    rr = np.uint64(r)
    below = (x < rr).all(axis=0)
    pm1 = (x[k - 1] == rr) & (x[: k - 1] == 0).all(axis=0)
    return below | pm1


def from_ints(vals, k: int, r: int, p: int) -> np.ndarray:
    """Canonical digits (k, n) of a list of ints (oracle-side encoding)."""
    from oracle.field import GFPField

    F = GFPField(k, r)
    out = np.empty((k, len(vals)), dtype=np.uint64)
    for i, v in enumerate(vals):
        out[:, i] = np.array(F.from_int(v), dtype=np.uint64)
    return out
