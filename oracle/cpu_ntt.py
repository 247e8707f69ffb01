"""Multithreaded C++ transform over Z/pZ (oracle side; test and measurement
infrastructure only).

Python side of ``cpu_ntt.cpp``: builds it with g++ into ``libcpu_ntt.so``
beside the source, loads it with ctypes and passes SoA digit arrays (shape
(k, n), uint64, the canonical encoding of section 2).  It is the timed CPU
baseline: the same values as ``oracle.transform.ntt`` / ``intt`` / the
schoolbook product (pinned by tests), computed by a textbook radix-2
transform with schoolbook multiprecision Montgomery arithmetic over all
given threads.  Roots of unity come from ``oracle.field`` (Alg. 1).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_ntt.cpp")
LIB = os.path.join(HERE, "libcpu_ntt.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile cpu_ntt.cpp (g++, -O2, pthreads) unless an up-to-date build exists."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-pthread", "-shared", "-fPIC", "-o", tmp, SRC])
    os.replace(tmp, LIB)
    return LIB


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        l_ = ctypes.CDLL(build())
        u64, p64 = ctypes.c_uint64, ctypes.c_void_p
        l_.cpu_ntt_transform.argtypes = [ctypes.c_int, u64, u64, p64, p64, p64, ctypes.c_int, ctypes.c_int]
        l_.cpu_ntt_transform.restype = ctypes.c_int
        l_.cpu_ntt_polymul.argtypes = [ctypes.c_int, u64, u64, p64, u64, p64, p64, u64, p64, p64, ctypes.c_int]
        l_.cpu_ntt_polymul.restype = ctypes.c_int
        _lib = l_
    return _lib


def default_threads() -> int:
    """Worker threads: OMP_NUM_THREADS when set, else the CPUs this process may run on."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def _digits(v: int, k: int, r: int) -> np.ndarray:
    """Canonical digits of a field element given as an integer < p."""
    if v == r ** k:
        return np.array([0] * (k - 1) + [r], dtype=np.uint64)
    out = []
    for _ in range(k):
        v, d = divmod(v, r)
        out.append(d)
    return np.array(out, dtype=np.uint64)


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


def transform(k: int, r: int, x: np.ndarray, w: int, inverse: bool = False, threads: int = 0) -> np.ndarray:
    """Y_i = sum_j X_j w^(ij) for x of shape (k, n); inverse=True also
    multiplies by 1/n (pass w^-1 for the inverse transform)."""
    x = np.ascontiguousarray(x, dtype=np.uint64)
    n = x.shape[1]
    y = np.empty_like(x)
    wd = _digits(w, k, r)
    rc = lib().cpu_ntt_transform(k, r, n, _ptr(x), _ptr(y), _ptr(wd), int(inverse), threads or default_threads())
    if rc:
        raise ValueError("cpu_ntt_transform: bad arguments")
    return y


def polymul(k: int, r: int, a: np.ndarray, b: np.ndarray, n: int, w: int, w_inv: int,
            threads: int = 0) -> np.ndarray:
    """c = a b (la + lb - 1 coefficients) through transforms of size n."""
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    la, lb = a.shape[1], b.shape[1]
    c = np.empty((k, la + lb - 1), dtype=np.uint64)
    wd, wid = _digits(w, k, r), _digits(w_inv, k, r)
    rc = lib().cpu_ntt_polymul(k, r, la, _ptr(a), lb, _ptr(b), _ptr(c), n, _ptr(wd), _ptr(wid),
                               threads or default_threads())
    if rc:
        raise ValueError("cpu_ntt_polymul: bad arguments")
    return c
