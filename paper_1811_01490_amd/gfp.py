"""Python binding of libgfpfft (ctypes).  Argument marshalling only: every
step of the transforms runs in the HIP library; PyTorch provides device
memory and streams.

Vectors are torch tensors of shape (k, ld), dtype int64 or uint64 (the bit
pattern is what matters), on a HIP device, row-major with unit stride along
the element axis: digit d of element i is t[d, i].  Only the first n
columns are read or written.
"""

from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgfpfft.so")

GFP_OK = 0
GFP_EINVAL = 1
GFP_EUNSUPPORTED = 2
GFP_ENOMEM = 3
GFP_EAGAIN = 4
GFP_EDEVICE = 5
GFP_ENOTPRIME = 6
GFP_ECANCELED = 7
GFP_EPENDING = 8
GFP_ENOTREADY = 9
STATIC_SCRATCH_BYTES = 32 << 20

OP_ADD, OP_SUB, OP_MUL, OP_MUL_POW_R, OP_MUL_CONST, OP_MUL_SCALE, OP_MUL_NTT = range(7)
BATCH_GRAPH = 1
BATCH_PERSISTENT = 2
SERVER_EAGER = 1
LAYOUT_DIGIT_MAJOR, LAYOUT_ELEMENT_MAJOR = 0, 1


class PolymulDesc(ctypes.Structure):
    """gfp_polymul_desc"""
    _fields_ = [("a", ctypes.c_void_p), ("la", ctypes.c_uint64), ("ld_a", ctypes.c_uint64),
                ("b", ctypes.c_void_p), ("lb", ctypes.c_uint64), ("ld_b", ctypes.c_uint64),
                ("c", ctypes.c_void_p), ("ld_c", ctypes.c_uint64)]

class ServerConfig(ctypes.Structure):
    """gfp_server_config"""
    _fields_ = [("workspace_bytes", ctypes.c_uint64), ("slots", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("max_pending", ctypes.c_uint32), ("max_wait_us", ctypes.c_uint32), ("device", ctypes.c_int32),
                ("express_log2n", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class Request(ctypes.Structure):
    """gfp_request"""
    _fields_ = [("field", ctypes.c_void_p), ("a", ctypes.c_void_p), ("la", ctypes.c_uint64), ("ld_a", ctypes.c_uint64),
                ("b", ctypes.c_void_p), ("lb", ctypes.c_uint64), ("ld_b", ctypes.c_uint64),
                ("c", ctypes.c_void_p), ("ld_c", ctypes.c_uint64), ("ready_event", ctypes.c_void_p)]


class Result(ctypes.Structure):
    """gfp_result"""
    _fields_ = [("status", ctypes.c_int32), ("batch_size", ctypes.c_uint32), ("batch_id", ctypes.c_uint64),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64), ("t_launch_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class ServerStats(ctypes.Structure):
    """gfp_server_stats"""
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("max_batch_size", ctypes.c_uint64),
                ("max_batch_workspace", ctypes.c_uint64), ("overlapped_batches", ctypes.c_uint64),
                ("slot_bytes", ctypes.c_uint64), ("graph_launches", ctypes.c_uint64),
                ("graph_captures", ctypes.c_uint64)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_u64 = ctypes.c_uint64
_u32 = ctypes.c_uint32
_i64 = ctypes.c_int64
_int = ctypes.c_int
_vp = ctypes.c_void_p
_pu64 = ctypes.POINTER(ctypes.c_uint64)

# name -> (restype, argtypes); mirrors include/gfp.h
SIGNATURES = {
    "gfp_field_create": (_int, [_u32, _u64, ctypes.POINTER(_vp)]),
    "gfp_field_destroy": (_int, [_vp]),
    "gfp_field_info": (_int, [_vp, ctypes.POINTER(_u32), ctypes.POINTER(_u64), ctypes.POINTER(_u32)]),
    "gfp_root_of_unity": (_int, [_vp, _u64, _int, _pu64]),
    "gfp_fft_workspace_size": (_int, [_vp, _u64, ctypes.POINTER(_u64)]),
    "gfp_fft_forward": (_int, [_vp, _u64, _vp, _u64, _vp, _u64, _vp, _u64, _vp]),
    "gfp_fft_inverse": (_int, [_vp, _u64, _vp, _u64, _vp, _u64, _vp, _u64, _vp]),
    "gfp_fft_noalloc": (_int, [_vp, _u64, _int, _vp, _u64, _vp, _u64, _vp]),
    "gfp_fft_pass": (_int, [_vp, _u64, _int, _int, _int, _vp, _u64, _vp, _u64, _vp]),
    "gfp_polymul_size": (_int, [_vp, _u64, _u64, ctypes.POINTER(_u64)]),
    "gfp_polymul_workspace_size": (_int, [_vp, _u64, _u64, ctypes.POINTER(_u64)]),
    "gfp_polymul": (_int, [_vp, _vp, _u64, _u64, _vp, _u64, _u64, _vp, _u64, _vp, _u64, _vp]),
    "gfp_polymul_batched_workspace_size": (_int, [_vp, _u32, _vp, ctypes.POINTER(_u64)]),
    "gfp_polymul_batched": (_int, [_vp, _u32, _vp, _vp, _u64, _int, _vp]),
    "gfp_elementwise": (_int, [_vp, _int, _vp, _u64, _vp, _u64, _vp, _u64, _u64, _i64, _pu64, _vp]),
    "gfp_bigint_mul_workspace_size": (_int, [_vp, _u64, _u64, ctypes.POINTER(_u64)]),
    "gfp_bigint_mul": (_int, [_vp, _vp, _u64, _vp, _u64, _vp, _vp, _u64, _vp]),
    "gfp_check_canonical": (_int, [_vp, _vp, _u64, _u64, _vp, ctypes.POINTER(_u64)]),
    "gfp_plan_get": (_int, [_vp, _u64, _u64, _int, ctypes.c_char_p, _u32]),
    "gfp_plan_set": (_int, [_vp, _u64, _u64, _int, ctypes.c_char_p]),
    "gfp_tune": (_int, [_vp, _u64, _u64, _int, _vp, ctypes.c_char_p, _u32, ctypes.POINTER(ctypes.c_double)]),
    "gfp_server_create": (_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(_vp)]),
    "gfp_server_submit": (_int, [_vp, ctypes.POINTER(Request), ctypes.POINTER(_u64)]),
    "gfp_server_poll": (_int, [_vp, _u64, ctypes.POINTER(Result)]),
    "gfp_server_wait": (_int, [_vp, _u64, _i64, ctypes.POINTER(Result)]),
    "gfp_server_drain": (_int, [_vp]),
    "gfp_server_get_stats": (_int, [_vp, ctypes.POINTER(ServerStats)]),
    "gfp_server_destroy": (_int, [_vp]),
    "gfp_strerror": (ctypes.c_char_p, [_int]),
}

_lib = None


class GFPError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__("%s: %s (code %d)" % (what, strerror(code), code))


def lib() -> ctypes.CDLL:
    """Load the HIP library; fails loudly if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libgfpfft.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def strerror(code: int) -> str:
    return lib().gfp_strerror(code).decode()


def _check(rc: int, what: str):
    if rc != GFP_OK:
        raise GFPError(rc, what)


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _vec(t: torch.Tensor, k: int, n: int, name: str):
    if t.dtype not in (torch.int64, torch.uint64) or t.dim() != 2 or t.shape[0] != k:
        raise ValueError("%s must be a (k, ld) int64/uint64 tensor" % name)
    if t.stride(1) != 1 or t.shape[1] < n or not t.is_cuda:
        raise ValueError("%s must be a HIP tensor with unit element stride and >= n columns" % name)
    return ctypes.c_void_p(t.data_ptr()), t.stride(0)


class Field:
    """Z/pZ with p = r^k + 1 (a handle on gfp_field)."""

    def __init__(self, k: int, r: int):
        h = _vp()
        _check(lib().gfp_field_create(k, r, ctypes.byref(h)), "gfp_field_create")
        self._h = h
        self.k = k
        self.r = r
        lg = _u32()
        _check(lib().gfp_field_info(h, None, None, ctypes.byref(lg)), "gfp_field_info")
        self.log2_max_n = lg.value

    def close(self):
        if getattr(self, "_h", None):
            lib().gfp_field_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def root_of_unity(self, n: int, inverse: bool = False) -> list:
        out = (ctypes.c_uint64 * self.k)()
        _check(lib().gfp_root_of_unity(self._h, n, int(inverse), out), "gfp_root_of_unity")
        return [int(v) for v in out]

    def fft_workspace_size(self, n: int) -> int:
        b = _u64()
        _check(lib().gfp_fft_workspace_size(self._h, n, ctypes.byref(b)), "gfp_fft_workspace_size")
        return b.value

    def polymul_size(self, la: int, lb: int) -> int:
        v = _u64()
        _check(lib().gfp_polymul_size(self._h, la, lb, ctypes.byref(v)), "gfp_polymul_size")
        return v.value

    def polymul_workspace_size(self, la: int, lb: int) -> int:
        v = _u64()
        _check(lib().gfp_polymul_workspace_size(self._h, la, lb, ctypes.byref(v)), "gfp_polymul_workspace_size")
        return v.value

    def _transform(self, fn, what, x, n, y, workspace, stream):
        px, ldx = _vec(x, self.k, n, "x")
        if y is None:
            y = torch.empty((self.k, n), dtype=x.dtype, device=x.device)
        py, ldy = _vec(y, self.k, n, "y")
        wp, wb = (ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()) \
            if workspace is not None else (None, 0)
        _check(fn(self._h, n, px, ldx, py, ldy, wp, wb, _stream(stream)), what)
        return y

    def fft_forward(self, x, n=None, y=None, workspace=None, stream=None):
        n = x.shape[1] if n is None else n
        return self._transform(lib().gfp_fft_forward, "gfp_fft_forward", x, n, y, workspace, stream)

    def fft_inverse(self, x, n=None, y=None, workspace=None, stream=None):
        n = x.shape[1] if n is None else n
        return self._transform(lib().gfp_fft_inverse, "gfp_fft_inverse", x, n, y, workspace, stream)

    def fft_noalloc(self, x, n=None, y=None, inverse=False, stream=None):
        """gfp_fft_noalloc: the transform with the library's static scratch
        (no device allocation inside the call); y must be given by callers
        that cannot allocate."""
        n = x.shape[1] if n is None else n
        px, ldx = _vec(x, self.k, n, "x")
        if y is None:
            y = torch.empty((self.k, n), dtype=x.dtype, device=x.device)
        py, ldy = _vec(y, self.k, n, "y")
        _check(lib().gfp_fft_noalloc(self._h, n, int(inverse), px, ldx, py, ldy, _stream(stream)), "gfp_fft_noalloc")
        return y

    def fft_pass(self, s, x, y, n, inverse=False, in_element_major=False, out_element_major=False, stream=None,
                 code="1"):
        """One launch of a plan starting at pass s: code '1' (one pass), '2'
        or 'w' (passes s and s+1 fused); element-major tensors are flat
        (n * k,) int64 device tensors."""
        def ptr(t, em, name):
            if em:
                if not t.is_cuda or t.numel() < n * self.k:
                    raise ValueError("%s: element-major needs n*k words on the device" % name)
                return ctypes.c_void_p(t.data_ptr()), 0
            return _vec(t, self.k, n, name)
        px, ldx = ptr(x, in_element_major, "x")
        py, ldy = ptr(y, out_element_major, "y")
        flags = (1 if in_element_major else 0) | (2 if out_element_major else 0) | {"1": 0, "2": 4, "w": 8, "n": 16}[code]
        _check(lib().gfp_fft_pass(self._h, n, s, int(inverse), flags, px, ldx, py, ldy, _stream(stream)),
               "gfp_fft_pass")
        return y

    def polymul(self, a, b, la=None, lb=None, c=None, workspace=None, stream=None):
        la = a.shape[1] if la is None else la
        lb = b.shape[1] if lb is None else lb
        pa, lda = _vec(a, self.k, la, "a")
        pb, ldb = _vec(b, self.k, lb, "b")
        if c is None:
            c = torch.empty((self.k, la + lb - 1), dtype=a.dtype, device=a.device)
        pc, ldc = _vec(c, self.k, la + lb - 1, "c")
        wp, wb = (ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()) \
            if workspace is not None else (None, 0)
        _check(lib().gfp_polymul(self._h, pa, la, lda, pb, lb, ldb, pc, ldc, wp, wb, _stream(stream)), "gfp_polymul")
        return c

    def batch_descs(self, reqs):
        """reqs: list of (a, b, c) tensors (shape (k, ld)); lengths = a.shape[1],
        b.shape[1].  Returns a ctypes array of gfp_polymul_desc (keep it alive
        with the tensors)."""
        arr = (PolymulDesc * len(reqs))()
        for i, (a, b, c) in enumerate(reqs):
            la, lb = a.shape[1], b.shape[1]
            pa, lda = _vec(a, self.k, la, "a")
            pb, ldb = _vec(b, self.k, lb, "b")
            pc, ldc = _vec(c, self.k, la + lb - 1, "c")
            arr[i] = PolymulDesc(pa, la, lda, pb, lb, ldb, pc, ldc)
        return arr

    def polymul_batched_workspace_size(self, descs) -> int:
        v = _u64()
        _check(lib().gfp_polymul_batched_workspace_size(self._h, len(descs), descs, ctypes.byref(v)),
               "gfp_polymul_batched_workspace_size")
        return v.value

    def polymul_batched(self, descs, workspace=None, graph=False, stream=None, persistent=False):
        wp, wb = (ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()) \
            if workspace is not None else (None, 0)
        flags = (BATCH_GRAPH if graph else 0) | (BATCH_PERSISTENT if persistent else 0)
        _check(lib().gfp_polymul_batched(self._h, len(descs), descs, wp, wb, flags, _stream(stream)),
               "gfp_polymul_batched")

    def check_canonical(self, x, n=None, stream=None) -> int:
        """Number of elements of x (a (k, ld) device tensor) that are not
        canonically encoded; synchronises the stream."""
        n = x.shape[1] if n is None else n
        px, ldx = _vec(x, self.k, n, "x")
        bad = _u64()
        _check(lib().gfp_check_canonical(self._h, px, ldx, n, _stream(stream), ctypes.byref(bad)),
               "gfp_check_canonical")
        return bad.value

    def bigint_mul(self, a, b, c=None, workspace=None, stream=None):
        """c = a * b for integers held as 1-D int64/uint64 device tensors of
        64-bit little-endian words; c gets len(a) + len(b) words."""
        for t, name in ((a, "a"), (b, "b")):
            if t.dim() != 1 or not t.is_cuda or t.dtype not in (torch.int64, torch.uint64) or t.stride(0) != 1:
                raise ValueError("%s must be a contiguous 1-D int64 device tensor" % name)
        na, nb = a.numel(), b.numel()
        if c is None:
            c = torch.empty(na + nb, dtype=a.dtype, device=a.device)
        if c.dim() != 1 or c.numel() < na + nb or c.stride(0) != 1:
            raise ValueError("c must be a contiguous 1-D tensor of at least na + nb words")
        wp, wb = (ctypes.c_void_p(workspace.data_ptr()), workspace.numel() * workspace.element_size()) \
            if workspace is not None else (None, 0)
        _check(lib().gfp_bigint_mul(self._h, ctypes.c_void_p(a.data_ptr()), na, ctypes.c_void_p(b.data_ptr()), nb,
                                    ctypes.c_void_p(c.data_ptr()), wp, wb, _stream(stream)), "gfp_bigint_mul")
        return c

    def bigint_mul_workspace_size(self, na: int, nb: int) -> int:
        v = _u64()
        _check(lib().gfp_bigint_mul_workspace_size(self._h, na, nb, ctypes.byref(v)), "gfp_bigint_mul_workspace_size")
        return v.value

    def plan(self, n: int, nvec: int = 1, layout: int = LAYOUT_DIGIT_MAJOR) -> str:
        """Stage grouping used for nvec transforms of size n, e.g. '1211'."""
        buf = ctypes.create_string_buffer(32)
        _check(lib().gfp_plan_get(self._h, n, nvec, layout, buf, 32), "gfp_plan_get")
        return buf.value.decode()

    def set_plan(self, n: int, plan, nvec: int = 1, layout: int = LAYOUT_DIGIT_MAJOR):
        """Set (or with None / '' reset) the stage grouping for (n, batch class, layout)."""
        _check(lib().gfp_plan_set(self._h, n, nvec, layout, plan.encode() if plan else None), "gfp_plan_set")

    def tune(self, n: int, nvec: int = 1, layout: int = LAYOUT_DIGIT_MAJOR, stream=None):
        """Autotune the stage grouping for (n, batch class, layout); returns (plan, us)."""
        buf = ctypes.create_string_buffer(32)
        us = ctypes.c_double()
        _check(lib().gfp_tune(self._h, n, nvec, layout, _stream(stream), buf, 32, ctypes.byref(us)), "gfp_tune")
        return buf.value.decode(), us.value

    def elementwise(self, op, x, y=None, z=None, n=None, s=0, c=None, stream=None):
        n = x.shape[1] if n is None else n
        px, ldx = _vec(x, self.k, n, "x")
        py, ldy = _vec(y, self.k, n, "y") if y is not None else (None, 0)
        if z is None:
            z = torch.empty((self.k, n), dtype=x.dtype, device=x.device)
        pz, ldz = _vec(z, self.k, n, "z")
        ch = (ctypes.c_uint64 * self.k)(*[int(v) for v in c]) if c is not None else None
        _check(lib().gfp_elementwise(self._h, op, px, ldx, py, ldy, pz, ldz, n, s, ch, _stream(stream)),
               "gfp_elementwise")
        return z


class Server:
    """Request loop (gfp_server): continuous batching of polynomial products.

    Operands and results are caller-owned (k, ld) device tensors; keep them
    alive until the ticket is done.  Pass ``ready`` (a recorded
    torch.cuda.Event) when the operands are still being written on some
    stream; otherwise they must be ready when submit is called."""

    def __init__(self, workspace_bytes: int, slots: int = 2, max_batch: int = 256, max_pending: int = 65536,
                 max_wait_us: int = 0, device: int = -1, express_log2n: int = 0, graphs: bool = True):
        cfg = ServerConfig(workspace_bytes, slots, max_batch, max_pending, max_wait_us, device, express_log2n,
                           0 if graphs else SERVER_EAGER)
        h = _vp()
        _check(lib().gfp_server_create(ctypes.byref(cfg), ctypes.byref(h)), "gfp_server_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().gfp_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def request(field: "Field", a, b, c, la=None, lb=None, ready=None) -> Request:
        la = a.shape[1] if la is None else la
        lb = b.shape[1] if lb is None else lb
        pa, lda = _vec(a, field.k, la, "a")
        pb, ldb = _vec(b, field.k, lb, "b")
        pc, ldc = _vec(c, field.k, la + lb - 1, "c")
        ev = ready.cuda_event if ready is not None else None
        return Request(field.handle, pa, la, lda, pb, lb, ldb, pc, ldc, ev)

    def submit_request(self, req: Request) -> int:
        """Returns the ticket; raises GFPError (code GFP_EAGAIN when full)."""
        t = _u64()
        _check(lib().gfp_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)), "gfp_server_submit")
        return t.value

    def submit(self, field: "Field", a, b, c, la=None, lb=None, ready=None) -> int:
        return self.submit_request(self.request(field, a, b, c, la, lb, ready))

    def poll(self, ticket: int):
        """Result dict when done, None while pending."""
        r = Result()
        rc = lib().gfp_server_poll(self._h, ticket, ctypes.byref(r))
        if rc == GFP_EPENDING:
            return None
        _check(rc, "gfp_server_poll")
        return r.as_dict()

    def wait(self, ticket: int, timeout_us: int = -1):
        r = Result()
        rc = lib().gfp_server_wait(self._h, ticket, timeout_us, ctypes.byref(r))
        if rc == GFP_EPENDING:
            return None
        _check(rc, "gfp_server_wait")
        return r.as_dict()

    def drain(self):
        _check(lib().gfp_server_drain(self._h), "gfp_server_drain")

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().gfp_server_get_stats(self._h, ctypes.byref(s)), "gfp_server_get_stats")
        return s.as_dict()


# ---- numpy <-> device helpers (marshalling only) --------------------------------
def to_device(digits_u64, device="cuda") -> torch.Tensor:
    """(k, n) numpy uint64 -> (k, n) int64 device tensor with the same bits."""
    import numpy as np

    arr = np.ascontiguousarray(digits_u64, dtype=np.uint64)
    return torch.from_numpy(arr.view(np.int64)).to(device)


def to_host(t: torch.Tensor):
    """Device tensor -> (k, n) numpy uint64."""
    import numpy as np

    return t.detach().cpu().contiguous().numpy().view(np.uint64)
