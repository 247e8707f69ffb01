"""C ABI checks that need no GPU: the library loads, exports every function
include/gfp.h declares, and its host-side field setup (probable-prime test,
Alg. 1 root of unity, error codes) agrees with the oracle."""

import ctypes
import os
import re

import pytest

from oracle.field import GFPField, P8, P16, P32, P64

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gfp.h")

gfp = pytest.importorskip("paper_1811_01490_amd.gfp")


def _lib():
    if not os.path.exists(gfp.LIB_PATH):
        pytest.skip("libgfpfft.so not built")
    return gfp.lib()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(gfp_\w+)\s*\(", text, re.M)))


def test_header_declares_the_bound_functions():
    names = declared_functions()
    assert names, "no declarations found"
    assert set(names) == set(gfp.SIGNATURES), (set(names) ^ set(gfp.SIGNATURES))


def test_library_exports_every_declared_symbol():
    L = _lib()
    for name in declared_functions():
        assert hasattr(L, name), name


@pytest.mark.parametrize("params", [P8, P16, P32, P64, dict(k=8, r=2 ** 59 + 2 ** 16), dict(k=16, r=2 ** 58 + 2 ** 10)])
def test_field_create_info_and_roots(params):
    _lib()
    F = GFPField(**params)
    f = gfp.Field(params["k"], params["r"])
    assert f.log2_max_n == F.max_log2_n
    for N in (2 * F.k, 4 * F.k * F.k, 2 ** 12, 2 ** 20):
        if N < 2 * F.k:
            continue
        w = F.paper_root_of_unity(N)
        assert f.root_of_unity(N) == F.from_int(w)
        assert f.root_of_unity(N, inverse=True) == F.from_int(F.inv(w))
    f.close()


def test_error_codes():
    L = _lib()
    h = ctypes.c_void_p()
    assert L.gfp_field_create(8, 2 ** 63 + 2 ** 30, ctypes.byref(h)) == gfp.GFP_ENOTPRIME  # composite (s = 30)
    assert L.gfp_field_create(6, 2 ** 63 + 2 ** 34, ctypes.byref(h)) == gfp.GFP_EINVAL    # k not a power of two
    assert L.gfp_field_create(8, 2 ** 63 + 2 ** 34 + 1, ctypes.byref(h)) == gfp.GFP_EINVAL  # r odd
    assert L.gfp_field_create(8, 2 ** 63 + 2 ** 34, None) == gfp.GFP_EINVAL
    # a prime outside the compiled shapes is accepted by create, rejected by transforms
    assert L.gfp_field_create(4, 2 ** 64 - 2 ** 50, ctypes.byref(h)) == gfp.GFP_OK  # Table 1 row 2
    out = (ctypes.c_uint64 * 4)()
    assert L.gfp_root_of_unity(h, 8, 0, out) == gfp.GFP_OK
    F = GFPField(4, 2 ** 64 - 2 ** 50)
    assert [int(v) for v in out] == F.from_int(F.paper_root_of_unity(8))
    assert L.gfp_fft_forward(h, 8, ctypes.c_void_p(8), 8, ctypes.c_void_p(8), 8, None, 0, None) == gfp.GFP_EUNSUPPORTED
    L.gfp_field_destroy(h)
    f = gfp.Field(**P8)
    b = ctypes.c_uint64()
    for bad_n in (0, 8, 24, 100, 2 ** 26):  # not a power of two, below K = 16, above 2^25
        assert L.gfp_fft_workspace_size(f.handle, bad_n, ctypes.byref(b)) in (gfp.GFP_EUNSUPPORTED, gfp.GFP_EINVAL)
    for n in (16, 32, 4096, 2 ** 13, 2 ** 25):  # any power of two from K on
        assert L.gfp_fft_workspace_size(f.handle, n, ctypes.byref(b)) == gfp.GFP_OK
        assert b.value == 2 * n * 8 * 8
    assert f.polymul_size(2048, 2048) == 4096
    assert f.polymul_size(1, 1) == 16
    assert f.polymul_size(9, 9) == 32 and f.polymul_size(1000, 1000) == 2048
    assert f.polymul_size(2 ** 19, 2 ** 19) == 2 ** 20 and f.polymul_size(2 ** 18, 2 ** 18) == 2 ** 19
    assert f.polymul_size(2 ** 18 + 2, 2 ** 18) == 2 ** 20 and f.polymul_size(8, 9) == 16
    # null / short-ld arguments are rejected before any device work
    assert L.gfp_fft_forward(f.handle, 4096, None, 4096, ctypes.c_void_p(8), 4096, None, 0, None) == gfp.GFP_EINVAL
    assert L.gfp_fft_forward(f.handle, 4096, ctypes.c_void_p(8), 4000, ctypes.c_void_p(8), 4096, None, 0, None) == gfp.GFP_EINVAL
    assert L.gfp_polymul(f.handle, ctypes.c_void_p(8), 0, 1, ctypes.c_void_p(8), 1, 1, ctypes.c_void_p(8), 1, None, 0, None) == gfp.GFP_EINVAL
    assert L.gfp_elementwise(f.handle, 99, ctypes.c_void_p(8), 1, None, 0, ctypes.c_void_p(8), 1, 1, 0, None, None) == gfp.GFP_EINVAL
    assert gfp.strerror(gfp.GFP_ENOTPRIME).startswith("r^k + 1")
    # batched flags: unknown bits, graph together with persistent, persistent for k = 32
    d = (gfp.PolymulDesc * 1)(gfp.PolymulDesc(8, 1, 1, 8, 1, 1, 8, 1))
    assert L.gfp_polymul_batched(f.handle, 1, d, None, 0, 4, None) == gfp.GFP_EINVAL
    assert L.gfp_polymul_batched(f.handle, 1, d, None, 0, gfp.BATCH_GRAPH | gfp.BATCH_PERSISTENT, None) == gfp.GFP_EINVAL
    f32 = gfp.Field(**P32)
    assert L.gfp_polymul_batched(f32.handle, 1, d, None, 0, gfp.BATCH_PERSISTENT, None) == gfp.GFP_EUNSUPPORTED


def test_server_argument_errors():
    """Argument checks of the request loop run before any device call."""
    L = _lib()
    h = ctypes.c_void_p()
    cfg = gfp.ServerConfig(1 << 30, 2, 16, 64, 0, -1, 0)
    assert L.gfp_server_create(None, ctypes.byref(h)) == gfp.GFP_EINVAL
    assert L.gfp_server_create(ctypes.byref(cfg), None) == gfp.GFP_EINVAL
    bad = gfp.ServerConfig(1 << 30, 1, 16, 64, 0, -1, 12)  # an express slot needs a second slot
    assert L.gfp_server_create(ctypes.byref(bad), ctypes.byref(h)) == gfp.GFP_EINVAL
    bad = gfp.ServerConfig(1 << 30, 2, 16, 64, 0, -1, 41)
    assert L.gfp_server_create(ctypes.byref(bad), ctypes.byref(h)) == gfp.GFP_EINVAL
    tiny = gfp.ServerConfig(100, 2, 16, 64, 0, -1, 0)  # under 256 bytes per slot
    assert L.gfp_server_create(ctypes.byref(tiny), ctypes.byref(h)) == gfp.GFP_EINVAL
    many = gfp.ServerConfig(1 << 30, 65, 16, 64, 0, -1, 0)
    assert L.gfp_server_create(ctypes.byref(many), ctypes.byref(h)) == gfp.GFP_EINVAL
    flags = gfp.ServerConfig(1 << 30, 2, 16, 64, 0, -1, 0, 6)  # unknown flag bits
    assert L.gfp_server_create(ctypes.byref(flags), ctypes.byref(h)) == gfp.GFP_EINVAL
    big = gfp.ServerConfig(1 << 30, 2, 70000, 64, 0, -1, 0)
    assert L.gfp_server_create(ctypes.byref(big), ctypes.byref(h)) == gfp.GFP_EINVAL
    t = ctypes.c_uint64()
    r = gfp.Result()
    assert L.gfp_server_submit(None, None, ctypes.byref(t)) == gfp.GFP_EINVAL
    assert L.gfp_server_poll(None, 1, ctypes.byref(r)) == gfp.GFP_EINVAL
    assert L.gfp_server_wait(None, 1, 0, ctypes.byref(r)) == gfp.GFP_EINVAL
    assert L.gfp_server_drain(None) == gfp.GFP_EINVAL
    assert L.gfp_server_destroy(None) == gfp.GFP_OK


def test_struct_layouts_match_the_header(tmp_path):
    """Every ctypes mirror has the size and field offsets that a C compiler
    gives the header's struct."""
    import shutil
    import subprocess

    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no C compiler")
    mirrors = {"gfp_server_config": gfp.ServerConfig, "gfp_request": gfp.Request, "gfp_result": gfp.Result,
               "gfp_server_stats": gfp.ServerStats, "gfp_polymul_desc": gfp.PolymulDesc}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gfp.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append('printf("%%s %%zu\\n", "%s", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('printf("%%s.%%s %%zu\\n", "%s", "%s", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.rsplit(" ", 1) for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                                check=True).stdout.split("\n") if line)
    for cname, py in mirrors.items():
        assert int(got[cname]) == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got["%s.%s" % (cname, fname)]) == getattr(py, fname).offset, (cname, fname)


def test_plan_strings():
    """Plan bookkeeping is host-only: defaults, per batch class and layout,
    validation."""
    _lib()
    f = gfp.Field(**P8)
    em = gfp.LAYOUT_ELEMENT_MAJOR
    assert f.plan(2 ** 20) == "w21" and f.plan(2 ** 20, layout=em) == "w12"
    assert f.plan(4096) == "12" and f.plan(256) == "2" and f.plan(16) == "1"
    f.set_plan(4096, "21", nvec=8)
    assert f.plan(4096, nvec=8) == "21" and f.plan(4096, nvec=63) == "21"
    assert f.plan(4096) == "12" and f.plan(4096, nvec=64) == "12" and f.plan(4096, nvec=8, layout=em) == "12"
    f.set_plan(4096, "w1", layout=em)  # wide pair at s = 0: 2^12 / (256 * 1) >= 8 blocks
    assert f.plan(4096, layout=em) == "w1"
    for bad in ("3", "22", "1", "1a1", "0111", "1w", "W1"):
        with pytest.raises(gfp.GFPError) as e:
            f.set_plan(4096, bad)
        assert e.value.code == gfp.GFP_EINVAL
    f.set_plan(4096, None, nvec=8)
    assert f.plan(4096, nvec=8) == "12"
    assert f.plan(2 ** 20, layout=em) == "w12"
    f.set_plan(2 ** 20, "1w11")
    assert f.plan(2 ** 20) == "1w11"
    # n = R K^e: the plan covers the e radix-K passes after the radix-R pass
    assert f.plan(2 ** 13) == "12" and f.plan(32) == "1" and f.plan(2 ** 19) == "121"
    f.set_plan(2 ** 13, "w1")  # 2^13 / (256 * 2) = 16 blocks per base
    with pytest.raises(gfp.GFPError):
        f.set_plan(2 ** 13, "1w")
    with pytest.raises(gfp.GFPError):
        f.set_plan(2 ** 20, "111w")  # the last pair has one block per twiddle base
    g = gfp.Field(**P16)
    assert g.plan(2 ** 20) == "1111"
    g.set_plan(32768, "21")  # fused pairs exist for k = 16 ...
    assert g.plan(32768) == "21"
    with pytest.raises(gfp.GFPError):
        g.set_plan(2 ** 20, "w11")  # ... the wide pair does not
    g.set_plan(32768, None)


def test_k32_field_host():
    """The k = 32 prime of Table 1 (r = 2^62 + 2^56, K = 64): root of unity
    from Alg. 1 as the oracle's, product sizes from K = 64 on, plans of
    radix-64 passes one per launch (no fused pair at k = 32)."""
    L = _lib()
    f = gfp.Field(**P32)
    F = GFPField(**P32)
    out = (ctypes.c_uint64 * 32)()
    for n in (64, 4096, 2 ** 18):
        assert L.gfp_root_of_unity(f.handle, n, 0, out) == gfp.GFP_OK
        assert [int(v) for v in out] == F.from_int(F.paper_root_of_unity(n))
    assert f.polymul_size(1, 1) == 64 and f.polymul_size(2048, 2048) == 4096
    assert f.plan(2 ** 18) == "111" and f.plan(8192) == "11" and f.plan(64) == "1"
    with pytest.raises(gfp.GFPError):
        f.set_plan(4096, "2")


def test_k64_field_host():
    """The k = 64 prime of Table 1 (r = 2^63 - 2^40, K = 128): roots as the
    oracle's, sizes from K = 128 on, one radix-128 pass per launch; integer
    products are offered."""
    L = _lib()
    f = gfp.Field(**P64)
    F = GFPField(**P64)
    out = (ctypes.c_uint64 * 64)()
    for n in (128, 2 ** 14, 2 ** 20):
        assert L.gfp_root_of_unity(f.handle, n, 0, out) == gfp.GFP_OK
        assert [int(v) for v in out] == F.from_int(F.paper_root_of_unity(n))
    assert f.polymul_size(1, 1) == 128 and f.polymul_size(2048, 2048) == 4096
    assert f.plan(2 ** 14) == "11" and f.plan(2 ** 13) == "1" and f.plan(128) == "1"
    b = ctypes.c_uint64()
    assert L.gfp_bigint_mul_workspace_size(f.handle, 10, 10, ctypes.byref(b)) == gfp.GFP_OK
    # 448-bit chunks: 10 words = 2 coefficients each, transform size 128 (K);
    # workspace at least the polynomial product's
    w = ctypes.c_uint64()
    assert L.gfp_polymul_workspace_size(f.handle, 2, 2, ctypes.byref(w)) == gfp.GFP_OK
    assert b.value >= w.value


def test_bigint_sizes():
    """Workspace sizing of integer products is host-only."""
    L = _lib()
    f = gfp.Field(**P8)
    b = ctypes.c_uint64()
    assert L.gfp_bigint_mul_workspace_size(f.handle, 0, 5, ctypes.byref(b)) == gfp.GFP_EINVAL
    assert L.gfp_bigint_mul_workspace_size(f.handle, 5, 5, None) == gfp.GFP_EINVAL
    assert L.gfp_bigint_mul(f.handle, None, 1, ctypes.c_void_p(8), 1, ctypes.c_void_p(8), None, 0, None) == gfp.GFP_EINVAL
    small = f.bigint_mul_workspace_size(10, 10)
    big = f.bigint_mul_workspace_size(2 ** 16, 2 ** 16)
    assert 0 < small < big
    # b = (8 63 - 2 - 24) / 2 = 239-bit coefficients for 2^18 words: la = 70198,
    # transform size 2^18; 2^26 words (b = 234) need more than 2^25 points
    assert f.bigint_mul_workspace_size(2 ** 18, 2 ** 18) > big
    f.bigint_mul_workspace_size(2 ** 25, 2 ** 25)
    with pytest.raises(gfp.GFPError):
        f.bigint_mul_workspace_size(2 ** 26, 2 ** 26)


def test_plan_cache_round_trip(tmp_path):
    """Plans exported to the JSON cache come back into a fresh field object;
    entries of another architecture or field are not applied."""
    _lib()
    from paper_1811_01490_amd import autotune

    em = gfp.LAYOUT_ELEMENT_MAJOR
    f = gfp.Field(**P8)
    f.set_plan(2 ** 20, "1121")
    f.set_plan(2 ** 20, "212", nvec=16, layout=em)
    f.set_plan(4096, "w1", nvec=100, layout=em)
    keys = [(2 ** 20, 1, 0), (2 ** 20, 16, em), (4096, 100, em), (256, 1, 0)]
    entries = autotune.export_plans(f, keys)
    assert entries == {"1048576|0|0": "1121", "1048576|2|1": "212", "4096|3|1": "w1", "256|0|0": "2"}
    path = str(tmp_path / "plans.json")
    autotune.save(path, f, entries, arch="gfx950")
    g = gfp.Field(**P8)
    assert g.plan(2 ** 20) == "w21"  # default before loading
    assert autotune.load(path, g, arch="gfx942") == 0  # another architecture
    assert autotune.load(path, gfp.Field(**P16), arch="gfx950") == 0  # another field
    assert autotune.load(path, g, arch="gfx950") == 4
    assert g.plan(2 ** 20) == "1121" and g.plan(2 ** 20, nvec=9, layout=em) == "212"
    assert g.plan(4096, nvec=64, layout=em) == "w1" and g.plan(256) == "2"
    assert autotune.batch_class(1) == 0 and autotune.batch_class(7) == 1 and autotune.batch_class(63) == 2
