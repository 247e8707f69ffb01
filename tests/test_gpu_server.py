"""Request loop (gfp_server_*): every result must equal gfp_polymul of the same
request alone (and the schoolbook product where the oracle is fast), batches
must respect the workspace budget and max_batch, requests that arrive while a
batch is on the device must be served by another slot meanwhile, a full queue
must answer GFP_EAGAIN, and shutdown must cancel what was not admitted.

To make the timing-dependent cases deterministic, a batch is held on the
device by giving its request a ready event recorded after a bounded spin
kernel (torch.cuda._sleep) on another stream.  The scheduling assertions use
the host-side admission and launch times: HIP maps streams onto a few
hardware queues, so the spin kernel may share a queue with another slot's
stream and delay its device work, but never its admission."""

import time

import numpy as np
import pytest

import gfp_inputs as gi
from oracle import transform as T
from oracle.field import GFPField, P8, P16, P32, P64
from tests.helpers import canonical_mask, to_ints

pytestmark = pytest.mark.gpu

SEED = gi.BASE_SEED + 400


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def fields(torch_mod):
    from paper_1811_01490_amd import Field

    return {8: Field(**P8), 16: Field(**P16), 32: Field(**P32), 64: Field(**P64)}


@pytest.fixture(scope="module")
def sleep_cycles(torch_mod):
    """Spin-kernel cycles for about 60 ms (the clock it counts is measured)."""
    import torch

    torch.cuda._sleep(1000)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    torch.cuda._sleep(2_000_000)
    e1.record()
    torch.cuda.synchronize()
    ms = max(e0.elapsed_time(e1), 1e-3)
    return int(2_000_000 * 60.0 / ms)


def _tables_ready(torch, f, *ops):
    """Build the twiddle tables of every product size a test submits while a
    batch is held.  A table build uploads from the submitting thread, and
    that copy can queue behind the held spin kernel when their streams share
    a hardware queue; submit would then wait out the hold."""
    for op in ops:
        f.polymul(op[2], op[3])
    torch.cuda.synchronize()


def _held_event(torch, cycles):
    """An event that completes after a ~60 ms spin on a side stream."""
    s = torch.cuda.Stream()
    ev = torch.cuda.Event()
    with torch.cuda.stream(s):
        torch.cuda._sleep(cycles)
        ev.record(s)
    return ev, s


def _operands(params, la, lb, stream):
    from paper_1811_01490_amd import to_device

    k, r = params["k"], params["r"]
    a = gi.operand(k, r, la, SEED, 2 * stream, edge_frac=0.05)
    b = gi.operand(k, r, lb, SEED, 2 * stream + 1, edge_frac=0.05)
    return a, b, to_device(a), to_device(b)


def _out(torch, k, n):
    return torch.full((k, n), -1, dtype=torch.int64, device="cuda")


def _check_alone(f, da, db, c):
    from paper_1811_01490_amd import to_host

    got = to_host(c)
    assert canonical_mask(got, f.r).all()
    assert np.array_equal(got, to_host(f.polymul(da, db)))
    return got


def test_mixed_fields_and_sizes_match_alone(torch_mod, fields):
    import torch

    from paper_1811_01490_amd import Server

    g = gi.rng(SEED, 1)
    reqs = []
    for i in range(48):
        params = P8 if g.integers(2) == 0 else P16
        la = int(2 ** g.uniform(0, 12))
        lb = int(2 ** g.uniform(0, 12)) if i % 3 else la
        a, b, da, db = _operands(params, la, lb, 10 + i)
        reqs.append((params, a, b, da, db, _out(torch, params["k"], la + lb - 1)))
    torch.cuda.synchronize()
    with Server(workspace_bytes=2 << 30, slots=2, max_batch=16) as srv:
        tickets = [srv.submit(fields[p["k"]], da, db, c) for p, a, b, da, db, c in reqs]
        res = [srv.wait(t) for t in tickets]
        st = srv.stats()
    assert all(r["status"] == 0 for r in res)
    assert st["submitted"] == st["completed"] == len(reqs)
    assert 1 <= st["max_batch_size"] <= 16
    for (params, a, b, da, db, c), r in zip(reqs, res):
        assert r["t_submit_ns"] <= r["t_admit_ns"] <= r["t_launch_ns"] <= r["t_done_ns"]
        got = _check_alone(fields[params["k"]], da, db, c)
        if a.shape[1] * b.shape[1] <= 40000:
            F = GFPField(**params)
            assert to_ints(got, F.r) == T.polymul(to_ints(a, F.r), to_ints(b, F.r), F.p)


def test_arrivals_during_a_batch_use_another_slot(torch_mod, fields, sleep_cycles):
    import torch

    from paper_1811_01490_amd import Server

    f = fields[8]
    a, b, da, db = _operands(P8, 3000, 2000, 100)
    small = [_operands(P8, 50 + 7 * i, 40 + 3 * i, 101 + i) for i in range(6)]
    c = _out(torch, 8, 4999)
    cs = [_out(torch, 8, x[2].shape[1] + x[3].shape[1] - 1) for x in small]
    _tables_ready(torch, f, (a, b, da, db), *small)
    with Server(workspace_bytes=1 << 30, slots=2, max_batch=64) as srv:
        ev, side = _held_event(torch, sleep_cycles)
        t_big = srv.submit(f, da, db, c, ready=ev)
        time.sleep(0.005)  # the first slot takes it and waits on the device
        ts = [srv.submit(f, x[2], x[3], cc) for x, cc in zip(small, cs)]
        rs = [srv.wait(t) for t in ts]
        r_big = srv.wait(t_big)
        st = srv.stats()
    side.synchronize()
    assert r_big["status"] == 0 and all(r["status"] == 0 for r in rs)
    assert all(r["batch_id"] != r_big["batch_id"] for r in rs)
    assert all(r["t_launch_ns"] < r_big["t_done_ns"] for r in rs)  # launched while the big batch was held
    assert st["overlapped_batches"] >= 1
    _check_alone(f, da, db, c)
    for x, cc in zip(small, cs):
        _check_alone(f, x[2], x[3], cc)


def test_wide_primes_in_one_stream(torch_mod, fields):
    """Requests over the k = 8, 16, 32 and 64 primes interleaved in one
    request stream: every result equals the same product alone."""
    import torch

    from paper_1811_01490_amd import Server

    g = gi.rng(SEED, 7)
    plist = [P8, P16, P32, P64]
    reqs = []
    for i in range(24):
        params = plist[i % 4]
        la, lb = int(2 ** g.uniform(0, 10)), int(2 ** g.uniform(0, 10))
        a, b, da, db = _operands(params, la, lb, 700 + i)
        reqs.append((params, da, db, _out(torch, params["k"], la + lb - 1)))
    torch.cuda.synchronize()
    with Server(workspace_bytes=2 << 30, slots=2, max_batch=16) as srv:
        tickets = [srv.submit(fields[p["k"]], da, db, c) for p, da, db, c in reqs]
        res = [srv.wait(t) for t in tickets]
    assert all(r["status"] == 0 for r in res)
    for params, da, db, c in reqs:
        _check_alone(fields[params["k"]], da, db, c)


def test_budget_limits_batch_and_rejects_oversize(torch_mod, fields, sleep_cycles):
    import torch

    from paper_1811_01490_amd import GFPError, Server, GFP_ENOMEM

    f = fields[8]
    per = f.polymul_workspace_size(2048, 2048)  # transform size 4096
    with Server(workspace_bytes=per * 5 // 2, slots=1, max_batch=64) as srv:
        assert srv.stats()["slot_bytes"] < 3 * per
        # a request whose transform workspace alone exceeds the slot (size 2^14)
        a, b, da, db = _operands(P8, 5000, 5000, 200)
        with pytest.raises(GFPError) as e:
            srv.submit(f, da, db, _out(torch, 8, 9999))
        assert e.value.code == GFP_ENOMEM
        # hold the only slot so the queue fills, then release it
        hold = _operands(P8, 10, 10, 201)
        ch = _out(torch, 8, 19)
        ops = [_operands(P8, 1500 + i, 1000 + i, 210 + i) for i in range(7)]  # transform size 4096
        outs = [_out(torch, 8, x[2].shape[1] + x[3].shape[1] - 1) for x in ops]
        _tables_ready(torch, f, hold, ops[0])
        ev, side = _held_event(torch, sleep_cycles)
        t0 = srv.submit(f, hold[2], hold[3], ch, ready=ev)
        time.sleep(0.005)
        ts = [srv.submit(f, x[2], x[3], c) for x, c in zip(ops, outs)]
        rs = [srv.wait(t) for t in ts]
        srv.wait(t0)
        st = srv.stats()
    side.synchronize()
    assert all(r["status"] == 0 for r in rs)
    assert max(r["batch_size"] for r in rs) == 2  # two transform-size-4096 requests fit 2.5x one's workspace
    assert st["max_batch_workspace"] <= st["slot_bytes"]
    for x, c in zip(ops, outs):
        _check_alone(f, x[2], x[3], c)


def test_full_queue_and_shutdown(torch_mod, fields, sleep_cycles):
    import torch

    from paper_1811_01490_amd import GFPError, Server, GFP_EAGAIN

    f = fields[16]
    srv = Server(workspace_bytes=1 << 30, slots=1, max_batch=64, max_pending=3)
    hold = _operands(P16, 40, 30, 300)
    ch = _out(torch, 16, 69)
    queued = [_operands(P16, 20 + i, 10 + i, 301 + i) for i in range(4)]
    outs = [_out(torch, 16, x[2].shape[1] + x[3].shape[1] - 1) for x in queued]
    _tables_ready(torch, f, hold, *queued)
    ev, side = _held_event(torch, sleep_cycles)
    t0 = srv.submit(f, hold[2], hold[3], ch, ready=ev)
    time.sleep(0.005)
    ts = [srv.submit(f, x[2], x[3], c) for x, c in zip(queued[:3], outs[:3])]
    with pytest.raises(GFPError) as e:
        srv.submit(f, queued[3][2], queued[3][3], outs[3])
    assert e.value.code == GFP_EAGAIN
    assert all(srv.poll(t) is None for t in ts)
    assert srv.stats()["rejected"] == 1
    srv.close()  # cancels the three queued requests, finishes the held one
    side.synchronize()
    torch.cuda.synchronize()
    _check_alone(f, hold[2], hold[3], ch)
    for c in outs:
        assert bool((c == -1).all())  # never written
    assert t0 not in ts


def test_express_slot_serves_small_requests_past_large_ones(torch_mod, fields, sleep_cycles):
    """With an express slot, a small request submitted behind queued large
    ones is served while they wait; the large ones keep their order."""
    import torch

    from paper_1811_01490_amd import Server

    f = fields[8]
    big = [_operands(P8, 3000, 3000, 500 + i) for i in range(3)]  # transform size 2^13
    small = _operands(P8, 100, 100, 510)  # transform size 2^8
    cb = [_out(torch, 8, 5999) for _ in big]
    cs = _out(torch, 8, 199)
    _tables_ready(torch, f, big[0], small)
    with Server(workspace_bytes=2 * f.polymul_workspace_size(3000, 3000), slots=2, max_batch=1,
                express_log2n=12) as srv:
        ev, side = _held_event(torch, sleep_cycles)
        tb = [srv.submit(f, big[0][2], big[0][3], cb[0], ready=ev)]
        time.sleep(0.005)
        tb += [srv.submit(f, x[2], x[3], c) for x, c in zip(big[1:], cb[1:])]
        ts = srv.submit(f, small[2], small[3], cs)
        r_small = srv.wait(ts)
        rb = [srv.wait(t) for t in tb]
    side.synchronize()
    assert r_small["status"] == 0 and all(r["status"] == 0 for r in rb)
    assert r_small["t_launch_ns"] < rb[0]["t_done_ns"]  # launched while the held large batch ran
    assert r_small["t_launch_ns"] < rb[1]["t_admit_ns"]  # ahead of the large ones queued before it
    assert rb[0]["t_done_ns"] <= rb[1]["t_launch_ns"] <= rb[2]["t_launch_ns"]  # one general slot, FIFO
    _check_alone(f, small[2], small[3], cs)
    for x, c in zip(big, cb):
        _check_alone(f, x[2], x[3], c)


def test_mixed_batch_completes_small_class_first(torch_mod, fields, sleep_cycles):
    """One batch with a small and a large class: the small class is done
    before the large one."""
    import torch

    from paper_1811_01490_amd import Server

    f = fields[16]
    hold = _operands(P16, 10, 10, 600)
    ch = _out(torch, 16, 19)
    large = _operands(P16, 2 ** 14, 2 ** 14, 601)  # transform size 32^3
    small = _operands(P16, 30, 20, 602)
    cl, cs = _out(torch, 16, 2 ** 15 - 1), _out(torch, 16, 49)
    _tables_ready(torch, f, hold, large, small)
    with Server(workspace_bytes=4 << 30, slots=1, max_batch=64) as srv:
        ev, side = _held_event(torch, sleep_cycles)
        t0 = srv.submit(f, hold[2], hold[3], ch, ready=ev)
        time.sleep(0.005)
        tl = srv.submit(f, large[2], large[3], cl)  # queued in arrival order, large first
        ts = srv.submit(f, small[2], small[3], cs)
        rl, rs = srv.wait(tl), srv.wait(ts)
        r0 = srv.wait(t0)
    side.synchronize()
    assert rl["batch_id"] == rs["batch_id"] and rl["batch_size"] == 2, (r0, rl, rs)
    assert rs["t_done_ns"] <= rl["t_done_ns"]
    _check_alone(f, large[2], large[3], cl)
    _check_alone(f, small[2], small[3], cs)


def test_graph_replay_matches_eager_and_alone(torch_mod, fields):
    """Batches run as replayed chunk graphs (the default) give the same
    products as eagerly launched batches and as each product alone, also when
    a graph captured for one chunk is replayed for later chunks of the same
    (field, size, count) with other operands, and when the count is rounded
    up to a power of two (padding entries copy nothing)."""
    import torch

    from paper_1811_01490_amd import Server, to_host

    g = gi.rng(SEED, 9)
    rounds = []
    for rnd in range(3):
        reqs = []
        for i in range(3 + rnd * 2):  # 3, 5, 7 requests: counts rounded up to 4 and 8
            params = P8 if i % 2 == 0 else P16
            la, lb = int(g.integers(100, 2000)), int(g.integers(100, 2000))
            a, b, da, db = _operands(params, la, lb, 300 + 20 * rnd + i)
            reqs.append((params, da, db, _out(torch, params["k"], la + lb - 1), _out(torch, params["k"], la + lb - 1)))
        rounds.append(reqs)
    torch.cuda.synchronize()
    with Server(workspace_bytes=1 << 30, slots=1, max_batch=64, max_wait_us=20000) as gsrv, \
            Server(workspace_bytes=1 << 30, slots=1, max_batch=64, max_wait_us=20000, graphs=False) as esrv:
        for reqs in rounds + rounds:  # every round twice: the second time replays its graphs
            tg = [gsrv.submit(fields[p["k"]], da, db, cg) for p, da, db, cg, ce in reqs]
            te = [esrv.submit(fields[p["k"]], da, db, ce) for p, da, db, cg, ce in reqs]
            assert all(r["status"] == 0 for r in [gsrv.wait(t) for t in tg] + [esrv.wait(t) for t in te])
            for p, da, db, cg, ce in reqs:
                got = to_host(cg)
                assert np.array_equal(got, to_host(ce))
                assert np.array_equal(got, _check_alone(fields[p["k"]], da, db, cg))
                cg.fill_(-1)
                ce.fill_(-1)
            torch.cuda.synchronize()
