"""Batched products (gfp_polymul_batched): mixed sizes in one call must give,
for every request, exactly gfp_polymul's result (and the schoolbook product
where the oracle is fast); the hipGraph path must give the same on every
replay, with unrelated eager work and synchronisations between replays."""

import numpy as np
import pytest

import gfp_inputs as gi
from oracle import transform as T
from oracle.field import GFPField, P8, P16, P32, P64
from tests.helpers import canonical_mask, to_ints

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _batch(params, sizes, seed):
    from paper_1811_01490_amd import to_device

    k, r = params["k"], params["r"]
    reqs = []
    for i, (la, lb) in enumerate(sizes):
        a = gi.operand(k, r, la, seed, 2 + 2 * i, edge_frac=0.05)
        b = gi.operand(k, r, lb, seed, 3 + 2 * i, edge_frac=0.05)
        reqs.append((a, b))
    dev = [(to_device(a), to_device(b)) for a, b in reqs]
    return reqs, dev


@pytest.mark.parametrize("params", [P8, P16, P32, P64], ids=["k8", "k16", "k32", "k64"])
def test_batched_mixed_sizes(torch_mod, params):
    import torch

    from paper_1811_01490_amd import Field, to_host

    F = GFPField(**params)
    f = Field(params["k"], params["r"])
    sizes = [(1, 1), (5, 3), (128, 128), (8, 9), (300, 200), (2048, 2048), (1, 2000), (513, 512), (100, 157),
             (4000, 96), (64, 64)] + [(7 + i, 11 + 2 * i) for i in range(20)]
    if params["k"] == 8:
        sizes.append((30000, 30000))  # transform size 16^4
    reqs, dev = _batch(params, sizes, gi.BASE_SEED + 300)
    outs = [torch.full((F.k, a.shape[1] + b.shape[1] - 1), 7, dtype=torch.int64, device="cuda") for a, b in dev]
    descs = f.batch_descs([(a, b, c) for (a, b), c in zip(dev, outs)])
    f.polymul_batched(descs)
    torch.cuda.synchronize()
    for i, ((a, b), (da, db), c) in enumerate(zip(reqs, dev, outs)):
        ch = to_host(c)
        assert canonical_mask(ch, F.r).all(), i
        single = to_host(f.polymul(da, db))
        assert np.array_equal(ch, single), i
        if a.shape[1] * b.shape[1] <= (2048 * 2048 if F.k < 32 else 600 * 600):
            assert to_ints(ch, F.r) == T.polymul(to_ints(a, F.r), to_ints(b, F.r), F.p), i


# (prime, operand sizes, count): every chunk has 2^18 elements.  k = 8: the
# inverse's first launch is one pass (4096 = 16^3, plan 12), a fused pair
# (256 = 16^2, plan 2) or the radix-8 pass (2048 = 8 16^2); k = 16: the
# radix-2 pass (4096 = 2 32^2).  k = 32, 64: with more than one launch the
# inverse takes 1/n from its second launch's tables and the product stays a
# launch of its own (4096); a transform of size K is one fused launch.
FUSED = [(P8, (2048, 2048), 64), (P8, (100, 100), 1024), (P8, (1000, 1000), 128), (P16, (2048, 2048), 64),
         (P32, (2048, 2048), 64), (P64, (2048, 2048), 64), (P32, (32, 33), 4096), (P64, (64, 65), 2048)]


@pytest.mark.parametrize("params,size,count", FUSED,
                         ids=["k8-one", "k8-pair", "k8-radix8", "k16", "k32", "k64", "k32-one", "k64-one"])
def test_fused_pointwise_product(torch_mod, params, size, count):
    """Products in a chunk of 2^18 elements take the pointwise product inside
    the inverse transform's first launch; one product alone takes the separate
    product launch.  Both must agree, and one of them with the schoolbook
    product."""
    import torch

    from paper_1811_01490_amd import Field, to_host

    F = GFPField(**params)
    f = Field(params["k"], params["r"])
    la, lb = size
    sizes = [(la, lb)] * (count - 1) + [(la - 1, lb + 1)]
    reqs, dev = _batch(params, sizes, gi.BASE_SEED + 310)
    outs = [torch.full((F.k, a.shape[1] + b.shape[1] - 1), 7, dtype=torch.int64, device="cuda") for a, b in dev]
    descs = f.batch_descs([(a, b, c) for (a, b), c in zip(dev, outs)])
    f.polymul_batched(descs)
    torch.cuda.synchronize()
    for i, ((da, db), c) in enumerate(zip(dev, outs)):
        ch = to_host(c)
        assert canonical_mask(ch, F.r).all(), i
        assert np.array_equal(ch, to_host(f.polymul(da, db))), i
    if F.k == 8:
        a, b = reqs[-1]
        assert to_ints(to_host(outs[-1]), F.r) == T.polymul(to_ints(a, F.r), to_ints(b, F.r), F.p)


def test_batched_graph_replays(torch_mod):
    import torch

    from paper_1811_01490_amd import Field, to_device, to_host

    F = GFPField(**P8)
    f = Field(P8["k"], P8["r"])
    sizes = [(100, 60), (2000, 2000), (20, 1), (600, 700), (3, 3), (1000, 30)]
    reqs, dev = _batch(P8, sizes, gi.BASE_SEED + 301)
    outs = [torch.zeros((F.k, a.shape[1] + b.shape[1] - 1), dtype=torch.int64, device="cuda") for a, b in dev]
    descs = f.batch_descs([(a, b, c) for (a, b), c in zip(dev, outs)])
    ws = torch.empty(f.polymul_batched_workspace_size(descs) // 8 + 1, dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    want = [T.polymul(to_ints(a, F.r), to_ints(b, F.r), F.p) for a, b in reqs]
    with torch.cuda.stream(stream):
        for rep in range(4):
            for c in outs:
                c.zero_()
            f.polymul_batched(descs, workspace=ws, graph=True, stream=stream)
            # unrelated eager work between replays
            junk = to_device(gi.uniform_digits(F.k, F.r, 4096, 5, rep))
            f.fft_forward(junk, stream=stream)
            stream.synchronize()
            for i, c in enumerate(outs):
                assert to_ints(to_host(c), F.r) == want[i], (rep, i)


def test_graph_cache_bound_and_plan_changes(torch_mod):
    """More distinct argument lists than the cache keeps (so old graphs are
    evicted), and a plan change between replays: every call still gives the
    single-product results."""
    import torch

    from paper_1811_01490_amd import Field, to_host
    from paper_1811_01490_amd.gfp import LAYOUT_ELEMENT_MAJOR

    f = Field(P8["k"], P8["r"])
    sizes = [(100, 60), (1500, 1000), (7, 9)]
    _, dev = _batch(P8, sizes, gi.BASE_SEED + 302)
    ref = [to_host(f.polymul(a, b)) for a, b in dev]
    n_out = sum(a.shape[1] + b.shape[1] - 1 for a, b in dev)
    pool = torch.zeros((8, n_out + 80), dtype=torch.int64, device="cuda")
    stream = torch.cuda.Stream()
    ws = None
    for call in range(70):  # 70 distinct output offsets -> 70 argument lists
        if call == 40:
            f.set_plan(4096, "111", nvec=2, layout=LAYOUT_ELEMENT_MAJOR)
        outs, off = [], call
        for a, b in dev:
            n = a.shape[1] + b.shape[1] - 1
            outs.append(pool[:, off:off + n])
            off += n
        descs = f.batch_descs([(a, b, c) for (a, b), c in zip(dev, outs)])
        if ws is None:
            ws = torch.empty(f.polymul_batched_workspace_size(descs) // 8 + 1, dtype=torch.int64, device="cuda")
        with torch.cuda.stream(stream):
            f.polymul_batched(descs, workspace=ws, graph=True, stream=stream)
            if call in (0, 39, 41, 69):
                f.polymul_batched(descs, workspace=ws, graph=True, stream=stream)  # a replay
        stream.synchronize()
        for i, c in enumerate(outs):
            assert np.array_equal(to_host(c.contiguous()), ref[i]), (call, i)


def test_graph_eviction_after_stream_destroyed(torch_mod):
    """A graph captured on a stream the caller has since destroyed is evicted
    (waiting on the library's own event, not on that stream), and a graph in
    steady use stays cached (least recently used eviction) and correct."""
    import torch

    from paper_1811_01490_amd import Field, to_host

    f = Field(P8["k"], P8["r"])
    _, dev = _batch(P8, [(50, 40), (300, 20)], gi.BASE_SEED + 303)
    ref = [to_host(f.polymul(a, b)) for a, b in dev]
    pool = torch.zeros((8, 2 * 400 + 80), dtype=torch.int64, device="cuda")

    def descs_at(off):
        outs = []
        for a, b in dev:
            n = a.shape[1] + b.shape[1] - 1
            outs.append(pool[:, off:off + n])
            off += n
        return outs, f.batch_descs([(a, b, c) for (a, b), c in zip(dev, outs)])

    outs0, d0 = descs_at(0)
    ws = torch.empty(f.polymul_batched_workspace_size(d0) // 8 + 1, dtype=torch.int64, device="cuda")
    s1 = torch.cuda.Stream()
    with torch.cuda.stream(s1):
        f.polymul_batched(d0, workspace=ws, graph=True, stream=s1)
    s1.synchronize()
    del s1
    torch.cuda.synchronize()
    s2 = torch.cuda.Stream()
    hot_outs, hot = descs_at(1)
    with torch.cuda.stream(s2):
        for call in range(70):  # 70 new lists: the s1 graph is evicted, `hot` is used between them
            outs, d = descs_at(2 + call)
            f.polymul_batched(d, workspace=ws, graph=True, stream=s2)
            s2.synchronize()
            for i, c in enumerate(outs):
                assert np.array_equal(to_host(c.contiguous()), ref[i]), (call, i)
            f.polymul_batched(hot, workspace=ws, graph=True, stream=s2)
            s2.synchronize()
            for i, c in enumerate(hot_outs):
                assert np.array_equal(to_host(c.contiguous()), ref[i]), ("hot", call, i)
