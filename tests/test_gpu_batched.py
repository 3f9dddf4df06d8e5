"""GPU tests of the batched form (persistent work-stealing kernels, autotuned
launch shapes, HIP-graph replay): outputs identical to the plain form."""
import numpy as np
import pytest

from gpu_helpers import compare_hits, compare_states, compare_tracks, host, to_dev
from synth import generate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def plain(b, params):
    import torch

    import paper_1912_09161_amd as velo
    px, off = to_dev(b.pixels, b.offsets)
    out = velo.reconstruct(px, off, params=params)
    torch.cuda.synchronize()
    return host(out)


def same(g, r, b):
    compare_hits(g["hits"], r["hits"], b.offsets)
    compare_tracks(g["tracks"], r["tracks"], b.offsets)
    compare_states(g["states"], r["states"], b.offsets, r["tracks"])
    for k in ("x", "y", "z", "tx", "ty", "chi2"):
        from gpu_helpers import track_slots
        sl = track_slots(r["tracks"], b.offsets)
        np.testing.assert_array_equal(g["states"][k][sl].view(np.uint32), r["states"][k][sl].view(np.uint32))


@pytest.mark.parametrize("name,n,xl", [("uneven", 1500, 5.94e-4), ("stress", 200, 2.38e-3)])
def test_batched_equals_plain_and_replays(name, n, xl):
    import torch

    import paper_1912_09161_amd as velo
    b = generate(name, n, workers=8)
    P = velo.default_params(x_over_x0=xl)
    ref = plain(b, P)
    px, off = to_dev(b.pixels, b.offsets)
    ctx = velo.Context()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        bufs = ctx.reconstruct(px, off, params=P, stream=stream)  # autotunes, then captures
    stream.synchronize()
    cfg = ctx.config()
    assert cfg["tuned"]
    first = host(bufs)
    same(first, ref, b)
    # replays of the captured graph, with eager work and synchronisation between them
    for r in range(3):
        for k in ("n_tracks", "nhits"):
            bufs["tracks"][k].zero_()
        bufs["states"]["accepted"].zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            ctx.reconstruct(px, off, params=P, bufs=bufs, stream=stream)
        stream.synchronize()
        _ = (px.to(torch.int64).sum() + r).item()
        same(host(bufs), ref, b)
    ctx.close()


FORKED = dict(cluster_grid=0, mid_grid=512, find_threads=256, find_grid=0, fit_threads=128,
              tier_grids=(16, 8, 8), route_hits=3000, fork=True, find_order=True)


@pytest.mark.parametrize("route", [0, 3000, 1])
def test_forked_routing_replays(route):
    """Events routed past the first track-finding tier, their middle tier on
    the context's side stream: the context's own graph (fork and join inside
    it) replayed, with eager work between replays, equals the plain form."""
    import torch

    import paper_1912_09161_amd as velo
    b = generate("stress", 120, first_event=40, workers=8)
    P = velo.default_params(x_over_x0=2.38e-3)
    ref = plain(b, P)
    px, off = to_dev(b.pixels, b.offsets)
    ctx = velo.Context()
    ctx.set_config(**dict(FORKED, route_hits=route, fork=route != 0, find_order=route != 1))
    stream = torch.cuda.Stream()
    bufs = None
    for r in range(4):
        if bufs is not None:
            for k in ("n_tracks", "nhits"):
                bufs["tracks"][k].fill_(9)
            torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            bufs = ctx.reconstruct(px, off, params=P, bufs=bufs, stream=stream)
        stream.synchronize()
        _ = (px.to(torch.int64).sum() + r).item()
        same(host(bufs), ref, b)
    ctx.close()


@pytest.mark.parametrize("forked", [False, True])
def test_batched_inside_a_caller_graph(forked):
    """A caller captures the (already tuned, or fixed with the routed tier
    forked onto the side stream) batched call into its own graph: the call
    only enqueues; every replay equals the plain form."""
    import torch

    import paper_1912_09161_amd as velo
    b = generate("uneven", 400, workers=8)
    P = velo.default_params()
    ref = plain(b, P)
    px, off = to_dev(b.pixels, b.offsets)
    ctx = velo.Context()
    if forked:
        ctx.set_config(**FORKED)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        bufs = ctx.reconstruct(px, off, params=P, stream=stream)  # tunes eagerly
    stream.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        ctx.reconstruct(px, off, params=P, bufs=bufs, stream=torch.cuda.current_stream())
    for r in range(3):
        for k in ("n_tracks", "nhits"):
            bufs["tracks"][k].zero_()
        bufs["hits"]["key"].zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        _ = (px.to(torch.int64).sum() + r).item()
        same(host(bufs), ref, b)
    ctx.close()


def test_batched_with_classifier_equals_plain_mlp():
    """The batched form with the classifier fused after the fit equals the plain
    reconstruction with the same classifier: hits, tracks, states, scores and
    decisions bit for bit (first call tuned and captured, then a replay)."""
    import torch

    import paper_1912_09161_amd as velo
    from gpu_helpers import track_slots
    from paper_1912_09161_amd import learn
    b = generate("uneven", 600, workers=8)
    P = velo.default_params()
    px, off = to_dev(b.pixels, b.offsets)
    p = learn.he_uniform(9)
    p[256:288] = np.random.default_rng(3).normal(0, 0.2, 32)
    p[1312:1344] = np.random.default_rng(4).normal(0, 0.2, 32)
    mean = torch.tensor([3.0, 10.0, 0.5, 0.0, 0.0, 3.5, 300.0, -100.0], device="cuda")
    std = torch.tensor([2.0, 4.0, 1.0, 0.1, 0.1, 0.8, 300.0, 300.0], device="cuda")
    probe = host(velo.reconstruct_mlp(px, off, velo.Mlp(torch.from_numpy(p).cuda(), mean, std, 0.0), params=P))
    sl = track_slots(probe["tracks"], b.offsets)
    mlp = velo.Mlp(torch.from_numpy(p).cuda(), mean, std, float(np.median(probe["states"]["score"][sl])))
    ref = velo.reconstruct_mlp(px, off, mlp, params=P)
    torch.cuda.synchronize()
    ref = host(ref)
    ctx = velo.Context()
    stream = torch.cuda.Stream()
    bufs = None
    for r in range(2):
        with torch.cuda.stream(stream):
            bufs = ctx.reconstruct(px, off, params=P, mlp=mlp, bufs=bufs, stream=stream)
        stream.synchronize()
        g = host(bufs)
        same(g, ref, b)
        for k in ("score", "accepted"):
            np.testing.assert_array_equal(g["states"][k][sl].view(np.uint8), ref["states"][k][sl].view(np.uint8))
        assert 0 < ref["states"]["accepted"][sl].sum() < len(sl)
    ctx.close()


def test_batched_edge_events():
    """Empty events, flagged events (bad words, hole pixels, plane order,
    duplicates) and an event with one huge cluster through the batched form:
    statuses, hits, tracks and states equal the plain form's."""
    import torch

    import paper_1912_09161_amd as velo
    from synth.raw import line_event, pack, word
    good = line_event([(0.02 * 600, 0.015 * 600, 0.02, 0.015), (-0.01 * 600, 0.02 * 600, -0.01, 0.02)])
    blob = [word(9, 400 + r, 400 + c, 1 + (r * 7 + c) % 15) for r in range(40) for c in range(40)]
    events = [[], good, good + [word(2, 20, 20, 3)], [word(0, 10, 10, 0)], [word(0, 768, 768, 3)],
              [word(4, 100, 100, 3), word(4, 100, 100, 5)], [word(4, 100, 100, 3), word(3, 100, 100, 5)],
              sorted(good + blob, key=lambda w: (w >> 22) & 31), [], good]
    px_h, off_h = pack(events)
    b = type("B", (), {"offsets": off_h})()
    P = velo.default_params()
    ref = plain(type("B", (), {"pixels": px_h, "offsets": off_h})(), P)
    px, off = to_dev(px_h, off_h)
    ctx = velo.Context()
    stream = torch.cuda.Stream()
    bufs = None
    for r in range(2):
        with torch.cuda.stream(stream):
            bufs = ctx.reconstruct(px, off, params=P, bufs=bufs, stream=stream)
        stream.synchronize()
        g = host(bufs)
        np.testing.assert_array_equal(g["hits"]["status"], ref["hits"]["status"])
        same(g, ref, b)
    assert ref["hits"]["status"].any() and ref["tracks"]["n_tracks"][-1] >= 1
    ctx.close()


def test_batched_graph_cache_alternating_batches():
    """One context, two batches of different sizes in different buffers, called
    alternately: every call replays the graph of its own buffers and equals the
    plain form (a replay of the wrong graph would write the other batch)."""
    import torch

    import paper_1912_09161_amd as velo
    P = velo.default_params()
    bs = [generate("nominal", 150, workers=8), generate("uneven", 220, first_event=500, workers=8)]
    refs = [plain(b, P) for b in bs]
    devs = [to_dev(b.pixels, b.offsets) for b in bs]
    ctx = velo.Context()
    stream = torch.cuda.Stream()
    bufs = [None, None]
    for r in range(5):
        k = r % 2
        px, off = devs[k]
        with torch.cuda.stream(stream):
            bufs[k] = ctx.reconstruct(px, off, params=P, bufs=bufs[k], stream=stream)
        stream.synchronize()
        same(host(bufs[k]), refs[k], bs[k])
    ctx.close()
