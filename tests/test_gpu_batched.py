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


def test_batched_inside_a_caller_graph():
    """A caller captures the (already tuned) batched call into its own graph:
    the call only enqueues; every replay equals the plain form."""
    import torch

    import paper_1912_09161_amd as velo
    b = generate("uneven", 400, workers=8)
    P = velo.default_params()
    ref = plain(b, P)
    px, off = to_dev(b.pixels, b.offsets)
    ctx = velo.Context()
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
