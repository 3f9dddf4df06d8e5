"""GPU parity of every launch shape the batched form's tuner may pick.

The tuner keeps a persistent (work-stealing) grid only when it wins on the
tuning stream, so which kernels run depends on the workload.  Here every
candidate shape is fixed through velo_context_set_config, one stage varied at
a time, and the outputs of each are compared with the oracle element by
element: clustering one workgroup per segment or persistent grids of 1024 to
8192 workgroups (with 64 to 1024 large-segment workgroups), track finding
with 128 or 256 lanes per event, one workgroup per event or persistent grids
of 512 to 1536, the fit with 64 to 256 lanes, the tiers that take the
escalated events with grids from their full size down to one workgroup,
events taken largest first by the first tier, events routed past it (by
plane capacity, by hits, all of them) with and without the fork onto the
context's side stream, the tiny tier ahead of the small one.
Events of uneven occupancy and high-occupancy events (where the larger
track-finding tiers run).
"""
import numpy as np
import pytest

from gpu_helpers import compare_all, host, to_dev
from synth import generate

pytestmark = pytest.mark.gpu

CLUSTER = [(cg, mg) for cg in (0, 1024, 2048, 4096, 8192) for mg in (64, 256, 512, 1024)]
FIND = [(nt, g) for nt in (128, 256) for g in (0, 512, 768, 1024, 1536)]
FIT = [64, 128, 256]
TIERS = [(64, 32, 32), (16, 8, 8), (1, 1, 1)]
# first tier largest event first; routing past the first tier: by plane
# capacity only, by hits, every event; unforked and forked, with full and with
# one-workgroup tier grids
ROUTE = [(0, False, True), (-1, False, False), (3000, False, True), (1, False, False), (3000, True, False),
         (1, True, True), (-1, True, True)]
BASE = dict(cluster_grid=0, mid_grid=512, find_threads=256, find_grid=0, fit_threads=128,
            tier_grids=(512, 256, 128))


def shapes():
    out = [dict(BASE, cluster_grid=cg, mid_grid=mg) for cg, mg in CLUSTER]
    out += [dict(BASE, find_threads=nt, find_grid=g) for nt, g in FIND]
    out += [dict(BASE, fit_threads=f) for f in FIT]
    out += [dict(BASE, tier_grids=t) for t in TIERS]
    out += [dict(BASE, route_hits=r, fork=f, find_order=o) for r, f, o in ROUTE]
    out += [dict(BASE, find_threads=128, route_hits=3000, fork=True, find_order=True, tier_grids=(1, 1, 1))]
    # the tiny tier ahead of the small one, alone, largest first, with one-workgroup hand-over tiers
    out += [dict(BASE, tiny=True), dict(BASE, tiny=True, find_order=True),
            dict(BASE, tiny=True, tier_grids=(1, 1, 1))]
    # all persistent at once
    out.append(dict(cluster_grid=2048, mid_grid=512, find_threads=256, find_grid=1024, fit_threads=128,
                    tier_grids=(16, 8, 8)))
    return out


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("name,n,xl", [("uneven", 1200, 5.94e-4), ("stress", 160, 2.38e-3)])
def test_every_launch_shape_equals_oracle(orc, name, n, xl):
    import torch

    import paper_1912_09161_amd as velo
    b = generate(name, n, first_event=700, workers=8)
    o = orc.reconstruct(b.pixels, b.offsets, params=dict(x_over_x0=xl), threads=8)
    P = velo.default_params(x_over_x0=xl)
    px, off = to_dev(b.pixels, b.offsets)
    stream = torch.cuda.Stream()
    bufs = None
    for sh in shapes():
        print(f"{name} {n} events, shape {sh}", flush=True)
        ctx = velo.Context()
        ctx.set_config(**sh)
        cfg = ctx.config()
        assert cfg["source"] == "set" and cfg["find_grid"] == sh["find_grid"]
        assert cfg["tier_grids"] == list(sh["tier_grids"])
        assert cfg["route_hits"] == sh.get("route_hits", 0) and cfg["fork"] == sh.get("fork", False)
        assert cfg["find_order"] == sh.get("find_order", False) and cfg["tiny"] == sh.get("tiny", False)
        if bufs is not None:  # stale outputs of the previous shape must be overwritten
            for k in ("n_tracks", "nhits"):
                bufs["tracks"][k].fill_(7)
            bufs["hits"]["n_hits"].fill_(-1)
        with torch.cuda.stream(stream):
            bufs = ctx.reconstruct(px, off, params=P, bufs=bufs, stream=stream)
        stream.synchronize()
        compare_all(host(bufs), o, b.offsets)
        ctx.close()
    if name == "stress":
        assert o["hits"]["layer_nhits"].max() > 352  # the middle tier ran


def test_set_config_rejects_bad_shapes():
    import paper_1912_09161_amd as velo
    ctx = velo.Context()
    for bad in (dict(find_threads=192), dict(fit_threads=32), dict(mid_grid=0), dict(cluster_grid=-1),
                dict(find_grid=70000), dict(tier_grids=(0, 8, 8)), dict(tier_grids=(513, 8, 8)),
                dict(tier_grids=(16, 257, 8)), dict(tier_grids=(16, 8, 129)),
                dict(route_hits=-2), dict(route_hits=3000, find_grid=512), dict(fork=True),
                dict(route_hits=1, fork=2), dict(find_order=True, find_grid=512), dict(find_order=2),
                dict(tiny=True, find_grid=512), dict(tiny=True, route_hits=-1), dict(tiny=True, find_threads=128),
                dict(tiny=2)):
        with pytest.raises(velo.VeloError):
            ctx.set_config(**dict(BASE, **bad))
    assert ctx.config()["source"] == "untuned"
    ctx.close()


def test_tune_cache_serves_a_new_context():
    """A second context meeting the same workload class takes the shapes the
    first one tuned, without timing anything, and gives identical outputs."""
    import torch

    import paper_1912_09161_amd as velo
    b = generate("nominal", 300, first_event=300, workers=8)
    P = velo.default_params(s_fwd=0.0401)  # parameters no other test tunes with
    px, off = to_dev(b.pixels, b.offsets)
    c1, c2 = velo.Context(), velo.Context()
    r1 = host(c1.reconstruct(px, off, params=P))
    torch.cuda.synchronize()
    r2 = host(c2.reconstruct(px, off, params=P))
    torch.cuda.synchronize()
    k1, k2 = c1.config(), c2.config()
    assert k1["source"] == "tuned" and k2["source"] == "tune cache"
    for k in ("cluster_grid", "mid_grid", "find_threads", "find_grid", "fit_threads", "tier_grids"):
        assert k1[k] == k2[k]
    for part in ("hits", "tracks"):
        for k, v in r1[part].items():
            np.testing.assert_array_equal(v, r2[part][k])
    c1.close()
    c2.close()
