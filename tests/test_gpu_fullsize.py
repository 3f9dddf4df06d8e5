"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (the whole batch in one call).

The oracle runs a seeded sample of the events on its own (events are
independent, so an event's outputs do not depend on the rest of the batch);
the GPU outputs of the same events, taken out of the full-batch buffers, must
match it to the parity bar (clusters bit-exact, identical track hit lists,
states within 1e-4).  Properties that hold for every event are checked on a
larger slice: statuses, hit counts, keys in ascending order inside every
(event, plane), each hit on at most one track, track lengths in [3, 26]."""
import numpy as np
import pytest

from gpu_helpers import compare_all
from synth import generate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def device_batch(b):
    import torch

    import paper_1912_09161_amd as velo
    px = torch.from_numpy(b.pixels.view(np.int32)).cuda()
    off = torch.from_numpy(b.offsets.view(np.int64)).cuda()
    N, E = b.n_pixels, b.n_events
    return velo, px, off, dict(hits=velo.alloc_hits(N, E), tracks=velo.alloc_tracks(N, E),
                               states=velo.alloc_states(N))


def gather(out, offsets, events):
    """Outputs of `events` out of the full-batch device buffers, in the layout
    of a batch holding only those events (as the oracle's sub-batch run)."""
    off = np.asarray(offsets, np.int64)
    ev = np.asarray(events, np.int64)
    sizes = off[ev + 1] - off[ev]
    sub_off = np.concatenate([[0], np.cumsum(sizes)])
    N = max(int(sub_off[-1]), 1)
    cap = max(int(sub_off[-1]) // 3, 1)
    H, T, S = out["hits"], out["tracks"], out["states"]
    row = lambda t, w: t.view(-1, w)[ev].cpu().numpy()  # noqa: E731
    h = dict(layer_start=row(H["layer_start"], 27).view(np.uint32),
             layer_nhits=row(H["layer_nhits"], 26).view(np.uint32),
             n_hits=H["n_hits"][ev].cpu().numpy().view(np.uint32),
             status=H["status"][ev].cpu().numpy().view(np.uint32))
    for k, dt in (("x", np.float32), ("y", np.float32), ("key", np.uint32), ("aux", np.uint32)):
        a = np.zeros(N, dt)
        for i, e in enumerate(ev):
            a[sub_off[i]:sub_off[i + 1]] = H[k][off[e]:off[e + 1]].cpu().numpy().view(dt)
        h[k] = a
    nt = T["n_tracks"][ev].cpu().numpy().view(np.uint32)
    t = dict(n_tracks=nt, status=T["status"][ev].cpu().numpy().view(np.uint32),
             nhits=np.zeros(cap, np.uint8), hit_idx=np.zeros((cap, 26), np.uint32))
    s = {k: np.zeros(cap, np.float32) for k in ("x", "y", "z", "tx", "ty", "chi2")}
    s.update(cov_x=np.zeros((cap, 3), np.float32), cov_y=np.zeros((cap, 3), np.float32),
             ndof=np.zeros(cap, np.int32), accepted=np.zeros(cap, np.uint8))
    hidx = T["hit_idx"].view(-1, 26)
    for i, e in enumerate(ev):
        a, d, n = off[e] // 3, sub_off[i] // 3, int(nt[i])
        if n == 0:
            continue
        t["nhits"][d:d + n] = T["nhits"][a:a + n].cpu().numpy()
        t["hit_idx"][d:d + n] = hidx[a:a + n].cpu().numpy().view(np.uint32)
        for k in ("x", "y", "z", "tx", "ty", "chi2"):
            s[k][d:d + n] = S[k][a:a + n].cpu().numpy()
        for k in ("cov_x", "cov_y"):
            s[k][d:d + n] = S[k].view(-1, 3)[a:a + n].cpu().numpy()
        s["ndof"][d:d + n] = S["ndof"][a:a + n].cpu().numpy()
        s["accepted"][d:d + n] = S["accepted"][a:a + n].cpu().numpy()
    return dict(hits=h, tracks=t, states=s), sub_off.astype(np.uint64)


def check_sample(orc, b, out, n_sample, seed, params=None):
    ev = np.sort(np.random.default_rng(seed).choice(b.n_events, n_sample, replace=False))
    g, sub_off = gather(out, b.offsets, ev)
    sub = b.select(ev)
    assert np.array_equal(sub.offsets, sub_off)
    o = orc.reconstruct(sub.pixels, sub.offsets, params=params, threads=16)
    return compare_all(g, o, sub.offsets)


def check_invariants(b, out, e0, e1):
    """Properties of every event in [e0, e1)."""
    off = np.asarray(b.offsets, np.int64)
    H, T = out["hits"], out["tracks"]
    st = H["status"][e0:e1].cpu().numpy()
    assert not st.any() and not T["status"][e0:e1].cpu().numpy().any()
    lnh = H["layer_nhits"].view(-1, 26)[e0:e1].cpu().numpy().astype(np.int64)
    lst = H["layer_start"].view(-1, 27)[e0:e1].cpu().numpy().astype(np.int64)
    assert np.array_equal(lnh.sum(1), H["n_hits"][e0:e1].cpu().numpy())
    key = H["key"][off[e0]:off[e1]].cpu().numpy().view(np.uint32).astype(np.int64)
    nt = T["n_tracks"][e0:e1].cpu().numpy().astype(np.int64)
    nh_all = T["nhits"].cpu().numpy()
    hidx = T["hit_idx"].view(-1, 26)
    for i, e in enumerate(range(e0, e1)):
        base = off[e] - off[e0]
        for l in range(26):
            k = key[base + lst[i, l]: base + lst[i, l] + lnh[i, l]]
            assert np.all(np.diff(k) > 0) and np.all((k >> 22) == l)
        a, n = off[e] // 3, nt[i]
        if n == 0:
            continue
        nh = nh_all[a:a + n].astype(np.int64)
        assert nh.min() >= 3 and nh.max() <= 26
        hi = hidx[a:a + n].cpu().numpy().view(np.uint32).astype(np.int64)
        used = hi[np.arange(26)[None, :] < nh[:, None]]
        valid = np.zeros(off[e + 1] - off[e], bool)  # event-relative slots holding a hit
        for l in range(26):
            valid[lst[i, l]:lst[i, l] + lnh[i, l]] = True
        assert valid[used].all(), f"event {e}: a track index outside the hits"
        assert len(np.unique(used)) == len(used), f"event {e}: a hit on two tracks"


def test_uneven_100k_batched(orc):
    """Batched form on 100k events of uneven occupancy (PVs/event uniform 1..15)
    in one call, as timed by the benchmark; 300 sampled events vs the oracle."""
    import torch
    b = generate("uneven", 100_000, workers=16)
    velo, px, off, bufs = device_batch(b)
    bufs["ws"] = velo.alloc_batched_workspace(b.n_pixels, b.n_events)
    ctx = velo.Context()
    ctx.reconstruct(px, off, params=velo.default_params(), bufs=bufs)
    ctx.reconstruct(px, off, params=velo.default_params(), bufs=bufs)  # graph replay
    torch.cuda.synchronize()
    ctx.close()
    nh, nt, ns = check_sample(orc, b, bufs, 300, 1)
    assert nt > 300 * 25
    check_invariants(b, bufs, 5000, 5300)


def test_stress_10k_plain(orc):
    """Plain form on 10k high-occupancy events in one call; 200 sampled events
    vs the oracle."""
    import torch
    b = generate("stress", 10_000, workers=16)
    velo, px, off, bufs = device_batch(b)
    bufs["ws"] = velo.alloc_workspace(b.n_pixels, b.n_events)
    velo.reconstruct(px, off, params=velo.default_params(x_over_x0=2.38e-3), bufs=bufs)
    torch.cuda.synchronize()
    check_sample(orc, b, bufs, 200, 2, params=dict(x_over_x0=2.38e-3))
    check_invariants(b, bufs, 100, 300)


def test_learned_10k_fused(orc):
    """Classifier fused after the fit on 10k nominal events: scores equal to the
    separate inference on every track; sampled tracks within the oracle's BF16
    emulation bar."""
    import torch

    from paper_1912_09161_amd import learn
    b = generate("nominal", 10_000, workers=16)
    velo, px, off, bufs = device_batch(b)
    bufs["ws"] = velo.alloc_workspace(b.n_pixels, b.n_events)
    P = velo.default_params()
    velo.reconstruct(px, off, params=P, bufs=bufs)
    feat = velo.track_features(bufs["hits"], bufs["tracks"], bufs["states"], off, b.n_pixels)
    torch.cuda.synchronize()
    nt = bufs["tracks"]["n_tracks"].cpu().numpy().astype(np.int64)
    base = b.offsets[:-1].astype(np.int64) // 3
    slot = np.concatenate([base[e] + np.arange(nt[e]) for e in range(b.n_events)])
    F = feat[torch.from_numpy(slot).cuda()].contiguous()
    mean, std = velo.feature_stats(F)
    p = learn.he_uniform(9)
    p[256:288] = np.random.default_rng(3).normal(0, 0.3, 32)
    mlp = velo.Mlp(torch.from_numpy(p).cuda(), mean, std, 0.1)
    z = velo.mlp_infer(mlp, F).cpu().numpy()
    s2 = velo.fit_mlp(bufs["hits"], bufs["tracks"], off, b.n_pixels, mlp, params=P)
    torch.cuda.synchronize()
    sc = s2["score"].cpu().numpy()[slot]
    np.testing.assert_array_equal(sc.view(np.uint32), z.view(np.uint32))
    np.testing.assert_array_equal(s2["accepted"].cpu().numpy()[slot], (z >= 0.1).astype(np.uint8))
    pick = np.random.default_rng(4).choice(len(slot), 5000, replace=False)
    Fh = F.cpu().numpy()[pick]
    zb = orc.mlp_forward_bf16(p, mean.cpu().numpy(), std.cpu().numpy(), Fh)
    assert np.all(np.abs(z[pick] - zb) <= 1e-3 * (1 + np.abs(zb)))
