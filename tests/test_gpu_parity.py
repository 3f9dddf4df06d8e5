"""GPU parity: libvelo (HIP, through its C ABI) against the CPU oracle.

Bar: clusters bit-exact (positions compared as bit patterns), track hit lists
identical in the canonical order, fitted states within 1e-4 relative (with
absolute floors, since beamline x and y sit near zero), identical ndof and
plain-cut decisions, identical per-event status codes.
"""
import numpy as np
import pytest

from gpu_helpers import compare_all, gpu_reconstruct, to_dev
from synth import generate
from synth.raw import line_event, pack, shuffle_within_layers, word

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def run_pair(orc, pixels, offsets, params=None):
    g = gpu_reconstruct(pixels, offsets, params)
    o = orc.reconstruct(pixels, offsets, params=params, threads=8)
    return g, o, compare_all(g, o, offsets)


def test_noiseless_straight(orc):
    b = generate("cpu10")
    g, o, (nh, nt, ns) = run_pair(orc, b.pixels, b.offsets)
    assert nt == 200


def test_nominal_200(orc):
    b = generate("nominal", 200)
    g, o, (nh, nt, ns) = run_pair(orc, b.pixels, b.offsets)
    assert nt > 30000


def test_stress_events(orc):
    """High occupancy: segments above the one-wave clustering capacity and
    planes above the small track-finding tables (the larger tiers run)."""
    b = generate("stress", 24)
    g, o, (nh, nt, ns) = run_pair(orc, b.pixels, b.offsets, params=dict(x_over_x0=2.38e-3))
    assert o["hits"]["layer_nhits"].max() > 384


def test_uneven_events(orc):
    b = generate("uneven", 300)
    run_pair(orc, b.pixels, b.offsets)


def test_statuses_and_empty_events(orc):
    good = line_event([(0.02 * 600, 0.015 * 600, 0.02, 0.015)])
    events = [
        [], good,
        good + [word(2, 20, 20, 3)],
        [word(0, 10, 10, 0)], [word(0, 1536, 10, 3)], [word(0, 10, 1600, 3)],
        [word(26, 10, 10, 3)], [word(0, 10, 10, 3) | (1 << 31)], [word(0, 768, 768, 3)],
        [word(4, 100, 100, 3), word(4, 100, 100, 5)],
        [word(4, 100, 100, 3), word(4, 100, 100, 5), word(0, 5, 5, 0)],
        [word(4, 100, 100, 3), word(3, 100, 100, 5)],
        [], [], good,
    ]
    px, off = pack(events)
    g, o, _ = run_pair(orc, px, off)
    assert o["hits"]["status"].any()
    assert g["tracks"]["n_tracks"][1] == 1 and g["tracks"]["n_tracks"][-1] == 1


def test_all_empty_batch(orc):
    px, off = pack([[], [], []])
    run_pair(orc, px, off)


def test_huge_segment_workspace_path(orc):
    """One plane with 70 x 70 touching pixels (one 4900-pixel cluster) next to
    normal events: clustering runs from the caller's workspace."""
    ws = [word(9, 400 + r, 400 + c, 1 + (r * 7 + c) % 15) for r in range(70) for c in range(70)]
    rng = np.random.default_rng(5)
    rng.shuffle(ws)
    b = generate("nominal", 3)
    evs = [b.event_pixels(0), ws, b.event_pixels(1)]
    px, off = pack(evs)
    g, o, _ = run_pair(orc, px, off)
    assert g["hits"]["n_hits"][1] == 1


def test_overflow_event(orc):
    ws = [word(l, 1000 + r, 1000 + c, 4) for l in (18, 19, 20) for r in range(0, 120, 2)
          for c in range(0, 120, 2)]
    good = line_event([(0.02 * 600, 0.015 * 600, 0.02, 0.015)])
    px, off = pack([good, ws, good])
    g, o, _ = run_pair(orc, px, off)
    assert g["tracks"]["status"][1] == 16


def test_permutation_and_repeat_determinism(orc):
    b = generate("nominal", 60)
    g1 = gpu_reconstruct(b.pixels, b.offsets)
    g2 = gpu_reconstruct(b.pixels, b.offsets)
    px3 = shuffle_within_layers(b.pixels, b.offsets, seed=11)
    g3 = gpu_reconstruct(px3, b.offsets)
    from gpu_helpers import compare_hits, compare_tracks
    for g in (g2, g3):
        compare_hits(g["hits"], g1["hits"], b.offsets)
        compare_tracks(g["tracks"], g1["tracks"], b.offsets)


def test_nominal_full_batch(orc):
    """The benchmark workload: 1000 nominal events in one launch, all compared."""
    b = generate("nominal", 1000)
    g, o, (nh, nt, ns) = run_pair(orc, b.pixels, b.offsets)
    assert nt > 150000


def test_fit_checks_caller_tracks():
    """velo_fit on caller-edited tracks: an oversized track count is clamped to
    the event's slots, slots with an invalid hit count or a hit outside the
    event are skipped and keep their previous state; every other slot equals
    the fit of the unedited tracks."""
    import torch

    import paper_1912_09161_amd as velo
    b = generate("nominal", 20)
    px, off = to_dev(b.pixels, b.offsets)
    out = velo.reconstruct(px, off)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in out["states"].items()}
    tr = {k: v.clone() for k, v in out["tracks"].items()}
    o = b.offsets.astype(np.int64)
    nt = tr["n_tracks"].cpu().numpy()
    e = 3
    base, cap = o[e] // 3, (o[e + 1] - o[e]) // 3
    assert nt[e] >= 2 and cap > nt[e]
    # slots after the event's real tracks hold no track; then a huge count
    tr["nhits"][base + nt[e]:base + cap] = 0
    tr["n_tracks"][e] = -16  # 0xFFFFFFF0
    bad_n, bad_i = base, base + 1
    tr["nhits"][bad_n] = 27
    tr["hit_idx"][26 * bad_i + 1] = int(o[e + 1] - o[e])
    st = {k: torch.full_like(v, 7) for k, v in ref.items()}
    velo.fit(out["hits"], tr, off, b.n_pixels, states=st)
    torch.cuda.synchronize()
    for k in ("x", "y", "z", "tx", "ty", "chi2", "ndof", "accepted"):
        g, r = st[k].cpu().numpy(), ref[k].cpu().numpy()
        for ev in range(20):
            sl = np.arange(o[ev] // 3, o[ev] // 3 + nt[ev])
            if ev == e:
                sl = sl[(sl != bad_n) & (sl != bad_i)]
            np.testing.assert_array_equal(g[sl].view(np.uint8), r[sl].view(np.uint8), err_msg=k)
        skipped = np.r_[bad_n, bad_i, np.arange(base + nt[e], base + cap)]
        assert np.all(g[skipped] == 7), k


def test_small_tier_capacity_edges(orc):
    """Events at the limits of the small track-finding tier: 288 hits on one
    plane (the most it holds) and 289 (handed to the middle tier before any
    work); 256 and 257 long straight lines from the origin (the most active
    tracks it holds, and one more), and 340, seen on both sides of it, with
    more active tracks and seed doublets than the small tier holds (handed
    over part way through); every event equals the oracle."""
    def grid_plane(l, n):  # n isolated pixels on plane l
        return [word(l, 100 + 2 * (k // 600), 100 + 2 * (k % 600), 3) for k in range(n)]

    def by_plane(ws):  # distinct addresses, grouped by plane
        return sorted(dict.fromkeys(int(w) for w in ws), key=lambda w: (w >> 22) & 31)

    good = line_event([(0.02 * 600, 0.015 * 600, 0.02, 0.015)])
    def lines(m):
        return [(0.0, 0.0, 0.05 * np.cos(2 * np.pi * k / m + 0.01), 0.05 * np.sin(2 * np.pi * k / m + 0.01))
                for k in range(m)]
    events = [by_plane(good + grid_plane(20, 287)), by_plane(good + grid_plane(20, 288)),
              by_plane(line_event(lines(340))), by_plane(line_event(lines(256))),
              by_plane(line_event(lines(257))), good]
    px, off = pack(events)
    g, o, _ = run_pair(orc, px, off)
    per_plane = o["hits"]["layer_nhits"].reshape(-1, 26).max(1)
    assert per_plane[0] == 288 and per_plane[1] == 289 and per_plane[2] == 340
    assert per_plane[3] == 256 and per_plane[4] == 257
    assert o["tracks"]["n_tracks"][2] > 600


def test_larger_tier_capacity_edges(orc):
    """One plane at the middle tier's limit (640 hits) and one above it (641,
    to the large tier), at the large tier's limit (1024) and above it (1025, to
    the workspace tier, which then completes normally): every event equals the
    oracle."""
    def grid_plane(l, n):  # n isolated pixels on plane l
        return [word(l, 100 + 2 * (k // 600), 100 + 2 * (k % 600), 3) for k in range(n)]

    good = line_event([(0.02 * 600, 0.015 * 600, 0.02, 0.015)])
    events = [sorted(good + grid_plane(20, n - 1), key=lambda w: (w >> 22) & 31) for n in (640, 641, 1024, 1025)]
    px, off = pack(events)
    g, o, _ = run_pair(orc, px, off)
    assert list(o["hits"]["layer_nhits"].reshape(-1, 26).max(1)) == [640, 641, 1024, 1025]
    assert list(g["tracks"]["n_tracks"]) == [1, 1, 1, 1] and not g["tracks"]["status"].any()


@pytest.mark.parametrize("name", ["good", "descent", "overlap", "beyond", "empty"])
def test_bad_offsets(orc, name):
    """Offset tables that break the usable-offsets rule (a decreasing pair, a
    start below an earlier offset, an end beyond the buffer) next to good
    events: statuses equal the oracle's, flagged events have no hits and no
    tracks, the good events' outputs equal the oracle's; plain and batched."""
    import torch

    import paper_1912_09161_amd as velo
    from gpu_helpers import host, compare_all
    from synth.raw import bad_offsets_case
    b, cases = bad_offsets_case()
    offs, exp = cases[name]
    off = np.array(offs, np.uint64)
    print(f"bad offsets case {name}: {offs} over {len(b.pixels)} words", flush=True)
    g, o, _ = run_pair(orc, b.pixels, off)
    np.testing.assert_array_equal(o["hits"]["status"], np.array(exp, np.uint32))
    np.testing.assert_array_equal(g["hits"]["status"], np.array(exp, np.uint32))
    px, doff = to_dev(b.pixels, off)
    ctx = velo.Context()
    ctx.set_config(cluster_grid=1024, mid_grid=256, find_threads=256, find_grid=512, fit_threads=128)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        bufs = ctx.reconstruct(px, doff, stream=stream)
    stream.synchronize()
    gb = host(bufs)
    np.testing.assert_array_equal(gb["hits"]["status"], np.array(exp, np.uint32))
    compare_all(gb, o, off)
    ctx.close()


def test_tiny_tier_capacity_edges(orc):
    """The batched form with the tiny track-finding tier ahead of the small
    one (fixed through velo_context_set_config, alone and with the
    largest-first order): 192 hits on one plane (the most it holds) and 193
    (handed on at once); 192 and 193 long straight lines from the origin (its
    active-track limit and one more); 250 lines (handed on part way, within
    the small tier) and 340 (on to the middle tier); every event equals the
    oracle, next to ordinary nominal events."""
    import torch

    import paper_1912_09161_amd as velo
    from gpu_helpers import host

    def grid_plane(l, n):  # n isolated pixels on plane l
        return [word(l, 100 + 2 * (k // 600), 100 + 2 * (k % 600), 3) for k in range(n)]

    def by_plane(ws):  # distinct addresses, grouped by plane
        return sorted(dict.fromkeys(int(w) for w in ws), key=lambda w: (w >> 22) & 31)

    def lines(m):
        return [(0.0, 0.0, 0.05 * np.cos(2 * np.pi * k / m + 0.01), 0.05 * np.sin(2 * np.pi * k / m + 0.01))
                for k in range(m)]
    good = line_event([(0.02 * 600, 0.015 * 600, 0.02, 0.015)])
    nom = generate("nominal", 40, first_event=1200)
    nom_events = [nom.pixels[nom.offsets[e]:nom.offsets[e + 1]].tolist() for e in range(nom.n_events)]
    events = [by_plane(good + grid_plane(20, 191)), by_plane(good + grid_plane(20, 192)),
              by_plane(line_event(lines(192))), by_plane(line_event(lines(193))),
              by_plane(line_event(lines(250))), by_plane(line_event(lines(340)))] + nom_events
    px_np, off_np = pack(events)
    o = orc.reconstruct(px_np, off_np, threads=8)
    per_plane = o["hits"]["layer_nhits"].reshape(-1, 26).max(1)
    assert list(per_plane[:6]) == [192, 193, 192, 193, 250, 340]
    px, off = to_dev(px_np, off_np)
    base = dict(cluster_grid=0, mid_grid=512, find_threads=256, find_grid=0, fit_threads=128,
                tier_grids=(512, 256, 128))
    for order in (False, True):
        ctx = velo.Context()
        ctx.set_config(**dict(base, tiny=True, find_order=order))
        assert ctx.config()["tiny"]
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            bufs = ctx.reconstruct(px, off, stream=stream)
        stream.synchronize()
        compare_all(host(bufs), o, off_np)
        ctx.close()
