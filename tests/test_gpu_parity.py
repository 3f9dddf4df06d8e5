"""GPU parity: libvelo (HIP, through its C ABI) against the CPU oracle.

Bar: clusters bit-exact (positions compared as bit patterns), track hit lists
identical in the canonical order, fitted states within 1e-4 relative (with
absolute floors, since beamline x and y sit near zero), identical ndof and
plain-cut decisions, identical per-event status codes.
"""
import numpy as np
import pytest

from gpu_helpers import compare_all, gpu_reconstruct
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
