"""Pins of the generator-truth matching and the tracking figures of merit
(Sec. 3.1: a track is correctly reconstructed when at least 70 % of its hits
come from one particle; a particle is reconstructible with hits on at least
three planes).  The readings pinned here: a hit belongs to the particle with
the most charge in it, ties to the lowest id, and to no particle when the
noise charge is at least that much; efficiency counts reconstructible
particles with an accepted matched track; ghost rate = accepted unmatched /
accepted; clone rate = (matched tracks - matched particles) / matched tracks.

The events are toy events built pixel by pixel, so every expected number
follows by counting.
"""
import numpy as np
import pytest

from synth.gen import EventBatch
from synth.truth import Truth, efficiency_ghosts, match_tracks, metrics, track_labels, \
    track_labels_parallel


def batch(events):
    """events: list of lists of (layer, row, col, charge, particle id or -1)."""
    words, pid, q, off = [], [], [], [0]
    for ev in events:
        ev = sorted(ev, key=lambda p: p[0])
        for l, r, c, qq, p in ev:
            words.append(c | (r << 11) | (l << 22) | (qq << 27))
            pid.append(p)
            q.append(qq)
        off.append(len(words))
    E = len(events)
    z = np.zeros(E + 1, np.uint64)
    return EventBatch(pixels=np.array(words, np.uint32), offsets=np.array(off, np.uint64),
                      pix_pid=np.array(pid, np.int32), pix_q=np.array(q, np.uint8),
                      part_off=z.copy(), part={}, pv_off=z.copy(), pv={})


def k(l, r, c):
    return (l << 22) | (r << 11) | c


def tracks_arrays(tracks):
    """[(event, [keys...]), ...] -> (ev, nh, keys[T, 26])."""
    T = len(tracks)
    ev = np.array([e for e, _ in tracks], np.int64)
    nh = np.array([len(t) for _, t in tracks], np.int64)
    keys = np.zeros((T, 26), np.int64)
    for i, (_, t) in enumerate(tracks):
        keys[i, :len(t)] = t
    return ev, nh, keys


def single_pixel_particle(pid, layers, col):
    return [(l, 400, col, 5, pid) for l in layers]


def test_seventy_percent_rule():
    p0 = single_pixel_particle(0, range(10), 300)
    p1 = single_pixel_particle(1, range(10, 14), 500)
    p2 = single_pixel_particle(2, range(14, 17), 700)
    b = batch([p0 + p1 + p2])
    T = Truth(b)
    K0 = [k(l, 400, 300) for l in range(10)]
    K1 = [k(l, 400, 500) for l in range(10, 14)]
    K2 = [k(l, 400, 700) for l in range(14, 17)]
    tracks = [
        (0, K0[:7] + K1[:3]),      # 7 of 10: matched to particle 0
        (0, K0[:6] + K1[:4]),      # 6 of 10: ghost
        (0, K2 + K1[:1]),          # 3 of 4 (75 %): particle 2
        (0, K2[:2] + K1[:1]),      # 2 of 3 (67 %): ghost
        (0, K1[:3]),               # all of particle 1
        (0, K0[:2] + K1[:2] + K2[:2]),  # no particle above a third: ghost
    ]
    m = match_tracks(T, *tracks_arrays(tracks))
    assert m.tolist() == [0, -1, 2, -1, 1, -1]


def test_hit_truth_by_charge_with_noise_and_ties():
    """Two-pixel clusters (the pixels touch): the truth of the hit."""
    cases = [
        ((0, 3), (-1, 5), -1),   # noise carries more charge: no particle
        ((0, 5), (-1, 3), 0),    # particle carries more
        ((0, 4), (-1, 4), -1),   # equal to the noise charge: no particle
        ((1, 4), (0, 4), 0),     # two particles, equal charge: the lower id
        ((1, 6), (0, 4), 1),     # two particles: the larger charge
    ]
    ev = []
    for i, ((pa, qa), (pb, qb), _) in enumerate(cases):
        ev.append((3, 100 + 10 * i, 200, qa, pa))
        ev.append((3, 100 + 10 * i, 201, qb, pb))
    # three contributors: particle 0 (3) beats particle 1 (2) but not the noise (4)
    ev += [(4, 50, 50, 3, 0), (4, 50, 51, 2, 1), (4, 51, 51, 4, -1)]
    T = Truth(batch([ev]))
    got = T.hit_particle(np.zeros(len(cases) + 1, np.int64),
                         np.array([k(3, 100 + 10 * i, 200) for i in range(len(cases))] + [k(4, 50, 50)]))
    assert got.tolist() == [c[2] for c in cases] + [-1]


def test_reconstructible_needs_three_distinct_planes():
    ev = (single_pixel_particle(0, [1, 2], 300)                  # two planes: no
          + single_pixel_particle(1, [1, 2, 3], 500)             # three planes: yes
          + [(5, 100, 100, 5, 2), (5, 300, 300, 5, 2), (6, 100, 100, 5, 2)]  # 3 hits, 2 planes: no
          # three planes, but the third plane's hit is noise-dominated: no
          + [(7, 10, 10, 5, 3), (8, 10, 10, 5, 3), (9, 10, 10, 2, 3), (9, 10, 11, 6, -1)])
    T = Truth(batch([ev]))
    assert T.n_reconstructible == 1
    assert sorted(T.reco_pid[T.reco_ok].tolist()) == [1]


def toy_metrics_event():
    """Particles 0, 1, 2 with 4 single-pixel hits each (all reconstructible)
    and particle 3 with three hits on two planes only (not reconstructible)."""
    ev = (single_pixel_particle(0, range(0, 4), 300) + single_pixel_particle(1, range(0, 4), 500)
          + single_pixel_particle(2, range(0, 4), 700) + single_pixel_particle(3, range(0, 2), 900)
          + [(1, 600, 950, 5, 3)])
    K = {p: [k(l, 400, c) for l in range(4)] for p, c in ((0, 300), (1, 500), (2, 700))}
    K[3] = [k(0, 400, 900), k(1, 400, 900), k(1, 600, 950)]
    return ev, K


def test_efficiency_ghost_and_clone_rates():
    ev, K = toy_metrics_event()
    b = batch([ev])
    T = Truth(b)
    tracks = [
        (0, K[0][:4]),                       # particle 0
        (0, K[0][:2] + K[3][:1]),            # particle 0 again, 2 of 3 hits: ghost
        (0, K[0][1:4]),                      # particle 0 again: a clone
        (0, K[1][:3]),                       # particle 1
        (0, [K[0][3], K[1][3], K[2][3]]),    # ghost
    ]
    ev_a, nh, keys = tracks_arrays(tracks)
    m = match_tracks(T, ev_a, nh, keys)
    assert m.tolist() == [0, -1, 0, 1, -1]
    acc = np.ones(len(tracks), bool)
    r = metrics(T, ev_a, nh, keys, acc)
    assert r["n_tracks"] == 5 and r["ghosts"] == 2
    assert r["ghost_rate"] == pytest.approx(2 / 5)
    assert r["n_reconstructible"] == 3 and r["found"] == 2
    assert r["efficiency"] == pytest.approx(2 / 3)
    assert r["clone_rate"] == pytest.approx((3 - 2) / 3)
    # a rejected track counts nowhere: dropping the clone and one ghost
    acc2 = np.array([True, False, False, True, True])
    r2 = metrics(T, ev_a, nh, keys, acc2)
    assert (r2["n_tracks"], r2["ghosts"], r2["found"]) == (3, 1, 2)
    assert r2["clone_rate"] == 0.0
    # dropping the only track of particle 1 loses it from the efficiency
    acc3 = np.array([True, True, True, False, True])
    assert metrics(T, ev_a, nh, keys, acc3)["efficiency"] == pytest.approx(1 / 3)


def fake_outputs(b, tracks_per_event):
    """Hit and track arrays in the reconstruction's layout for given key lists:
    each event's hits are listed in slot order at offsets[e] + i."""
    N = b.n_pixels
    key = np.zeros(max(N, 1), np.uint32)
    E = b.n_events
    cap = max(N // 3, 1)
    nt = np.zeros(E, np.uint32)
    nhits = np.zeros(cap, np.uint8)
    hidx = np.zeros((cap, 26), np.uint32)
    for e in range(E):
        a = int(b.offsets[e])
        ks = sorted(set(int(w) & 0x07FFFFFF for w in b.event_pixels(e)))
        slot_of = {kk: i for i, kk in enumerate(ks)}
        key[a:a + len(ks)] = ks
        base = a // 3
        for t, trk in enumerate(tracks_per_event[e]):
            nhits[base + t] = len(trk)
            hidx[base + t, :len(trk)] = [slot_of[kk] for kk in trk]
        nt[e] = len(tracks_per_event[e])
    return dict(key=key), dict(n_tracks=nt, nhits=nhits, hit_idx=hidx)


@pytest.mark.parametrize("workers,chunk", [(1, 250), (3, 1)])
def test_track_labels_over_events(workers, chunk):
    """Labels and figures over a multi-event batch agree with the per-track
    counting above, whether computed in one piece or over event chunks."""
    ev, K = toy_metrics_event()
    b = batch([ev, ev, ev])
    per_event = [[K[0][:4], K[1][:3], [K[0][3], K[1][3], K[2][3]]],   # 2 matched, 1 ghost
                 [K[2][:4], K[3]],             # 1 matched, 1 of a non-reconstructible particle
                 []]                                                   # nothing found
    hits, tracks = fake_outputs(b, per_event)
    slot, lab, uid, reco = track_labels_parallel(b, tracks, hits, workers=workers, chunk=chunk)
    assert lab.tolist() == [1, 1, 0, 1, 1]
    assert len(np.unique(reco)) == 9
    r = efficiency_ghosts(uid, np.ones(len(slot), bool), reco)
    assert (r["n_tracks"], r["ghosts"], r["found"]) == (5, 1, 3)
    assert r["efficiency"] == pytest.approx(3 / 9)
    s1, l1, u1, r1 = track_labels(Truth(b), tracks, hits, b.offsets)
    assert np.array_equal(s1, slot) and np.array_equal(l1, lab) and np.array_equal(u1, uid)
    assert np.array_equal(np.sort(r1), np.sort(reco))
