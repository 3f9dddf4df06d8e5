"""Pins of the oracle's search by triplet (Sec. 2.3.1, second paragraph).

References independent of the oracle: generator truth (noiseless straight
tracks must come back exactly), hand-built events whose answer follows from
the rules by inspection, and invariants (hit exclusivity, permutation
invariance, three consecutive planes per seed).
"""
import numpy as np
import pytest

from synth import generate
from synth.gen import layer_z_mm
from synth.raw import line_event, pack, shuffle_within_layers, word
from synth.truth import Truth, match_tracks, metrics, track_list


def tracks_as_keysets(r, offsets):
    ev, slot, nh, keys = track_list(r["tracks"], r["hits"], offsets)
    out = {}
    for e, n, k in zip(ev, nh, keys):
        out.setdefault(int(e), []).append(tuple(int(v) for v in k[:n]))
    return out


def test_noiseless_straight_tracks_are_found_exactly(orc):
    """Configuration with 1 PV, 20 straight tracks, full efficiency, 1-pixel
    clusters and no noise: every particle with >= 3 hits is found with
    exactly its own hits and nothing else is found."""
    b = generate("cpu10")
    r = orc.reconstruct(b.pixels, b.offsets)
    truth = Truth(b)
    found = tracks_as_keysets(r, b.offsets)
    exceptions = []
    for e in range(b.n_events):
        w = b.event_pixels(e)
        pid = b.pix_pid[int(b.offsets[e]):int(b.offsets[e + 1])]
        want = {}
        for k, p in zip(w & 0x07FFFFFF, pid):
            want.setdefault(int(p), set()).add(int(k))
        # truth sets whose pixels touch another particle's pixel would merge
        got = [set(t) for t in found.get(e, [])]
        for p, ks in want.items():
            if len(ks) < 3:
                continue
            if ks not in got:
                exceptions.append((e, p))
        assert len(got) == sum(1 for ks in want.values() if len(ks) >= 3) - sum(1 for x in exceptions if x[0] == e)
    # no merged clusters happen in this sample: every particle is exact
    assert exceptions == []
    ev, slot, nh, keys = track_list(r["tracks"], r["hits"], b.offsets)
    m = metrics(truth, ev, nh, keys, np.ones(len(ev), bool))
    assert m["ghosts"] == 0 and m["efficiency"] == 1.0 and m["clone_rate"] == 0.0


def test_hits_exclusive_and_tracks_ordered(orc):
    b = generate("nominal", 30)
    r = orc.reconstruct(b.pixels, b.offsets)
    found = tracks_as_keysets(r, b.offsets)
    for e, ts in found.items():
        allk = [k for t in ts for k in t]
        assert len(allk) == len(set(allk)), "a hit is used by two tracks"
        firsts = [t[0] for t in ts]
        assert firsts == sorted(firsts, reverse=True)
        for t in ts:
            lay = [k >> 22 for k in t]
            assert len(t) >= 3
            # decreasing z, first three planes consecutive (seed), gaps <= max_skip
            assert all(a > b for a, b in zip(lay, lay[1:]))
            assert lay[0] - lay[1] == 1 and lay[1] - lay[2] == 1
            assert all(a - b <= 2 for a, b in zip(lay, lay[1:]))


def test_permutation_invariance(orc):
    b = generate("nominal", 20)
    r1 = orc.reconstruct(b.pixels, b.offsets)
    px2 = shuffle_within_layers(b.pixels, b.offsets, seed=3)
    r2 = orc.reconstruct(px2, b.offsets)
    assert tracks_as_keysets(r1, b.offsets) == tracks_as_keysets(r2, b.offsets)
    # event order does not matter either
    perm = np.random.default_rng(0).permutation(b.n_events)
    b3 = b.select(perm)
    r3 = orc.reconstruct(b3.pixels, b3.offsets)
    t1 = tracks_as_keysets(r1, b.offsets)
    t3 = tracks_as_keysets(r3, b3.offsets)
    for i, e in enumerate(perm):
        assert t3.get(i, []) == t1.get(int(e), [])


def from_pv(tx, ty, zpv=-600.0):
    """Line through (0, 0, zpv) as (x0, y0, tx, ty) at z = 0.  With zpv = -600 mm
    and a total slope in (0.016, 0.031) it stays inside the sensor and outside
    the beam hole on all 26 planes."""
    return (-tx * zpv, -ty * zpv, tx, ty)


def keys_of_line(x0, y0, tx, ty, layers):
    z = layer_z_mm()
    out = []
    for l in layers:
        xr = x0 + tx * z[l]
        yr = y0 + ty * z[l]
        c = int(np.floor(xr / 0.055 + 768))
        rr = int(np.floor(yr / 0.055 + 768))
        out.append((l << 22) | (rr << 11) | c)
    return out


def test_one_missing_plane_is_bridged_two_split_the_track(orc):
    trk = from_pv(0.02, 0.015)
    # one gap at layer 12: one track of 25 hits
    px, off = pack([line_event([trk], skip={(0, 12)})])
    r = orc.reconstruct(px, off)
    ts = tracks_as_keysets(r, off)[0]
    assert len(ts) == 1 and len(ts[0]) == 25
    assert sorted(ts[0], reverse=True) == list(ts[0])
    # two consecutive gaps at 12 and 11: the track closes; a new one is seeded below
    px, off = pack([line_event([trk], skip={(0, 12), (0, 11)})])
    r = orc.reconstruct(px, off)
    ts = tracks_as_keysets(r, off)[0]
    assert sorted(len(t) for t in ts) == [11, 13]
    up = [t for t in ts if len(t) == 13][0]
    assert [k >> 22 for k in up] == list(range(25, 12, -1))


def test_isolated_three_hit_track_survives(orc):
    trk = from_pv(-0.012, 0.02)
    px, off = pack([line_event([trk], layers=[5, 4, 3])])
    r = orc.reconstruct(px, off)
    ts = tracks_as_keysets(r, off)[0]
    assert len(ts) == 1 and [k >> 22 for k in ts[0]] == [5, 4, 3]


def test_non_consecutive_hits_do_not_seed(orc):
    trk = from_pv(0.018, -0.016)
    px, off = pack([line_event([trk], layers=[20, 18, 16, 14, 12])])
    r = orc.reconstruct(px, off)
    assert r["tracks"]["n_tracks"][0] == 0


def test_competing_hits_go_to_the_closer_prediction(orc):
    """Two candidate hits for one track on a plane: the one nearer the line wins;
    the farther one is left unused (too few neighbours to seed its own track)."""
    trk = from_pv(0.025, 0.0)
    words = line_event([trk], layers=range(10, 26))
    z = layer_z_mm()
    # extra pixel two columns away (0.11 mm) from the track crossing on layer 9,
    # and the true crossing pixel on layer 9
    x9 = trk[0] + 0.025 * z[9]
    rt, ct = int(np.floor(0.0 / 0.055 + 768)), int(np.floor(x9 / 0.055 + 768))
    words += [word(9, rt, ct, 5), word(9, rt, ct + 2, 5)]
    words.sort(key=lambda w: (w >> 22) & 31)
    px, off = pack([words])
    r = orc.reconstruct(px, off)
    ts = tracks_as_keysets(r, off)[0]
    assert len(ts) == 1 and len(ts[0]) == 17
    assert ts[0][-1] == (9 << 22) | (rt << 11) | ct


def test_seed_conflict_lower_priority_loses(orc):
    """Two seeds share the middle hit: A is exactly collinear (s = 0) while B
    bends by one pixel (s = 0.055^2 mm^2, inside the seed window).  Greedy by
    ascending s keeps A; B's other two hits stay unused and nothing else can
    be seeded from three planes."""
    h1 = (800, 1102)
    a0, a2 = (800, 1100), (800, 1104)
    b0, b2 = (802, 1100), (798, 1105)
    words = [word(10, *a2, 5), word(10, *b2, 5), word(11, *h1, 5), word(12, *a0, 5), word(12, *b0, 5)]
    px, off = pack([words])
    r = orc.reconstruct(px, off)
    ts = tracks_as_keysets(r, off).get(0, [])
    key = lambda l, rc: (l << 22) | (rc[0] << 11) | rc[1]  # noqa: E731
    assert ts == [(key(12, a0), key(11, h1), key(10, a2))]
    # without A's third hit, B is the only seed
    px, off = pack([[word(10, *b2, 5), word(11, *h1, 5), word(12, *a0, 5), word(12, *b0, 5)]])
    r = orc.reconstruct(px, off)
    assert tracks_as_keysets(r, off).get(0, []) == [(key(12, b0), key(11, h1), key(10, b2))]


def test_overflow_flag(orc):
    """A pathological dense patch produces more seed candidates than the limit:
    the event is flagged and gets no tracks; its neighbours are unaffected."""
    ws = []
    for l in (18, 19, 20):
        for r in range(0, 120, 2):
            for c in range(0, 120, 2):
                ws.append(word(l, 1000 + r, 1000 + c, 4))
    good = line_event([from_pv(0.02, 0.015)], layers=range(26))
    px, off = pack([good, ws, good])
    r = orc.reconstruct(px, off)
    st = r["tracks"]["status"]
    assert st[1] == orc.EV_OVERFLOW and r["tracks"]["n_tracks"][1] == 0
    assert st[0] == 0 and st[2] == 0
    assert r["tracks"]["n_tracks"][0] == 1 and r["tracks"]["n_tracks"][2] == 1


def test_nominal_physics_sanity(orc):
    b = generate("nominal", 50)
    r = orc.reconstruct(b.pixels, b.offsets)
    truth = Truth(b)
    ev, slot, nh, keys = track_list(r["tracks"], r["hits"], b.offsets)
    m = metrics(truth, ev, nh, keys, r["states"]["accepted"][slot])
    assert m["efficiency"] > 0.98
    assert m["ghost_rate"] < 0.01
