"""Pins of the oracle's decoding and clustering (Sec. 2.3.1, first paragraph).

Independent references: scipy.ndimage.label (8-connectivity) for the
components, a float64 charge-weighted mean of pixel centres for the
centroid, float64 radii for the hole, and exact closed forms for 1- and
2-pixel clusters.
"""
import numpy as np
import pytest
from scipy import ndimage

from synth import generate
from synth.raw import pack, shuffle_within_layers, word

PITCH = 0.055


def hits_of_event(h, offsets, e):
    b = int(offsets[e])
    out = []
    for l in range(26):
        a = b + int(h["layer_start"][e, l])
        n = int(h["layer_nhits"][e, l])
        out.append(dict(x=h["x"][a:a + n], y=h["y"][a:a + n], key=h["key"][a:a + n],
                        aux=h["aux"][a:a + n]))
    return out


def test_single_pixel_is_pixel_centre(orc):
    rng = np.random.default_rng(1)
    words, expect = [], []
    for l in range(26):
        # far-apart pixels, one per (layer, position)
        for k in range(6):
            r, c = int(rng.integers(0, 1536)), int(rng.integers(0, 1536))
            if (2 * c - 1535) ** 2 + (2 * r - 1535) ** 2 <= 34393:
                continue
            words.append(word(l, r, c, int(rng.integers(1, 16))))
    # keep pixels isolated: drop any that touch another on the same layer
    w = np.array(words, np.uint32)
    lay, row, col = (w >> 22) & 31, (w >> 11) & 0x7FF, w & 0x7FF
    keep = np.ones(len(w), bool)
    for i in range(len(w)):
        near = (lay == lay[i]) & (np.abs(row.astype(int) - int(row[i])) <= 1) & (np.abs(col.astype(int) - int(col[i])) <= 1)
        keep[i] = near.sum() == 1
    w = w[keep]
    px, off = pack([w])
    h = orc.cluster(px, off)
    assert h["status"][0] == 0 and h["n_hits"][0] == len(w)
    n = int(h["n_hits"][0])
    # every hit sits exactly on the centre of its pixel: x = (c - 767.5) * pitch in binary32
    key = h["key"][:n]
    ex = (np.float32(key & 0x7FF) - np.float32(767.5)) * np.float32(PITCH)
    ey = (np.float32((key >> 11) & 0x7FF) - np.float32(767.5)) * np.float32(PITCH)
    np.testing.assert_array_equal(h["x"][:n], ex)
    np.testing.assert_array_equal(h["y"][:n], ey)
    # charge and size round-trip through aux
    q_of = {int(a & 0x07FFFFFF): int(a >> 27) for a in w}
    for k, a in zip(key, h["aux"][:n]):
        assert int(a) >> 16 == 1 and int(a) & 0xFFFF == q_of[int(k)]


def test_two_pixel_equal_charge_is_midpoint(orc):
    ws = []
    cases = []
    for i, (dr, dc) in enumerate([(0, 1), (1, 0), (1, 1), (1, -1)]):
        r, c = 200 + 10 * i, 300 + 10 * i
        ws += [word(3, r, c, 7), word(3, r + dr, c + dc, 7)]
        cases.append((r, c, dr, dc))
    px, off = pack([ws])
    h = orc.cluster(px, off)
    hl = hits_of_event(h, off, 0)[3]
    assert len(hl["x"]) == 4
    for (r, c, dr, dc) in cases:
        k = (3 << 22) | (min(r, r + dr) << 11) | (c if dr == 0 or dc >= 0 else c)
        j = np.nonzero(hl["key"] == ((3 << 22) | (r << 11) | c))[0]
        assert len(j) == 1, (r, c)
        j = j[0]
        # (c + c + dc)/2 is exact in binary32
        assert hl["x"][j] == np.float32((np.float32(c + dc / 2) - np.float32(767.5)) * np.float32(PITCH))
        assert hl["y"][j] == np.float32((np.float32(r + dr / 2) - np.float32(767.5)) * np.float32(PITCH))
        assert int(hl["aux"][j]) == (2 << 16) | 14


def random_blob_event(rng, n_layers=4, size=24, density=0.35, origin=(400, 900)):
    """Dense random pixels in a small window on a few layers (many touching)."""
    words = []
    grids = {}
    for l in sorted(rng.choice(26, n_layers, replace=False)):
        g = rng.random((size, size)) < density
        grids[int(l)] = g
        rr, cc = np.nonzero(g)
        q = rng.integers(1, 16, len(rr))
        ws = [word(int(l), origin[0] + int(r), origin[1] + int(c), int(qq)) for r, c, qq in zip(rr, cc, q)]
        rng.shuffle(ws)
        words += ws
    return words, grids


@pytest.mark.parametrize("seed", range(12))
def test_components_match_scipy_label(orc, seed):
    rng = np.random.default_rng(100 + seed)
    words, grids = random_blob_event(rng, density=[0.15, 0.35, 0.55][seed % 3])
    px, off = pack([words])
    h = orc.cluster(px, off)
    assert h["status"][0] == 0
    hl = hits_of_event(h, off, 0)
    w = np.asarray(words, np.uint32)
    qmap = {int(a & 0x07FFFFFF): int(a >> 27) for a in w}
    for l, g in grids.items():
        lab, nlab = ndimage.label(g, structure=np.ones((3, 3), int))
        hh = hl[l]
        assert len(hh["key"]) == nlab
        exp = []
        for k in range(1, nlab + 1):
            rr, cc = np.nonzero(lab == k)
            rows = 400 + rr
            cols = 900 + cc
            addr = (rows << 11) | cols
            kmin = int(addr.min())
            q = np.array([qmap[(l << 22) | int(a)] for a in addr], float)
            xc = np.average((cols - 767.5) * PITCH, weights=q)
            yc = np.average((rows - 767.5) * PITCH, weights=q)
            exp.append(((l << 22) | kmin, xc, yc, len(rr), int(q.sum())))
        exp.sort()
        # hits come out in ascending key order
        assert np.all(np.diff(hh["key"].astype(np.int64)) > 0)
        for j, (k, xc, yc, n, Q) in enumerate(exp):
            assert int(hh["key"][j]) == k
            assert abs(float(hh["x"][j]) - xc) <= 2e-6 * max(1.0, abs(xc))
            assert abs(float(hh["y"][j]) - yc) <= 2e-6 * max(1.0, abs(yc))
            assert int(hh["aux"][j]) == (n << 16) | Q


def test_conservation_and_order_invariance(orc):
    b = generate("nominal", 40)
    h = orc.cluster(b.pixels, b.offsets)
    assert np.all(h["status"] == 0)
    for e in range(b.n_events):
        hl = hits_of_event(h, b.offsets, e)
        w = b.event_pixels(e)
        sizes = np.concatenate([x["aux"] >> 16 for x in hl])
        charges = np.concatenate([x["aux"] & 0xFFFF for x in hl])
        assert sizes.sum() == len(w)
        assert charges.sum() == ((w >> 27) & 15).sum()
        for l in range(26):
            assert int(h["layer_start"][e, l]) == int(np.count_nonzero(((w >> 22) & 31) < l))
    px2 = shuffle_within_layers(b.pixels, b.offsets, seed=7)
    assert not np.array_equal(px2, b.pixels)
    h2 = orc.cluster(px2, b.offsets)
    for k in ("x", "y", "key", "aux", "layer_start", "layer_nhits", "n_hits", "status"):
        np.testing.assert_array_equal(h[k], h2[k])


def test_hole_boundary_matches_float_radius(orc):
    # every pixel whose centre radius lies within 0.3 mm of 5.1 mm, one per event
    c = np.arange(1536)
    xc = (c - 767.5) * PITCH
    R = np.sqrt(xc[:, None] ** 2 + xc[None, :] ** 2)
    rr, cc = np.nonzero(np.abs(R - 5.1) < 0.3)
    events = [[word(5, int(r), int(col), 3)] for r, col in zip(rr, cc)]
    px, off = pack(events)
    h = orc.cluster(px, off)
    inside = R[rr, cc] < 5.1
    assert inside.any() and (~inside).any()
    np.testing.assert_array_equal(h["status"] == orc.EV_HOLE, inside)
    np.testing.assert_array_equal(h["status"] == 0, ~inside)
    np.testing.assert_array_equal(h["n_hits"], (~inside).astype(np.uint32))


def test_status_flags_and_empty_events(orc):
    good = [word(0, 10, 10, 3), word(1, 500, 500, 4), word(25, 1535, 1535, 15)]
    events = [
        [],                                              # empty event
        good,                                            # fine
        good + [word(2, 20, 20, 3)],                     # layer order (2 after 25)
        [word(0, 10, 10, 0)],                            # charge 0
        [word(0, 1536, 10, 3)],                          # row out of range
        [word(0, 10, 1600, 3)],                          # col out of range
        [word(26, 10, 10, 3)],                           # layer 26
        [word(0, 10, 10, 3) | (1 << 31)],                # bit 31
        [word(0, 768, 768, 3)],                          # beam hole
        [word(4, 100, 100, 3), word(4, 100, 100, 5)],    # duplicate address
        [word(4, 100, 100, 3), word(4, 100, 100, 5), word(0, 5, 5, 0)],  # dup + bad: bad only
        [word(4, 100, 100, 3), word(3, 100, 100, 5)],    # order
        good,                                            # fine again after bad neighbours
    ]
    px, off = pack(events)
    h = orc.cluster(px, off)
    exp = [0, 0, orc.EV_LAYER_ORDER, orc.EV_BAD_WORD, orc.EV_BAD_WORD, orc.EV_BAD_WORD,
           orc.EV_BAD_WORD, orc.EV_BAD_WORD, orc.EV_HOLE, orc.EV_DUPLICATE,
           orc.EV_BAD_WORD | orc.EV_LAYER_ORDER, orc.EV_LAYER_ORDER, 0]
    np.testing.assert_array_equal(h["status"], np.array(exp, np.uint32))
    for e, s in enumerate(exp):
        if s or e == 0:
            assert h["n_hits"][e] == 0
            assert not h["layer_start"][e].any() and not h["layer_nhits"][e].any()
    assert h["n_hits"][1] == 3 and h["n_hits"][12] == 3
    assert int(h["layer_start"][1, 26]) == 3


def test_large_component_without_size_cap(orc):
    # a full 60 x 60 block is one cluster of 3600 pixels
    ws = [word(7, 300 + r, 300 + c, 1 + (r + c) % 15) for r in range(60) for c in range(60)]
    px, off = pack([ws[::-1]])
    h = orc.cluster(px, off)
    assert h["n_hits"][0] == 1
    a = int(h["aux"][int(h["layer_start"][0, 7])])
    assert a >> 16 == 3600
    q = np.array([1 + (r + c) % 15 for r in range(60) for c in range(60)], float)
    cols = np.array([300 + c for r in range(60) for c in range(60)])
    xc = np.average((cols - 767.5) * PITCH, weights=q)
    assert abs(float(h["x"][0]) - xc) < 1e-5


@pytest.mark.parametrize("name", ["good", "descent", "overlap", "beyond", "empty"])
def test_bad_offsets(orc, name):
    """An event is usable only if offsets[e] <= offsets[e+1] <= n_pixels and no
    earlier offset exceeds offsets[e]; the others are flagged BAD_OFFSETS and
    have no hits, and every usable event's hits equal those of the same words
    clustered alone."""
    from synth.raw import bad_offsets_case
    b, cases = bad_offsets_case()
    offs, exp = cases[name]
    off = np.array(offs, np.uint64)
    h = orc.cluster(b.pixels, off)
    np.testing.assert_array_equal(h["status"], np.array(exp, np.uint32))
    for e, s in enumerate(exp):
        a, z = int(off[e]), int(off[e + 1])
        if s:
            assert h["n_hits"][e] == 0 and not h["layer_start"][e].any() and not h["layer_nhits"][e].any()
            continue
        alone = orc.cluster(b.pixels[a:z], np.array([0, z - a], np.uint64))
        assert h["n_hits"][e] == alone["n_hits"][0]
        np.testing.assert_array_equal(h["layer_nhits"][e], alone["layer_nhits"][0])
        for l in range(26):
            s0 = int(alone["layer_start"][0, l])
            m = int(alone["layer_nhits"][0, l])
            np.testing.assert_array_equal(h["key"][a + s0:a + s0 + m], alone["key"][s0:s0 + m])
            np.testing.assert_array_equal(h["x"][a + s0:a + s0 + m], alone["x"][s0:s0 + m])
    # the whole chain accepts the flagged events and gives them no tracks
    r = orc.reconstruct(b.pixels, off)
    for e, s in enumerate(exp):
        if s:
            assert r["tracks"]["n_tracks"][e] == 0
