"""Pins of the oracle's Velo-to-UT search windows (Sec. 2.3.2: UT hits decoded
into sorted regions for fast look-up; Velo tracks extrapolated to the UT with
the largest bending of a particle above 3 GeV).

The expected values come from the detector model itself, evaluated in
double precision away from rounding boundaries, and from numpy's sort:
  - the sorted hits and region starts equal numpy's sort of each event's
    words and a search of the region boundaries;
  - status rules at their limits (duplicates, bad fields, the hit limit,
    unusable offsets), flagged events next to good ones;
  - windows over dense strips (every strip of a region fired), so the first
    index and the count are fixed by the window's two edges: straight and
    stereo planes, the bending half width with and without its tolerance,
    sensor rows at their half-open limits;
  - generated events: a particle above 3 GeV has its UT hits inside the
    windows of its Velo track; a particle far below does not.
"""
import math

import numpy as np
import pytest

from synth import generate
from synth.gen import (UT_ANGLE_DEG, UT_KICK_MEV, UT_PITCH_MM, UT_SECTOR_MM, UT_U0_MM, UT_Y0_MM,
                       UT_Z_KICK_MM, UT_Z_MM)
from synth.truth import Truth, match_tracks, track_list

P_MIN, TOL_U, TOL_Y = 3000.0, 1.0, 10.0


def word(strip, sector, layer):
    return int(strip) | int(sector) << 13 | int(layer) << 17


def strip_u(n):
    return (n + 0.5) * UT_PITCH_MM + UT_U0_MM


def one_track(x, y, tx, ty, z=0.0, accepted=1):
    """States and track tables of one event with one track (slot 0)."""
    st = {k: np.array([v], np.float32) for k, v in dict(x=x, y=y, z=z, tx=tx, ty=ty).items()}
    st["accepted"] = np.array([accepted], np.uint8)
    return st, dict(n_tracks=np.array([1], np.uint32)), np.array([0, 3], np.uint64)


def dense(layer, sector, n0=0, n1=8192):
    """Every strip n0 <= n < n1 of one region fired."""
    return np.array([word(n, sector, layer) for n in range(n0, n1)], np.uint32)


def window_strips(up, w):
    """Strips whose centre lies within [up - w, up + w] (double)."""
    lo = math.ceil((up - w - UT_U0_MM) / UT_PITCH_MM - 0.5)
    hi = math.floor((up + w - UT_U0_MM) / UT_PITCH_MM - 0.5)
    # no edge within 1e-4 mm of a strip centre: the binary32 result is the same
    for e in (up - w, up + w):
        t = (e - UT_U0_MM) / UT_PITCH_MM - 0.5
        assert abs(t - round(t)) * UT_PITCH_MM > 1e-4
    return lo, hi


def half_width(k, tol=TOL_U):
    return UT_KICK_MEV / P_MIN * (UT_Z_MM[k] - UT_Z_KICK_MM) * math.cos(math.radians(UT_ANGLE_DEG[k])) + tol


def test_sorted_regions_equal_numpy(orc):
    b = generate("ut", 60, workers=8)
    r = orc.reconstruct(b.pixels, b.offsets, threads=8)
    o = orc.ut_windows(b.ut_words, b.ut_offsets, b.offsets, r["tracks"], r["states"])
    assert not o["status"].any()
    for e in range(b.n_events):
        u0, u1 = int(b.ut_offsets[e]), int(b.ut_offsets[e + 1])
        ref = np.sort(b.ut_words[u0:u1])
        np.testing.assert_array_equal(o["sorted"][u0:u1], ref)
        reg = (ref >> 17) * 14 + ((ref >> 13) & 15)
        np.testing.assert_array_equal(o["region"][e], np.searchsorted(reg, np.arange(57), side="left"))


def test_status_rules(orc):
    good = [word(5, 3, 0), word(7, 3, 0), word(9, 0, 3)]
    evs = [good,
           good + [word(7, 3, 0)],                      # the same strip twice
           good + [word(1, 14, 2)],                     # sensor row 14 does not exist
           good + [word(1, 2, 2) | 1 << 19],            # a high bit
           good + [word(1, 14, 2), word(5, 3, 0)],      # bad field and duplicate: only BAD_WORD
           [word(n % 8192, n // 8192, 1) for n in range(8192)],      # at the limit
           [word(n % 8192, n // 8192, 1) for n in range(8193)],      # one above
           good]
    words = np.concatenate([np.array(e, np.uint32) for e in evs])
    uo = np.concatenate([[0], np.cumsum([len(e) for e in evs])]).astype(np.uint64)
    E = len(evs)
    st, tr, _ = one_track(0.0, 0.0, 0.01, 0.01)
    off = np.arange(E + 1, dtype=np.uint64) * 3
    tracks = dict(n_tracks=np.ones(E, np.uint32))
    states = {k: np.repeat(v, E) for k, v in st.items()}
    o = orc.ut_windows(words, uo, off, tracks, states)
    assert list(o["status"]) == [0, orc.EV_DUPLICATE, orc.EV_BAD_WORD, orc.EV_BAD_WORD, orc.EV_BAD_WORD, 0,
                                 orc.EV_UT_OVERFLOW, 0]
    for e in (1, 2, 3, 4, 6):
        assert not o["region"][e].any() and not o["win"][e].any()
    assert o["region"][5][56] == 8192 and o["region"][7][56] == 3
    # unusable offsets: decreasing, beyond the buffer, below an earlier offset
    uo2 = np.array([0, 3, 2, 6, 9, 12, 100], np.uint64)
    w2 = np.array([word(n, 5, 1) for n in range(12)], np.uint32)
    o2 = orc.ut_windows(w2, uo2, np.arange(7, dtype=np.uint64) * 3, dict(n_tracks=np.zeros(6, np.uint32)),
                        {k: np.repeat(v, 6) for k, v in st.items()})
    bad = orc.EV_BAD_OFFSETS
    assert list(o2["status"]) == [0, bad, bad, 0, 0, bad]
    np.testing.assert_array_equal(o2["sorted"][6:12], w2[6:12])


@pytest.mark.parametrize("k", range(4))
@pytest.mark.parametrize("tx,ty", [(0.013, 0.0412), (-0.05, -0.1013), (0.0021, 0.1605)])
def test_dense_window_edges(orc, k, tx, ty):
    """Track from (x, y) = (0.3, -0.2) mm at z = -11 mm: the window on plane k
    covers exactly the strips whose centre lies within the half width of the
    extrapolated u (straight line; u = x cos a + y sin a)."""
    x0, z0 = 0.3, -11.0
    zk = UT_Z_MM[k]
    sec = int((ty * (zk - z0) - UT_Y0_MM) // UT_SECTOR_MM)
    y0 = UT_Y0_MM + (sec + 0.5) * UT_SECTOR_MM + 13.7 - ty * (zk - z0)  # 13.7 mm from the row's middle
    y0 = float(np.float32(y0))
    xp, yp = x0 + tx * (zk - z0), y0 + ty * (zk - z0)
    a = math.radians(UT_ANGLE_DEG[k])
    up = xp * math.cos(a) + yp * math.sin(a)
    assert yp - TOL_Y > UT_Y0_MM + sec * UT_SECTOR_MM and yp + TOL_Y < UT_Y0_MM + (sec + 1) * UT_SECTOR_MM
    lo, hi = window_strips(up, half_width(k))
    words = dense(k, sec)
    st, tr, off = one_track(x0, y0, tx, ty, z0)
    o = orc.ut_windows(words, np.array([0, len(words)], np.uint64), off, tr, st)
    w = o["win"][0]
    assert w[2 * k] == lo | (hi - lo + 1) << 16
    assert not np.delete(w, 2 * k).any()
    # without the tolerance the window narrows accordingly
    lo0, hi0 = window_strips(up, half_width(k, tol=0.0))
    o0 = orc.ut_windows(words, np.array([0, len(words)], np.uint64), off, tr, st, orc.ut_params(tol_u=0.0))
    assert o0["win"][0][2 * k] == lo0 | (hi0 - lo0 + 1) << 16
    assert 5 <= hi - hi0 <= 6 and 5 <= lo0 - lo <= 6   # 1 mm = 5.3 strips on each side
    # a track that is not accepted gets no window
    st["accepted"][0] = 0
    assert not orc.ut_windows(words, np.array([0, len(words)], np.uint64), off, tr, st)["win"].any()


def test_sensor_rows_half_open(orc):
    """y_p + tol_y reaching a row's lower edge includes the row; y_p - tol_y
    reaching a row's upper edge excludes it (rows are [lo, hi))."""
    words = np.concatenate([dense(0, 3, 3800, 4400), dense(0, 4, 3800, 4400)])
    words.sort()
    uo = np.array([0, len(words)], np.uint64)
    for y, rows in ((-310.0, (3, 4)), (-290.0, (4,)), (-310.01, (3,)), (-350.0, (3,))):
        st, tr, off = one_track(10.0, y, 0.0, 0.0)
        o = orc.ut_windows(words, uo, off, tr, st)
        w = o["win"][0]
        lo, hi = window_strips(10.0, half_width(0))
        got = [(int(v) & 0xFFFF, int(v) >> 16) for v in w[:2] if v]
        want = [(lo - 3800 + 600 * (r - 3), hi - lo + 1) for r in rows]
        assert got == want, (y, got, want)
        assert not w[2:].any()
    # outside the sensor rows: nothing
    st, tr, off = one_track(10.0, -715.0, 0.0, 0.0)
    assert not orc.ut_windows(words, uo, off, tr, st)["win"].any()


def test_stereo_planes_use_y(orc):
    """At y = 450 mm the tilted strips sit 39 mm away from the vertical ones:
    the track's own strip is the centre of its window on the u and v planes."""
    for k in (1, 2):
        a = math.radians(UT_ANGLE_DEG[k])
        zk = UT_Z_MM[k]
        tx, ty = 0.004, 450.0 / zk
        xp, yp = tx * zk, ty * zk
        n = int(math.floor((xp * math.cos(a) + yp * math.sin(a) - UT_U0_MM) / UT_PITCH_MM))
        sec = int((yp - UT_Y0_MM) // UT_SECTOR_MM)
        words = np.array([word(n, sec, k)], np.uint32)
        st, tr, off = one_track(0.0, 0.0, tx, ty)
        o = orc.ut_windows(words, np.array([0, 1], np.uint64), off, tr, st)
        assert o["win"][0][2 * k] == 0 | 1 << 16, k
        # the strip of the other tilt is far outside
        m = int(math.floor((xp * math.cos(a) - yp * math.sin(a) - UT_U0_MM) / UT_PITCH_MM))
        assert abs(strip_u(m) - strip_u(n)) > 60
        o = orc.ut_windows(np.array([word(m, sec, k)], np.uint32), np.array([0, 1], np.uint64), off, tr, st)
        assert not o["win"].any()


def test_counts_are_clamped(orc):
    """A track count above a third of the event's words touches no slot of
    the next event."""
    st, _, _ = one_track(0.0, 0.0, 0.01, 0.01)
    states = {k: np.repeat(v, 4) for k, v in st.items()}
    win_before = np.full((4, 8), 7, np.uint32)
    o = orc.ut_windows(np.zeros(0, np.uint32), np.zeros(3, np.uint64), np.array([0, 6, 12], np.uint64),
                       dict(n_tracks=np.array([9, 0], np.uint32)), states)
    assert not o["win"][:2].any()
    del win_before


def test_generated_particles_inside_their_windows(orc):
    """Velo tracks matched to particles: above 3.3 GeV (margin for the Velo
    extrapolation) every UT hit of the particle lies inside the track's
    window on its plane; below 1.4 GeV (bending more than twice the largest
    allowed) none does."""
    b = generate("ut", 150, workers=8)
    r = orc.reconstruct(b.pixels, b.offsets, threads=8)
    o = orc.ut_windows(b.ut_words, b.ut_offsets, b.offsets, r["tracks"], r["states"])
    T = Truth(b)
    ev, slot, nh, keys = track_list(r["tracks"], r["hits"], b.offsets)
    m = match_tracks(T, ev, nh, keys)
    first = b.part_off[:-1].astype(np.int64)
    inside = {True: [0, 0], False: [0, 0]}
    for e, s, pid in zip(ev, slot, m):
        if pid < 0 or not r["states"]["accepted"][s]:
            continue
        p = b.part["p"][first[e] + pid]
        if 1400.0 <= p <= 3300.0:
            continue
        u0, u1 = int(b.ut_offsets[e]), int(b.ut_offsets[e + 1])
        srt = o["sorted"][u0:u1]
        own = set(b.ut_words[u0:u1][b.ut_pid[u0:u1] == pid].tolist())
        for wd in own:
            k = wd >> 17
            idx = int(np.searchsorted(srt, wd))
            hit = any((v & 0xFFFF) <= idx < (v & 0xFFFF) + (v >> 16) for v in o["win"][s][2 * k:2 * k + 2])
            inside[p > 3300.0][0] += hit
            inside[p > 3300.0][1] += 1
    hi_in, hi_n = inside[True]
    lo_in, lo_n = inside[False]
    assert hi_n > 2000 and lo_n > 500
    assert hi_in == hi_n, (hi_in, hi_n)
    assert lo_in <= 0.01 * lo_n, (lo_in, lo_n)


def test_window_edges_are_inclusive(orc):
    """A strip centre exactly on either edge of the window belongs to it.  On
    the first plane a track with zero slope has up = x exactly, so x is
    chosen (in binary32) with x - w or x + w equal to a strip centre."""
    f = np.float32
    w = f(f(f(45.0) / f(3000.0)) * f(f(2327.5) - f(1000.0))) * f(1.0) + f(1.0)
    cases = 0
    for n in range(3000, 5000):
        u = f(strip_u(n))
        for side in (-1, 1):
            x = f(u - w) if side > 0 else f(u + w)
            edge = f(x + w) if side > 0 else f(x - w)
            if edge != u:
                continue
            words = dense(0, 7, n - 300, n + 300)
            st, tr, off = one_track(float(x), 50.0, 0.0, 0.0)
            v = int(orc.ut_windows(words, np.array([0, len(words)], np.uint64), off, tr, st)["win"][0][0])
            first, count = v & 0xFFFF, v >> 16
            if side < 0:
                assert first == 300, (n, first)
            else:
                assert first + count - 1 == 300, (n, first, count)
            cases += 1
        if cases >= 20:
            break
    assert cases >= 20
