"""Pins of the oracle's Velo-only filter with a measured momentum (Sec.
2.3.5: the Velo segment fitted with the momentum estimated from the full
track, for a better impact-parameter resolution; here the generator's true
momentum stands in for the downstream estimate).

The reading: the filter of the plain fit, with the slope variance per plane
crossed 13.6^2 X/X0 / p^2 from the track's own momentum, and the transport to
the beamline point taken through every plane in between, each adding that
noise.  Pins: it reduces to the plain fit when the momentum equals the plain
fit's constant-pT estimate, apart from the closed-form noise of the planes
crossed on the way to the beamline, and exactly when there is no material;
invalid momenta fall back to the plain fit; and on events whose scattering
follows each particle's momentum, the pulls of the beamline position and
slope against the true trajectory have unit width, while the constant-pT
model misjudges low-momentum tracks.
"""
import numpy as np
import pytest

from synth import generate
from synth.truth import Truth, match_tracks, track_list


def line_hits(rng, n=12, l0=24):
    layers = np.arange(l0, l0 - n, -1)
    z = np.array([-280.0 + 1030.0 * l / 25.0 for l in layers], np.float32)
    tx, ty = rng.uniform(-0.2, 0.2, 2)
    x0, y0 = rng.uniform(-0.05, 0.05, 2)
    hx = (x0 + tx * z + rng.normal(0, 0.012, n)).astype(np.float32)
    hy = (y0 + ty * z + rng.normal(0, 0.012, n)).astype(np.float32)
    return hx, hy, z, layers.astype(np.int32)


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("l0", [24, 14])
def test_reduces_to_the_constant_pt_fit(orc, seed, l0):
    """With p = pt0 sqrt(1 + t2) / sqrt(t2) (t2 from the first two hits) the
    momentum fit is the plain fit (up to the rounding of the noise term),
    except that its transport adds the slope noise of each plane between the
    last hit and the beamline point, with the closed form of a transport
    through k planes: C11 grows by k ms2, C01 and C00 by the terms of each
    plane's lever arm."""
    rng = np.random.default_rng(seed)
    hx, hy, hz, hl = line_hits(rng, l0=l0)
    d = float(hz[1] - hz[0])
    t2 = ((float(hx[1]) - float(hx[0])) / d) ** 2 + ((float(hy[1]) - float(hy[0])) / d) ** 2
    p = 400.0 * np.sqrt(1 + t2) / np.sqrt(t2)
    a = orc.fit_points(hx, hy, hz, hl)
    b = orc.fit_points_p(hx, hy, hz, hl, p)
    for k in ("z", "tx", "ty", "chi2"):
        assert abs(float(a[k]) - float(b[k])) <= 1e-5 * max(abs(float(a[k])), 1e-3), k
    for k in ("x", "y"):  # the transport in pieces rounds differently
        assert abs(float(a[k]) - float(b[k])) <= 2e-5, k
    ms2 = 184.96 * 5.94e-4 / p ** 2
    zb = float(a["z"])
    planes = [-280.0 + 1030.0 * l / 25.0 for l in range(int(hl[-1]))]
    lever = [zp - zb for zp in planes if zp > zb]  # planes between the beamline point and the last hit
    assert len(lever) == int(hl[-1]) - (0 if zb < -280 else sum(1 for zp in planes if zp <= zb))
    for c in ("cov_x", "cov_y"):
        ca, cb = np.asarray(a[c], np.float64), np.asarray(b[c], np.float64)
        assert cb[2] - ca[2] == pytest.approx(len(lever) * ms2, rel=2e-3, abs=1e-11)
        assert cb[1] - ca[1] == pytest.approx(-sum(lever) * ms2, rel=2e-3, abs=1e-9)
        assert cb[0] - ca[0] == pytest.approx(sum(x * x for x in lever) * ms2, rel=2e-3, abs=1e-7)


def test_no_material_is_the_plain_fit_and_invalid_momenta_fall_back(orc):
    """Without material the filter is the plain fit bit for bit and the
    beamline position differs only by the rounding of the transport in
    pieces; a momentum that is not a positive finite number gives the plain
    fit exactly."""
    rng = np.random.default_rng(7)
    for l0 in (24, 10):
        hx, hy, hz, hl = line_hits(rng, l0=l0)
        nm = dict(x_over_x0=0.0)
        a = orc.fit_points(hx, hy, hz, hl, params=nm)
        b = orc.fit_points_p(hx, hy, hz, hl, 2000.0, params=nm)
        for k in ("z", "tx", "ty"):
            assert np.float32(a[k]).view(np.uint32) == np.float32(b[k]).view(np.uint32), k
        assert a["chi2"] == b["chi2"]
        np.testing.assert_array_equal(a["cov_x"][2], b["cov_x"][2])
        for k in ("x", "y"):
            assert abs(float(a[k]) - float(b[k])) <= 2e-5
        for p in (0.0, -5.0, np.inf, np.nan):
            a = orc.fit_points(hx, hy, hz, hl)
            b = orc.fit_points_p(hx, hy, hz, hl, p)
            for k in ("x", "y", "z", "tx", "ty"):
                assert np.float32(a[k]).view(np.uint32) == np.float32(b[k]).view(np.uint32), (p, k)
            assert a["chi2"] == b["chi2"]
            np.testing.assert_array_equal(a["cov_x"], b["cov_x"])


def test_noise_falls_with_momentum(orc):
    """More momentum, less scattering: the slope variance of the beamline
    state decreases monotonically with p and tends to the no-material value."""
    rng = np.random.default_rng(8)
    hx, hy, hz, hl = line_hits(rng)
    v = [float(orc.fit_points_p(hx, hy, hz, hl, p)["cov_x"][2]) for p in (300.0, 1e3, 1e4, 1e5, 1e7)]
    assert all(a > b for a, b in zip(v, v[1:]))
    v0 = float(orc.fit_points(hx, hy, hz, hl, params=dict(x_over_x0=0.0))["cov_x"][2])
    assert abs(v[-1] - v0) <= 1e-4 * v0


def truth_of_tracks(b, r):
    """Particle of every found track (or -1) and its index in b.part."""
    T = Truth(b)
    ev, slot, nh, keys = track_list(r["tracks"], r["hits"], b.offsets)
    m = match_tracks(T, ev, nh, keys)
    first = b.part_off[:-1].astype(np.int64)
    gp = np.where(m >= 0, first[ev] + np.maximum(m, 0), -1)
    return slot, nh, gp


def pulls(b, states, slot, gp, sel):
    s = slot[sel]
    g = gp[sel]
    z = states["z"][s].astype(np.float64)
    xt = b.part["pv_x"][g] + b.part["tx"][g] * (z - b.part["pv_z"][g])
    yt = b.part["pv_y"][g] + b.part["ty"][g] * (z - b.part["pv_z"][g])
    px = (states["x"][s] - xt) / np.sqrt(states["cov_x"][s, 0])
    py = (states["y"][s] - yt) / np.sqrt(states["cov_y"][s, 0])
    ptx = (states["tx"][s] - b.part["tx"][g]) / np.sqrt(states["cov_x"][s, 2])
    return np.concatenate([px, py]), ptx, np.concatenate([states["x"][s] - xt, states["y"][s] - yt])


def test_pulls_with_the_true_momentum(orc):
    """Events whose scattering follows each particle's momentum: with the
    true momentum the beamline pulls have about unit width at low and high
    momentum; the constant-pT model's pulls are too wide at low momentum,
    and the true momentum gives the smaller position residuals there."""
    b = generate("momentum", 120, workers=8)
    r = orc.reconstruct(b.pixels, b.offsets, threads=8)
    slot, nh, gp = truth_of_tracks(b, r)
    cap = len(r["tracks"]["nhits"])
    pm = np.zeros(cap, np.float32)
    pm[slot[gp >= 0]] = b.part["p"][gp[gp >= 0]]
    rp = orc.fit_momentum(r["hits"], r["tracks"], b.offsets, pm)
    good = (gp >= 0) & (nh >= 8)
    p = np.where(gp >= 0, b.part["p"][np.maximum(gp, 0)], 0)
    low, high = good & (p < 3000), good & (p > 20000)
    assert low.sum() > 200 and high.sum() > 200
    for sel in (low, high):
        pull, pull_t, _ = pulls(b, rp, slot, gp, sel)
        assert 0.85 < np.std(pull) < 1.15
        assert 0.85 < np.std(pull_t) < 1.15
    pull_c, pull_tc, res_c = pulls(b, r["states"], slot, gp, low)
    _, _, res_p = pulls(b, rp, slot, gp, low)
    assert np.std(pull_c) > 1.5 and np.std(pull_tc) > 2.0
    assert np.sqrt(np.mean(res_p ** 2)) < 0.97 * np.sqrt(np.mean(res_c ** 2))
