"""Pins of the oracle's track fit (Sec. 2.3.1, third and fourth paragraphs).

Independent references: exact lines (the filter must reproduce them),
weighted linear least squares from numpy (a Kalman filter without process
noise, initialised from two points, is recursive least squares), and the
statistics of Gaussian-smeared tracks (pulls of unit width, chi2/ndof ~ 1).
"""
import numpy as np
import pytest

from synth.gen import layer_z_mm

SIG = 0.055 / 12 ** 0.5


def zs(layers):
    return np.array([np.float32(-280.0 + 1030.0 * l / 25.0) for l in layers], np.float32)


def pca_of_line(x0, y0, tx, ty):
    """Point of closest approach to the z axis of x = x0 + tx z, y = y0 + ty z."""
    zb = -(x0 * tx + y0 * ty) / (tx * tx + ty * ty)
    return x0 + tx * zb, y0 + ty * zb, zb


@pytest.mark.parametrize("seed", range(20))
def test_exact_line_refit(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 27))
    top = int(rng.integers(n - 1, 26))
    layers = np.arange(top, top - n, -1)
    z = zs(layers)
    zpv = rng.normal(0, 45)
    eta = rng.uniform(2, 5)
    phi = rng.uniform(0, 2 * np.pi)
    t = np.tan(2 * np.arctan(np.exp(-eta)))
    tx, ty = t * np.cos(phi), t * np.sin(phi)
    xpv, ypv = rng.normal(0, 0.01, 2)
    x0, y0 = xpv - tx * zpv, ypv - ty * zpv
    hx = (x0 + tx * z.astype(np.float64)).astype(np.float32)
    hy = (y0 + ty * z.astype(np.float64)).astype(np.float32)
    s = orc.fit_points(hx, hy, z, layers, params=dict(x_over_x0=5.94e-4))
    xb, yb, zb = pca_of_line(x0, y0, tx, ty)
    assert abs(s["x"] - xb) < 1e-5 + 1e-5 * abs(xb)
    assert abs(s["y"] - yb) < 1e-5 + 1e-5 * abs(yb)
    assert abs(s["tx"] - tx) < 1e-5 * max(1, abs(tx))
    assert abs(s["ty"] - ty) < 1e-5 * max(1, abs(ty))
    # z of closest approach: conditioning ~ 1/t^2, allow the float32 input rounding
    assert abs(s["z"] - zb) < 2e-3 * (1 + 1 / (tx * tx + ty * ty)) ** 0.5
    assert s["ndof"] == 2 * n - 4
    assert s["chi2"] < 1e-3 * s["ndof"] + 1e-3


@pytest.mark.parametrize("seed", range(20))
def test_no_scattering_equals_weighted_least_squares(orc, seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(3, 27))
    top = int(rng.integers(n - 1, 26))
    layers = np.arange(top, top - n, -1)
    # with gaps: drop some planes but keep the first two
    if n > 5 and seed % 2:
        keep = np.ones(n, bool)
        keep[rng.choice(np.arange(3, n), 2, replace=False)] = False
        layers = layers[keep]
        n = len(layers)
    z = zs(layers)
    tx, ty = rng.uniform(-0.3, 0.3, 2)
    x0, y0 = rng.normal(0, 3, 2)
    hx = (x0 + tx * z + rng.normal(0, SIG, n)).astype(np.float32)
    hy = (y0 + ty * z + rng.normal(0, SIG, n)).astype(np.float32)
    s = orc.fit_points(hx, hy, z, layers, params=dict(x_over_x0=0.0))
    z64 = z.astype(np.float64)
    A = np.stack([np.ones(n), z64], 1)
    chi = 0.0
    for proj, m, st, cov in (("x", hx, s["x"], s["cov_x"]), ("y", hy, s["y"], s["cov_y"])):
        coef, *_ = np.linalg.lstsq(A, m.astype(np.float64), rcond=None)
        Cab = np.linalg.inv(A.T @ A) * SIG ** 2
        zb = float(s["z"])
        J = np.array([[1.0, zb], [0.0, 1.0]])
        Cb = J @ Cab @ J.T
        u = coef[0] + coef[1] * zb
        slope = coef[1]
        assert abs(st - u) < 2e-4 * (1 + abs(u))
        assert abs(s["t" + proj] - slope) < 1e-5 * (1 + abs(slope)) + 3e-5 * np.sqrt(Cb[1, 1])
        np.testing.assert_allclose(cov, [Cb[0, 0], Cb[0, 1], Cb[1, 1]], rtol=2e-3, atol=1e-12)
        res = m.astype(np.float64) - A @ coef
        chi += float(res @ res) / SIG ** 2
    assert abs(s["chi2"] - chi) < 2e-3 * (1 + chi)


def test_pulls_and_chi2_with_scattering(orc):
    """Tracks with per-plane scattering kinks of the size the filter assumes and
    Gaussian hit smearing: pulls at the beamline have unit width, <chi2/ndof> ~ 1."""
    rng = np.random.default_rng(7)
    xl = 2.38e-3
    pulls_x, pulls_tx, chis = [], [], []
    z_all = layer_z_mm()
    for i in range(3000):
        eta = rng.uniform(2, 5)
        phi = rng.uniform(0, 2 * np.pi)
        t = np.tan(2 * np.arctan(np.exp(-eta)))
        tx, ty = t * np.cos(phi), t * np.sin(phi)
        t2 = tx * tx + ty * ty
        p = 400.0 * np.sqrt(1 + t2) / np.sqrt(t2)
        sig_ms = np.sqrt(184.96 * xl) / p
        zpv = rng.normal(0, 45)
        layers = np.array([l for l in range(26) if z_all[l] > zpv])[::-1]
        # propagate from the PV upstream to downstream, kink after each plane
        lay_up = layers[::-1]
        x, y = rng.normal(0, 0.01, 2)
        zc = zpv
        cx, cy, ctx, cty = x, y, tx, ty
        xs, ys = {}, {}
        for l in lay_up:
            dz = z_all[l] - zc
            cx += ctx * dz
            cy += cty * dz
            zc = z_all[l]
            xs[l], ys[l] = cx, cy
            ctx += rng.normal(0, sig_ms)
            cty += rng.normal(0, sig_ms)
        hx = np.array([xs[l] for l in layers]) + rng.normal(0, SIG, len(layers))
        hy = np.array([ys[l] for l in layers]) + rng.normal(0, SIG, len(layers))
        s = orc.fit_points(hx.astype(np.float32), hy.astype(np.float32), zs(layers), layers,
                           params=dict(x_over_x0=xl))
        # truth at the fitted z: straight line from the PV with the initial slope
        xt = x + tx * (s["z"] - zpv)
        pulls_x.append((s["x"] - xt) / np.sqrt(s["cov_x"][0]))
        pulls_tx.append((s["tx"] - tx) / np.sqrt(s["cov_x"][2]))
        chis.append(s["chi2"] / s["ndof"])
    px = np.std(pulls_x)
    ptx = np.std(pulls_tx)
    assert 0.85 < px < 1.15, px
    assert 0.85 < ptx < 1.15, ptx
    assert 0.85 < np.mean(chis) < 1.15, np.mean(chis)


def test_beamline_z_close_to_pv(orc):
    """Noise-free straight tracks from a PV at (0, 0, z_pv), pixelised by the
    generator: the fitted z of closest approach recovers z_pv within the
    resolution expected for the track angle."""
    from synth import generate
    b = generate("cpu10")
    r = orc.reconstruct(b.pixels, b.offsets)
    from synth.truth import Truth, match_tracks, track_list
    ev, slot, nh, keys = track_list(r["tracks"], r["hits"], b.offsets)
    m = match_tracks(Truth(b), ev, nh, keys)
    zpv = b.part["pv_z"][b.part_off[ev].astype(int) + m]
    dz = r["states"]["z"][slot] - zpv
    t = np.hypot(r["states"]["tx"][slot], r["states"]["ty"][slot])
    # hit resolution ~16 um at ~z distances of 100s of mm: sigma_z ~ sigma / t
    assert np.median(np.abs(dz * t)) < 0.02
