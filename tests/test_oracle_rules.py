"""Pins of the oracle's seeding and forwarding rules, decision by decision
(search by triplet, Sec. 2.3.1, second paragraph; the cut forms and the
conflict order are this project's reading of it).

Every event here is placed hit by hit (coordinates and keys chosen by hand)
and fed to track finding directly, so each test isolates one rule:

* the slope cut of a seed doublet, |tx| and |ty| against max_t, decided at
  the last representable binary32 value on each side of the limit;
* the same-azimuth cone cr^2 <= (sin2_phi r0) r1 at its binary32 boundary,
  and the same-side condition x0 x1 + y0 y1 > 0 (opposite sides of the beam,
  and exactly zero);
* the third-hit and forwarding windows s <= s_seed, s <= s_fwd at their
  binary32 boundaries, with the forward prediction from the last two hits;
* the order of exactly equal priorities: seeds by key of h1, then h0, then
  h2; extensions by key of the track's first hit, then of the hit.

Exact ties come from a symmetry rather than from tuning numbers: swapping
x and y maps every expression of the rules onto itself with its operands
commuted (IEEE addition and multiplication are commutative), so a seed or a
track and its mirror image in the diagonal x = y have bit-identical s.

The boundary values are computed here in binary32 from the rule as written;
the tests fail when the oracle's comparison, operand or order differs (each
was checked against one-line mutations of the oracle).
"""
import numpy as np
import pytest

from synth.raw import hit_event

F = np.float32
SQ2 = F(np.sqrt(2.0))


def z(orc, l):
    return F(orc.layer_z(l))


def prev(v):
    return np.nextafter(F(v), F(0))


def run(orc, planes, **params):
    hits, off = hit_event(planes)
    t = orc.find_tracks(hits, off, params=params or None)
    n = int(t["n_tracks"][0])
    out = []
    for i in range(n):
        m = int(t["nhits"][i])
        out.append(tuple(int(hits["key"][j]) for j in t["hit_idx"][i, :m]))
    return out, int(t["status"][0])


def key(l, i):
    return (l << 22) | i


# ---------------------------------------------------------------------------
# seed doublet: slope cut


def radial_triplet(orc, R1, phi, t, l=10, d2=(0.0, 0.0)):
    """h0 on l+2, h1 on l+1 at radius R1 and azimuth phi, h2 on l, on a line of
    slope t in the radial direction (h2 displaced by d2 mm)."""
    c, s = np.cos(phi), np.sin(phi)
    z0, z1, z2 = (float(z(orc, l + 2)), float(z(orc, l + 1)), float(z(orc, l)))
    x1, y1 = R1 * c, R1 * s
    h0 = (x1 + t * c * (z0 - z1), y1 + t * s * (z0 - z1))
    h2 = (x1 + t * c * (z2 - z1) + d2[0], y1 + t * s * (z2 - z1) + d2[1])
    return {l + 2: [(*h0, 0)], l + 1: [(x1, y1, 0)], l: [(*h2, 0)]}


def doublet_slopes(orc, planes, l=10):
    (x0, y0, _), = planes[l + 2]
    (x1, y1, _), = planes[l + 1]
    dz = z(orc, l + 1) - z(orc, l + 2)
    return (F(x1) - F(x0)) / dz, (F(y1) - F(y0)) / dz


@pytest.mark.parametrize("phi", [0.1, 1.45, np.pi + 0.2, -1.3])
def test_slope_cut_boundary(orc, phi):
    """|tx| and |ty| <= max_t: the seed is found with max_t equal to the larger
    slope magnitude (binary32) and lost one representable value below it,
    whichever of tx, ty is the larger and whatever its sign."""
    planes = radial_triplet(orc, 15.0, phi, 0.1)
    tx, ty = doublet_slopes(orc, planes)
    lim = max(abs(tx), abs(ty))
    assert lim > 0.05
    found, _ = run(orc, planes, max_t=float(lim))
    assert len(found) == 1 and len(found[0]) == 3
    found, _ = run(orc, planes, max_t=float(prev(lim)))
    assert found == []


# ---------------------------------------------------------------------------
# seed doublet: azimuth cone and same side of the beam


def cone_terms(planes, l=10):
    (x0, y0, _), = planes[l + 2]
    (x1, y1, _), = planes[l + 1]
    x0, y0, x1, y1 = F(x0), F(y0), F(x1), F(y1)
    cr = x0 * y1 - y0 * x1
    r0 = x0 * x0 + y0 * y0
    r1 = x1 * x1 + y1 * y1
    return cr * cr, r0, r1


def smallest_passing_sin2(cc, r0, r1):
    """Smallest binary32 s with (s * r0) * r1 >= cc, evaluated in binary32."""
    s = F(float(cc) / (float(r0) * float(r1)))
    while (s * r0) * r1 < cc:
        s = np.nextafter(s, F(np.inf))
    while (np.nextafter(s, F(0)) * r0) * r1 >= cc:
        s = np.nextafter(s, F(0))
    return s


@pytest.mark.parametrize("seed", range(8))
def test_azimuth_cone_boundary(orc, seed):
    """cr^2 <= (sin2_phi r0) r1 with cr = x0 y1 - y0 x1, r = x^2 + y^2: a doublet
    whose azimuths differ is found exactly from the smallest sin2_phi that
    admits it, not one representable value below."""
    rng = np.random.default_rng(100 + seed)
    R1 = rng.uniform(8, 30)
    phi = rng.uniform(-np.pi, np.pi)
    dphi = rng.uniform(0.004, 0.02) * rng.choice([-1, 1])
    planes = radial_triplet(orc, R1, phi, 0.08)
    # turn h0 about the beam axis by dphi, and put h2 back on the doublet's line
    (x0, y0, _), = planes[12]
    c, s = np.cos(dphi), np.sin(dphi)
    planes[12] = [(x0 * c - y0 * s, x0 * s + y0 * c, 0)]
    (x1, y1, _), = planes[11]
    x0n, y0n = planes[12][0][:2]
    k = (float(z(orc, 10)) - float(z(orc, 11))) / (float(z(orc, 11)) - float(z(orc, 12)))
    planes[10] = [(x1 + (x1 - x0n) * k, y1 + (y1 - y0n) * k, 0)]
    cc, r0, r1 = cone_terms(planes)
    lim = smallest_passing_sin2(cc, r0, r1)
    found, _ = run(orc, planes, sin2_phi=float(lim))
    assert len(found) == 1
    found, _ = run(orc, planes, sin2_phi=float(prev(lim)))
    assert found == []


def test_doublet_across_the_beam_is_rejected(orc):
    """Two hits on opposite sides of the beam (x0 x1 + y0 y1 < 0) are within the
    azimuth cone of a straight line through the beam axis, since the cone is
    tested on sin^2; the same-side condition rejects them, and no track is
    seeded even with a third hit exactly on their line."""
    planes = {12: [(6.0, 0.03, 0)], 11: [(-6.0, 0.03, 0)]}
    k = (float(z(orc, 10)) - float(z(orc, 11))) / (float(z(orc, 11)) - float(z(orc, 12)))
    planes[10] = [(-6.0 + (-12.0) * k, 0.03, 0)]
    cc, r0, r1 = cone_terms(planes)
    assert cc <= (F(9e-4) * r0) * r1
    assert run(orc, planes)[0] == []


def test_same_side_condition_is_strict(orc):
    """x0 x1 + y0 y1 = 0 exactly (perpendicular radius vectors (8, 6) and
    (-6, 8); with sin2_phi = 1 the cone admits them with equality): rejected,
    since the condition is '> 0'.  The same doublet turned so that the dot
    product is positive is accepted."""
    k = (float(z(orc, 10)) - float(z(orc, 11))) / (float(z(orc, 11)) - float(z(orc, 12)))

    def planes_for(h0, h1):
        return {12: [(*h0, 0)], 11: [(*h1, 0)],
                10: [(h1[0] + (h1[0] - h0[0]) * k, h1[1] + (h1[1] - h0[1]) * k, 0)]}

    planes = planes_for((8.0, 6.0), (-6.0, 8.0))
    x0, y0, x1, y1 = F(8), F(6), F(-6), F(8)
    assert x0 * x1 + y0 * y1 == 0
    assert run(orc, planes, sin2_phi=1.0)[0] == []
    planes = planes_for((8.0, 6.0), (-5.5, 8.25))
    assert len(run(orc, planes, sin2_phi=1.0)[0]) == 1


# ---------------------------------------------------------------------------
# third hit and forwarding windows


def seed_s(orc, planes, l=10):
    (x0, y0, _), = planes[l + 2]
    (x1, y1, _), = planes[l + 1]
    (x2, y2, _), = planes[l]
    x0, y0, x1, y1, x2, y2 = map(F, (x0, y0, x1, y1, x2, y2))
    z0, z1, z2 = z(orc, l + 2), z(orc, l + 1), z(orc, l)
    dz = z1 - z0
    tx = (x1 - x0) / dz
    ty = (y1 - y0) / dz
    d = z2 - z1
    xp = x1 + tx * d
    yp = y1 + ty * d
    dx, dy = x2 - xp, y2 - yp
    return dx * dx + dy * dy


@pytest.mark.parametrize("d2", [(0.1, 0.05), (-0.03, 0.12), (0.0, -0.15)])
def test_third_hit_window_boundary(orc, d2):
    """s <= s_seed, s the squared distance of h2 to the doublet's line at h2's
    plane: found with s_seed = s, lost one representable value below."""
    planes = radial_triplet(orc, 12.0, 0.7, 0.06, d2=d2)
    s = seed_s(orc, planes)
    assert 0.001 < s < 0.025
    assert len(run(orc, planes, s_seed=float(s))[0]) == 1
    assert run(orc, planes, s_seed=float(prev(s)))[0] == []


def fwd_s(orc, a, b, h, la, lb, lh):
    """s of hit h for the line through the last hit a and the one before, b."""
    xa, ya, xb, yb, xh, yh = map(F, (*a, *b, *h))
    za, zb, zl = z(orc, la), z(orc, lb), z(orc, lh)
    dza = za - zb
    tx = (xa - xb) / dza
    ty = (ya - yb) / dza
    d = zl - za
    xp = xa + tx * d
    yp = ya + ty * d
    dx, dy = xh - xp, yh - yp
    return dx * dx + dy * dy


@pytest.mark.parametrize("kink", [0.0, 0.002])
def test_forwarding_window_boundary(orc, kink):
    """A seed on planes 25, 24, 23 and one hit on 22: s <= s_fwd, with the
    prediction along the line through the track's last two hits (a kink
    between the first and the second pair makes the first pair's line
    predict elsewhere): 4 hits with s_fwd = s, 3 hits one value below."""
    zz = [float(z(orc, l)) for l in range(26)]
    t = np.array([0.04, 0.025])
    p25 = np.array([0.04, 0.025]) * 500.0
    p24 = p25 + t * (zz[24] - zz[25])
    t2 = t + kink
    p23 = p24 + t2 * (zz[23] - zz[24])
    p22 = p23 + t2 * (zz[22] - zz[23]) + np.array([0.09, -0.07])
    planes = {25: [(*p25, 0)], 24: [(*p24, 0)], 23: [(*p23, 0)], 22: [(*p22, 0)]}
    s = fwd_s(orc, planes[23][0][:2], planes[24][0][:2], planes[22][0][:2], 23, 24, 22)
    assert 0.005 < s < 0.04
    found, _ = run(orc, planes, s_fwd=float(s))
    assert [len(f) for f in found] == [4]
    found, _ = run(orc, planes, s_fwd=float(prev(s)))
    assert [len(f) for f in found] == [3]


# ---------------------------------------------------------------------------
# exact ties


def diag(R, o):
    """Point at distance R along the diagonal x = y and o across it; the
    mirror image in the diagonal is diag(R, -o), and diag(R, 0) has x == y."""
    if o == 0:
        v = F(R) / SQ2
        return (v, v)
    return (F((R - o) / np.sqrt(2.0)), F((R + o) / np.sqrt(2.0)))


def mirror(p):
    return (p[1], p[0])


def radius(orc, l, t=0.05, zpv=-400.0):
    return t * (float(z(orc, l)) - zpv)


def test_seed_tie_h1_key_before_h0_key(orc):
    """Seeds A = (h0, h1, h2) and its mirror B = (h0', h1', h2) share h2 on the
    diagonal and have equal s.  A's h1 has the smaller key, B's h0 has the
    smaller key: A wins, B's hits stay unused."""
    d = 0.1
    h2 = diag(radius(orc, 10), 0)
    h1 = diag(radius(orc, 11), d)
    h0 = diag(radius(orc, 12), 2 * d)
    planes = {12: [(*h0, 1), (*mirror(h0), 0)], 11: [(*h1, 0), (*mirror(h1), 1)], 10: [(*h2, 0)]}
    assert seed_s(orc, {12: [(*h0, 0)], 11: [(*h1, 0)], 10: [(*h2, 0)]}) == \
        seed_s(orc, {12: [(*mirror(h0), 0)], 11: [(*mirror(h1), 0)], 10: [(*h2, 0)]})
    found, _ = run(orc, planes)
    assert found == [(key(12, 1), key(11, 0), key(10, 0))]


def test_seed_tie_h0_key_before_h2_key(orc):
    """A = (h0, h1, h2) and its mirror B = (h0', h1, h2') share h1 on the
    diagonal (the line crosses it).  A's h0 has the smaller key, B's h2 has
    the smaller key: A wins."""
    d = 0.1
    h1 = diag(radius(orc, 11), 0)
    h0 = diag(radius(orc, 12), d)
    h2 = diag(radius(orc, 10), -d)
    planes = {12: [(*h0, 0), (*mirror(h0), 1)], 11: [(*h1, 0)], 10: [(*h2, 1), (*mirror(h2), 0)]}
    found, _ = run(orc, planes)
    assert found == [(key(12, 0), key(11, 0), key(10, 1))]


@pytest.mark.parametrize("a_first", [True, False])
def test_seed_tie_h2_key(orc, a_first):
    """A = (h0, h1, h2) and B = (h0, h1, h2') share h0 and h1 on the diagonal;
    h2, h2' are mirror images: the smaller key of the third hit wins."""
    h0 = diag(radius(orc, 12), 0)
    h1 = diag(radius(orc, 11), 0)
    h2 = diag(radius(orc, 10), 0.05)
    ia, ib = (0, 1) if a_first else (1, 0)
    planes = {12: [(*h0, 0)], 11: [(*h1, 0)], 10: [(*h2, ia), (*mirror(h2), ib)]}
    found, _ = run(orc, planes)
    assert found == [(key(12, 0), key(11, 0), key(10, 0))]
    # and the winner is the hit given key 0
    winner = h2 if a_first else mirror(h2)
    hits, _ = hit_event(planes)
    j = int(np.nonzero(hits["key"] == key(10, 0))[0][0])
    assert (hits["x"][j], hits["y"][j]) == winner


@pytest.mark.parametrize("t1_first", [True, False])
def test_extension_tie_first_hit_key(orc, t1_first):
    """Tracks T1 (planes 25, 24, 23 approaching the diagonal) and its mirror T2
    compete for one hit on the diagonal at plane 22 with equal s: the track
    whose first hit has the smaller key takes it."""
    d = 0.1
    R = {l: radius(orc, l, t=0.03, zpv=0.0) for l in (25, 24, 23, 22)}
    t1 = {25: diag(R[25], 3 * d), 24: diag(R[24], 2 * d), 23: diag(R[23], d)}
    i1, i2 = (0, 1) if t1_first else (1, 0)
    planes = {l: [(*p, i1), (*mirror(p), i2)] for l, p in t1.items()}
    planes[22] = [(*diag(R[22], 0), 0)]
    found, _ = run(orc, planes)
    assert sorted(len(f) for f in found) == [3, 4]
    long = [f for f in found if len(f) == 4][0]
    assert long == (key(25, 0), key(24, 0), key(23, 0), key(22, 0))
    # canonical order: decreasing key of the first hit
    assert [f[0] for f in found] == [key(25, 1), key(25, 0)]


@pytest.mark.parametrize("a_first", [True, False])
def test_extension_tie_hit_key(orc, a_first):
    """A track on the diagonal meets two mirror-image hits on plane 22 at equal
    s: it takes the one with the smaller key."""
    R = {l: radius(orc, l, t=0.03, zpv=0.0) for l in (25, 24, 23, 22)}
    planes = {l: [(*diag(R[l], 0), 0)] for l in (25, 24, 23)}
    h = diag(R[22], 0.05)
    ia, ib = (0, 1) if a_first else (1, 0)
    planes[22] = [(*h, ia), (*mirror(h), ib)]
    found, _ = run(orc, planes)
    assert found == [(key(25, 0), key(24, 0), key(23, 0), key(22, 0))]
