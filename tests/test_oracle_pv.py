"""Pins of the oracle's primary-vertex finding (Sec. 2.3.1, last paragraph:
PV candidates are clusters in a histogram of the tracks' beamline z, and
every track is given a weight for every candidate, so all candidates are
fitted in parallel; Sec. 3.1: a reconstructed PV matches a simulated one
within five times its z uncertainty).

Hand-built track states pin each rule: admission, the histogram counts and
the candidate rule (seeds at bin centres, read with no fit rounds), the
weighted fit against its closed form, the sharing of a track between two
candidates, and the limits.  Generated events pin the whole chain against
the generator's true vertices.
"""
import numpy as np
import pytest

from synth import generate
from synth.truth import pv_metrics, pv_truth_tracks

TX = 0.1  # every hand-built track has slope (0.1, 0): var_z = var_x / 0.01


def states_of(events, accepted=None, slopes=None):
    """events: list of lists of (z, var) per track -> (states, tracks, offsets)."""
    T = sum(len(e) for e in events)
    off = np.zeros(len(events) + 1, np.uint64)
    off[1:] = np.cumsum([3 * len(e) for e in events])
    cap = max(T, 1)
    st = dict(z=np.zeros(cap, np.float32), tx=np.zeros(cap, np.float32), ty=np.zeros(cap, np.float32),
              cov_x=np.zeros((cap, 3), np.float32), cov_y=np.zeros((cap, 3), np.float32),
              accepted=np.ones(cap, np.uint8))
    i = 0
    for e in events:
        for z, var in e:
            tx, ty = (TX, 0.0) if slopes is None else slopes[i]
            st["z"][i], st["tx"][i], st["ty"][i] = z, tx, ty
            st["cov_x"][i, 0] = var * TX * TX
            i += 1
    if accepted is not None:
        st["accepted"][:T] = accepted
    tracks = dict(n_tracks=np.array([len(e) for e in events], np.uint32))
    return st, tracks, off


def seen_var(var):
    """The beamline-z variance the admission rule computes in binary32."""
    f = np.float32
    cx = f(var * TX * TX)
    t = f(TX)
    return float((t * t * cx + f(0) * f(0) * f(0)) / ((t * t) * (t * t)))


def tukey(c, cut=9.0):
    return (1 - c / cut) ** 2 if c < cut else 0.0


def find(orc, events, **kw):
    acc = kw.pop("accepted", None)
    slopes = kw.pop("slopes", None)
    st, tr, off = states_of(events, acc, slopes)
    return orc.find_pvs(st, tr, off, orc.pv_params(**kw))


def test_single_vertex_closed_form(orc):
    """Tracks symmetric about z = 10 with equal variance: the fit stays at 10;
    var = 1 / sum(r_i / var_i) and the weight sum = sum(r_i) with the Tukey
    weights r of the final position."""
    d = [0.0, 0.05, -0.05, 0.1, -0.1, 0.2, -0.2]
    var = 0.04
    r = find(orc, [[(10.0 + x, var) for x in d]])
    assert r["n_pv"][0] == 1
    z = float(r["z"][0, 0])
    assert abs(z - 10.0) < 2e-6
    v = seen_var(var)
    w = [tukey((10.0 + x - z) ** 2 / v) for x in d]
    assert float(r["weight"][0, 0]) == pytest.approx(sum(w), rel=1e-5)
    assert float(r["var"][0, 0]) == pytest.approx(1.0 / sum(wi / v for wi in w), rel=1e-5)


def test_weighted_mean_with_unequal_variances(orc):
    """Tracks all at one z except a far one (beyond the Tukey cut of the
    converged vertex): the vertex is the inverse-variance mean of the rest."""
    trk = [(-20.0, 0.01), (-20.3, 0.04), (-19.9, 0.02), (-20.1, 0.09), (-20.05, 0.01), (-17.0, 0.01)]
    r = find(orc, [trk], n_iter=30)
    assert r["n_pv"][0] == 1
    near = trk[:5]
    vv = [seen_var(v) for _, v in near]
    z = float(r["z"][0, 0])
    # fixed point of the Tukey-weighted inverse-variance mean, in double
    zz = -20.0
    for _ in range(200):
        w = [tukey((zi - zz) ** 2 / v) / v for (zi, _), v in zip(near, vv)]
        zz = sum(wi * zi for wi, (zi, _) in zip(w, near)) / sum(w)
    assert abs(z - zz) < 1e-5


def test_track_shared_between_two_vertices(orc):
    """A track exactly half way between two vertices (mirror images about
    z = 0) has the same Tukey weight r for both and gives each r (r / 2r) =
    r / 2: each weight sum is its own five tracks (weight 1) plus r / 2."""
    A = [(-0.8, 0.0004)] * 5
    B = [(0.8, 0.0004)] * 5
    mid = [(0.0, 0.16)]
    r = find(orc, [A + mid + B])
    assert r["n_pv"][0] == 2
    za, zb = float(r["z"][0, 0]), float(r["z"][0, 1])
    assert za == pytest.approx(-zb, abs=1e-6) and za < 0
    rm = tukey(za * za / seen_var(0.16))
    assert 0.2 < rm < 0.5
    ra = tukey((-0.8 - za) ** 2 / seen_var(0.0004))
    for k in (0, 1):
        assert float(r["weight"][0, k]) == pytest.approx(5 * ra + rm / 2, rel=1e-5)


def bin_center(orc, b):
    P = orc.pv_params()
    return P.z0 + (b + 0.5) * P.bin_w


def at_bin(orc, b, n, var=0.01):
    P = orc.pv_params()
    return [(P.z0 + (b + 0.5) * P.bin_w, var)] * n


def test_seed_threshold_and_counts(orc):
    """A track adds 2 to its bin and 1 to each neighbour; a candidate needs a
    count of at least seed_min (8): four tracks in one bin seed, three there
    and one in the next bin (count 7) do not, unless seed_min is 7."""
    r = find(orc, [at_bin(orc, 600, 4)], n_iter=0, min_weight=0.0)
    assert r["n_pv"][0] == 1 and r["z"][0, 0] == np.float32(bin_center(orc, 600))
    ev = at_bin(orc, 600, 3) + at_bin(orc, 601, 1)
    assert find(orc, [ev], n_iter=0, min_weight=0.0)["n_pv"][0] == 0
    r = find(orc, [ev], n_iter=0, min_weight=0.0, seed_min=7)
    assert r["n_pv"][0] == 1 and r["z"][0, 0] == np.float32(bin_center(orc, 600))


def test_candidate_dominance_and_ties(orc):
    """Equal peaks two bins apart (within nms = 2): the earlier bin is the
    candidate (strictly above the bins before it, at least the bins after);
    three bins apart both are; a lower peak within nms bins of a higher one
    is none."""
    ev = at_bin(orc, 300, 4) + at_bin(orc, 302, 4)
    r = find(orc, [ev], n_iter=0, min_weight=0.0)
    assert r["n_pv"][0] == 1 and r["z"][0, 0] == np.float32(bin_center(orc, 300))
    ev = at_bin(orc, 300, 4) + at_bin(orc, 303, 4)
    r = find(orc, [ev], n_iter=0, min_weight=0.0)
    assert r["n_pv"][0] == 2
    assert list(r["z"][0, :2]) == [np.float32(bin_center(orc, 300)), np.float32(bin_center(orc, 303))]
    ev = at_bin(orc, 300, 5) + at_bin(orc, 302, 4)
    r = find(orc, [ev], n_iter=0, min_weight=0.0)
    assert r["n_pv"][0] == 1 and r["z"][0, 0] == np.float32(bin_center(orc, 300))
    # with nms = 1 the lower peak still sits next to its neighbour's count 9
    assert find(orc, [ev], n_iter=0, min_weight=0.0, nms=1)["n_pv"][0] == 1
    ev = at_bin(orc, 300, 5) + at_bin(orc, 303, 4)
    assert find(orc, [ev], n_iter=0, min_weight=0.0)["n_pv"][0] == 2


def test_admission(orc):
    """Rejected tracks, tracks along the beam, tracks with too large a z
    variance and tracks outside the histogram take no part: the result equals
    the one without them."""
    good = at_bin(orc, 500, 4)
    extra = at_bin(orc, 500, 4, var=0.02)
    base = find(orc, [good])
    assert base["n_pv"][0] == 1

    def same(r, ref):
        assert r["n_pv"][0] == ref["n_pv"][0]
        for k in ("z", "var", "weight"):
            assert r[k][0, 0] == ref[k][0, 0]

    same(find(orc, [good + extra], accepted=[1] * 4 + [0] * 4), base)
    same(find(orc, [good + [(z, 5.0) for z, _ in extra]]), base)
    # slope (5e-4, 5e-4): t^2 = 5e-7 < 1e-6, with a variance that would pass
    slopes = [(TX, 0.0)] * 4 + [(5e-4, 5e-4)] * 4
    same(find(orc, [good + [(z, 1e-9) for z, _ in extra]], slopes=slopes), base)
    # at the top of the histogram: z = 256 is outside [z0, z0 + 1024 * 0.5)
    top = at_bin(orc, 1023, 4)
    ref = find(orc, [top])
    assert ref["n_pv"][0] == 1
    same(find(orc, [top + [(256.0, 0.01)] * 3]), ref)
    assert find(orc, [top + [(255.999, 0.01)] * 3])["z"][0, 0] != ref["z"][0, 0]


def test_minimum_weight(orc):
    """A candidate whose weight sum stays below min_weight is no PV."""
    ev = at_bin(orc, 100, 4, var=0.01)
    assert find(orc, [ev], min_weight=4.0)["n_pv"][0] == 1
    assert find(orc, [ev], min_weight=np.nextafter(np.float32(4.0), np.float32(5.0)))["n_pv"][0] == 0


def test_limits(orc):
    """More than 64 candidates: the first 64 in z order are kept and the
    event is flagged; more than 2048 admitted tracks: no PVs and flagged."""
    ev = []
    for k in range(70):
        ev += at_bin(orc, 10 + 6 * k, 4)
    r = find(orc, [ev], n_iter=0, min_weight=0.0)
    assert r["status"][0] == orc.EV_PV_OVERFLOW and r["n_pv"][0] == 64
    assert r["z"][0, 63] == np.float32(bin_center(orc, 10 + 6 * 63))
    r = find(orc, [at_bin(orc, 500, 2049)])
    assert r["status"][0] == orc.EV_PV_OVERFLOW and r["n_pv"][0] == 0
    r = find(orc, [at_bin(orc, 500, 2048)])
    assert r["status"][0] == 0 and r["n_pv"][0] == 1


def test_order_of_events_and_empty_events(orc):
    a = at_bin(orc, 200, 6)
    b = at_bin(orc, 800, 5)
    r = find(orc, [a, [], b])
    assert list(r["n_pv"]) == [1, 0, 1]
    assert r["z"][2, 0] == find(orc, [b])["z"][0, 0]


def test_generated_events_against_true_vertices(orc):
    """Nominal events through the whole oracle chain: simulated PVs with at
    least 5 reconstructible particles are found within 5 sigma_z, few
    reconstructed PVs match nothing, and the pulls have about unit width."""
    b = generate("nominal", 150, first_event=1000, workers=8)
    r = orc.reconstruct(b.pixels, b.offsets, threads=8)
    pv = orc.find_pvs(r["states"], r["tracks"], b.offsets)
    m = pv_metrics(b, pv["n_pv"], pv["z"], pv["var"], pv_truth_tracks(b))
    assert m["n_true"] > 800
    assert m["efficiency"] > 0.9
    assert m["fake_rate"] < 0.02
    assert 0.8 < m["pull_std"] < 1.4 and abs(m["pull_mean"]) < 0.2
