"""Seeded generator of VELO-like collision events (input infrastructure).

Detector model: 26 planar pixel layers perpendicular to the beam (z) axis,
evenly spaced from z = -280 mm to z = +750 mm (the paper's Velo has 26
planes, Sec. 2.3.1), 1536 x 1536 pixels of 55 um pitch centred on the beam,
with the pixels whose centre lies within r < 5.1 mm left inactive (the
beam-pipe hole).

Physics model per event: primary vertices (PVs) with z ~ N(0, 45 mm) and
x, y ~ N(0, 0.01 mm); charged particles per PV with pseudorapidity uniform in
[2, 5] and azimuth uniform in [0, 2 pi), travelling in +z as straight lines
with a Gaussian multiple-scattering kink added to both slopes at every plane
they cross; an independent hit efficiency per crossing; a 1-3 pixel cluster
around the crossing point with integer charges 1..15; uniform noise pixels;
pixels fired twice are merged into one word (charge summed, clipped at 15,
truth = largest contributor).

Raw format (one uint32 word per fired pixel):
bits [0,11) column, [11,22) row, [22,27) layer, [27,31) charge, bit 31 = 0.
Words of one event are grouped by ascending layer; the order inside a layer
is a random permutation (the reconstruction must not depend on it).

Optional upstream-tracker (UT) hits, for the Velo-to-UT search windows
(Sec. 2.3.2): four planes of silicon strips behind the Velo, the outer two
with vertical strips (x layers), the inner two tilted by +5 and -5 degrees
around z; here at z = 2327.5, 2372.5, 2597.5, 2642.5 mm, strips of
0.1875 mm pitch measuring u = x cos(a) + y sin(a) over u in [-768, 768) mm
(8192 strips), each strip cut into 14 sensors of 100 mm in y from
y = -700 mm, an inactive square |x|, |y| < 40 mm around the beam.  Particles
continue in a straight line from their state after the last Velo plane and
are bent in x by the field between the Velo and the UT: a single kick of
transverse momentum 45 MeV at z = 1000 mm, so x gains
q (45 MeV / p)(z - 1000 mm) (charge q = +-1).  One strip fires per crossing
(the paper: most UT hits are single strips, so there is no clustering) with
an efficiency, plus uniform noise strips; strips fired twice are one hit
(truth = lower particle id, noise last).  Raw UT word: bits [0,13) strip,
[13,17) sensor row (sector), [17,19) layer, the rest 0; the words of an
event in random order.

Randomness: numpy's Philox counter-based generator keyed by
(seed, chunk index); events are produced in fixed chunks of CHUNK events, so
the first n events of a config are the same whatever the total requested.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

N_LAYERS = 26
N_PIX = 1536
PITCH_MM = 0.055
Z_FIRST_MM = -280.0
Z_LAST_MM = 750.0
# (2c-1535)^2 + (2r-1535)^2 <= HOLE_Q  <=>  pixel-centre radius < 5.1 mm
HOLE_Q = 34393
CHUNK = 512
NOISE_PID = -1


def layer_z_mm() -> np.ndarray:
    """z of each layer (float64) used to propagate particles."""
    return Z_FIRST_MM + (Z_LAST_MM - Z_FIRST_MM) * np.arange(N_LAYERS) / (N_LAYERS - 1)


def _in_hole(c, r):
    dc = 2 * np.asarray(c, np.int64) - 1535
    dr = 2 * np.asarray(r, np.int64) - 1535
    return dc * dc + dr * dr <= HOLE_Q


def _n_active() -> int:
    d = (2 * np.arange(N_PIX, dtype=np.int64) - 1535) ** 2
    return int(N_PIX * N_PIX - np.count_nonzero(d[:, None] + d[None, :] <= HOLE_Q))


N_ACTIVE = _n_active()


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    n_events: int
    seed: int
    pv_mode: str            # "fixed" | "poisson" | "uniform"
    pv_param: tuple
    trk_mode: str           # "fixed" | "poisson"
    trk_param: float
    kink_sigma: float       # rad per crossed plane, applied to tx and ty
    hit_eff: float
    cluster_sizes: tuple    # equiprobable pixel counts of a particle's cluster
    noise_p: float          # noise probability per active pixel per layer
    pv_z_sigma: float = 45.0
    pv_xy_sigma: float = 0.01
    eta_range: tuple = (2.0, 5.0)
    # momentum-dependent scattering (0: fixed kink_sigma, no momentum): every
    # particle gets pT = 100 MeV + exponential(pt_mean) and p = pT cosh(eta);
    # the kink per crossed plane is N(0, 13.6 MeV / p * sqrt(ms_x0)) on each slope
    ms_x0: float = 0.0
    pt_mean: float = 0.0
    # upstream-tracker hits (needs a momentum per particle, ms_x0 > 0)
    ut: bool = False
    ut_eff: float = 0.99
    ut_noise: float = 100.0  # mean noise strips per (event, UT layer)


CONFIGS = {
    # small noiseless straight-track sample (oracle scale)
    "cpu10": Config("cpu10", 10, 0, "fixed", (1,), "fixed", 20, 0.0, 1.0, (1,), 0.0),
    # nominal occupancy, 1000 events
    "nominal": Config("nominal", 1000, 2, "poisson", (7.6,), "poisson", 25, 5e-5, 0.98,
                      (1, 2, 3), 1e-5),
    # uneven occupancy, 100k events
    "uneven": Config("uneven", 100_000, 3, "uniform", (1, 15), "poisson", 25, 5e-5, 0.98,
                     (1, 2, 3), 1e-5),
    # nominal occupancy, training / validation / test seeds for the ghost classifier
    "learn_train": Config("learn_train", 5500, 4, "poisson", (7.6,), "poisson", 25, 5e-5, 0.98,
                          (1, 2, 3), 1e-5),
    "learn_val": Config("learn_val", 2000, 40, "poisson", (7.6,), "poisson", 25, 5e-5, 0.98,
                        (1, 2, 3), 1e-5),
    "learn_test": Config("learn_test", 10_000, 41, "poisson", (7.6,), "poisson", 25, 5e-5, 0.98,
                         (1, 2, 3), 1e-5),
    # high occupancy stress, 10k events
    "stress": Config("stress", 10_000, 5, "poisson", (20.0,), "poisson", 25, 1e-4, 0.95,
                     (1, 2, 3), 1e-4),
    # nominal occupancy with a momentum per particle and scattering that depends on it
    # (the fit that takes a measured momentum)
    "momentum": Config("momentum", 1000, 6, "poisson", (7.6,), "poisson", 25, 0.0, 0.98,
                       (1, 2, 3), 1e-5, ms_x0=5.94e-4, pt_mean=500.0),
    # the same with upstream-tracker hits (the Velo-to-UT search windows)
    "ut": Config("ut", 1000, 7, "poisson", (7.6,), "poisson", 25, 0.0, 0.98,
                 (1, 2, 3), 1e-5, ms_x0=5.94e-4, pt_mean=500.0, ut=True),
}

# upstream tracker (generator's model; see the module docstring)
UT_Z_MM = (2327.5, 2372.5, 2597.5, 2642.5)
UT_ANGLE_DEG = (0.0, 5.0, -5.0, 0.0)
UT_PITCH_MM = 0.1875
UT_U0_MM = -768.0
UT_STRIPS = 8192
UT_Y0_MM = -700.0
UT_SECTOR_MM = 100.0
UT_SECTORS = 14
UT_HOLE_MM = 40.0
UT_KICK_MEV = 45.0
UT_Z_KICK_MM = 1000.0


def make_config(name: str, **overrides) -> Config:
    return dataclasses.replace(CONFIGS[name], **overrides)


@dataclasses.dataclass
class EventBatch:
    """Packed raw events plus generator truth.

    pixels      uint32 [N]      raw words, events back to back
    offsets     uint64 [E+1]    event e owns pixels[offsets[e]:offsets[e+1]]
    pix_pid     int32  [N]      event-local particle id of each word (-1 = noise)
    pix_q       uint8  [N]      charge of each word (same as bits 27..30)
    part_off    uint64 [E+1]    particles of event e are rows part_off[e]:part_off[e+1]
    part        dict of arrays  per particle: eta, phi, tx, ty, p (MeV, 0 when the
                                config draws no momentum), pv (event-local), pv_z, pv_x, pv_y
    pv_off      uint64 [E+1]    PVs of event e
    pv          dict            per PV: z, x, y, ntrk
    ut_words    uint32 [M]      raw UT words (None when the config has no UT)
    ut_offsets  uint64 [E+1]    event e owns ut_words[ut_offsets[e]:ut_offsets[e+1]]
    ut_pid      int32  [M]      event-local particle id of each UT word (-1 = noise)
    """
    pixels: np.ndarray
    offsets: np.ndarray
    pix_pid: np.ndarray
    pix_q: np.ndarray
    part_off: np.ndarray
    part: dict
    pv_off: np.ndarray
    pv: dict
    ut_words: np.ndarray | None = None
    ut_offsets: np.ndarray | None = None
    ut_pid: np.ndarray | None = None

    @property
    def n_events(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_pixels(self) -> int:
        return int(self.offsets[-1])

    def event_pixels(self, e: int) -> np.ndarray:
        return self.pixels[int(self.offsets[e]):int(self.offsets[e + 1])]

    def range(self, e0: int, e1: int) -> "EventBatch":
        """New batch holding events [e0, e1)."""
        return _slice(self, int(e0), int(e1))

    def select(self, events) -> "EventBatch":
        """New batch holding the given events (in the given order)."""
        ev = np.asarray(events, np.int64)
        return concat([_slice(self, int(e), int(e) + 1) for e in ev]) if len(ev) else _slice(self, 0, 0)


def _slice(b: EventBatch, e0: int, e1: int) -> EventBatch:
    p0, p1 = int(b.offsets[e0]), int(b.offsets[e1])
    q0, q1 = int(b.part_off[e0]), int(b.part_off[e1])
    v0, v1 = int(b.pv_off[e0]), int(b.pv_off[e1])
    ut = {}
    if b.ut_words is not None:
        u0, u1 = int(b.ut_offsets[e0]), int(b.ut_offsets[e1])
        ut = dict(ut_words=b.ut_words[u0:u1].copy(),
                  ut_offsets=(b.ut_offsets[e0:e1 + 1] - b.ut_offsets[e0]).astype(np.uint64),
                  ut_pid=b.ut_pid[u0:u1].copy())
    return EventBatch(
        pixels=b.pixels[p0:p1].copy(),
        offsets=(b.offsets[e0:e1 + 1] - b.offsets[e0]).astype(np.uint64),
        pix_pid=b.pix_pid[p0:p1].copy(),
        pix_q=b.pix_q[p0:p1].copy(),
        part_off=(b.part_off[e0:e1 + 1] - b.part_off[e0]).astype(np.uint64),
        part={k: v[q0:q1].copy() for k, v in b.part.items()},
        pv_off=(b.pv_off[e0:e1 + 1] - b.pv_off[e0]).astype(np.uint64),
        pv={k: v[v0:v1].copy() for k, v in b.pv.items()},
        **ut,
    )


def concat(batches) -> EventBatch:
    batches = list(batches)

    def cat_off(offs):
        out = [np.zeros(1, np.uint64)]
        base = 0
        for o in offs:
            out.append(o[1:].astype(np.uint64) + np.uint64(base))
            base += int(o[-1])
        return np.concatenate(out)

    return EventBatch(
        pixels=np.concatenate([b.pixels for b in batches]).astype(np.uint32),
        offsets=cat_off([b.offsets for b in batches]),
        pix_pid=np.concatenate([b.pix_pid for b in batches]).astype(np.int32),
        pix_q=np.concatenate([b.pix_q for b in batches]).astype(np.uint8),
        part_off=cat_off([b.part_off for b in batches]),
        part={k: np.concatenate([b.part[k] for b in batches]) for k in batches[0].part},
        pv_off=cat_off([b.pv_off for b in batches]),
        pv={k: np.concatenate([b.pv[k] for b in batches]) for k in batches[0].pv},
        **(dict(ut_words=np.concatenate([b.ut_words for b in batches]).astype(np.uint32),
                ut_offsets=cat_off([b.ut_offsets for b in batches]),
                ut_pid=np.concatenate([b.ut_pid for b in batches]).astype(np.int32))
           if batches[0].ut_words is not None else {}),
    )


def _draw_counts(rng, mode, param, n):
    if mode == "fixed":
        return np.full(n, int(param[0] if isinstance(param, tuple) else param), np.int64)
    if mode == "poisson":
        return rng.poisson(param[0] if isinstance(param, tuple) else param, n).astype(np.int64)
    if mode == "uniform":
        lo, hi = param
        return rng.integers(lo, hi + 1, n).astype(np.int64)
    raise ValueError(mode)


_NEIGH = np.array([(dc, dr) for dr in (-1, 0, 1) for dc in (-1, 0, 1) if (dc, dr) != (0, 0)],
                  np.int64)


def _gen_chunk(cfg: Config, chunk: int, n_ev: int) -> EventBatch:
    rng = np.random.Generator(np.random.Philox(key=np.array([cfg.seed, chunk], np.uint64)))
    zl = layer_z_mm()
    dzl = zl[1] - zl[0]

    # primary vertices
    npv = _draw_counts(rng, cfg.pv_mode, cfg.pv_param, n_ev)
    n_pv = int(npv.sum())
    pv_ev = np.repeat(np.arange(n_ev), npv)
    pv_z = rng.normal(0.0, cfg.pv_z_sigma, n_pv)
    pv_x = rng.normal(0.0, cfg.pv_xy_sigma, n_pv)
    pv_y = rng.normal(0.0, cfg.pv_xy_sigma, n_pv)

    # particles
    ntrk = _draw_counts(rng, cfg.trk_mode, cfg.trk_param, n_pv)
    n_t = int(ntrk.sum())
    t_pv = np.repeat(np.arange(n_pv), ntrk)
    t_ev = pv_ev[t_pv]
    eta = rng.uniform(cfg.eta_range[0], cfg.eta_range[1], n_t)
    phi = rng.uniform(0.0, 2.0 * math.pi, n_t)
    tan_theta = np.tan(2.0 * np.arctan(np.exp(-eta)))
    tx0 = tan_theta * np.cos(phi)
    ty0 = tan_theta * np.sin(phi)
    p_mev = np.zeros(n_t)

    # propagation through the planes downstream of the PV
    crossed = zl[None, :] > pv_z[t_pv][:, None]                 # [T, 26]
    first = np.argmax(crossed, axis=1)
    if cfg.ms_x0 > 0:
        pt = 100.0 + rng.exponential(cfg.pt_mean, n_t)
        p_mev = pt * np.cosh(eta)
        sig = 13.6 / p_mev * math.sqrt(cfg.ms_x0)
        kx = rng.normal(0.0, 1.0, (n_t, N_LAYERS)) * sig[:, None]
        ky = rng.normal(0.0, 1.0, (n_t, N_LAYERS)) * sig[:, None]
    elif cfg.kink_sigma > 0:
        kx = rng.normal(0.0, cfg.kink_sigma, (n_t, N_LAYERS))
        ky = rng.normal(0.0, cfg.kink_sigma, (n_t, N_LAYERS))
    else:
        kx = np.zeros((n_t, N_LAYERS))
        ky = np.zeros((n_t, N_LAYERS))
    cr = crossed.astype(np.float64)
    tx_after = tx0[:, None] + np.cumsum(kx * cr, axis=1)        # slope after each crossing
    ty_after = ty0[:, None] + np.cumsum(ky * cr, axis=1)
    sx = np.cumsum(tx_after * cr, axis=1)
    sy = np.cumsum(ty_after * cr, axis=1)
    sx_prev = np.concatenate([np.zeros((n_t, 1)), sx[:, :-1]], axis=1)
    sy_prev = np.concatenate([np.zeros((n_t, 1)), sy[:, :-1]], axis=1)
    zf = zl[first]
    x = (pv_x[t_pv] + tx0 * (zf - pv_z[t_pv]))[:, None] + dzl * sx_prev
    y = (pv_y[t_pv] + ty0 * (zf - pv_z[t_pv]))[:, None] + dzl * sy_prev

    eff = rng.random((n_t, N_LAYERS)) < cfg.hit_eff
    hit = crossed & eff
    ti, li = np.nonzero(hit)
    hx, hy = x[ti, li], y[ti, li]
    c = np.floor(hx / PITCH_MM + 768.0).astype(np.int64)
    r = np.floor(hy / PITCH_MM + 768.0).astype(np.int64)
    ok = (c >= 0) & (c < N_PIX) & (r >= 0) & (r < N_PIX)
    ok &= ~_in_hole(np.clip(c, 0, N_PIX - 1), np.clip(r, 0, N_PIX - 1))
    ti, li, hx, hy, c, r = ti[ok], li[ok], hx[ok], hy[ok], c[ok], r[ok]
    n_h = len(ti)

    # cluster shape: seed pixel plus the (s-1) neighbour pixels nearest the crossing point
    sizes = np.asarray(cfg.cluster_sizes, np.int64)
    s = sizes[rng.integers(0, len(sizes), n_h)]
    pc = [c]
    pr = [r]
    pt = [ti]
    pl = [li]
    if sizes.max() > 1:
        nc = c[:, None] + _NEIGH[None, :, 0]
        nr = r[:, None] + _NEIGH[None, :, 1]
        d2 = ((nc - 767.5) * PITCH_MM - hx[:, None]) ** 2 + ((nr - 767.5) * PITCH_MM - hy[:, None]) ** 2
        order = np.argsort(d2, axis=1, kind="stable")
        for k in range(int(sizes.max()) - 1):
            sel = s > k + 1
            j = order[sel, k]
            cc = nc[sel, j]
            rr = nr[sel, j]
            good = (cc >= 0) & (cc < N_PIX) & (rr >= 0) & (rr < N_PIX)
            good &= ~_in_hole(np.clip(cc, 0, N_PIX - 1), np.clip(rr, 0, N_PIX - 1))
            pc.append(cc[good])
            pr.append(rr[good])
            pt.append(ti[sel][good])
            pl.append(li[sel][good])
    pc = np.concatenate(pc)
    pr = np.concatenate(pr)
    pt = np.concatenate(pt)
    pl = np.concatenate(pl)
    pe = t_ev[pt]
    pq = rng.integers(1, 16, len(pc))

    # noise pixels, uniform over the active area of every (event, layer)
    if cfg.noise_p > 0:
        nn = rng.poisson(cfg.noise_p * N_ACTIVE, (n_ev, N_LAYERS))
        n_noise = int(nn.sum())
        ne = np.repeat(np.repeat(np.arange(n_ev), N_LAYERS), nn.ravel())
        nl = np.repeat(np.tile(np.arange(N_LAYERS), n_ev), nn.ravel())
        ncc = rng.integers(0, N_PIX, n_noise)
        nrr = rng.integers(0, N_PIX, n_noise)
        bad = _in_hole(ncc, nrr)
        while bad.any():
            k = int(bad.sum())
            ncc[bad] = rng.integers(0, N_PIX, k)
            nrr[bad] = rng.integers(0, N_PIX, k)
            bad = _in_hole(ncc, nrr)
        nq = rng.integers(1, 16, n_noise)
        pc = np.concatenate([pc, ncc])
        pr = np.concatenate([pr, nrr])
        pl = np.concatenate([pl, nl])
        pe = np.concatenate([pe, ne])
        pq = np.concatenate([pq, nq])
        pt = np.concatenate([pt, np.full(n_noise, -1, np.int64)])

    # merge pixels fired more than once
    addr = (((pe * N_LAYERS + pl) << 22) | (pr << 11) | pc).astype(np.int64)
    # one int64 sort key: address, then larger charge first, then lower particle id (noise last)
    assert n_t < (1 << 23) - 1 and n_ev * N_LAYERS < (1 << 14)
    pid_key = np.where(pt < 0, (1 << 23) - 1, pt)
    order = np.argsort((addr << 27) | ((15 - np.minimum(pq, 15)) << 23) | pid_key)
    addr_s = addr[order]
    start = np.ones(len(addr_s), bool)
    start[1:] = addr_s[1:] != addr_s[:-1]
    gi = np.nonzero(start)[0]
    win = order[gi]
    qsum = np.add.reduceat(pq[order], gi) if len(gi) else np.zeros(0, np.int64)
    m_e, m_l, m_r, m_c = pe[win], pl[win], pr[win], pc[win]
    m_q = np.minimum(qsum, 15)
    m_t = pt[win]

    # event-local particle ids
    t_off = np.zeros(n_ev + 1, np.int64)
    np.cumsum(np.bincount(t_ev, minlength=n_ev), out=t_off[1:])
    m_pid = np.where(m_t < 0, NOISE_PID, m_t - t_off[np.clip(m_e, 0, n_ev - 1)] if len(m_t) else m_t)

    # event-major, layer-ascending, random order within a layer
    rnd = rng.integers(0, 1 << 32, len(m_e), dtype=np.int64)
    order = np.argsort((m_e << 40) | (m_l << 35) | rnd)
    m_e, m_l, m_r, m_c, m_q, m_pid = (a[order] for a in (m_e, m_l, m_r, m_c, m_q, m_pid))
    words = (m_c | (m_r << 11) | (m_l << 22) | (m_q << 27)).astype(np.uint32)
    offsets = np.zeros(n_ev + 1, np.uint64)
    np.cumsum(np.bincount(m_e, minlength=n_ev), out=offsets[1:])

    pv_off = np.zeros(n_ev + 1, np.uint64)
    np.cumsum(npv, out=pv_off[1:])
    pv_first = pv_off[:-1].astype(np.int64)
    ut = {}
    if cfg.ut:
        # state after the last Velo plane (every particle crosses it: its PV lies upstream)
        ut = _ut_hits(rng, cfg, n_ev, t_ev, t_off, p_mev, x[:, -1], y[:, -1], tx_after[:, -1],
                      ty_after[:, -1], zl[-1])
    return EventBatch(
        pixels=words,
        offsets=offsets,
        pix_pid=m_pid.astype(np.int32),
        pix_q=m_q.astype(np.uint8),
        part_off=t_off.astype(np.uint64),
        part=dict(eta=eta, phi=phi, tx=tx0, ty=ty0, p=p_mev, pv=(t_pv - pv_first[t_ev]).astype(np.int32),
                  pv_z=pv_z[t_pv], pv_x=pv_x[t_pv], pv_y=pv_y[t_pv]),
        pv_off=pv_off,
        pv=dict(z=pv_z, x=pv_x, y=pv_y, ntrk=ntrk),
        **ut,
    )


def _ut_hits(rng, cfg, n_ev, t_ev, t_off, p_mev, x_end, y_end, tx_end, ty_end, z_end):
    """Raw UT words of the chunk's particles (model in the module docstring)."""
    n_t = len(t_ev)
    q = np.where(rng.random(n_t) < 0.5, -1.0, 1.0)
    words, ev, pid = [], [], []
    for k, (zk, ang) in enumerate(zip(UT_Z_MM, UT_ANGLE_DEG)):
        a = math.radians(ang)
        xk = x_end + tx_end * (zk - z_end) + q * (UT_KICK_MEV / p_mev) * (zk - UT_Z_KICK_MM)
        yk = y_end + ty_end * (zk - z_end)
        u = xk * math.cos(a) + yk * math.sin(a)
        strip = np.floor((u - UT_U0_MM) / UT_PITCH_MM).astype(np.int64)
        sec = np.floor((yk - UT_Y0_MM) / UT_SECTOR_MM).astype(np.int64)
        ok = (strip >= 0) & (strip < UT_STRIPS) & (sec >= 0) & (sec < UT_SECTORS)
        ok &= ~((np.abs(xk) < UT_HOLE_MM) & (np.abs(yk) < UT_HOLE_MM))
        ok &= rng.random(n_t) < cfg.ut_eff
        idx = np.nonzero(ok)[0]
        words.append(strip[idx] | (sec[idx] << 13) | (k << 17))
        ev.append(t_ev[idx])
        pid.append(idx - t_off[t_ev[idx]])
        nn = rng.poisson(cfg.ut_noise, n_ev)
        tot = int(nn.sum())
        words.append(rng.integers(0, UT_STRIPS, tot) | (rng.integers(0, UT_SECTORS, tot) << 13) | (k << 17))
        ev.append(np.repeat(np.arange(n_ev), nn))
        pid.append(np.full(tot, -1, np.int64))
    w = np.concatenate(words).astype(np.int64)
    e = np.concatenate(ev).astype(np.int64)
    pid = np.concatenate(pid).astype(np.int64)
    # one hit per fired strip: lowest particle id wins, noise last
    pk = np.where(pid < 0, (1 << 23) - 1, pid)
    order = np.argsort((e << 42) | (w << 23) | pk)
    key = (e << 19 | w)[order]
    first = np.ones(len(key), bool)
    first[1:] = key[1:] != key[:-1]
    sel = order[first]
    w, e, pid = w[sel], e[sel], pid[sel]
    # random order inside an event
    order = np.argsort((e << 32) | rng.integers(0, 1 << 32, len(e), dtype=np.int64))
    w, e, pid = w[order], e[order], pid[order]
    off = np.zeros(n_ev + 1, np.uint64)
    np.cumsum(np.bincount(e, minlength=n_ev), out=off[1:])
    return dict(ut_words=w.astype(np.uint32), ut_offsets=off, ut_pid=pid.astype(np.int32))


def _chunk_part(args):
    cfg, ch, lo, hi = args
    return _slice(_gen_chunk(cfg, ch, CHUNK), lo, hi)


def generate(cfg, n_events: int | None = None, first_event: int = 0, workers: int = 1) -> EventBatch:
    """Events [first_event, first_event + n_events) of a config (name or Config).

    workers > 1 draws the chunks on a thread pool (the result is identical;
    numpy releases the interpreter lock in the bulk work).  No process is
    forked, so it may be called at any time, also after a GPU is in use."""
    if isinstance(cfg, str):
        cfg = CONFIGS[cfg]
    if n_events is None:
        n_events = cfg.n_events
    if n_events == 0:
        return _slice(_gen_chunk(cfg, 0, CHUNK), 0, 0)
    c0 = first_event // CHUNK
    c1 = (first_event + n_events - 1) // CHUNK
    jobs = [(cfg, ch, max(first_event - ch * CHUNK, 0), min(first_event + n_events - ch * CHUNK, CHUNK))
            for ch in range(c0, c1 + 1)]
    if workers > 1 and len(jobs) > 1:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(min(workers, len(jobs))) as pool:
            parts = list(pool.map(_chunk_part, jobs))
    else:
        parts = [_chunk_part(j) for j in jobs]
    return parts[0] if len(parts) == 1 else concat(parts)
