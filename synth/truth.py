"""Generator-truth matching and tracking metrics (test / benchmark infrastructure).

Definitions (paper Sec. 3.1): a track is correctly reconstructed when at least
70 % of its hits belong to one simulated particle; a particle is
reconstructible when it has hits on at least three different planes.
Readings for the rest: the truth of a hit is the particle that contributes
most charge to its pixels (ties to the lower id; noise pixels count for no
particle and a noise-majority hit has no particle); ghost rate = accepted
tracks matched to no particle / accepted tracks; clone rate =
(matched tracks - matched particles) / matched tracks.

Hit membership (which raw pixels form the hit with a given key) is computed
here with scipy's graph connected components, independently of both the
oracle and the GPU library.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components


def pixel_components(pixels: np.ndarray, offsets: np.ndarray):
    """Label the 8-connected pixel groups of every (event, plane).

    Returns (label[N], key_of_label[L]) where key is the group's smallest
    27-bit pixel address (layer << 22 | row << 11 | col).
    """
    pixels = np.asarray(pixels, np.uint32)
    n = len(pixels)
    if n == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.uint32)
    ev = np.repeat(np.arange(len(offsets) - 1), np.diff(offsets.astype(np.int64)))
    addr = (pixels & 0x07FFFFFF).astype(np.int64)
    g = (ev.astype(np.int64) << 27) | addr          # global address, unique per pixel
    order = np.argsort(g, kind="stable")
    gs = g[order]
    rows, cols = [], []
    # forward neighbours: (r, c+1), (r+1, c-1), (r+1, c), (r+1, c+1)
    col = gs & 0x7FF
    row = (gs >> 11) & 0x7FF
    for dr, dc in ((0, 1), (1, -1), (1, 0), (1, 1)):
        ok = (col + dc >= 0) & (col + dc < 1536) & (row + dr < 1536)
        tgt = gs + (dr << 11) + dc
        j = np.searchsorted(gs, tgt)
        j = np.minimum(j, n - 1)
        hit = ok & (gs[j] == tgt)
        rows.append(np.nonzero(hit)[0])
        cols.append(j[hit])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    A = coo_matrix((np.ones(len(r), np.int8), (r, c)), shape=(n, n))
    _, lab_sorted = connected_components(A, directed=False)
    label = np.empty(n, np.int64)
    label[order] = lab_sorted
    nl = int(label.max()) + 1
    key = np.full(nl, np.iinfo(np.int64).max, np.int64)
    np.minimum.at(key, label, addr)
    return label, key.astype(np.uint32)


class Truth:
    """Per-event map hit key -> particle, and particle reconstructibility."""

    def __init__(self, batch):
        self.batch = batch
        label, lkey = pixel_components(batch.pixels, batch.offsets)
        E = batch.n_events
        ev = np.repeat(np.arange(E), np.diff(batch.offsets.astype(np.int64)))
        pid = batch.pix_pid.astype(np.int64)
        q = batch.pix_q.astype(np.int64)
        # charge per (label, particle); noise (-1) never wins
        real = pid >= 0
        lp = label[real] * (1 << 24) + pid[real]
        uniq, inv = np.unique(lp, return_inverse=True)
        qs = np.bincount(inv, weights=q[real])
        lab_u = uniq >> 24
        pid_u = uniq & ((1 << 24) - 1)
        # noise charge per label
        qn = np.bincount(label[~real], weights=q[~real], minlength=len(lkey))
        # best particle per label: max charge, then lowest id
        o = np.lexsort((pid_u, -qs, lab_u))
        first = np.ones(len(o), bool)
        first[1:] = lab_u[o][1:] != lab_u[o][:-1]
        best_lab = lab_u[o][first]
        best_pid = pid_u[o][first]
        best_q = qs[o][first]
        lab_pid = np.full(len(lkey), -1, np.int64)
        keep = best_q > qn[best_lab]
        lab_pid[best_lab[keep]] = best_pid[keep]
        lab_ev = np.zeros(len(lkey), np.int64)
        lab_ev[label] = ev
        self.lab_ev = lab_ev
        self.lab_key = lkey
        self.lab_pid = lab_pid
        # lookup (event, key) -> particle
        self._gk = (lab_ev << 27) | lkey.astype(np.int64)
        o = np.argsort(self._gk)
        self._gk = self._gk[o]
        self._gp = lab_pid[o]
        # reconstructible particles: hits on >= 3 distinct planes
        has = lab_pid >= 0
        pl = (lab_ev[has] << 40) | (lab_pid[has] << 5) | (lkey[has].astype(np.int64) >> 22)
        pl = np.unique(pl)
        part = pl >> 5
        up, cnt = np.unique(part, return_counts=True)
        self.reco_ev = up >> 35
        self.reco_pid = up & ((1 << 35) - 1)
        self.reco_ok = cnt >= 3
        self.n_reconstructible = int(np.count_nonzero(self.reco_ok))

    def hit_particle(self, ev: np.ndarray, key: np.ndarray) -> np.ndarray:
        gk = (np.asarray(ev, np.int64) << 27) | np.asarray(key, np.int64)
        j = np.searchsorted(self._gk, gk)
        j = np.minimum(j, len(self._gk) - 1)
        out = np.where(self._gk[j] == gk, self._gp[j], -1)
        return out


def track_list(tracks: dict, hits: dict, offsets: np.ndarray):
    """Flatten per-event track outputs: (event, slot, n_hits, keys[T, 26] (0 pad))."""
    offsets = np.asarray(offsets, np.int64)
    E = len(offsets) - 1
    base = offsets[:-1] // 3
    nt = np.asarray(tracks["n_tracks"], np.int64)
    ev = np.repeat(np.arange(E), nt)
    slot = np.concatenate([base[e] + np.arange(nt[e]) for e in range(E)]) if E else np.zeros(0, np.int64)
    slot = slot.astype(np.int64)
    nh = np.asarray(tracks["nhits"])[slot].astype(np.int64)
    hidx = np.asarray(tracks["hit_idx"]).reshape(-1, 26)[slot].astype(np.int64)
    mask = np.arange(26)[None, :] < nh[:, None]
    # entries past a track's hit count are unspecified: mask them before indexing
    absidx = np.where(mask, offsets[ev][:, None] + hidx, 0)
    keys = np.where(mask, np.asarray(hits["key"])[absidx], 0)
    return ev, slot, nh, keys


def match_tracks(truth: Truth, ev, nh, keys):
    """Particle matched to each track by the 70 % rule (-1 = ghost)."""
    T = len(ev)
    if T == 0:
        return np.zeros(0, np.int64)
    mask = np.arange(26)[None, :] < nh[:, None]
    pk = truth.hit_particle(np.repeat(ev, 26).reshape(T, 26), keys)
    pk = np.where(mask, pk, -2)
    out = np.full(T, -1, np.int64)
    srt = np.sort(pk, axis=1)
    # most frequent non-negative id per row
    best_cnt = np.zeros(T, np.int64)
    best_id = np.full(T, -1, np.int64)
    run_id = srt[:, 0].copy()
    run_cnt = np.ones(T, np.int64)
    for j in range(1, 27):
        cur = srt[:, j] if j < 26 else np.full(T, -3, np.int64)
        same = cur == run_id
        run_cnt = np.where(same, run_cnt + 1, run_cnt)
        end = ~same
        better = end & (run_id >= 0) & (run_cnt > best_cnt)
        best_cnt = np.where(better, run_cnt, best_cnt)
        best_id = np.where(better, run_id, best_id)
        run_id = np.where(end, cur, run_id)
        run_cnt = np.where(end, 1, run_cnt)
    ok = best_cnt * 10 >= 7 * nh
    out[ok] = best_id[ok]
    return out


def metrics(truth: Truth, ev, nh, keys, accepted) -> dict:
    m = match_tracks(truth, ev, nh, keys)
    acc = np.asarray(accepted, bool)
    n_acc = int(acc.sum())
    ghosts = int(np.count_nonzero(acc & (m < 0)))
    matched = acc & (m >= 0)
    pairs = np.unique((np.asarray(ev, np.int64)[matched] << 35) | m[matched])
    reco = set(((truth.reco_ev[truth.reco_ok] << 35) | truth.reco_pid[truth.reco_ok]).tolist())
    found = sum(1 for p in pairs.tolist() if p in reco)
    n_m = int(matched.sum())
    return dict(
        n_tracks=n_acc, ghosts=ghosts, ghost_rate=ghosts / max(n_acc, 1),
        efficiency=found / max(truth.n_reconstructible, 1),
        n_reconstructible=truth.n_reconstructible, found=found,
        clone_rate=(n_m - len(pairs)) / max(n_m, 1),
    )


def track_labels(truth: Truth, tracks: dict, hits: dict, offsets):
    """Generator-truth labels of every found track.

    Returns (slot, label, particle_uid, reco_uid): track slots in canonical
    order, label 1 for tracks matched to a particle by the 70 % rule (clones
    included) and 0 for ghosts, a unique id (event << 35 | particle) of the
    matched particle (-1 for ghosts), and the unique ids of the
    reconstructible particles."""
    ev, slot, nh, keys = track_list(tracks, hits, offsets)
    m = match_tracks(truth, ev, nh, keys)
    uid = np.where(m >= 0, (np.asarray(ev, np.int64) << 35) | np.maximum(m, 0), -1)
    reco = (truth.reco_ev[truth.reco_ok] << 35) | truth.reco_pid[truth.reco_ok]
    return slot, (m >= 0).astype(np.float32), uid, reco


def efficiency_ghosts(particle_uid, accepted, reco_uid) -> dict:
    """Efficiency, ghost rate and clone rate of accepted tracks."""
    acc = np.asarray(accepted, bool)
    n_acc = int(acc.sum())
    ghosts = int(np.count_nonzero(acc & (particle_uid < 0)))
    matched = acc & (particle_uid >= 0)
    pairs = np.unique(particle_uid[matched])
    found = int(np.isin(np.unique(reco_uid), pairs).sum())
    n_m = int(matched.sum())
    return dict(n_tracks=n_acc, ghosts=ghosts, ghost_rate=ghosts / max(n_acc, 1),
                efficiency=found / max(len(np.unique(reco_uid)), 1), found=found,
                clone_rate=(n_m - len(pairs)) / max(n_m, 1))


def _label_chunk(job):
    b, ev, nh, keys, (e0, e1, t0, t1) = job
    T = Truth(b.range(e0, e1))
    m = match_tracks(T, ev[t0:t1] - e0, nh[t0:t1], keys[t0:t1])
    reco = ((T.reco_ev[T.reco_ok] + e0) << 35) | T.reco_pid[T.reco_ok]
    return m, reco


def track_labels_parallel(batch, tracks: dict, hits: dict, workers: int = 8, chunk: int = 250):
    """track_labels(Truth(batch), ...) computed over chunks of events on a
    thread pool (no process is forked)."""
    from concurrent.futures import ThreadPoolExecutor
    ev, slot, nh, keys = track_list(tracks, hits, batch.offsets)
    E = batch.n_events
    if workers <= 1 or E <= chunk:
        T = Truth(batch)
        m = match_tracks(T, ev, nh, keys)
        reco = (T.reco_ev[T.reco_ok] << 35) | T.reco_pid[T.reco_ok]
    else:
        bounds = np.searchsorted(ev, np.arange(0, E + chunk, chunk).clip(max=E))
        jobs = [(batch, ev, nh, keys, (e0, min(e0 + chunk, E), int(bounds[i]), int(bounds[i + 1])))
                for i, e0 in enumerate(range(0, E, chunk))]
        with ThreadPoolExecutor(min(workers, len(jobs))) as pool:
            res = list(pool.map(_label_chunk, jobs))
        m = np.concatenate([r[0] for r in res]) if res else np.zeros(0, np.int64)
        reco = np.concatenate([r[1] for r in res]) if res else np.zeros(0, np.int64)
    uid = np.where(m >= 0, (np.asarray(ev, np.int64) << 35) | np.maximum(m, 0), -1)
    return slot, (m >= 0).astype(np.float32), uid, reco


def pv_truth_tracks(batch, truth: Truth | None = None) -> np.ndarray:
    """Number of reconstructible particles of every simulated PV (flat over
    the batch's PVs, in batch.pv order)."""
    truth = truth if truth is not None else Truth(batch)
    n_pv = len(batch.pv["z"])
    part_pv = batch.part["pv"].astype(np.int64)
    part_ev = np.repeat(np.arange(batch.n_events), np.diff(batch.part_off.astype(np.int64)))
    pv_first = batch.pv_off[:-1].astype(np.int64)
    ok = truth.reco_ok
    ev, pid = truth.reco_ev[ok], truth.reco_pid[ok]
    part_first = batch.part_off[:-1].astype(np.int64)
    gpart = part_first[ev] + pid
    gpv = pv_first[part_ev[gpart]] + part_pv[gpart]
    return np.bincount(gpv, minlength=n_pv)


def pv_metrics(batch, n_pv, pv_z, pv_var, n_reco_tracks=None, min_tracks: int = 5, n_sigma: float = 5.0):
    """PV efficiency and fake rate (Sec. 3.1: a reconstructed PV matches a
    simulated one closer than n_sigma times its z uncertainty).  Matching per
    event, one to one, closest pairs first.  Efficiency counts simulated PVs
    with at least min_tracks reconstructible particles; a reconstructed PV
    matched to no simulated PV (of any multiplicity) is a fake."""
    if n_reco_tracks is None:
        n_reco_tracks = pv_truth_tracks(batch)
    E = batch.n_events
    tz = np.asarray(batch.pv["z"], np.float64)
    found = np.zeros(len(tz), bool)
    resid = []
    n_rec = n_fake = 0
    for e in range(E):
        a, b = int(batch.pv_off[e]), int(batch.pv_off[e + 1])
        k = int(n_pv[e])
        rz = np.asarray(pv_z[e, :k], np.float64)
        rs = np.sqrt(np.maximum(np.asarray(pv_var[e, :k], np.float64), 0.0))
        n_rec += k
        pairs = sorted((abs(rz[i] - tz[a + j]), i, j) for i in range(k) for j in range(b - a)
                       if abs(rz[i] - tz[a + j]) < n_sigma * rs[i])
        used_r, used_t = set(), set()
        for d, i, j in pairs:
            if i in used_r or j in used_t:
                continue
            used_r.add(i)
            used_t.add(j)
            found[a + j] = True
            resid.append((rz[i] - tz[a + j]) / rs[i])
        n_fake += k - len(used_r)
    sel = n_reco_tracks >= min_tracks
    pulls = np.asarray(resid)
    return dict(n_true=int(sel.sum()), n_found=int((found & sel).sum()),
                efficiency=float((found & sel).sum() / max(sel.sum(), 1)),
                n_rec=n_rec, n_fake=n_fake, fake_rate=n_fake / max(n_rec, 1),
                pull_mean=float(pulls.mean()) if len(pulls) else 0.0,
                pull_std=float(pulls.std()) if len(pulls) > 1 else 0.0)
