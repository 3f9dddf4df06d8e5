"""Helpers of the GPU parity tests: run libvelo through its C ABI and compare
with the oracle element by element."""
import numpy as np

HIT_KEYS = ("x", "y", "key", "aux")


def to_dev(pixels, offsets, device="cuda"):
    import torch
    px = torch.from_numpy(np.ascontiguousarray(pixels, np.uint32).view(np.int32)).to(device)
    off = torch.from_numpy(np.ascontiguousarray(offsets, np.uint64).view(np.int64)).to(device)
    return px, off


def gpu_reconstruct(pixels, offsets, params=None):
    import torch

    import paper_1912_09161_amd as velo
    px, off = to_dev(pixels, offsets)
    p = velo.default_params(**(params or {}))
    out = velo.reconstruct(px, off, params=p)
    torch.cuda.synchronize()
    return host(out)


def host(out):
    h = {k: v.cpu().numpy() for k, v in out["hits"].items()}
    t = {k: v.cpu().numpy() for k, v in out["tracks"].items()}
    s = {k: v.cpu().numpy() for k, v in out["states"].items()}
    for k in ("key", "aux", "layer_start", "layer_nhits", "n_hits", "status"):
        h[k] = h[k].view(np.uint32)
    E = len(h["n_hits"]) if len(h["n_hits"]) else 0
    h["layer_start"] = h["layer_start"].reshape(-1, 27)
    h["layer_nhits"] = h["layer_nhits"].reshape(-1, 26)
    for k in ("n_tracks", "hit_idx", "status"):
        t[k] = t[k].view(np.uint32)
    t["hit_idx"] = t["hit_idx"].reshape(-1, 26)
    s["cov_x"] = s["cov_x"].reshape(-1, 3)
    s["cov_y"] = s["cov_y"].reshape(-1, 3)
    return dict(hits=h, tracks=t, states=s)


def hit_slots(h, offsets):
    """Absolute slots of all valid hits (per the layer tables of `h`)."""
    E = len(offsets) - 1
    starts = (np.asarray(offsets[:-1], np.int64)[:, None] + h["layer_start"][:E, :26].astype(np.int64)).ravel()
    counts = h["layer_nhits"][:E].astype(np.int64).ravel()
    if counts.sum() == 0:
        return np.zeros(0, np.int64)
    rep = np.repeat(starts - np.concatenate([[0], np.cumsum(counts)[:-1]]), counts)
    return rep + np.arange(counts.sum())


def track_slots(t, offsets):
    E = len(offsets) - 1
    base = np.asarray(offsets[:-1], np.int64) // 3
    nt = t["n_tracks"][:E].astype(np.int64)
    if nt.sum() == 0:
        return np.zeros(0, np.int64)
    rep = np.repeat(base - np.concatenate([[0], np.cumsum(nt)[:-1]]), nt)
    return rep + np.arange(nt.sum())


def compare_hits(g, o, offsets):
    E = len(offsets) - 1
    for k in ("status", "n_hits"):
        np.testing.assert_array_equal(g[k][:E], o[k][:E], err_msg=k)
    np.testing.assert_array_equal(g["layer_start"][:E], o["layer_start"][:E], err_msg="layer_start")
    np.testing.assert_array_equal(g["layer_nhits"][:E], o["layer_nhits"][:E], err_msg="layer_nhits")
    sl = hit_slots(o, offsets)
    for k in HIT_KEYS:
        a, b = g[k][sl], o[k][sl]
        if a.dtype.kind == "f":
            # bit-exact, including signed zeros
            np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32), err_msg=k)
        else:
            np.testing.assert_array_equal(a, b, err_msg=k)
    return len(sl)


def compare_tracks(g, o, offsets):
    E = len(offsets) - 1
    np.testing.assert_array_equal(g["status"][:E], o["status"][:E], err_msg="track status")
    np.testing.assert_array_equal(g["n_tracks"][:E], o["n_tracks"][:E], err_msg="n_tracks")
    sl = track_slots(o, offsets)
    np.testing.assert_array_equal(g["nhits"][sl], o["nhits"][sl], err_msg="track nhits")
    nh = o["nhits"][sl].astype(np.int64)
    mask = np.arange(26)[None, :] < nh[:, None]
    np.testing.assert_array_equal(np.where(mask, g["hit_idx"][sl], 0), np.where(mask, o["hit_idx"][sl], 0),
                                  err_msg="track hit indices")
    return len(sl)


# |gpu - oracle| <= 1e-4 * max(|gpu|, |oracle|) + floor
FLOORS = dict(x=1e-6, y=1e-6, z=1e-5, tx=1e-8, ty=1e-8, chi2=1e-6, cov_x=1e-12, cov_y=1e-12)


def compare_states(g, o, offsets, tracks):
    sl = track_slots(tracks, offsets)
    for k, fl in FLOORS.items():
        a = g[k][sl].astype(np.float64)
        b = o[k][sl].astype(np.float64)
        tol = 1e-4 * np.maximum(np.abs(a), np.abs(b)) + fl
        bad = np.abs(a - b) > tol
        assert not bad.any(), f"{k}: {bad.sum()} states differ, first {np.nonzero(bad.ravel())[0][:5]}"
    np.testing.assert_array_equal(g["ndof"][sl], o["ndof"][sl], err_msg="ndof")
    np.testing.assert_array_equal(g["accepted"][sl], o["accepted"][sl], err_msg="accepted")
    return len(sl)


def compare_all(g, o, offsets):
    n_h = compare_hits(g["hits"], o["hits"], offsets)
    n_t = compare_tracks(g["tracks"], o["tracks"], offsets)
    n_s = compare_states(g["states"], o["states"], offsets, o["tracks"])
    return n_h, n_t, n_s
