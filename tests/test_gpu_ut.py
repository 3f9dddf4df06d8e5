"""GPU parity of the Velo-to-UT search windows (velo_ut_windows) with the
oracle (Sec. 2.3.2).

Sorting distinct integers and counting hits inside a window are exact
operations, and the extrapolation is the same binary32 expression on both
sides, so given the same track states every output must agree bit for bit:
per-event status, region starts, the sorted words of good events and the
window words of every track slot.  Covered: the benchmark's batch size of
generated events with UT hits (on the GPU's own states), the status rules
(duplicates, bad fields, the hit limit and one above, unusable offsets)
next to good events, dense strips at the window edges of every plane with
and without the tolerance, sensor rows at their half-open limits, and strip
centres exactly on a window edge.
"""
import numpy as np
import pytest

from gpu_helpers import host, to_dev
from synth import generate
from test_oracle_ut import dense, one_track, strip_u, word

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def gpu_ut(words, uo, offsets, tracks, states, n_pixels=None, **kw):
    import torch

    import paper_1912_09161_amd as velo
    w = torch.from_numpy(np.ascontiguousarray(words, np.uint32).view(np.int32)).cuda()
    u = torch.from_numpy(np.ascontiguousarray(uo, np.uint64).view(np.int64)).cuda()
    off = torch.from_numpy(np.ascontiguousarray(offsets, np.uint64).view(np.int64)).cuda()
    st = {k: torch.from_numpy(np.ascontiguousarray(states[k])).cuda() for k in ("x", "y", "z", "tx", "ty", "accepted")}
    nt = torch.from_numpy(np.ascontiguousarray(tracks["n_tracks"], np.uint32).view(np.int32)).cuda()
    tr = dict(n_tracks=nt, nhits=nt, hit_idx=nt, status=nt)  # only n_tracks is read
    npx = int(offsets[-1]) if n_pixels is None else int(n_pixels)
    out = velo.alloc_ut(len(words), len(uo) - 1, npx)
    out["win"].fill_(0x5A5A5A5A)  # slots beyond the counts must stay untouched
    out = velo.ut_windows(w, u, tr, st, off, npx, params=velo.default_ut_params(**kw), out=out)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy().view(np.uint32) for k, v in out.items()}


def compare(g, o, uo, offsets, tracks, n_pixels=None):
    E = len(uo) - 1
    np.testing.assert_array_equal(g["status"][:E], o["status"], err_msg="status")
    np.testing.assert_array_equal(g["region"][:E * 57].reshape(E, 57), o["region"], err_msg="region")
    for e in np.nonzero(o["status"] == 0)[0]:
        a, b = int(uo[e]), int(uo[e + 1])
        np.testing.assert_array_equal(g["sorted"][a:b], o["sorted"][a:b], err_msg=f"sorted, event {e}")
    npx = int(offsets[-1]) if n_pixels is None else int(n_pixels)
    win = g["win"].reshape(-1, 8)
    n = 0
    for e in range(E):
        b, end = int(offsets[e]), int(offsets[e + 1])
        cap = (end - b) // 3 if b <= end <= npx else 0
        nt = min(int(tracks["n_tracks"][e]), cap)
        s = b // 3
        np.testing.assert_array_equal(win[s:s + nt], o["win"][s:s + nt], err_msg=f"windows, event {e}")
        n += int((o["win"][s:s + nt] != 0).sum())
    return n


def test_generated_events_at_batch_size(orc):
    """1000 events with UT hits, reconstructed on the GPU; windows from the
    GPU's states by the kernel and by the oracle."""
    import torch

    import paper_1912_09161_amd as velo
    b = generate("ut", 1000, workers=8)
    print(f"ut: {b.n_events} events, {len(b.ut_words)} UT words", flush=True)
    px, off = to_dev(b.pixels, b.offsets)
    out = velo.reconstruct(px, off)
    torch.cuda.synchronize()
    h = host(out)
    g = gpu_ut(b.ut_words, b.ut_offsets, b.offsets, h["tracks"], h["states"])
    o = orc.ut_windows(b.ut_words, b.ut_offsets, b.offsets, h["tracks"], h["states"])
    assert not o["status"].any()
    assert compare(g, o, b.ut_offsets, b.offsets, h["tracks"]) > 100000


def test_status_rules_next_to_good_events(orc):
    good = [word(5, 3, 0), word(7, 3, 0), word(9, 0, 3), word(8191, 13, 2), word(0, 0, 0)]
    evs = [good,
           good + [word(7, 3, 0)],
           good + [word(1, 14, 2)],
           good + [word(1, 2, 2) | 1 << 19],
           good + [word(1, 14, 2), word(5, 3, 0)],
           [word(n % 8192, n // 8192, 1) for n in range(8192)][::-1],
           [word(n % 8192, n // 8192, 1) for n in range(8193)],
           [],
           good[::-1]]
    words = np.concatenate([np.array(e, np.uint32) for e in evs])
    uo = np.concatenate([[0], np.cumsum([len(e) for e in evs])]).astype(np.uint64)
    E = len(evs)
    st, _, _ = one_track(0.0, -640.0, 0.01, 0.01)
    off = np.arange(E + 1, dtype=np.uint64) * 3
    tracks = dict(n_tracks=np.ones(E, np.uint32))
    states = {k: np.repeat(v, E) for k, v in st.items()}
    o = orc.ut_windows(words, uo, off, tracks, states)
    g = gpu_ut(words, uo, off, tracks, states)
    compare(g, o, uo, off, tracks)
    assert o["status"][5] == 0 and o["status"][6] == orc.EV_UT_OVERFLOW
    # unusable UT offsets: decreasing, beyond the buffer, below an earlier offset
    uo2 = np.array([0, 3, 2, 6, 9, 12, 100], np.uint64)
    w2 = np.array([word(n, 5, 1) for n in range(12)][::-1], np.uint32)
    tr2 = dict(n_tracks=np.ones(6, np.uint32))
    st2 = {k: np.repeat(v, 6) for k, v in st.items()}
    off2 = np.arange(7, dtype=np.uint64) * 3
    o2 = orc.ut_windows(w2, uo2, off2, tr2, st2)
    g2 = gpu_ut(w2, uo2, off2, tr2, st2)
    compare(g2, o2, uo2, off2, tr2)
    assert list(o2["status"]) == [0, 32, 32, 0, 0, 32]


def dense_cases():
    """One-track events over dense strips of every plane, the track placed at
    several slopes and rows (as in the oracle's pins), with counts above the
    event's slots and a track that is not accepted."""
    from test_oracle_ut import UT_SECTOR_MM, UT_Y0_MM, UT_Z_MM
    evs = []
    for k in range(4):
        for tx, ty in ((0.013, 0.0412), (-0.05, -0.1013), (0.0021, 0.1605)):
            x0, z0 = 0.3, -11.0
            zk = UT_Z_MM[k]
            sec = int((ty * (zk - z0) - UT_Y0_MM) // UT_SECTOR_MM)
            y0 = float(np.float32(UT_Y0_MM + (sec + 0.5) * UT_SECTOR_MM + 13.7 - ty * (zk - z0)))
            evs.append((dense(k, sec), (x0, y0, tx, ty, z0, 1)))
    rows = np.concatenate([dense(0, 3, 3800, 4400), dense(0, 4, 3800, 4400)])
    for y in (-310.0, -290.0, -310.01, -350.0, -715.0):
        evs.append((rows, (10.0, y, 0.0, 0.0, 0.0, 1)))
    evs.append((rows, (10.0, -310.0, 0.0, 0.0, 0.0, 0)))
    return evs


@pytest.mark.parametrize("tol_u", [1.0, 0.0])
def test_dense_windows_and_rows(orc, tol_u):
    evs = dense_cases()
    words = np.concatenate([w for w, _ in evs])
    uo = np.concatenate([[0], np.cumsum([len(w) for w, _ in evs])]).astype(np.uint64)
    E = len(evs)
    st = {k: np.array([t[i] for _, t in evs], np.float32) for i, k in enumerate(("x", "y", "tx", "ty", "z"))}
    st["accepted"] = np.array([t[5] for _, t in evs], np.uint8)
    # one track slot per event (3 words each), event 2 claims more than it owns
    off = np.arange(E + 1, dtype=np.uint64) * 3
    tracks = dict(n_tracks=np.ones(E, np.uint32))
    tracks["n_tracks"][2] = 5
    o = orc.ut_windows(words, uo, off, tracks, st, orc.ut_params(tol_u=tol_u))
    g = gpu_ut(words, uo, off, tracks, st, tol_u=tol_u)
    assert compare(g, o, uo, off, tracks) >= 12


def test_edges_exactly_on_strip_centres(orc):
    f = np.float32
    w = f(f(f(45.0) / f(3000.0)) * f(f(2327.5) - f(1000.0))) * f(1.0) + f(1.0)
    evs = []
    for n in range(3000, 5000):
        u = f(strip_u(n))
        for side in (-1, 1):
            x = f(u - w) if side > 0 else f(u + w)
            edge = f(x + w) if side > 0 else f(x - w)
            if edge == u:
                evs.append((dense(0, 7, n - 300, n + 300), float(x)))
        if len(evs) >= 24:
            break
    words = np.concatenate([d for d, _ in evs])
    uo = np.concatenate([[0], np.cumsum([len(d) for d, _ in evs])]).astype(np.uint64)
    E = len(evs)
    states = dict(x=np.array([x for _, x in evs], np.float32), y=np.full(E, 50.0, np.float32),
                  z=np.zeros(E, np.float32), tx=np.zeros(E, np.float32), ty=np.zeros(E, np.float32),
                  accepted=np.ones(E, np.uint8))
    off = np.arange(E + 1, dtype=np.uint64) * 3
    tracks = dict(n_tracks=np.ones(E, np.uint32))
    o = orc.ut_windows(words, uo, off, tracks, states)
    g = gpu_ut(words, uo, off, tracks, states)
    assert compare(g, o, uo, off, tracks) == E
