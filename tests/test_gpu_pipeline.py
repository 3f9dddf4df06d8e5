"""GPU test of the streaming form (velo_pipeline_run): raw events from host
memory through several host-thread / stream pairs, global event cut on the
host, compact tracks and vertices back.

Every event's rows must equal, bit for bit, the states velo_reconstruct and
velo_find_pvs give for the same event in an ordinary batch (results of an
event do not depend on its batch), and its track count and status must
equal the oracle's; events above the cut and events with unusable offsets
are flagged and not processed.
"""
import numpy as np
import pytest

from gpu_helpers import host, to_dev
from synth import generate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def reference(b, sel):
    """velo_reconstruct + velo_find_pvs of the selected events in one batch."""
    import torch

    import paper_1912_09161_amd as velo
    s = b.select(sel)
    px, off = to_dev(s.pixels, s.offsets)
    out = velo.reconstruct(px, off)
    pv = velo.find_pvs(out["tracks"], out["states"], off, s.n_pixels)
    torch.cuda.synchronize()
    return s, host(out), {k: v.cpu().numpy() for k, v in pv.items()}


@pytest.mark.parametrize("streams,events", [(1, 1000), (3, 96), (4, 37)])
def test_pipeline_equals_batch_reconstruction(orc, streams, events):
    import paper_1912_09161_amd as velo
    b = generate("nominal", 600, first_event=6000, workers=8)
    sizes = np.diff(b.offsets.astype(np.int64))
    gec = int(np.percentile(sizes, 90))
    print(f"pipeline: {streams} streams, {events} events per batch, cut {gec} words", flush=True)
    p = velo.Pipeline(streams, events, 1_500_000, gec_max_words=gec)
    r = p.run(b.pixels, b.offsets)
    p.close()
    cut = sizes > gec
    assert cut.sum() > 30
    np.testing.assert_array_equal(r["status"][cut], velo.EV_GEC)
    assert not r["n_tracks"][cut].any()
    sel = np.nonzero(~cut)[0]
    s, g, pv = reference(b, sel)
    o = orc.reconstruct(s.pixels, s.offsets, threads=8)
    np.testing.assert_array_equal(r["status"][sel], g["hits"]["status"] | g["tracks"]["status"]
                                  | pv["status"].view(np.uint32))
    np.testing.assert_array_equal(r["n_tracks"][sel], o["tracks"]["n_tracks"])
    np.testing.assert_array_equal(r["n_tracks"][sel], g["tracks"]["n_tracks"])
    assert len(r["tracks"]) == int(g["tracks"]["n_tracks"].sum())
    base = (s.offsets[:-1] // 3).astype(np.int64)
    st = g["states"]
    for i, ev in enumerate(sel):
        n = int(r["n_tracks"][ev])
        rows = r["tracks"][int(r["first_track"][ev]):int(r["first_track"][ev]) + n]
        sl = base[i] + np.arange(n)
        for k in ("x", "y", "z", "tx", "ty", "chi2"):
            np.testing.assert_array_equal(rows[k].view(np.uint32), st[k][sl].view(np.uint32), err_msg=k)
        np.testing.assert_array_equal(rows["ndof"], st["ndof"][sl])
        np.testing.assert_array_equal(rows["accepted"], st["accepted"][sl])
        np.testing.assert_array_equal(rows["nhits"], g["tracks"]["nhits"][sl])
        k = int(pv["n_pv"][i])
        assert r["n_pv"][ev] == k
        np.testing.assert_array_equal(r["pv_z"][ev, :k].view(np.uint32),
                                      pv["z"][i * 64:i * 64 + k].view(np.uint32))


def test_pipeline_flags_bad_offsets_and_oversized_events():
    import paper_1912_09161_amd as velo
    from synth.raw import bad_offsets_case
    b, cases = bad_offsets_case()
    offs, exp = cases["descent"]
    p = velo.Pipeline(2, 2, 10_000)
    r = p.run(b.pixels, np.array(offs, np.uint64))
    np.testing.assert_array_equal(r["status"], np.array(exp, np.uint32))
    assert r["n_tracks"][0] > 0 and not r["n_tracks"][1:].any()
    # an event larger than a batch's words is cut like an event above the GEC
    p2 = velo.Pipeline(1, 4, 100)
    r2 = p2.run(b.pixels, b.offsets)
    assert (r2["status"] == velo.EV_GEC).all()
    p.close()
    p2.close()
