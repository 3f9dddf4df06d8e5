"""GPU parity of primary-vertex finding (velo_find_pvs) with the oracle.

The kernel and the oracle evaluate the same binary32 expressions in the same
order (histogram counts are integers; the fit sums run over tracks in slot
order), so given the same fitted states the outputs must agree bit for bit:
PV counts, positions, variances, weight sums and statuses.  Hand-built
states cover every rule; generated events cover the states the
reconstruction produces, at the benchmark's batch size and at high
occupancy.
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


def gpu_pvs(states, tracks, offsets, n_pixels, **kw):
    import torch

    import paper_1912_09161_amd as velo
    off = torch.from_numpy(np.ascontiguousarray(offsets, np.uint64).view(np.int64)).cuda()
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in states.items()}
    for k in ("cov_x", "cov_y"):
        dev[k] = dev[k].reshape(-1)
    tr = dict(n_tracks=torch.from_numpy(np.ascontiguousarray(tracks["n_tracks"], np.uint32).view(np.int32)).cuda())
    # the other track arrays are not read
    tr.update(nhits=tr["n_tracks"], hit_idx=tr["n_tracks"], status=tr["n_tracks"])
    out = velo.find_pvs(tr, dev, off, n_pixels, params=velo.default_pv_params(**kw))
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def compare(g, o):
    E = len(o["n_pv"])
    np.testing.assert_array_equal(g["n_pv"][:E].view(np.uint32), o["n_pv"])
    np.testing.assert_array_equal(g["status"][:E].view(np.uint32), o["status"])
    for k in ("z", "var", "weight"):
        a = g[k][:E * 64].reshape(E, 64)
        np.testing.assert_array_equal(a.view(np.uint32), o[k].view(np.uint32), err_msg=k)
    return int(o["n_pv"].sum())


def hand_cases(orc):
    from test_oracle_pv import at_bin, states_of
    evs = [
        [(10.0 + x, 0.04) for x in (0.0, 0.05, -0.05, 0.1, -0.1, 0.2, -0.2)],
        [(-0.8, 0.0004)] * 5 + [(0.0, 0.16)] + [(0.8, 0.0004)] * 5,
        at_bin(orc, 300, 4) + at_bin(orc, 302, 4),
        at_bin(orc, 300, 5) + at_bin(orc, 303, 4),
        at_bin(orc, 600, 3) + at_bin(orc, 601, 1),
        [],
        at_bin(orc, 1023, 4) + [(256.0, 0.01)] * 3 + [(255.999, 0.01)] * 2,
        [(-20.0, 0.01), (-20.3, 0.04), (-19.9, 0.02), (-20.1, 0.09), (-20.05, 0.01), (-17.0, 0.01)],
    ]
    many = []
    for k in range(70):
        many += at_bin(orc, 10 + 6 * k, 4)
    evs.append(many)
    evs.append(at_bin(orc, 500, 2049))
    evs.append(at_bin(orc, 500, 2048))
    return states_of(evs)


@pytest.mark.parametrize("kw", [{}, dict(n_iter=0, min_weight=0.0), dict(nms=1, seed_min=7, n_iter=3)])
def test_hand_built_states(orc, kw):
    st, tr, off = hand_cases(orc)
    o = orc.find_pvs(st, tr, off, orc.pv_params(**kw))
    g = gpu_pvs(st, tr, off, int(off[-1]), **kw)
    compare(g, o)
    assert o["status"][-2] == orc.EV_PV_OVERFLOW and o["status"][-3] == orc.EV_PV_OVERFLOW


@pytest.mark.parametrize("name,n,xl", [("nominal", 1000, 5.94e-4), ("stress", 150, 2.38e-3)])
def test_reconstructed_states(orc, name, n, xl):
    """PVs from the GPU's own fitted states: kernel and oracle on the same
    states; and the GPU chain's PVs against the generator's true vertices."""
    import torch

    import paper_1912_09161_amd as velo
    from synth.truth import pv_metrics
    b = generate(name, n, first_event=4000, workers=8)
    print(f"{name}: {n} events, {b.n_pixels} words", flush=True)
    px, off = to_dev(b.pixels, b.offsets)
    out = velo.reconstruct(px, off, params=velo.default_params(x_over_x0=xl))
    pv = velo.find_pvs(out["tracks"], out["states"], off, b.n_pixels)
    torch.cuda.synchronize()
    h = host(out)
    g = {k: v.cpu().numpy() for k, v in pv.items()}
    st = {k: h["states"][k] for k in ("z", "tx", "ty", "cov_x", "cov_y", "accepted")}
    o = orc.find_pvs(st, h["tracks"], b.offsets)
    assert compare(g, o) > 2 * n
    m = pv_metrics(b, o["n_pv"], o["z"], o["var"])
    assert m["efficiency"] > (0.9 if name == "nominal" else 0.75)
