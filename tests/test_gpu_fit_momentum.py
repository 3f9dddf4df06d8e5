"""GPU parity of the fit with a measured momentum (velo_fit_momentum, Sec.
2.3.5) with the oracle.

Both sides evaluate the same binary32 filter in the same order, so states
agree within the fit's bar (1e-4 relative plus small floors) and ndof and
the cut decisions exactly.  Inputs: the benchmark's batch size of events
whose scattering follows each particle's momentum, reconstructed on the GPU,
with the generator's momentum of the matched particle in each track slot;
and the same tracks with momenta at the limits (very low and very high,
zero, negative, infinite, NaN: the last four fall back to the plain fit).
"""
import numpy as np
import pytest

from gpu_helpers import compare_states, host, to_dev
from synth import generate
from synth.truth import Truth, match_tracks, track_list

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def momenta_of_tracks(b, h):
    """The generator's momentum of the particle each track matches (0 for
    ghosts), per track slot."""
    T = Truth(b)
    ev, slot, nh, keys = track_list(h["tracks"], h["hits"], b.offsets)
    m = match_tracks(T, ev, nh, keys)
    first = b.part_off[:-1].astype(np.int64)
    pm = np.zeros(len(h["tracks"]["nhits"]), np.float32)
    ok = m >= 0
    pm[slot[ok]] = b.part["p"][first[ev[ok]] + m[ok]]
    return pm, slot


@pytest.mark.parametrize("mode", ["truth", "limits"])
def test_momentum_fit_equals_oracle(orc, mode):
    import torch

    import paper_1912_09161_amd as velo
    b = generate("momentum", 1000, workers=8)
    print(f"momentum: {b.n_events} events, {b.n_pixels} words, {mode}", flush=True)
    px, off = to_dev(b.pixels, b.offsets)
    out = velo.reconstruct(px, off)
    torch.cuda.synchronize()
    h = host(out)
    pm, slot = momenta_of_tracks(b, h)
    if mode == "limits":
        rng = np.random.default_rng(3)
        choice = np.array([20.0, 150.0, 1e6, 1e9, 0.0, -5.0, np.inf, np.nan, -np.inf, 3.0e38], np.float32)
        pm[slot] = choice[rng.integers(0, len(choice), len(slot))]
    st = velo.fit_momentum(out["hits"], out["tracks"], off, b.n_pixels,
                           torch.from_numpy(pm).cuda())
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in st.items()}
    g["cov_x"] = g["cov_x"].reshape(-1, 3)
    g["cov_y"] = g["cov_y"].reshape(-1, 3)
    o = orc.fit_momentum(h["hits"], h["tracks"], b.offsets, pm)
    assert compare_states(g, o, b.offsets, h["tracks"]) > 150000
    # the fallback tracks equal the plain fit exactly
    if mode == "limits":
        fb = slot[~((pm[slot] > 0) & np.isfinite(pm[slot]))]
        for k in ("x", "y", "z", "tx", "ty", "chi2"):
            np.testing.assert_array_equal(g[k][fb].view(np.uint32), h["states"][k][fb].view(np.uint32), err_msg=k)
    else:
        # a measured momentum changes the states of low-momentum tracks
        low = slot[(pm[slot] > 0) & (pm[slot] < 2000)]
        assert len(low) > 1000
        assert (g["cov_x"][low, 2] != h["states"]["cov_x"][low, 2]).mean() > 0.99
