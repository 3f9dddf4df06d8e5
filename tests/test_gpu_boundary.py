"""GPU tests of the boundary's service calls: the synchronous status check
(velo_check_status) and the classifier held by a batched-form context
(velo_mlp_load / velo_mlp_save / velo_mlp_train_step, and its use by
velo_reconstruct_batched when the call names no classifier)."""
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


def test_check_status():
    import torch

    import paper_1912_09161_amd as velo
    from synth.raw import line_event, pack, word
    good = line_event([(0.02 * 600, 0.015 * 600, 0.02, 0.015)])
    px, off = pack([good, good + [word(2, 20, 20, 3)], good, [word(0, 768, 768, 3)]])
    dpx, doff = to_dev(px, off)
    out = velo.reconstruct(dpx, doff)
    rc, bits = velo.check_status(out["hits"]["status"], out["tracks"]["status"])
    assert rc == 2 and bits == velo.EV_LAYER_ORDER | velo.EV_HOLE
    px, off = pack([good, good])
    dpx, doff = to_dev(px, off)
    out = velo.reconstruct(dpx, doff)
    assert velo.check_status(out["hits"]["status"], out["tracks"]["status"]) == (0, 0)
    torch.cuda.synchronize()


def test_context_classifier_load_train_save_and_use():
    import torch

    import paper_1912_09161_amd as velo
    from paper_1912_09161_amd import learn
    from synth.truth import Truth, track_labels
    b = generate("nominal", 200, first_event=9000, workers=8)
    px, off = to_dev(b.pixels, b.offsets)
    out = velo.reconstruct(px, off)
    feat = velo.track_features(out["hits"], out["tracks"], out["states"], off, b.n_pixels)
    torch.cuda.synchronize()
    h = host(out)
    slot, lab, _, _ = track_labels(Truth(b), h["tracks"], h["hits"], b.offsets)
    F = feat[torch.from_numpy(slot).cuda()].contiguous()
    L = torch.from_numpy(lab).cuda()
    mean, std = velo.feature_stats(F)
    p0 = learn.he_uniform(11)
    ctx = velo.Context()
    ctx.mlp_load(velo.mlp_blob(p0, mean.cpu().numpy(), std.cpu().numpy(), 0.25))
    # the same steps through the stand-alone kernels
    P = torch.from_numpy(p0).cuda()
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    rng = np.random.default_rng(5)
    n = min(4096, F.shape[0])
    for step in range(1, 6):
        idx = torch.from_numpy(rng.permutation(F.shape[0])[:n].astype(np.int32)).cuda()
        g, _ = velo.mlp_fwd_bwd(P, mean, std, F, L, n, idx=idx)
        velo.mlp_adam_step(P, m, v, g, step, 1e-3)
        ctx.mlp_train_step(F, L, n, 1e-3, step, idx=idx)
    torch.cuda.synchronize()
    pc, mc, sc, thr = velo.parse_mlp_blob(ctx.mlp_save())
    np.testing.assert_array_equal(pc.view(np.uint32), P.cpu().numpy().view(np.uint32))
    np.testing.assert_array_equal(mc, mean.cpu().numpy())
    assert thr == np.float32(0.25)
    # the context applies its own classifier when the call names none
    ref = host(velo.reconstruct_mlp(px, off, velo.Mlp(P, mean, std, 0.25)))
    g = host(ctx.reconstruct(px, off))
    torch.cuda.synchronize()
    from gpu_helpers import track_slots
    sl = track_slots(ref["tracks"], b.offsets)
    for k in ("score", "accepted", "x", "tx"):
        np.testing.assert_array_equal(g["states"][k][sl], ref["states"][k][sl], err_msg=k)
    ctx.close()
