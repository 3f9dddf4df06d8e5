"""GPU tests of the learned track classifier against the CPU oracle.

Bars: features within 1e-6 relative (binary32 vs double); FP32 gradients
within 1e-4 of the double-precision oracle (relative to the gradient's
largest component); BF16 inference vs the oracle's emulation of the same
precision within 1e-3 (1 + |logit|) and vs the double-precision network
within 2e-2 (1 + |logit|); accept decisions identical except for logits
within 1e-3 (1 + |threshold|) of the threshold; the fused fit+classifier
equal to the separate fit and inference.  The gain test trains the network
on the GPU and requires equal-or-better efficiency with a ghost rate at
least 20 % below the plain chi2/hit-count cut on held-out events.
"""
import numpy as np
import pytest

from gpu_helpers import host
from synth import generate
from synth.truth import Truth, efficiency_ghosts, track_labels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def reco(b, xl=5.94e-4):
    import torch

    import paper_1912_09161_amd as velo
    px = torch.from_numpy(b.pixels.view(np.int32)).cuda()
    off = torch.from_numpy(b.offsets.view(np.int64)).cuda()
    P = velo.default_params(x_over_x0=xl)
    out = velo.reconstruct(px, off, params=P)
    feat = velo.track_features(out["hits"], out["tracks"], out["states"], off, b.n_pixels)
    torch.cuda.synchronize()
    return dict(px=px, off=off, out=out, feat=feat, P=P, h=host(out), b=b)


def labelled(d):
    slot, lab, uid, rec = track_labels(Truth(d["b"]), d["h"]["tracks"], d["h"]["hits"], d["b"].offsets)
    return slot, lab, uid, rec


def test_features_match_oracle(orc):
    b = generate("nominal", 40)
    d = reco(b)
    F = d["feat"].cpu().numpy()
    ref = orc.features(d["h"]["hits"], d["h"]["tracks"], d["h"]["states"], b.offsets)
    slot, *_ = labelled(d)
    np.testing.assert_allclose(F[slot], ref[slot], rtol=1e-6, atol=1e-6)


def test_gradients_match_oracle(orc):
    import torch

    import paper_1912_09161_amd as velo
    from paper_1912_09161_amd import learn
    b = generate("nominal", 40)
    d = reco(b)
    slot, lab, *_ = labelled(d)
    F = d["feat"][torch.from_numpy(slot).cuda()].contiguous()
    Y = torch.from_numpy(lab).cuda()
    mean, std = velo.feature_stats(F)
    Fh = F.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(mean.cpu().numpy(), Fh.mean(0), rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(std.cpu().numpy(), Fh.std(0), rtol=1e-4, atol=1e-6)
    p = learn.he_uniform(11)
    p[256:288] = np.random.default_rng(1).normal(0, 0.2, 32)
    P = torch.from_numpy(p).cuda()
    idx = torch.from_numpy(np.random.default_rng(2).permutation(len(slot))[:3000].astype(np.int32)).cuda()
    grad, loss = velo.mlp_fwd_bwd(P, mean, std, F, Y, idx.numel(), idx=idx)
    torch.cuda.synchronize()
    sel = idx.cpu().numpy()
    g = (Fh[sel] - mean.cpu().numpy().astype(np.float32)) / std.cpu().numpy().astype(np.float32)
    l_ref, g_ref = orc.mlp_fwd_bwd(p.astype(np.float64), g.astype(np.float32).astype(np.float64), lab[sel])
    gg = grad.cpu().numpy().astype(np.float64)
    scale = np.abs(g_ref).max()
    assert np.abs(gg - g_ref).max() <= 1e-4 * scale, np.abs(gg - g_ref).max() / scale
    assert abs(float(loss.item()) - l_ref) <= 1e-5 * (1 + l_ref)
    # deterministic: the same call gives the same bits
    grad2, _ = velo.mlp_fwd_bwd(P, mean, std, F, Y, idx.numel(), idx=idx)
    assert torch.equal(grad, grad2)


def test_adam_step():
    import torch

    import paper_1912_09161_amd as velo
    rng = np.random.default_rng(0)
    p = rng.normal(0, 1, 1377).astype(np.float32)
    m = rng.normal(0, 0.1, 1377).astype(np.float32)
    v = rng.uniform(0, 0.1, 1377).astype(np.float32)
    g = rng.normal(0, 1, 1377).astype(np.float32)
    P, M, V, G = (torch.from_numpy(a.copy()).cuda() for a in (p, m, v, g))
    velo.mlp_adam_step(P, M, V, G, step=3, lr=1e-3)
    torch.cuda.synchronize()
    m2 = 0.9 * m + 0.1 * g
    v2 = 0.999 * v + 0.001 * g.astype(np.float64) ** 2
    ref = p - 1e-3 * (m2 / (1 - 0.9 ** 3)) / (np.sqrt(v2 / (1 - 0.999 ** 3)) + 1e-8)
    np.testing.assert_allclose(P.cpu().numpy(), ref, rtol=2e-6, atol=1e-7)


def test_inference_matches_oracle_precision(orc):
    import torch

    import paper_1912_09161_amd as velo
    from paper_1912_09161_amd import learn
    b = generate("nominal", 60)
    d = reco(b)
    slot, *_ = labelled(d)
    F = d["feat"][torch.from_numpy(slot).cuda()].contiguous()
    mean, std = velo.feature_stats(F)
    rng = np.random.default_rng(4)
    p = learn.he_uniform(5)
    p[256:288] = rng.normal(0, 0.3, 32)
    p[1312:1344] = rng.normal(0, 0.3, 32)
    p[1376] = 0.7
    P = torch.from_numpy(p).cuda()
    thr = 0.4
    mlp = velo.Mlp(P, mean, std, thr)
    z = velo.mlp_infer(mlp, F).cpu().numpy()
    Fh = F.cpu().numpy()
    zb = orc.mlp_forward_bf16(p, mean.cpu().numpy(), std.cpu().numpy(), Fh)
    zd = orc.mlp_forward(p.astype(np.float64),
                         (Fh.astype(np.float64) - mean.cpu().numpy()) / std.cpu().numpy())
    assert np.all(np.abs(z - zb) <= 1e-3 * (1 + np.abs(zb))), np.abs(z - zb).max()
    assert np.all(np.abs(z - zd) <= 2e-2 * (1 + np.abs(zd)))
    near = np.abs(zb - thr) <= 1e-3 * (1 + abs(thr))
    assert np.array_equal((z >= thr)[~near], (zb >= thr)[~near])
    # the fused fit + classifier equals the separate fit and inference
    s2 = velo.fit_mlp(d["out"]["hits"], d["out"]["tracks"], d["off"], b.n_pixels, mlp, params=d["P"])
    torch.cuda.synchronize()
    sc = s2["score"].cpu().numpy()[slot]
    np.testing.assert_array_equal(sc.view(np.uint32), z.view(np.uint32))
    np.testing.assert_array_equal(s2["accepted"].cpu().numpy()[slot], (z >= thr).astype(np.uint8))
    for k in ("x", "y", "z", "tx", "ty", "chi2", "ndof"):
        np.testing.assert_array_equal(s2[k].cpu().numpy()[slot], d["h"]["states"][k][slot])


@pytest.mark.slow
def test_trained_classifier_beats_plain_cut():
    """High-occupancy events (PVs Poisson(20), noise 1e-4, 95 % hit efficiency,
    100 urad scattering), where ghosts are frequent: train on method-produced
    tracks of such events, choose the threshold on validation events for an
    efficiency 1e-4 above the plain cut's, and compare on held-out events:
    efficiency at least the plain cut's (within 1e-4, the statistical
    resolution of the sample) and a ghost rate at least 20 % lower."""
    import torch

    from paper_1912_09161_amd import learn
    import paper_1912_09161_amd as velo
    xl = 2.38e-3
    tr = reco(generate("stress", 800, workers=16), xl)
    va = reco(generate("stress", 500, first_event=2048, workers=16), xl)
    te = reco(generate("stress", 800, first_event=4096, workers=16), xl)
    slot, lab, *_ = labelled(tr)
    F = tr["feat"][torch.from_numpy(slot).cuda()].contiguous()
    T = learn.Trainer(F, torch.from_numpy(lab).cuda(), seed=7)
    losses = [T.epoch() for _ in range(12)]
    assert losses[-1] < losses[0]

    def evaluate(d):
        s, _, uid, rec = labelled(d)
        z = velo.mlp_infer(T.mlp(0.0), d["feat"][torch.from_numpy(s).cuda()].contiguous()).cpu().numpy()
        plain = efficiency_ghosts(uid, d["h"]["states"]["accepted"][s], rec)
        return z, uid, rec, plain

    z, uid, rec, plain_va = evaluate(va)
    thr = learn.choose_threshold(z, uid, rec, plain_va["efficiency"] + 1e-4)
    z, uid, rec, plain = evaluate(te)
    learned = efficiency_ghosts(uid, z >= thr, rec)
    print("plain", plain, "learned", learned, "threshold", thr)
    assert learned["efficiency"] >= plain["efficiency"] - 1e-4
    assert learned["ghost_rate"] <= 0.8 * plain["ghost_rate"]
