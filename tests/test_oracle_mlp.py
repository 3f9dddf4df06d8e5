"""Pins of the oracle's learned track-quality classifier.

References independent of the oracle's code: central finite differences of
its own loss (the analytic backward pass must agree), closed forms of tiny
networks, torch's bfloat16 conversion (round to nearest even) for the
inference-precision emulation, and features recomputed from their definition
on tracks with known hits.
"""
import numpy as np
import pytest
import torch

N = 1377


def he_init(rng):
    p = np.zeros(N)
    p[0:256] = rng.uniform(-1, 1, 256) * np.sqrt(6 / 8)
    p[256:288] = rng.normal(0, 0.1, 32)
    p[288:1312] = rng.uniform(-1, 1, 1024) * np.sqrt(6 / 32)
    p[1312:1344] = rng.normal(0, 0.1, 32)
    p[1344:1376] = rng.uniform(-1, 1, 32) * np.sqrt(6 / 32)
    p[1376] = 0.3
    return p


def test_gradient_matches_central_differences(orc):
    rng = np.random.default_rng(3)
    p = he_init(rng)
    g = rng.normal(0, 1, (40, 8))
    y = (rng.random(40) < 0.3).astype(float)
    loss, grad = orc.mlp_fwd_bwd(p, g, y)
    h = 1e-6
    idx = np.concatenate([rng.choice(256, 40, replace=False), np.arange(256, 288),
                          288 + rng.choice(1024, 80, replace=False), np.arange(1312, 1377)])
    for i in idx:
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        fd = (orc.mlp_fwd_bwd(pp, g, y)[0] - orc.mlp_fwd_bwd(pm, g, y)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(abs(fd), abs(grad[i])) + 1e-9, (i, fd, grad[i])


def test_zero_network_closed_form(orc):
    rng = np.random.default_rng(4)
    g = rng.normal(0, 1, (25, 8))
    y = (rng.random(25) < 0.5).astype(float)
    loss, grad = orc.mlp_fwd_bwd(np.zeros(N), g, y)
    assert abs(loss - np.log(2)) < 1e-12
    # only the output bias moves: d/db3 = mean(sigmoid(0) - y)
    assert abs(grad[1376] - np.mean(0.5 - y)) < 1e-12
    assert np.all(grad[:1376] == 0)


def test_single_path_network_closed_form(orc):
    """W1 routes feature 2 to unit 0, W2 copies unit 0, w3 reads it: z = max(x2, 0)
    + b3; the loss for label y is softplus(z) - y z."""
    p = np.zeros(N)
    p[0 * 8 + 2] = 1.0      # W1[0][2]
    p[288 + 0 * 32 + 0] = 1.0  # W2[0][0]
    p[1344 + 0] = 1.0       # w3[0]
    p[1376] = -0.25
    g = np.zeros((6, 8))
    g[:, 2] = [-2.0, -0.1, 0.0, 0.3, 1.7, 4.0]
    z = orc.mlp_forward(p, g)
    np.testing.assert_allclose(z, np.maximum(g[:, 2], 0) - 0.25, rtol=0, atol=1e-15)
    y = np.array([0, 1, 0, 1, 1, 0], float)
    loss, _ = orc.mlp_fwd_bwd(p, g, y)
    ref = np.mean(np.logaddexp(0, z) - y * z)
    assert abs(loss - ref) < 1e-12


def test_bf16_emulation_matches_torch_rounding_and_double_forward(orc):
    rng = np.random.default_rng(5)
    p = he_init(rng).astype(np.float32)
    mean = rng.normal(0, 1, 8).astype(np.float32)
    std = rng.uniform(0.5, 3, 8).astype(np.float32)
    f = (mean + std * rng.normal(0, 1, (500, 8))).astype(np.float32)
    z16 = orc.mlp_forward_bf16(p, mean, std, f)
    # independent re-evaluation with torch's bfloat16 rounding
    bf = lambda a: torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()  # noqa: E731
    g = bf(((f - mean) / std).astype(np.float32))
    W1 = bf(p[0:256].reshape(32, 8)); b1 = p[256:288].astype(np.float64)
    W2 = bf(p[288:1312].reshape(32, 32)); b2 = p[1312:1344].astype(np.float64)
    w3 = bf(p[1344:1376]); b3 = float(p[1376])
    h1 = bf(np.maximum((g @ W1.T).astype(np.float32) + b1.astype(np.float32), 0).astype(np.float32))
    h2 = bf(np.maximum((h1 @ W2.T).astype(np.float32) + b2.astype(np.float32), 0).astype(np.float32))
    zt = (h2 @ w3).astype(np.float32) + np.float32(b3)
    np.testing.assert_allclose(z16, zt, rtol=1e-5, atol=1e-5)
    # and it stays within the inference tolerance of the double-precision network
    zd = orc.mlp_forward(p.astype(np.float64), (f.astype(np.float64) - mean) / std)
    assert np.all(np.abs(z16 - zd) <= 2e-2 * (1 + np.abs(zd)))


def test_features_from_definition(orc):
    from synth import generate
    b = generate("nominal", 6)
    r = orc.reconstruct(b.pixels, b.offsets)
    F = orc.features(r["hits"], r["tracks"], r["states"], b.offsets)
    base = (b.offsets[:-1] // 3).astype(int)
    for e in range(b.n_events):
        for t in range(int(r["tracks"]["n_tracks"][e])):
            s = base[e] + t
            n = int(r["tracks"]["nhits"][s])
            keys = r["hits"]["key"][int(b.offsets[e]) + r["tracks"]["hit_idx"][s, :n]]
            lay = keys >> 22
            tx, ty = float(r["states"]["tx"][s]), float(r["states"]["ty"][s])
            want = [r["states"]["chi2"][s] / r["states"]["ndof"][s], n, (lay[0] - lay[-1] + 1) - n,
                    tx, ty, np.arcsinh(1 / np.hypot(tx, ty)),
                    -280 + 1030 * lay[0] / 25, -280 + 1030 * lay[-1] / 25]
            np.testing.assert_allclose(F[s], want, rtol=1e-6, atol=1e-4)
