"""Training and working point of the learned track-quality classifier.

Orchestration only: every forward, backward, optimiser, statistics and
inference step runs in libvelo's kernels (velo_mlp_fwd_bwd,
velo_mlp_adam_step, velo_feature_stats, velo_mlp_infer); this module draws
the seeded initial weights and minibatch permutations on the host and keeps
the checkpoint format.

Training set: tracks produced by the method itself (velo_reconstruct on
simulated events) with their raw features (velo_track_features) and a label
1 for tracks matched to a simulated particle (clones included), 0 for ghosts;
the caller supplies the labels from its generator truth.
"""
from __future__ import annotations

import io
import json

import numpy as np
import torch

from . import velo

CHECKPOINT_VERSION = 1


def he_uniform(seed: int) -> np.ndarray:
    """He-uniform weights (bound sqrt(6 / fan_in)) and zero biases, float32 [1377]."""
    rng = np.random.default_rng(seed)
    p = np.zeros(velo.N_PARAMS, np.float32)
    p[0:256] = rng.uniform(-1, 1, 256) * np.sqrt(6 / 8)
    p[288:1312] = rng.uniform(-1, 1, 1024) * np.sqrt(6 / 32)
    p[1344:1376] = rng.uniform(-1, 1, 32) * np.sqrt(6 / 32)
    return p


class Trainer:
    """Adam (lr 1e-3, betas 0.9 / 0.999, eps 1e-8) on minibatches of the mean
    binary cross-entropy; features standardised with the training set's mean
    and standard deviation."""

    def __init__(self, feat: torch.Tensor, label: torch.Tensor, seed: int = 0, lr: float = 1e-3,
                 batch: int = 4096, mean=None, std=None, ghost_weight: float = 1.0):
        assert feat.dtype == torch.float32 and feat.dim() == 2 and feat.shape[1] == velo.N_FEATURES
        self.feat = feat.contiguous()
        self.label = label.to(torch.float32).contiguous()
        self.n = feat.shape[0]
        self.dev = feat.device
        self.lr = lr
        self.batch = batch
        if mean is None:
            mean, std = velo.feature_stats(self.feat)
        self.mean, self.std = mean, std
        self.params = torch.from_numpy(he_uniform(seed)).to(self.dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self.rng = np.random.default_rng(seed + 1)
        # an epoch visits every track once and every ghost (label 0) about
        # ghost_weight times: the rare class weighted by repetition, which in
        # expectation is the loss with weight ghost_weight on ghosts
        self.rows = np.arange(self.n, dtype=np.int32)
        reps = int(round(ghost_weight)) - 1
        if reps > 0:
            ghosts = np.nonzero(self.label.cpu().numpy() == 0)[0].astype(np.int32)
            self.rows = np.concatenate([self.rows] + [ghosts] * reps)
        self.ws = velo.mlp_workspace(batch, self.dev)
        self.grad = torch.empty(velo.N_PARAMS, dtype=torch.float32, device=self.dev)
        self.loss = torch.empty(1, dtype=torch.float32, device=self.dev)

    def epoch(self) -> float:
        perm = torch.from_numpy(self.rng.permutation(self.rows).astype(np.int32)).to(self.dev)
        losses = []
        for b0 in range(0, perm.numel(), self.batch):
            idx = perm[b0:b0 + self.batch]
            nb = idx.numel()
            velo.mlp_fwd_bwd(self.params, self.mean, self.std, self.feat, self.label, nb, idx=idx,
                             grad=self.grad, loss=self.loss, ws=self.ws)
            self.step += 1
            velo.mlp_adam_step(self.params, self.m, self.v, self.grad, self.step, self.lr)
            losses.append(self.loss.clone())
        return float(torch.stack(losses).mean().item())

    def mlp(self, threshold: float = 0.0) -> velo.Mlp:
        return velo.Mlp(self.params, self.mean, self.std, threshold)

    # checkpoint: weights, statistics, optimiser state and the permutation rng
    def state(self) -> dict:
        return dict(version=CHECKPOINT_VERSION, params=self.params.cpu().numpy(),
                    m=self.m.cpu().numpy(), v=self.v.cpu().numpy(), step=self.step,
                    mean=self.mean.cpu().numpy(), std=self.std.cpu().numpy(), lr=self.lr,
                    batch=self.batch, rng=json.dumps(self.rng.bit_generator.state))

    def load_state(self, st: dict):
        assert int(st["version"]) == CHECKPOINT_VERSION
        f = lambda a: torch.from_numpy(np.asarray(a, np.float32)).to(self.dev)  # noqa: E731
        self.params, self.m, self.v = f(st["params"]), f(st["m"]), f(st["v"])
        self.mean, self.std = f(st["mean"]), f(st["std"])
        self.step = int(st["step"])
        self.lr = float(st["lr"])
        self.batch = int(st["batch"])
        self.rng.bit_generator.state = json.loads(str(st["rng"]))


def save_checkpoint(path, trainer: Trainer, threshold: float | None = None):
    st = trainer.state()
    st["threshold"] = np.nan if threshold is None else threshold
    np.savez(path, **st)


def load_checkpoint(path) -> dict:
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


def choose_threshold(logit: np.ndarray, particle: np.ndarray, reconstructible: np.ndarray,
                     target_eff: float) -> float:
    """Largest logit threshold whose efficiency is at least target_eff.

    logit[t]: classifier output of track t; particle[t]: unique id of the
    particle the track is matched to, or -1; reconstructible: unique ids of
    the reconstructible particles.  A particle counts as found when one of its
    matched tracks is accepted, so it is found at threshold c iff its best
    matched logit is >= c.  The result is always a finite binary32 value: if
    no threshold reaches target_eff, the one of the highest reachable
    efficiency; if any does (target <= 0), the largest finite value."""
    f32 = np.finfo(np.float32)
    reco = np.unique(reconstructible)
    n_reco = len(reco)
    m = particle >= 0
    best = {}
    for p, z in zip(particle[m].tolist(), logit[m].tolist()):
        if p not in best or z > best[p]:
            best[p] = z
    vals = np.sort(np.array([best[p] for p in reco.tolist() if p in best], np.float64))[::-1]
    need = int(np.ceil(target_eff * n_reco - 1e-9))
    if need <= 0:
        return float(f32.max)
    if len(vals) == 0:
        return float(f32.min)
    return float(np.float32(vals[min(need, len(vals)) - 1]))
