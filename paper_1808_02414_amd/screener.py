"""Learned covariance screener: training and screening on the GPU.

A network predicts each camera's 9x9 covariance from 55 features, as the
log-Cholesky factor of the covariance normalised per camera by its
block-diagonal estimate (Z_ii)^-1 and a training-set scale; cameras whose
predicted spread (trace of the normalised covariance) exceeds a threshold
fall back to the exact computation.  Every numeric step runs in the
library's kernels: features (``ucov_screener_features``), the network's
forward, gradient and Adam steps (``ucov_mlp_*``), the statistics that
standardise inputs and outputs (``ucov_screener_stats``), the label
transforms (``ucov_screener_labels`` / ``ucov_screener_covariance``) and the
screener file (``ucov_screener_save`` / ``ucov_screener_load``).  This module
holds the training loop: the learning-rate schedule and the sample order.

The exact covariances that label the training set come from
``Context.camera_covariance`` and remain the reference for the network's error.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from ._binding import N_FEATURES, N_OUTPUTS, Context, DeviceScene


def training_set(ctx: Context, scenes):
    """Features (n, 55) float32 and exact covariances (n, 9, 9) float64 of
    every camera of ``scenes`` (host ``scenegen.Scene`` objects or
    ``DeviceScene``), concatenated on the device."""
    torch = ctx.torch
    feats, covs = [], []
    for s in scenes:
        d = s if isinstance(s, DeviceScene) else DeviceScene.from_scene(s)
        feats.append(ctx.screener_features(d))
        cov, _ = ctx.camera_covariance(d)
        covs.append(cov)
    return torch.cat(feats), torch.cat(covs)


@dataclasses.dataclass
class Screener:
    params: object      # (P,) float32, device
    in_mean: object     # (55,) float32
    in_std: object      # (55,) float32
    scale: object       # (9,) float64: per-parameter training-set scale
    out_mean: object    # (45,) float32
    out_std: object     # (45,) float32
    adam_m: object = None   # (P,) float32 Adam moments, to resume training
    adam_v: object = None
    step: int = 0           # Adam steps taken

    def predict(self, ctx: Context, features):
        """Predicted covariances (n, 9, 9) and spreads (n,) for features (n, 55)."""
        y = ctx.mlp_forward(self.params, features, self.in_mean, self.in_std)
        return ctx.screener_covariance(y, features, self.scale, self.out_mean, self.out_std)

    def screen(self, ctx: Context, scene: DeviceScene, threshold: float):
        """Covariances of every camera of ``scene``: the network's where the
        predicted spread is at most ``threshold``, the exact ones elsewhere
        (computed only when some camera falls back).  Returns the blocks, the
        spreads and the fallback mask."""
        feats = ctx.screener_features(scene)
        cov, spread = self.predict(ctx, feats)
        # a spread that is not a number (a network output out of range) also
        # falls back
        fallback = ~(spread <= threshold)
        if bool(fallback.any()):
            exact, _ = ctx.camera_covariance(scene)
            cov[fallback] = exact[fallback]
        return cov, spread, fallback

    def tensors(self):
        names = ("params", "in_mean", "in_std", "scale", "out_mean", "out_std", "adam_m", "adam_v")
        return {k: getattr(self, k) for k in names if getattr(self, k) is not None}

    def save(self, ctx: Context, path: str):
        """Write the screener file (``ucov_screener_save``), Adam state included
        when the screener carries it."""
        ctx.screener_save(path, self.tensors(), self.step)

    @classmethod
    def load(cls, ctx: Context, path: str, adam: bool = False, device="cuda"):
        t, step = ctx.screener_load(path, adam=adam, device=device)
        return cls(step=step, **t)


def fit(ctx: Context, features, covs, init, epochs: int = 30, batch: int = 512,
        lr: float = 2e-3, lr_final: float = 1e-4, seed: int = 0, log=None):
    """Train a screener on features (n, 55) and exact covariances (n, 9, 9).

    ``init`` holds the initial parameters (ucov_mlp_param_count() values, e.g.
    He-normal weights and zero biases).  The learning rate decays
    geometrically from ``lr`` to ``lr_final``; each epoch visits the samples
    in a seeded random order.  Returns the screener and the mean loss of each
    epoch.
    """
    torch = ctx.torch
    dev = features.device
    P = ctx.mlp_param_count()
    params = torch.as_tensor(np.asarray(init), dtype=torch.float32).to(dev).contiguous()
    assert params.numel() == P, (params.numel(), P)
    covs = covs.contiguous()
    features = features.contiguous()
    in_mean, in_std, scale, out_mean, out_std = ctx.screener_stats(features, covs)
    labels = ctx.screener_labels(covs, features, scale, out_mean, out_std)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    gen = torch.Generator(device="cpu").manual_seed(seed)
    n = features.shape[0]
    step = 1
    history = []
    for ep in range(epochs):
        rate = lr * (lr_final / lr) ** (ep / max(1, epochs - 1))
        perm = torch.randperm(n, generator=gen).to(dev)
        x = features[perm].contiguous()
        t = labels[perm].contiguous()
        losses = ctx.mlp_train(params, m, v, step, rate, batch, x, t, in_mean, in_std)
        step += losses.numel()
        history.append(float(losses.mean().item()))
        if log:
            log(f"epoch {ep}: lr {rate:.2e} loss {history[-1]:.4f}")
    return Screener(params, in_mean, in_std, scale, out_mean, out_std, m, v, step - 1), history


__all__ = ["Screener", "fit", "training_set", "N_FEATURES", "N_OUTPUTS"]
