"""Seeded synthetic latents for the GMM entropy coder.

This module holds input generation only: none of the coder's arithmetic.
It serves both the CPU oracle (tests) and the GPU library (tests, bench).

The paper times its coder on Kodak latents of a trained Checkerboard model
(FlashGMM, Sec. IV-B); neither the images nor the weights are available, so
seeded synthetic latents of the same shapes stand in for them: a 768x512
Kodak image at 1/16 resolution gives a 320x48x32 latent, a 4K frame a
320x135x240 latent.

Recipe for one latent of n = C*H*W elements with K components:
  1. logits (n, K) ~ Normal(0, s_logit)
  2. w = softmax(logits) in float64, stored as float32
  3. mu (n, K) ~ Normal(0, s_mu), stored as float32
  4. sigma (n, K) = exp(Uniform(ln 0.11, ln sigma_max)), stored as float32
  5. component k ~ Categorical(w): one Uniform(0,1) per element against the
     running sum of w
  6. y ~ Normal(mu_k, sigma_k) from the float32 parameters, symbol =
     clip(rint(y), lo, hi) as int32 (rint rounds half to even)
  7. parameters are returned as [K][n] planes (structure of arrays)
Batch shapes H, W ~ Uniform{a..b} are drawn first from the same generator.

Two generators implement the recipe: numpy's PCG64 (``backend="numpy"``,
bit-reproducible everywhere, used wherever the oracle checks every element)
and torch's device Philox (``backend="torch"``, used for the full-size
batched workloads whose parameters reach tens of GB).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class LatentCfg:
    name: str
    shapes: tuple            # ((C, H, W), ...) or None for a sampled batch
    K: int = 3
    lo: int = -128
    hi: int = 127
    precision: int = 16
    streams: tuple = (256,)  # per latent (fixed) or () for the rule
    s_logit: float = 1.0
    s_mu: float = 2.0
    sigma_max: float = 20.0
    seed: int = 1
    batch: int = 0           # number of latents for sampled batches
    channels: int = 0
    hw_range: tuple = (0, 0)


def streams_rule(n: int) -> int:
    """Stream count for batched latents: 64 streams per 12,288 symbols
    (about 192 symbols per stream, like the 192x16x16 latent with 256)."""
    return 64 * max(1, math.ceil(n / 12288))


CONFIGS = {
    # plain method, one 192x16x16 latent, 256 streams
    "c1": LatentCfg("c1", ((192, 16, 16),), K=3, lo=-128, hi=127, streams=(256,), seed=1),
    # plain method at the paper's scale: a Kodak latent and a 4K latent
    "c2a": LatentCfg("c2a", ((320, 48, 32),), K=3, lo=-255, hi=255, streams=(4096,), seed=2),
    "c2b": LatentCfg("c2b", ((320, 135, 240),), K=3, lo=-255, hi=255, streams=(65536,), seed=3),
    # 64 uneven latents, 192 channels, H and W uniform on 8..128
    "c3": LatentCfg("c3", None, K=3, lo=-128, hi=127, streams=(), seed=4, batch=64,
                    channels=192, hw_range=(8, 128)),
    # learned-bracket evaluation latent (4K, support as the 4K plain case)
    "c4": LatentCfg("c4", ((320, 135, 240),), K=3, lo=-255, hi=255, streams=(65536,), seed=5),
    # 256 uneven latents, K=5, wider parameters and support
    "c5": LatentCfg("c5", None, K=5, lo=-511, hi=511, streams=(), seed=7, batch=256,
                    channels=320, hw_range=(16, 135), s_logit=1.5, s_mu=4.0, sigma_max=40.0),
}
TRAIN_SEED_C4 = 6
TRAIN_SEED_C5 = 8
TRAIN_SEED_C1 = 9


@dataclass
class Latent:
    symbols: object          # int32 [n]
    weights: object          # float32 [K][n]
    means: object
    scales: object
    shape: tuple
    streams: int

    @property
    def n(self) -> int:
        return int(self.symbols.shape[0])


def batch_shapes(cfg: LatentCfg, rng_numpy=None):
    """(C, H, W) of each latent of a sampled batch (drawn first)."""
    if cfg.shapes is not None:
        return list(cfg.shapes)
    rng = rng_numpy if rng_numpy is not None else np.random.default_rng(cfg.seed)
    a, b = cfg.hw_range
    hw = rng.integers(a, b + 1, size=(cfg.batch, 2))
    return [(cfg.channels, int(h), int(w)) for h, w in hw]


def _latent_numpy(rng, n, K, lo, hi, s_logit, s_mu, sigma_max):
    logits = rng.normal(0.0, s_logit, size=(n, K))
    logits -= logits.max(axis=1, keepdims=True)
    e = np.exp(logits)
    w64 = e / e.sum(axis=1, keepdims=True)
    w = w64.astype(np.float32)
    mu = rng.normal(0.0, s_mu, size=(n, K)).astype(np.float32)
    sig = np.exp(rng.uniform(math.log(0.11), math.log(sigma_max), size=(n, K))).astype(np.float32)
    u = rng.uniform(0.0, 1.0, size=n)
    cw = np.cumsum(w64, axis=1)
    comp = np.minimum((u[:, None] >= cw).sum(axis=1), K - 1)
    rows = np.arange(n)
    y = rng.normal(0.0, 1.0, size=n) * sig[rows, comp].astype(np.float64) + mu[rows, comp]
    sym = np.clip(np.rint(y), lo, hi).astype(np.int32)
    return (sym, np.ascontiguousarray(w.T), np.ascontiguousarray(mu.T),
            np.ascontiguousarray(sig.T))


def _latent_torch(gen, device, n, K, lo, hi, s_logit, s_mu, sigma_max):
    import torch
    f64 = torch.float64
    logits = torch.randn((n, K), generator=gen, device=device, dtype=f64) * s_logit
    w64 = torch.softmax(logits, dim=1)
    del logits
    w = w64.float()
    mu = (torch.randn((n, K), generator=gen, device=device, dtype=f64) * s_mu).float()
    lu = torch.rand((n, K), generator=gen, device=device, dtype=f64)
    sig = torch.exp(math.log(0.11) + lu * (math.log(sigma_max) - math.log(0.11))).float()
    del lu
    u = torch.rand((n,), generator=gen, device=device, dtype=f64)
    cw = torch.cumsum(w64, dim=1)
    del w64
    comp = torch.clamp((u[:, None] >= cw).sum(dim=1), max=K - 1)
    del cw, u
    idx = comp[:, None]
    ms = torch.gather(mu, 1, idx).squeeze(1).double()
    ss = torch.gather(sig, 1, idx).squeeze(1).double()
    y = torch.randn((n,), generator=gen, device=device, dtype=f64) * ss + ms
    sym = torch.clamp(torch.round(y), lo, hi).to(torch.int32)
    return sym, w.t().contiguous(), mu.t().contiguous(), sig.t().contiguous()


def make_latents(cfg: LatentCfg, backend: str = "numpy", device=None, limit=None,
                 scale_hw=None):
    """All latents of a config. ``limit`` keeps only the first latents of a
    batch; ``scale_hw`` replaces a fixed shape (used for reduced test sizes).
    """
    rng = np.random.default_rng(cfg.seed)
    shapes = batch_shapes(cfg, rng)
    if scale_hw is not None:
        shapes = [scale_hw]
    if limit is not None:
        shapes = shapes[:limit]
    out = []
    if backend == "numpy":
        for (C, H, W) in shapes:
            n = C * H * W
            sym, w, mu, sig = _latent_numpy(rng, n, cfg.K, cfg.lo, cfg.hi, cfg.s_logit,
                                            cfg.s_mu, cfg.sigma_max)
            S = cfg.streams[0] if cfg.streams else streams_rule(n)
            out.append(Latent(sym, w, mu, sig, (C, H, W), S))
    elif backend == "torch":
        import torch
        gen = torch.Generator(device=device)
        gen.manual_seed(cfg.seed)
        for (C, H, W) in shapes:
            n = C * H * W
            sym, w, mu, sig = _latent_torch(gen, device, n, cfg.K, cfg.lo, cfg.hi, cfg.s_logit,
                                            cfg.s_mu, cfg.sigma_max)
            S = cfg.streams[0] if cfg.streams else streams_rule(n)
            out.append(Latent(sym, w, mu, sig, (C, H, W), S))
    else:
        raise ValueError(backend)
    return out


def random_params(rng, n, K, s_logit=1.0, s_mu=2.0, sigma_max=20.0, sigma_min=0.11):
    """Parameters only (no symbols), [K][n] float32 planes."""
    logits = rng.normal(0.0, s_logit, size=(n, K))
    logits -= logits.max(axis=1, keepdims=True)
    e = np.exp(logits)
    w = (e / e.sum(axis=1, keepdims=True)).astype(np.float32)
    mu = rng.normal(0.0, s_mu, size=(n, K)).astype(np.float32)
    sig = np.exp(rng.uniform(math.log(sigma_min), math.log(sigma_max), size=(n, K))).astype(
        np.float32)
    return (np.ascontiguousarray(w.T), np.ascontiguousarray(mu.T), np.ascontiguousarray(sig.T))


def raw_params(rng, n, K, s_logit=1.0, s_mu=2.0, sigma_max=20.0, sigma_min=0.11):
    """A network's raw outputs for the same distributions as random_params:
    weight logits ~ N(0, s_logit), means ~ N(0, s_mu), log-scales
    ~ U(ln sigma_min, ln sigma_max); [K][n] float32 planes. A few elements
    get extreme logits and log-scales (the mapping's clamps)."""
    logits = rng.normal(0.0, s_logit, size=(K, n)).astype(np.float32)
    mu = rng.normal(0.0, s_mu, size=(K, n)).astype(np.float32)
    log_s = rng.uniform(math.log(sigma_min), math.log(sigma_max), size=(K, n)).astype(np.float32)
    m = min(n, 64)
    logits[:, :m] = rng.uniform(-90.0, 90.0, size=(K, m)).astype(np.float32)
    log_s[:, :m] = rng.uniform(-12.0, 12.0, size=(K, m)).astype(np.float32)
    return logits, mu, log_s


def adversarial_params(rng, n, K):
    """Parameters at the edges of the numeric range: tiny and huge scales,
    zero and denormal-range weights, means far outside the support, ties."""
    w, mu, sig = random_params(rng, n, K)
    kinds = rng.integers(0, 8, size=n)
    for i in np.nonzero(kinds == 0)[0]:
        sig[:, i] = 1e-6
    for i in np.nonzero(kinds == 1)[0]:
        sig[:, i] = 5e3
    for i in np.nonzero(kinds == 2)[0]:
        w[:, i] = 0.0
        w[0, i] = 1.0
    for i in np.nonzero(kinds == 3)[0]:
        w[:, i] = 1e-30
        w[-1, i] = 1.0
    for i in np.nonzero(kinds == 4)[0]:
        mu[:, i] = rng.choice([-1e6, 1e6, -600.0, 600.0], size=K)
    for i in np.nonzero(kinds == 5)[0]:
        mu[:, i] = np.round(mu[:, i]) + 0.5   # means on boundaries
        sig[:, i] = 0.11
    for i in np.nonzero(kinds == 6)[0]:
        w[:, i] = np.float32(1.0 / K) * 1.000001   # sum slightly above one
    for i in np.nonzero(kinds == 7)[0]:
        w[0, i] = -0.5                              # outside the precondition w >= 0
    return w, mu, sig


def random_params_torch(gen, device, n, K, s_logit=1.0, s_mu=2.0, sigma_max=20.0,
                        sigma_min=0.11):
    """random_params on a torch device generator: [K][n] float32 planes."""
    import torch
    f64 = torch.float64
    w = torch.softmax(torch.randn((n, K), generator=gen, device=device, dtype=f64) * s_logit,
                      dim=1).float()
    mu = (torch.randn((n, K), generator=gen, device=device, dtype=f64) * s_mu).float()
    lu = torch.rand((n, K), generator=gen, device=device, dtype=f64)
    sig = torch.exp(math.log(sigma_min) + lu * (math.log(sigma_max) - math.log(sigma_min))).float()
    return w.t().contiguous(), mu.t().contiguous(), sig.t().contiguous()
