"""Training of the decoder's learned search bracket on the GPU.

Tuples: mixture parameters drawn from a workload's distributions, a rANS
slot uniform on [0, 2^P) (the decoder's slots are uniform), and the exact
decoded symbol for that slot — the unique j with c_j <= slot < c_{j+1},
computed by the library's inverse-CDF kernel (the same function the decoder
inverts, bit-exact with the CPU reference coder).

Network and loss: D = 3K+1 features -> 64 -> ReLU -> 64 -> ReLU -> 1 with
bfloat16 weights (float32 master copy, Adam) and the Huber loss at one
symbol, all forward, backward and update steps in the library's kernels.
Features are normalised and rounded to bfloat16 exactly as the decoder's
matrix-core inference sees them.

CLI: python -m paper_2509_18815_amd.train --K 3 --lo -255 --hi 255 --out m.npz
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import time

import numpy as np
import torch

from . import api, synth


@dataclasses.dataclass
class BracketModel:
    K: int
    lo: int
    hi: int
    precision: int
    params: np.ndarray       # float32 [P] (bfloat16-rounded on load)
    in_mean: np.ndarray      # float32 [D]
    in_std: np.ndarray       # float32 [D]
    out_mean: float
    out_std: float
    radius: int = 4
    history: list = dataclasses.field(default_factory=list)

    def load(self) -> "api.Bracket":
        return api.Bracket(self.K, self.params, self.in_mean, self.in_std, self.out_mean,
                           self.out_std, self.radius)

    def save(self, path: str) -> None:
        """Plain arrays and a JSON string of the training history (loadable
        without pickling)."""
        np.savez(path, K=self.K, lo=self.lo, hi=self.hi, precision=self.precision,
                 params=self.params, in_mean=self.in_mean, in_std=self.in_std,
                 out_mean=self.out_mean, out_std=self.out_std, radius=self.radius,
                 history=np.array(json.dumps(self.history)))

    @staticmethod
    def from_file(path: str) -> "BracketModel":
        z = np.load(path, allow_pickle=False)
        hist = json.loads(str(z["history"])) if "history" in z.files else []
        return BracketModel(int(z["K"]), int(z["lo"]), int(z["hi"]), int(z["precision"]),
                            z["params"], z["in_mean"], z["in_std"], float(z["out_mean"]),
                            float(z["out_std"]), int(z["radius"]), hist)


def make_tuples(K, lo, hi, precision, n, gen, device, s_logit=1.0, s_mu=2.0, sigma_max=20.0):
    """(weights, means, scales) [K][n], slots (int32 view of uint32) and the
    exact symbol index j for each (parameters, slot)."""
    w, mu, sg = synth.random_params_torch(gen, device, n, K, s_logit, s_mu, sigma_max)
    slot = torch.randint(0, 1 << precision, (n,), generator=gen, device=device,
                         dtype=torch.int32)
    j = api.inverse_cdf(api.make_cfg(K, lo, hi, precision, 1), w, mu, sg, slot)
    return w, mu, sg, slot, j


def bracket_hits(pred, j, slot, lo, N, M, radius):
    """Per-sample hit of the decoder's bracket rule for predictions pred."""
    s = slot.to(torch.int64) & 0xFFFFFFFF
    jmin = torch.clamp(s - (M - N), min=0)
    jmax = torch.clamp(s, max=N - 1)
    jh = torch.round(torch.clamp(pred - lo, -1.0, float(N))).to(torch.int64)
    jh = torch.minimum(torch.maximum(jh, jmin), jmax)
    return (jh - j.to(torch.int64)).abs() <= radius


def init_params(D, seed):
    rng = np.random.default_rng(seed)
    H = 64
    parts = [rng.normal(0, math.sqrt(2.0 / D), size=H * D), np.zeros(H),
             rng.normal(0, math.sqrt(2.0 / H), size=H * H), np.zeros(H),
             rng.normal(0, math.sqrt(1.0 / H), size=H), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def train_bracket(K, lo, hi, precision=16, n_train=10_000_000, n_eval=262_144, epochs=6,
                  batch=8192, lr=3e-3, seed=6, s_logit=1.0, s_mu=2.0, sigma_max=20.0,
                  radius=4, device="cuda", log=None, plateau=None) -> BracketModel:
    """Trains the bracket network. With plateau, training stops before
    `epochs` once the held-out hit rate has gained less than plateau in each
    of two consecutive epochs (the learning rate follows a cosine over
    `epochs` either way)."""
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    t0 = time.perf_counter()
    n = n_train + n_eval
    w, mu, sg, slot, j = make_tuples(K, lo, hi, precision, n, gen, dev, s_logit, s_mu, sigma_max)
    D = 3 * K + 1
    raw = api.mlp_features(K, w, mu, sg, slot, precision)
    mean = raw[:n_train].mean(0)
    std = raw[:n_train].std(0).clamp_min(1e-6)
    del raw
    X = api.mlp_features(K, w, mu, sg, slot, precision, mean.contiguous(),
                         (1.0 / std).contiguous(), round_bf16=True)
    sym = (j + lo).to(torch.float32)
    out_mean = float(sym[:n_train].mean().item())
    out_std = float(sym[:n_train].std().item())
    y = ((sym - out_mean) / out_std).contiguous()
    t_data = time.perf_counter() - t0
    P = api.mlp_num_params(D)
    master = torch.from_numpy(init_params(D, seed)).to(dev)
    shadow = master.to(torch.bfloat16).to(torch.float32)
    m = torch.zeros_like(master)
    v = torch.zeros_like(master)
    ws = torch.empty(int(api.lib().gmm_mlp_workspace_bytes(D, batch)), dtype=torch.uint8,
                     device=dev)
    steps_per_epoch = n_train // batch
    total = epochs * steps_per_epoch
    delta = 1.0 / out_std      # one symbol
    N, M = hi - lo + 1, 1 << precision
    ev = slice(n_train, n)
    history = []
    step = 0
    t1 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n_train, generator=gen, device=dev)
        loss_sum = torch.zeros((), dtype=torch.float64, device=dev)
        for b in range(steps_per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            g = api.mlp_loss_grad(X[idx].contiguous(), y[idx].contiguous(), shadow, delta,
                                  round_act=True, ws=ws)
            step += 1
            lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * step / total))
            api.mlp_adam(master, g, m, v, lr_t, step, 1.0 / batch, shadow)
            loss_sum += g[P].double()
        pred = api.mlp_forward(X[ev].contiguous(), shadow) * out_std + out_mean
        hit = bracket_hits(pred, j[ev], slot[ev], lo, N, M, radius)
        h = float(hit.float().mean().item())
        groups = hit[: (hit.numel() // 64) * 64].view(-1, 64).all(dim=1)
        rec = {"epoch": ep, "loss_per_sample": float(loss_sum.item()) / (steps_per_epoch * batch),
               "hit_rate": h, "wave_all_hit": float(groups.float().mean().item())}
        history.append(rec)
        if log:
            log(rec)
        if (plateau is not None and len(history) >= 3
                and history[-1]["hit_rate"] - history[-2]["hit_rate"] < plateau
                and history[-2]["hit_rate"] - history[-3]["hit_rate"] < plateau):
            break
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    model = BracketModel(K, lo, hi, precision, master.cpu().numpy(), mean.cpu().numpy(),
                         std.cpu().numpy(), out_mean, out_std, radius, history)
    model.history.append({"tuples": n_train, "steps": step, "batch": batch,
                          "data_s": t_data, "train_s": t_train})
    return model


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--K", type=int, default=3)
    ap.add_argument("--lo", type=int, default=-255)
    ap.add_argument("--hi", type=int, default=255)
    ap.add_argument("--precision", type=int, default=16)
    ap.add_argument("--tuples", type=int, default=10_000_000)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--seed", type=int, default=synth.TRAIN_SEED_C4)
    ap.add_argument("--plateau", type=float, default=None)
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    model = train_bracket(a.K, a.lo, a.hi, a.precision, n_train=a.tuples, epochs=a.epochs,
                          seed=a.seed, log=print, plateau=a.plateau)
    model.save(a.out)
    print(model.history[-1])


if __name__ == "__main__":
    main()
