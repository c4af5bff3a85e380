"""Learned projection around the library's kernels: mining labelled pairs
with the exhaustive search, training with msm_mlp_train, and saving or
loading the trained parameters.

The network (two layers, GELU, tanh output; the sign of the output layer's
pre-activation is the bit) replaces the random projection R of eq. (3), the
non-random hashing the paper names in Section 6. Training pairs come from
the exact method on a sample: epsilon-pairs found by msm_bruteforce_eps
(label 1), and pairs beyond epsilon (label 0) drawn half from the exhaustive search's
pairs within 2 eps (hard negatives) and half uniformly. Host code here only
draws indices and orders the pair list; all arithmetic runs in libmsm.
"""
from __future__ import annotations

import json
from dataclasses import asdict, dataclass

import numpy as np
import torch

from . import msm as M


@dataclass
class TrainConfig:
    hid: int = 512
    ell: int = 128
    h: int = 4
    lam: float = 0.05
    lr: float = 1e-3
    batch: int = 4096
    epochs: int = 20
    seed: int = 7


def _codes(p: np.ndarray) -> np.ndarray:
    p = p.astype(np.uint64)
    return (p[:, 0] << np.uint64(32)) | p[:, 1]


def mine_pairs(ctx: M.Context, Xs: torch.Tensor, eps: float, n_pos: int, n_neg: int, seed: int,
               metric="euclidean"):
    """(pairs int32 (P, 2) on the device, labels float32 (P,), stats) from a sample Xs.

    Positives: up to n_pos epsilon-pairs of the sample (all of them if fewer).
    Negatives: n_neg pairs with distance > eps, half from the pairs within
    2 eps that are not epsilon-pairs, half uniform random pairs checked by
    msm_verify.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = Xs.shape[0]
    pos_t, m_pos = M.bruteforce_eps(ctx, Xs, metric, eps, cap_hint=max(1024, 4 * n))
    pos = _pairs_np(pos_t)
    near_t, _ = M.bruteforce_eps(ctx, Xs, metric, 2.0 * eps, cap_hint=max(1024, 4 * pos.shape[0]))
    near = _pairs_np(near_t)
    near = near[~np.isin(_codes(near), _codes(pos))]
    if pos.shape[0] > n_pos:
        pos = pos[rng.choice(pos.shape[0], n_pos, replace=False)]
    n_hard = min(n_neg // 2, near.shape[0])
    hard = near[rng.choice(near.shape[0], n_hard, replace=False)] if n_hard > 0 else np.zeros((0, 2), np.uint32)
    # uniform pairs (i < j), minus those within eps
    need = n_neg - n_hard
    rand = np.zeros((0, 2), np.uint32)
    while rand.shape[0] < need:
        k = 2 * (need - rand.shape[0]) + 64
        a = rng.integers(0, n, k)
        b = rng.integers(0, n, k)
        keep = a != b
        cand = np.stack([np.minimum(a, b), np.maximum(a, b)], axis=1)[keep].astype(np.uint32)
        cand_t = torch.from_numpy(cand.view(np.int32)).to(Xs.device)
        close, _ = M.msm_verify(ctx, Xs, cand_t, metric, eps, cap=cand.shape[0])
        close_codes = _codes(_pairs_np(close))
        far = cand[~np.isin(_codes(cand), close_codes)]
        rand = np.concatenate([rand, far])[:need]
    neg = np.concatenate([hard, rand])
    pairs = np.concatenate([pos, neg]).astype(np.uint32)
    labels = np.concatenate([np.ones(pos.shape[0], np.float32), np.zeros(neg.shape[0], np.float32)])
    order = rng.permutation(pairs.shape[0])
    pairs, labels = pairs[order], labels[order]
    stats = {"sample": int(n), "eps_pairs_in_sample": int(m_pos), "positives": int(pos.shape[0]),
             "hard_negatives": int(n_hard), "random_negatives": int(rand.shape[0])}
    return (torch.from_numpy(np.ascontiguousarray(pairs).view(np.int32)).to(Xs.device),
            torch.from_numpy(labels).to(Xs.device), stats)


def _pairs_np(t: torch.Tensor | None) -> np.ndarray:
    if t is None:
        return np.zeros((0, 2), np.uint32)
    return np.ascontiguousarray(t.cpu().numpy()).view(np.uint32).reshape(-1, 2)


def train(ctx: M.Context, X: torch.Tensor, pairs: torch.Tensor, labels: torch.Tensor, cfg: TrainConfig,
          params0: np.ndarray):
    """Adam on the pair loss for cfg.epochs passes over the pair list, in a
    new host-drawn order each epoch. Returns (params, m, v, losses, next
    Adam step) with params, m, v on the device."""
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    params = torch.from_numpy(np.asarray(params0, np.float32)).to(X.device)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    pairs_h = pairs.cpu().numpy()
    labels_h = labels.cpu().numpy()
    P = pairs_h.shape[0]
    B = min(cfg.batch, P)
    steps_per_epoch = max(1, P // B)
    losses = []
    step = 1
    for _ in range(cfg.epochs):
        perm = rng.permutation(P)
        ep_pairs = torch.from_numpy(np.ascontiguousarray(pairs_h[perm])).to(X.device)
        ep_labels = torch.from_numpy(np.ascontiguousarray(labels_h[perm])).to(X.device)
        losses += M.msm_mlp_train(ctx, X, params, m, v, cfg.hid, cfg.ell, ep_pairs, ep_labels, B,
                                  steps_per_epoch, step, cfg.lr, cfg.h, cfg.lam)
        step += steps_per_epoch
    return params, m, v, losses, step


def save(path: str, params: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, d: int,
         cfg: TrainConfig):
    """Parameters and Adam state as raw little-endian FP32 (<path>.bin) plus
    <path>.json with the shapes, step and training configuration."""
    host = [t.detach().cpu().numpy().astype("<f4") for t in (params, m, v)]
    with open(path + ".bin", "wb") as f:
        for a in host:
            f.write(a.tobytes())
    meta = {"d": int(d), "count": int(params.numel()), "step": int(step), "layout": "W1|b1|W2|b2 row-major",
            "arrays": ["params", "adam_m", "adam_v"], "config": asdict(cfg)}
    with open(path + ".json", "w") as f:
        json.dump(meta, f, indent=1)


def load(path: str, device="cuda"):
    """Inverse of save: (params, m, v, step, d, cfg)."""
    with open(path + ".json") as f:
        meta = json.load(f)
    cfg = TrainConfig(**meta["config"])
    count = int(meta["count"])
    if count != M.mlp_param_count(int(meta["d"]), cfg.hid, cfg.ell):
        raise ValueError("checkpoint size does not match its shapes")
    raw = np.fromfile(path + ".bin", dtype="<f4")
    if raw.size != 3 * count:
        raise ValueError("checkpoint data has the wrong length")
    arrs = [torch.from_numpy(raw[i * count:(i + 1) * count].astype(np.float32)).to(device) for i in range(3)]
    return arrs[0], arrs[1], arrs[2], int(meta["step"]), int(meta["d"]), cfg
