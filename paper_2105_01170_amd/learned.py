"""Training utilities for the rank/sketch-width predictor (tsvdm_mlp_*).

The predictor maps the sketch features of a transform-domain face
(tsvdm_rank_features) to (k/32, l/48): the rank the energy rule keeps and
the sketch width the randomized truncation needs.  Its labels come from the
library itself, on the caller's data:
  * width label: the smallest width of 16, 32, 40 whose certified error
    (tsvdm_truncate, PREC_MIXED, energy rule, rank caps 13, 26, 32) meets tau;
  * rank label: the rank the width-40 truncation keeps.
Every computation is a call into libtsvdm.so; PyTorch supplies memory.
"""
from __future__ import annotations

import torch

from . import api
from . import tsvdm as C

WIDTHS = (16, 32, 40)
CAPS = (13, 26, 32)


def labels(xhat: torch.Tensor, m: int, p: int, nf: int, omega: torch.Tensor, tau: float,
           power_iters: int = 1):
    """(rank label, width label) int32 tensors of the nf faces of xhat."""
    dev = xhat.device
    width = torch.full((nf,), WIDTHS[-1], dtype=torch.int32, device=dev)
    done = torch.zeros(nf, dtype=torch.bool, device=dev)
    rank = None
    for w, k in zip(WIDTHS, CAPS):
        tr = api.Truncator(m, p, nf, torch.float32, rank_mode=C.RANK_ENERGY, k=k, tau=tau,
                           precision=C.PREC_MIXED, oversample=w - k, power_iters=power_iters,
                           omega=omega, kmax=k, device=dev)
        F = tr(xhat)
        ok = F.cert <= tau * F.fro
        width = torch.where(ok & ~done, torch.full_like(width, w), width)
        done |= ok
        if w == WIDTHS[-1]:
            rank = F.ranks.clone()
    return rank, width


def targets(rank: torch.Tensor, width: torch.Tensor) -> torch.Tensor:
    """Regression targets (k / 32, l / 48), (n, 2) FP32."""
    return torch.stack([rank.float() / 32.0, width.float() / 48.0], dim=1).contiguous()


def train(pred: api.RankPredictor, feats: torch.Tensor, tgt: torch.Tensor, epochs: int = 20,
          batch: int = 1024, lr: float = 1e-3, seed: int = 0) -> list:
    """Mini-batch Adam on (feats (n, 32) half, tgt (n, 2) FP32); returns the
    mean loss of every epoch."""
    n = feats.shape[0]
    g = torch.Generator(device="cpu").manual_seed(seed)
    hist = []
    for _ in range(epochs):
        order = torch.randperm(n, generator=g).to(feats.device)
        tot, cnt = 0.0, 0
        for s in range(0, n, batch):
            idx = order[s:s + batch]
            x = feats.index_select(0, idx).contiguous()
            t = tgt.index_select(0, idx).contiguous()
            pred.train_step(x, t, lr=lr)
            tot += float(pred.loss.item()) * idx.numel()
            cnt += idx.numel()
        hist.append(tot / cnt)
    return hist
