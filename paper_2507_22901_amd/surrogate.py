"""Training and evaluation of the surrogate network on the exact search's
own whole-cube table.  Every step runs in the library's kernels (table
batches, forward, loss, backward, Adam); this module only orders the calls,
shuffles the training colours and reads results back."""
from __future__ import annotations

import math
import time

import torch

from . import MLP, Grid, Rule, context, pair_reduce, permute_ids


def cube_colours_device(device="cuda") -> torch.Tensor:
    ids = torch.arange(1 << 24, dtype=torch.int32, device=device)
    return torch.stack([(ids >> 16) & 255, (ids >> 8) & 255, ids & 255], dim=1).to(torch.uint8)


def cube_table(grid: Grid, rule: Rule, ctx=None) -> torch.Tensor:
    """Angle-bin table of all 2^24 colours (uint8 [2^24, 40]) from the exact search."""
    _, tab = pair_reduce(cube_colours_device(), grid, rule, summaries=False, table=True, ctx=ctx)
    return tab


def train(mlp: MLP, table: torch.Tensor, train_ids: torch.Tensor, dr: float, epochs: float = 32.0,
          batch: int = 8192, lr: float = 4e-3, lr_min: float = 2e-5, delta: float = 0.05,
          seed: int = 0, log_every: int = 200, step0: int = 0):
    """Adam with cosine decay from lr to lr_min over the run; rows are the
    training colour ids (int32 on the GPU) in a new pseudorandom order every
    epoch (the library's keyed permutation, key = (seed, epoch)); each epoch
    is one call of the library's training loop.  Returns (steps,
    [(step, loss)], seconds)."""
    n = train_ids.shape[0]
    per_epoch = math.ceil(n / batch)
    total = max(1, int(round(epochs * per_epoch)))
    log = []
    ids = torch.empty_like(train_ids)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step = 0
    epoch = 0
    while step < total:
        take = min(per_epoch, total - step)
        permute_ids(train_ids, (seed << 32) + epoch, out=ids, ctx=mlp.ctx)
        losses = mlp.train_steps(ids[:min(n, take * batch)], table, dr, batch, delta, lr, lr_min,
                                 step0 + step, total, log=bool(log_every))
        epoch += 1
        if log_every:
            lv = losses.cpu().numpy()
            for k in range(0, take, log_every):
                log.append((step + k, float(lv[k])))
            log.append((step + take - 1, float(lv[-1])))
        step += take
    torch.cuda.synchronize()
    return total, log, time.perf_counter() - t0


@torch.no_grad()
def evaluate(mlp: MLP, table: torch.Tensor, ids: torch.Tensor, dr: float, chunk: int = 1 << 20):
    """Radius error (MAE / p95 / max, in Delta E 1976 units) over the
    (colour, bin) pairs with a valid radius, and feasibility precision /
    recall (logit > 0 against count > 0), on the given colour ids."""
    errs, tp, fp, fn = [], 0, 0, 0
    for a in range(0, ids.shape[0], chunk):
        b = ids[a:a + chunk].long()
        rgb = torch.stack([(b >> 16) & 255, (b >> 8) & 255, b & 255], dim=1).to(torch.uint8)
        out = mlp.forward(rgb)
        rows = table[b]
        ridx = rows[:, 4:40].float()
        count = rows[:, :4].contiguous().view(torch.int32).squeeze(1)
        true_r = ridx * dr
        mask = ridx > 0
        errs.append((out[:, :36] * 50.0 - true_r)[mask].abs())
        feas_p = out[:, 36] > 0
        feas_t = count > 0
        tp += int((feas_p & feas_t).sum())
        fp += int((feas_p & ~feas_t).sum())
        fn += int((~feas_p & feas_t).sum())
    e = torch.cat(errs)
    es = e.float().sort().values
    q = es[int(0.95 * (es.numel() - 1))]
    return {"radius_mae": float(e.mean()), "radius_p95": float(q), "radius_max": float(es[-1]),
            "bins": int(e.numel()), "feasible_precision": tp / max(1, tp + fp),
            "feasible_recall": tp / max(1, tp + fn), "colours": int(ids.shape[0])}
