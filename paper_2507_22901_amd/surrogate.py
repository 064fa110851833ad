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
          seed: int = 0, log_every: int = 200, step0: int = 0, start: int = 0, stop: int | None = None,
          checkpoint: str | None = None):
    """Adam with cosine decay from lr to lr_min over the run; rows are the
    training colour ids (int32 on the GPU) in a new pseudorandom order every
    epoch (the library's keyed permutation, key = (seed, epoch)); each epoch
    (or the part of one between start / stop) is one call of the library's
    training loop.  start: the steps already done (a resumed run, e.g. from
    load_checkpoint); stop: end after that many steps of the run (default:
    all); checkpoint: a path that receives the training checkpoint (parameters,
    Adam moments, step, seed) when the call ends.  Returns (steps, [(step,
    loss)], seconds)."""
    n = train_ids.shape[0]
    per_epoch = math.ceil(n / batch)
    total = max(1, int(round(epochs * per_epoch)))
    end = total if stop is None else min(int(stop), total)
    log = []
    ids = torch.empty_like(train_ids)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step = int(start)
    while step < end:
        epoch, off = divmod(step, per_epoch)
        take = min(per_epoch - off, end - step)
        permute_ids(train_ids, (seed << 32) + epoch, out=ids, ctx=mlp.ctx)
        losses = mlp.train_steps(ids[off * batch:min(n, (off + take) * batch)], table, dr, batch, delta, lr,
                                 lr_min, step0 + step, total, log=bool(log_every))
        if log_every:
            lv = losses.cpu().numpy()
            for k in range(0, take, log_every):
                log.append((step + k, float(lv[k])))
            log.append((step + take - 1, float(lv[-1])))
        step += take
    torch.cuda.synchronize()
    if checkpoint:
        mlp.save_checkpoint(checkpoint, step, seed)
    return end - int(start), log, time.perf_counter() - t0


def table_signature(grid: Grid, rule: Rule, ctx=None) -> dict:
    """What a cached cube table depends on: the grid, the rule and the
    library's colour constants (the L*a*b* of the eight cube corners and a
    mid grey, as the library converts them)."""
    from . import rgb8_to_lab
    probe = torch.tensor([[r, g, b] for r in (0, 255) for g in (0, 255) for b in (0, 255)] + [[128, 128, 128]],
                         dtype=torch.uint8, device="cuda")
    lab = rgb8_to_lab(probe, ctx=ctx).cpu().numpy().astype(float).round(6).tolist()
    return {"format": "cube-table-1", "rows": 1 << 24, "row_bytes": 40,
            "grid": [grid.dr, grid.nr, grid.dtheta_deg, grid.ntheta],
            "rule": [rule.v_th, rule.r_novib, rule.pattern_mask, rule.flags], "lab_probe": lab}


def save_table(path: str, table: torch.Tensor, grid: Grid, rule: Rule, ctx=None) -> None:
    """Cache a whole-cube table: a JSON header line (signature and the
    SHA-256 of the rows) followed by the 2^24 x 40 bytes."""
    import hashlib
    import json
    rows = table.contiguous().cpu().numpy().tobytes()
    head = dict(table_signature(grid, rule, ctx), sha256=hashlib.sha256(rows).hexdigest())
    with open(path, "wb") as f:
        f.write((json.dumps(head, sort_keys=True) + "\n").encode())
        f.write(rows)


def load_table(path: str, grid: Grid, rule: Rule, ctx=None) -> torch.Tensor | None:
    """A cached table for this grid, rule and library, or None when the file
    is missing, was made for something else or fails its hash."""
    import hashlib
    import json
    try:
        with open(path, "rb") as f:
            head = json.loads(f.readline().decode())
            rows = f.read()
    except (OSError, ValueError, UnicodeDecodeError):
        return None
    want = table_signature(grid, rule, ctx)
    if any(head.get(k) != v for k, v in want.items()) or len(rows) != (1 << 24) * 40:
        return None
    if hashlib.sha256(rows).hexdigest() != head.get("sha256"):
        return None
    import numpy as np
    return torch.from_numpy(np.frombuffer(rows, dtype=np.uint8).reshape(1 << 24, 40).copy()).cuda()


# Baseline proposers for the honest gain test: the same verify-and-fallback
# path fed with proposals that need no network.

def colour_ids(rgb: torch.Tensor) -> torch.Tensor:
    """uint8 [n, 3] -> int64 ids R << 16 | G << 8 | B."""
    r = rgb.long()
    return (r[:, 0] << 16) | (r[:, 1] << 8) | r[:, 2]


@torch.no_grad()
def table_pred(table: torch.Tensor, rgb: torch.Tensor, dr: float) -> torch.Tensor:
    """Proposals looked up in the whole-cube table: each colour's own 36 bin
    radii (in the network's units, radius / 50) and a logit of +10 / -10 for a
    colour with / without a survivor on the table's grid (float32 [n, 37])."""
    rows = table[colour_ids(rgb)]
    pred = torch.empty((rgb.shape[0], 37), dtype=torch.float32, device=rgb.device)
    pred[:, :36] = rows[:, 4:40].float() * (dr / 50.0)
    cnt = rows[:, :4].contiguous().view(torch.int32).squeeze(1)
    pred[:, 36] = torch.where(cnt > 0, 10.0, -10.0)
    return pred


@torch.no_grad()
def constant_prior(table: torch.Tensor, train_ids: torch.Tensor, dr: float) -> torch.Tensor:
    """One proposal for every colour: the mean radius of each bin over the
    training colours that have one (network units), and a logit of +10
    (float32 [37])."""
    out = torch.zeros(37, dtype=torch.float64, device=table.device)
    cnt = torch.zeros(36, dtype=torch.float64, device=table.device)
    for a in range(0, train_ids.shape[0], 1 << 22):
        r = table[train_ids[a:a + (1 << 22)].long(), 4:40].double()
        out[:36] += r.sum(0)
        cnt += (r > 0).double().sum(0)
    out[:36] = out[:36] / cnt.clamp(min=1.0) * (dr / 50.0)
    out[36] = 10.0
    return out.float()


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
