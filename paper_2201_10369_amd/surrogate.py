"""Surrogate-guided search for good point-family parameters.

The paper finds good points by sweeping the error curve over c, which it
observes to be smooth (arXiv:2201.10369, Sections 1 and 6.1).  Here a small
network trained on sweep results predicts the log10 mean absolute error of a
family (c1, c2) for a tile size F(m, r); its best predictions are re-scored
by the exact sweep, which has the final word.

Everything numeric runs in the HIP library: the sweep (wg_sweep_*), training
(wg_mlp_train), inference (wg_mlp_predict) and selection (wg_topk_min).  This
module only arranges the calls.  Random inputs (parameter pairs, sample
counts, initial weights, minibatch orders) come from the `synth` module.
"""
from __future__ import annotations

import numpy as np

import synth

from . import wg

POOL = 2000


def _torch():
    import torch
    return torch


def sweep_for(m, r, dims=2, pool_n=POOL, max_cand=65536, seed=2):
    """A sweep object for one tile size with its own seeded sample pool."""
    torch = _torch()
    d, g = synth.tile_pool(pool_n, m + r - 1, r, dims, seed=seed)
    return wg.Sweep(m, r, dims, torch.from_numpy(d).cuda(), torch.from_numpy(g).cuda(), max_cand)


def score(S, c1, c2, counts):
    """Exact sweep scores: mean absolute error per candidate (inf if flagged),
    in runs of at most S.max_cand candidates."""
    torch = _torch()
    c1, c2, counts = np.asarray(c1, np.float64), np.asarray(c2, np.float64), np.asarray(counts, np.int32)
    means = []
    for a in range(0, len(c1), S.max_cand):
        b = min(len(c1), a + S.max_cand)
        out = S.run(torch.from_numpy(c1[a:b].copy()).cuda(), torch.from_numpy(c2[a:b].copy()).cuda(),
                    torch.from_numpy(counts[a:b].copy()).cuda()).cpu().numpy()
        mean = out[:, 0] / np.maximum(out[:, 2], 1)
        mean[out[:, 3] > 0] = np.inf
        means.append(mean)
    return np.concatenate(means)


def make_dataset(sizes, n_per_size, dims=2, seed=5, sweeps=None):
    """Labelled samples: (c1, c2) log-uniform over [0.05, 20]^2, each scored by
    the sweep of its size on an uneven 500-2000 sample prefix; the label is
    log10 of the mean absolute error, capped at 0 (flagged sets get 0)."""
    rows = []
    for k, (m, r) in enumerate(sizes):
        S = sweeps[(m, r)] if sweeps is not None else sweep_for(m, r, dims)
        pairs = synth.surrogate_pairs(n_per_size, seed=seed * 1000 + k)
        counts = synth.sample_counts(n_per_size, seed=seed * 1000 + k)
        mean = score(S, pairs[:, 0], pairs[:, 1], counts)
        lab = np.minimum(np.log10(np.where(np.isfinite(mean) & (mean > 0), mean, 1.0)), 0.0)
        rows.append((pairs[:, 0], pairs[:, 1], np.full(n_per_size, m), np.full(n_per_size, r), lab))
    c1, c2, mm, rr, lab = (np.concatenate(x) for x in zip(*rows))
    return dict(c1=c1, c2=c2, m=mm.astype(np.int32), r=rr.astype(np.int32), target=lab.astype(np.float32))


class Model:
    """Trained parameters plus the affine map from network output to log10
    error (targets are standardised before training)."""

    def __init__(self, params, mean, std):
        self.params, self.mean, self.std = params, mean, std


def train(data, epochs=20, batch=4096, lr=1e-3, seed=7):
    """Adam on the mean squared error of standardised log10 errors; returns
    (Model, per-step losses)."""
    torch = _torch()
    n = len(data["c1"])
    t = np.asarray(data["target"], np.float64)
    mean, std = float(t.mean()), float(t.std()) or 1.0
    params = torch.from_numpy(wg.mlp_pack(synth.mlp_init((4, 128, 128, 128, 1), seed=seed))).cuda()
    adam = torch.zeros(2 * params.numel(), dtype=torch.float32, device="cuda")
    perm = torch.from_numpy(synth.minibatch_order(n, epochs, seed=seed + 1)).cuda()
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in data.items() if k != "target"}
    tz = torch.from_numpy(((t - mean) / std).astype(np.float32)).cuda()
    ctx = wg.Mlp(batch)
    losses = ctx.train(params, adam, 1, lr, dev["c1"], dev["c2"], dev["m"], dev["r"], tz, perm, batch)
    return Model(params, mean, std), losses


def predict(model, c1, c2, m, r):
    """Network outputs (standardised log10 error; lower is better)."""
    torch = _torch()
    n = len(c1)
    return wg.mlp_predict(model.params, torch.from_numpy(np.asarray(c1, np.float64)).cuda(),
                          torch.from_numpy(np.asarray(c2, np.float64)).cuda(),
                          torch.full((n,), m, dtype=torch.int32, device="cuda"),
                          torch.full((n,), r, dtype=torch.int32, device="cuda"))


def predict_log10(model, c1, c2, m, r):
    return predict(model, c1, c2, m, r).cpu().numpy() * model.std + model.mean


def propose(model, m, r, grid_c1, grid_c2, k=32):
    """Indices into the grid of the k lowest predicted errors."""
    pred = predict(model, grid_c1, grid_c2, m, r)
    return wg.topk_min(pred, k).cpu().numpy()


def guided_search(model, S, m, r, grid_c1, grid_c2, k=32, refine=32, spans=(0.25, 0.05, 0.01),
                  n_eval=POOL, refine_c2=False):
    """Re-score the k best proposals exactly, then refine: for each span,
    `refine` log-spaced values of c1 within a factor (1 +- span) of the best
    so far (the error curve is smooth, Section 6.1), and with refine_c2 the
    same for c2 (the two-parameter families).
    Returns (best error, best c1, best c2, exact evaluations used)."""
    idx = propose(model, m, r, grid_c1, grid_c2, k)
    idx = idx[idx >= 0]
    c1, c2 = np.asarray(grid_c1)[idx], np.asarray(grid_c2)[idx]
    errs = score(S, c1, c2, np.full(len(idx), n_eval))
    b = int(np.argmin(errs))
    best = (errs[b], c1[b], c2[b])
    used = len(idx)
    for span in (spans if refine else ()):
        for axis in ((0, 1) if refine_c2 else (0,)):
            f = np.exp(np.linspace(np.log(1 - span), np.log(1 + span), refine))
            rc1 = best[1] * f if axis == 0 else np.full(refine, best[1])
            rc2 = best[2] * f if axis == 1 else np.full(refine, best[2])
            rerr = score(S, rc1, rc2, np.full(refine, n_eval))
            j = int(np.argmin(rerr))
            if rerr[j] < best[0]:
                best = (rerr[j], rc1[j], rc2[j])
            used += refine
    return best[0], best[1], best[2], used
