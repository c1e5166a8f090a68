"""Surrogate-guided search for good point-family parameters.

The paper finds good points by sweeping the error curve over c, which it
observes to be smooth (arXiv:2201.10369, Sections 1 and 6.1).  Here a small
network trained on sweep results predicts the log10 mean absolute error of a
family (c1, c2) for a tile size F(m, r); its best predictions are re-scored
by the exact sweep, which has the final word.

Everything numeric runs in the HIP library: the sweep (wg_sweep_*), training
(wg_mlp_train), inference (wg_mlp_predict) and selection (wg_topk_min).  This
module only arranges the calls.  Every random input (sample pools, parameter
pairs, sample counts, initial weights, minibatch orders) is an argument.
"""
from __future__ import annotations

import numpy as np

from . import wg

POOL = 2000


def _torch():
    import torch
    return torch


def sweep_for(m, r, d_pool, g_pool, dims=2, max_cand=65536):
    """A sweep object for one tile size over the given sample pool (host
    float32 arrays: d_pool n x alpha (x alpha), g_pool n x r (x r))."""
    torch = _torch()
    return wg.Sweep(m, r, dims, torch.from_numpy(np.ascontiguousarray(d_pool, np.float32)).cuda(),
                    torch.from_numpy(np.ascontiguousarray(g_pool, np.float32)).cuda(), max_cand)


def score(S, c1, c2, counts):
    """Exact sweep scores: mean absolute error per candidate, in runs of at
    most S.max_cand candidates.  A flagged candidate, or one whose float32
    evaluation overflowed (a NaN or infinite sum: extreme points make the
    transformed values exceed float32), scores inf."""
    torch = _torch()
    c1, c2, counts = np.asarray(c1, np.float64), np.asarray(c2, np.float64), np.asarray(counts, np.int32)
    means = []
    for a in range(0, len(c1), S.max_cand):
        b = min(len(c1), a + S.max_cand)
        out = S.run(torch.from_numpy(c1[a:b].copy()).cuda(), torch.from_numpy(c2[a:b].copy()).cuda(),
                    torch.from_numpy(counts[a:b].copy()).cuda()).cpu().numpy()
        mean = out[:, 0] / np.maximum(out[:, 2], 1)
        mean[(out[:, 3] > 0) | ~np.isfinite(mean)] = np.inf
        means.append(mean)
    return np.concatenate(means)


def make_dataset(sweeps, pairs, counts):
    """Labelled samples for the tile sizes keyed in `pairs`: each (c1, c2) of
    pairs[(m, r)] (n x 2) scored by sweeps[(m, r)] on the pool prefix
    counts[(m, r)][i]; the label is log10 of the mean absolute error, capped
    at 0 (flagged sets get 0)."""
    rows = []
    for (m, r), pr in pairs.items():
        mean = score(sweeps[(m, r)], pr[:, 0], pr[:, 1], counts[(m, r)])
        lab = np.minimum(np.log10(np.where(np.isfinite(mean) & (mean > 0), mean, 1.0)), 0.0)
        n = len(pr)
        rows.append((pr[:, 0], pr[:, 1], np.full(n, m), np.full(n, r), lab))
    c1, c2, mm, rr, lab = (np.concatenate(x) for x in zip(*rows))
    return dict(c1=c1, c2=c2, m=mm.astype(np.int32), r=rr.astype(np.int32), target=lab.astype(np.float32))


def best_samples(data, k):
    """(c1, c2) of the k samples of `data` with the lowest labels."""
    j = np.argsort(data["target"], kind="stable")[:k]
    return data["c1"][j], data["c2"][j]


def select(data, keep):
    """The samples of `data` where the boolean mask `keep` is set."""
    return {k: v[keep] for k, v in data.items()}


def concat(*parts):
    return {k: np.concatenate([p[k] for p in parts]) for k in parts[0]}


class Model:
    """Trained parameters plus the affine map from network output to log10
    error (targets are standardised before training)."""

    def __init__(self, params, mean, std):
        self.params, self.mean, self.std = params, mean, std


def train(data, init_params, perm, batch=4096, lr=1e-3):
    """Adam on the mean squared error of standardised log10 errors from the
    initial parameters init_params ([(W, b), ...] per layer, W (out, in)),
    one epoch per row of perm (int32 permutations of the n samples, on the
    host or as a contiguous int32 tensor on the GPU);
    returns (Model, per-step losses)."""
    torch = _torch()
    n = len(data["c1"])
    if isinstance(perm, torch.Tensor):
        if perm.dtype != torch.int32 or not perm.is_cuda or not perm.is_contiguous():
            raise ValueError("perm as a tensor must be contiguous int32 on the GPU")
        permd = perm
    else:
        permd = None
        perm = np.ascontiguousarray(perm, np.int32)
    if perm.ndim != 2 or perm.shape[1] != n:
        raise ValueError("perm must have shape (epochs, n)")
    t = np.asarray(data["target"], np.float64)
    mean, std = float(t.mean()), float(t.std()) or 1.0
    params = torch.from_numpy(wg.mlp_pack(init_params)).cuda()
    adam = torch.zeros(2 * params.numel(), dtype=torch.float32, device="cuda")
    if permd is None:
        permd = torch.from_numpy(perm).cuda()
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in data.items() if k != "target"}
    tz = torch.from_numpy(((t - mean) / std).astype(np.float32)).cuda()
    ctx = wg.Mlp(batch)
    losses = ctx.train(params, adam, 1, lr, dev["c1"], dev["c2"], dev["m"], dev["r"], tz, permd, batch)
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


def search_grids(alpha, lo=0.05, hi=20.0):
    """Candidate grids of the held-out protocol for a family of alpha points:
    (plain c1, plain c2, proposal c1, proposal c2, two-parameter).  Families
    with at most 8 points are searched over c alone (c2 = 1; the family of 8
    points then holds +-1): 4096 log-spaced values, on which the surrogate
    also proposes.  The families of 9 and 10 points need c2 away from 1
    (+-1/d and +-d coincide at d = 1): a 64 x 64 log grid over (c1, c2) for
    the plain search and a 128 x 128 one for the proposals."""
    from .search import log_grid
    if alpha <= 8:
        g = log_grid(lo, hi, 4096)
        return g, np.ones_like(g), g, np.ones_like(g), False
    a, b = np.meshgrid(log_grid(lo, hi, 64), log_grid(lo, hi, 64), indexing="ij")
    p, q = np.meshgrid(log_grid(lo, hi, 128), log_grid(lo, hi, 128), indexing="ij")
    return a.ravel(), b.ravel(), p.ravel(), q.ravel(), True


def guided_search(model, S, m, r, grid_c1, grid_c2, k=32, refine=32, spans=(0.25, 0.05, 0.01),
                  n_eval=POOL, refine_c2=False, extra=None):
    """Re-score the k best proposals exactly, and the points of `extra` (a
    pair of arrays (c1, c2), e.g. the best exact samples the network was
    given for this size), then refine: for each span, `refine` log-spaced
    values of c1 within a factor (1 +- span) of the best so far (the error
    curve is smooth, Section 6.1), and with refine_c2 the same for c2 (the
    two-parameter families).  A one-parameter search refines from the best
    proposal and, separately, from the best extra point; a two-parameter
    search from the best of both.
    Returns (best error, best c1, best c2, exact evaluations used)."""
    idx = propose(model, m, r, grid_c1, grid_c2, k)
    idx = idx[idx >= 0]
    c1, c2 = np.asarray(grid_c1)[idx], np.asarray(grid_c2)[idx]
    errs = score(S, c1, c2, np.full(len(c1), n_eval))
    used = len(c1)
    b = int(np.argmin(errs))
    seeds = [(errs[b], c1[b], c2[b])]
    if extra is not None and len(extra[0]):
        x1, x2 = np.asarray(extra[0], np.float64), np.asarray(extra[1], np.float64)
        xe = score(S, x1, x2, np.full(len(x1), n_eval))
        used += len(x1)
        j = int(np.argmin(xe))
        if refine_c2:
            if xe[j] < seeds[0][0]:
                seeds = [(xe[j], x1[j], x2[j])]
        else:
            seeds.append((xe[j], x1[j], x2[j]))
    results = []
    for best in seeds:
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
        results.append(best)
    best = min(results, key=lambda t: t[0])
    return best[0], best[1], best[2], used
