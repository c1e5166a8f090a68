"""Point searches on the batched sweep: the two-parameter (c, d) families
and the base-point subsets.

The paper scores point sets by the L1 error of float32 Winograd results
against a float64 reference on random inputs, sweeping the parameters
(arXiv:2201.10369, Sections 6.1-6.3).  For the largest tiles it proposes
two-parameter sets {0, +-c, +-1/c, plus some of +-d, +-1/d} (n = 9 and 10,
Tables tab:sota_1d and tab:sota_2d) and for small tiles it fixes base points
and picks a subset of {-1/c, -c, c, 1/c} (Section 6.2, eq. subset_points).

Every score comes from the sweep kernels (wg_sweep_run for families,
wg_sweep_run_points for explicit lists); this module only builds the
candidate lists and picks minima.  Ties go to the earlier candidate.
"""
from __future__ import annotations

import math

import numpy as np

from . import pointsets


def _torch():
    import torch
    return torch


def _means(out):
    out = out.cpu().numpy()
    mean = out[:, 0] / np.maximum(out[:, 2], 1)
    mean[out[:, 3] > 0] = np.inf
    return mean


def score_family(S, c1, c2, n_eval):
    """Mean absolute error per (c1[i], c2[i]) on the first n_eval pool
    samples (inf when flagged), in runs of at most S.max_cand."""
    torch = _torch()
    c1 = np.ascontiguousarray(c1, np.float64)
    c2 = np.ascontiguousarray(np.broadcast_to(np.asarray(c2, np.float64), c1.shape))
    res = []
    for a in range(0, len(c1), S.max_cand):
        b = min(len(c1), a + S.max_cand)
        counts = torch.full((b - a,), int(n_eval), dtype=torch.int32, device="cuda")
        res.append(_means(S.run(torch.from_numpy(c1[a:b].copy()).cuda(),
                                torch.from_numpy(c2[a:b].copy()).cuda(), counts)))
    return np.concatenate(res)


def score_points(S, pts, n_eval):
    """Mean absolute error per explicit point list (rows of pts)."""
    torch = _torch()
    pts = np.ascontiguousarray(np.atleast_2d(pts), np.float64)
    res = []
    for a in range(0, len(pts), S.max_cand):
        b = min(len(pts), a + S.max_cand)
        counts = torch.full((b - a,), int(n_eval), dtype=torch.int32, device="cuda")
        res.append(_means(S.run_points(torch.from_numpy(pts[a:b].copy()).cuda(), counts)))
    return np.concatenate(res)


def log_grid(lo, hi, n):
    return np.exp(np.linspace(math.log(lo), math.log(hi), n))


def two_param_search(S, grid=64, lo=0.05, hi=20.0, keep=8, local=16, rounds=3, n_coarse=500,
                     n_eval=None):
    """Grid-and-refine search over (c, d) for the family of S's tile size.

    A grid x grid log-spaced grid over [lo, hi]^2 is scored on n_coarse
    samples; the `keep` best are re-scored on n_eval samples (default: the
    whole pool); then `rounds` times a local x local log-spaced grid around
    the best so far, of half-width one coarse step halved each round, is
    scored on n_eval samples.  Returns a dict with the best (c, d), its mean
    absolute error on n_eval samples, the number of scored candidates and
    the best value after each stage."""
    n_eval = S.n_pool if n_eval is None else n_eval
    g = log_grid(lo, hi, grid)
    C1, C2 = np.meshgrid(g, g, indexing="ij")
    c1, c2 = C1.ravel(), C2.ravel()
    coarse = score_family(S, c1, c2, n_coarse)
    order = np.argsort(coarse, kind="stable")[:keep]
    order = order[np.isfinite(coarse[order])]
    fine = score_family(S, c1[order], c2[order], n_eval)
    b = int(np.argmin(fine))
    best = (float(fine[b]), float(c1[order[b]]), float(c2[order[b]]))
    used = len(c1) + len(order)
    history = [best[0]]
    step = (math.log(hi) - math.log(lo)) / (grid - 1)
    for k in range(rounds):
        h = step / 2 ** k
        lc = best[1] * np.exp(np.linspace(-h, h, local))
        ld = best[2] * np.exp(np.linspace(-h, h, local))
        L1, L2 = np.meshgrid(lc, ld, indexing="ij")
        errs = score_family(S, L1.ravel(), L2.ravel(), n_eval)
        j = int(np.argmin(errs))
        if errs[j] < best[0]:
            best = (float(errs[j]), float(L1.ravel()[j]), float(L2.ravel()[j]))
        used += local * local
        history.append(best[0])
    return {"mean_abs": best[0], "c": best[1], "d": best[2], "evaluations": used, "history": history}


def subset_search(S, base, cs, n_eval=None):
    """For every subset of {-1/c, -c, c, 1/c} that completes 0, the base
    points and infinity to S's tile size, the error curve over cs (one
    batched run of all subsets and values).  Returns a list of dicts
    (subset, best c, best mean absolute error, curve), best subset first."""
    n_eval = S.n_pool if n_eval is None else n_eval
    subsets = pointsets.base_subsets(S.alpha, base)
    lists = np.concatenate([pointsets.subset_lists(base, sub, cs) for sub in subsets])
    errs = score_points(S, lists, n_eval).reshape(len(subsets), len(cs))
    rows = []
    for sub, curve in zip(subsets, errs):
        j = int(np.argmin(curve))
        rows.append({"subset": list(sub), "c": float(cs[j]), "mean_abs": float(curve[j]), "curve": curve})
    rows.sort(key=lambda r: r["mean_abs"])
    return rows
