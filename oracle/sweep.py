"""Error sweep over the point parameter c (oracle).  Test infrastructure only.

Section 6.1 evaluates the error of a point family as a function of c (e.g.
F(4,3) with {-1/c, -c, 0, c, 1/c} for c in [1.1, 2.5], step 1e-3) and
Section 6.3 searches many such combinations; each evaluation scores float32
Winograd results on random inputs against a float64 direct convolution.

For every candidate: build the family's points (as float64 numbers), the
exact matrices of those points and their float32 roundings (toomcook / fp), evaluate float32 tiles on the first n_i
samples of a shared pool (common random numbers), and accumulate the L1 error
against the float64 reference.  A candidate whose points coincide is
reported with infinite error.
"""
from __future__ import annotations

import math

import numpy as np

from . import fp
from . import toomcook as tc


def pool_reference(d, g):
    """float64 direct correlation of every pool sample (computed once)."""
    return fp.direct_tile_f64(d, g)


def candidate_error(alpha, m, r, dims, c1, c2, d, g, yref, n):
    """L1 error sums of one candidate on the pool prefix [0, n).  The
    family's points are float64 numbers (1/c rounded to the nearest float64,
    as for the points of a layer plan); the matrices are built exactly from
    them."""
    try:
        pts = tc.family_points_f64(alpha, c1, c2)
        mats = fp.mats_f32(pts, m, r)
    except tc.SingularPoints:
        return dict(abs_sum=math.inf, ref_sum=float(np.abs(yref[:n]).sum()),
                    rel_l1=math.inf, mean_abs=math.inf, count=0, singular=True)
    tile = fp.tile_1d_f32 if dims == 1 else fp.tile_2d_f32
    y = tile(mats, d[:n], g[:n])
    e = fp.l1_errors(y, yref[:n])
    e["singular"] = False
    return e


def sweep(m, r, dims, c1, c2, counts, d, g, yref=None):
    """Error curve: one dict per candidate (c1[i], c2[i]) scored on counts[i]
    pool samples.  c2 may be None for families that need one parameter."""
    alpha = m + r - 1
    if yref is None:
        yref = pool_reference(d, g)
    out = []
    for i in range(len(c1)):
        cc2 = None if c2 is None else float(c2[i])
        out.append(candidate_error(alpha, m, r, dims, float(c1[i]), cc2, d, g, yref,
                                   int(counts[i])))
    return out


def argmin(values, grid):
    """Index and grid value of the smallest finite value; ties go to the
    smaller grid value."""
    best = None
    for i, v in enumerate(values):
        if not math.isfinite(v):
            continue
        if best is None or v < values[best] or (v == values[best] and grid[i] < grid[best]):
            best = i
    return best, (None if best is None else grid[best])


def candidate_error_points(pts, m, r, dims, d, g, yref, n):
    """L1 error sums of one explicit point list (finite points, infinity
    implied last) on the pool prefix [0, n).  Float points are taken as the
    exact rationals they denote."""
    from fractions import Fraction
    try:
        exact = [p if isinstance(p, Fraction) else Fraction(float(p)) for p in pts]
        mats = fp.mats_f32(exact, m, r)
    except tc.SingularPoints:
        return dict(abs_sum=math.inf, ref_sum=float(np.abs(yref[:n]).sum()),
                    rel_l1=math.inf, mean_abs=math.inf, count=0, singular=True)
    tile = fp.tile_1d_f32 if dims == 1 else fp.tile_2d_f32
    y = tile(mats, d[:n], g[:n])
    e = fp.l1_errors(y, yref[:n])
    e["singular"] = False
    return e


def candidate_error_mixed(mats64, m, r, dims, d, g, yref, n):
    """L1 error sums of the mixed-precision evaluation (float64 transforms,
    float32 Hadamard product; Section 6) with the given float64 matrices on
    the pool prefix [0, n)."""
    tile = fp.tile_1d_mixed if dims == 1 else fp.tile_2d_mixed
    y = tile(mats64, d[:n], g[:n])
    e = fp.l1_errors(y, yref[:n])
    e["singular"] = False
    return e
