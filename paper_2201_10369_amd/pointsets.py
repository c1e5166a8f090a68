"""Explicit point sets for the sweep's point-list mode (wg_sweep_run_points).

Every set is an ordered list of alpha - 1 finite float64 points; the point
at infinity is implied last (the modified construction of arXiv:2201.10369,
Section 4.2).  The order fixes the rows of the transform matrices and so the
order of the float32 sums.

* comparison_set: the point sets the paper compares its proposals against
  (Tables tab:sota_1d and tab:sota_2d, the sets P_n of Barabasz et al.), in
  the order the tables list them.
* chebyshev: the Chebyshev nodes x_k = cos((2k - 1) pi / (2n)), k = 1..n,
  n = alpha - 1 (Section 2), with the middle node of an odd n taken as
  exactly 0 (its mathematical value).
* base_subsets / subset_lists: fixed base points plus a subset of the
  proposed points {-1/c, -c, c, 1/c} (Section 5.1, eq. subset_points; the
  base-point study of Section 6.2, Tables tab:optimal_f23 to tab:pattern_2d).
* family_lists: the families of wg_family_points as explicit lists (the same
  float64 values the device builds from (c1, c2)).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import wg

# P4 = {0, -1, 1, inf}; larger sets add points in the order the tables list
_P4 = [0.0, -1.0, 1.0]
_P8 = _P4 + [0.5, -0.5, 2.0, -2.0]
_COMPARISON = {
    1: {4: _P4, 5: _P4 + [0.5], 6: _P4 + [0.5, -3.0], 7: _P4 + [0.5, -0.5, -3.0],
        8: _P8, 9: _P8 + [-0.25], 10: _P8 + [-0.25, 4.0]},
    2: {4: _P4, 5: _P4 + [0.5], 6: _P4 + [0.5, -2.0], 7: _P4 + [0.5, -2.0, -0.5],
        8: _P8, 9: _P8 + [-0.25], 10: _P8 + [-0.25, 4.0]},
}

# the paper's proposed parameters for the two-parameter families
# (Tables tab:sota_1d and tab:sota_2d, n = 9 and 10)
PROPOSED_CD = {
    (9, 1): (1.313, 2.478), (10, 1): (1.953, 1.229),
    (9, 2): (1.305, 2.485), (10, 2): (1.272, 2.099),
}

# the proposed points a subset is drawn from (Section 5.1)
PROPOSED = ("-1/c", "-c", "c", "1/c")


def comparison_set(alpha, dims):
    """Finite points of the comparison set with alpha points (infinity last)."""
    try:
        return list(_COMPARISON[dims][alpha])
    except KeyError:
        raise ValueError(f"no comparison set for alpha={alpha}, dims={dims}") from None


def chebyshev(alpha):
    """The alpha - 1 Chebyshev nodes of the first kind, k = 1..alpha-1."""
    n = alpha - 1
    pts = []
    for k in range(1, n + 1):
        if 2 * (2 * k - 1) == 2 * n:                 # angle pi/2: the node is 0
            pts.append(0.0)
        else:
            pts.append(math.cos((2 * k - 1) * math.pi / (2 * n)))
    return pts


def _value(name, c):
    return {"-1/c": -1.0 / c, "-c": -c, "c": c, "1/c": 1.0 / c}[name]


def base_subsets(alpha, base):
    """All subsets (as tuples of PROPOSED names, in PROPOSED order) that,
    with 0, the base points and infinity, make alpha points."""
    k = alpha - 2 - len(base)
    if k < 0 or k > len(PROPOSED):
        raise ValueError(f"alpha={alpha} does not fit base {base} plus a subset of {PROPOSED}")
    return list(itertools.combinations(PROPOSED, k))


def subset_lists(base, subset, cs):
    """Point lists [0, *base, *subset(c)] for every c in cs: array
    [len(cs), 1 + len(base) + len(subset)]."""
    cs = np.asarray(cs, np.float64)
    out = np.empty((len(cs), 1 + len(base) + len(subset)), np.float64)
    out[:, 0] = 0.0
    for j, b in enumerate(base):
        out[:, 1 + j] = b
    for j, name in enumerate(subset):
        out[:, 1 + len(base) + j] = [_value(name, float(c)) for c in cs]
    return out


def family_lists(alpha, c1, c2=None):
    """wg_family_points for every (c1[i], c2[i]): array [n, alpha - 1]."""
    c1 = np.atleast_1d(np.asarray(c1, np.float64))
    c2 = np.ones_like(c1) if c2 is None else np.broadcast_to(np.asarray(c2, np.float64), c1.shape)
    return np.array([wg.family_points(alpha, float(a), float(b)) for a, b in zip(c1, c2)], np.float64)
