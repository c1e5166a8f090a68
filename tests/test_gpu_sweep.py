"""GPU parity of the batched error sweep against the oracle sweep."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import synth
from oracle import fp, sweep
from oracle import toomcook as tc

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _wg():
    from paper_2201_10369_amd import wg
    return wg


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dtype is None else t.to(dtype)).to("cuda")


def _make(m, r, dims, n_pool, max_cand, seed=2):
    wg = _wg()
    alpha = m + r - 1
    d, g = synth.tile_pool(n_pool, alpha, r, dims, seed=seed)
    dd, gd = _dev(d), _dev(g)
    return wg.Sweep(m, r, dims, dd, gd, max_cand), d, g


def _oracle_mats(alpha, m, r, c1, c2):
    return fp.mats_f32(tc.family_points(alpha, Fr(float(c1)), Fr(float(c2))), m, r)


def _ordinal(v):
    """float32 -> integers ordered like the floats (+0 and -0 both map to 0)."""
    i = np.ascontiguousarray(v, np.float32).view(np.int32).astype(np.int64)
    return np.where(i < 0, -(i & 0x7FFFFFFF), i)


SIZES = [(2, 3), (3, 3), (4, 3), (6, 3), (8, 3), (2, 5), (4, 5), (6, 5)]


@pytest.mark.parametrize("m,r", SIZES)
def test_device_construction_matches_exact(m, r):
    """The float64 device construction rounds to the same float32 matrices as
    the exact rational construction (entries that cancel exactly are zero)."""
    alpha = m + r - 1
    S, d, g = _make(m, r, 2, 64, 64)
    rng = np.random.default_rng(m * 10 + r)
    c1 = np.concatenate([[2.0, 1.622, 0.5, 1.5], np.exp(rng.uniform(np.log(0.05), np.log(20), 28))])
    c2 = np.concatenate([[1.0, 2.5, 3.0, 0.7], np.exp(rng.uniform(np.log(0.05), np.log(20), 28))])
    counts = np.full(len(c1), 64, np.int32)
    S.run(_dev(c1), _dev(c2), _dev(counts))
    torch.cuda.synchronize()
    mismatched = 0
    for i in range(len(c1)):
        AT, G, BT, flag = S.matrices(i)
        try:
            o = _oracle_mats(alpha, m, r, c1[i], c2[i])
        except tc.SingularPoints:
            assert flag == 1
            continue
        assert flag == 0
        for mine, ref in zip((AT, G, BT), o):
            # zero pattern identical; nonzero entries within one float32 ulp
            assert np.array_equal(mine == 0, ref == 0), (i, c1[i], c2[i])
            ulps = np.abs(_ordinal(mine) - _ordinal(ref))
            assert ulps.max() <= 1
            mismatched += int((ulps > 0).sum())
    assert mismatched <= 2


@pytest.mark.parametrize("dims", [1, 2])
@pytest.mark.parametrize("m,r", [(2, 3), (4, 3), (6, 3), (8, 3), (4, 5), (6, 5)])
def test_sweep_errors_match_oracle(m, r, dims):
    """Per-candidate error sums on uneven pool prefixes equal the oracle's
    (identical float32 tiles; the float64 sums differ only in order)."""
    alpha = m + r - 1
    n_pool = 700
    S, d, g = _make(m, r, dims, n_pool, 40)
    rng = np.random.default_rng(7 + m + 10 * dims)
    c1 = np.exp(rng.uniform(np.log(0.3), np.log(4.0), 24))
    c2 = np.exp(rng.uniform(np.log(0.3), np.log(4.0), 24))
    c1[0], c2[0] = 2.0, 1.0
    counts = rng.integers(0, n_pool + 50, 24).astype(np.int32)
    counts[1], counts[2] = 0, n_pool
    out = S.run(_dev(c1), _dev(c2), _dev(counts)).cpu().numpy()
    yref = sweep.pool_reference(d, g)
    ref = sweep.sweep(m, r, dims, c1, c2, np.minimum(counts, n_pool), d, g, yref)
    outs = m if dims == 1 else m * m
    for i, e in enumerate(ref):
        n = min(int(counts[i]), n_pool)
        assert out[i, 2] == n * outs
        assert out[i, 3] == (1.0 if e["singular"] else 0.0)
        assert out[i, 1] == pytest.approx(e["ref_sum"], rel=1e-12, abs=1e-300)
        if e["singular"]:
            assert math.isinf(out[i, 0])
            continue
        AT, G, BT, _ = S.matrices(i)
        same = all(np.array_equal(a_, b_) for a_, b_ in zip((AT, G, BT), _oracle_mats(alpha, m, r, c1[i], c2[i])))
        tol = 1e-12 if same else 1e-3
        assert out[i, 0] == pytest.approx(e["abs_sum"], rel=tol, abs=1e-300), (i, c1[i], c2[i], same)


def test_singular_and_invalid_candidates_are_flagged():
    S, d, g = _make(4, 3, 2, 100, 8)
    c1 = np.array([1.0, -1.0, 0.0, np.nan, np.inf, 2.0, 1e-200, 1.5])
    counts = np.full(8, 100, np.int32)
    out = S.run(_dev(c1), None, _dev(counts)).cpu().numpy()
    assert list(out[:, 3]) == [1, 1, 1, 1, 1, 0, 1, 0]
    assert np.all(np.isinf(out[[0, 1, 2, 3, 4, 6], 0]))
    assert np.isfinite(out[[5, 7], 0]).all() and (out[[5, 7], 0] > 0).all()


def test_graph_replay_and_autotune_are_consistent():
    S, d, g = _make(6, 3, 2, 2000, 512)
    c1 = synth.candidate_grid(512)
    counts = synth.sample_counts(512)
    c1d, c2d, cd = _dev(c1), _dev(np.ones(512)), _dev(counts)
    a = S.run(c1d, c2d, cd).clone()
    b = S.run(c1d, c2d, cd).clone()                     # graph replay
    assert torch.equal(a, b)
    S.autotune(c1d, c2d, cd)
    t = S.tuning()
    assert t["tuned"] and t["block"] in (64, 128, 256)
    c = S.run(c1d, c2d, cd)
    fin = torch.isfinite(a[:, 0])
    assert torch.equal(fin, torch.isfinite(c[:, 0]))
    assert torch.allclose(a[fin], c[fin], rtol=1e-12, atol=0)


@pytest.mark.parametrize("dims", [1, 2])
def test_full_candidate_grid_sampled(dims):
    """4096 candidates log-spaced over [0.05, 20] with uneven 500-2000 sample
    counts (F(6,3) / F(6x6,3x3), family {0, inf, +-1, +-c, +-1/c}): 48 sampled
    candidates match the oracle; the curve is symmetric in log c and its
    minimum over the grid agrees with the oracle's minimum over the samples
    near it."""
    n = 4096
    S, d, g = _make(6, 3, dims, 2000, n)
    c1 = synth.candidate_grid(n)
    counts = synth.sample_counts(n)
    out = S.run(_dev(c1), _dev(np.ones(n)), _dev(counts)).cpu().numpy()
    mean = out[:, 0] / np.maximum(out[:, 2], 1)
    yref = sweep.pool_reference(d, g)
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([rng.integers(0, n, 44), [0, n - 1, int(np.nanargmin(mean)), 2048]]))
    for i in idx:
        e = sweep.candidate_error(8, 6, 3, dims, float(c1[i]), 1.0, d, g, yref, int(counts[i]))
        if e["singular"]:
            assert out[i, 3] == 1
            continue
        AT, G, BT, _ = S.matrices(int(i))
        same = all(np.array_equal(a_, b_) for a_, b_ in zip((AT, G, BT), _oracle_mats(8, 6, 3, c1[i], 1.0)))
        assert out[i, 0] == pytest.approx(e["abs_sum"], rel=1e-12 if same else 1e-3)
    # log-symmetry of the family: c and 1/c give the same point set
    for i in (300, 800, 1500):
        j = n - 1 - i                                    # grid is symmetric in log c
        assert abs(mean[i] / mean[j] - 1) < 0.05
    best = int(np.nanargmin(mean))
    assert 0.2 < c1[best] < 5.0
