"""Pins for the sweep oracle (Section 6.1 curve) and the surrogate reference."""
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

import synth
from oracle import fp, mlp, sweep
from oracle import toomcook as tc


# ----------------------------------------------------------------------------
# Sweep
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dims", [1, 2])
def test_f43_curve_minimum_location(dims):
    """Section 6.1: for {-1/c, -c, 0, c, 1/c} the error over c in [1.1, 2.5]
    is smallest for c in roughly 1.6-1.8; this oracle's curve (ascending
    summation) must have its minimum within [1.5, 1.9]."""
    grid = synth.linear_grid(1.1, 2.5, 0.02)
    d, g = synth.tile_pool(3000, 6, 3, dims, seed=2)
    res = sweep.sweep(4, 3, dims, grid, None, np.full(len(grid), 3000), d, g)
    errs = [e["mean_abs"] for e in res]
    i, c = sweep.argmin(errs, grid)
    assert 1.5 <= c <= 1.9, (dims, c)
    # a rough curve: the ends are clearly worse than the minimum
    assert errs[0] > 1.1 * errs[i] and errs[-1] > 1.1 * errs[i]


def test_reciprocal_symmetry():
    """{+-c, +-1/c} is the same point set for c and 1/c (only the order of
    the points differs), so the error curve is symmetric in log c."""
    d, g = synth.tile_pool(3000, 8, 3, 2, seed=2)
    yref = sweep.pool_reference(d, g)
    for c in (1.3, 1.9, 3.1):
        a = sweep.candidate_error(8, 6, 3, 2, c, 1.0, d, g, yref, 3000)["mean_abs"]
        b = sweep.candidate_error(8, 6, 3, 2, 1.0 / c, 1.0, d, g, yref, 3000)["mean_abs"]
        assert abs(a / b - 1) < 0.03, (c, a, b)


def test_singular_candidate_is_flagged():
    d, g = synth.tile_pool(100, 8, 3, 2, seed=2)
    res = sweep.sweep(6, 3, 2, np.array([1.0, 2.0]), np.array([1.0, 1.0]), np.array([100, 100]), d, g)
    assert res[0]["singular"] and math.isinf(res[0]["mean_abs"])
    assert not res[1]["singular"] and res[1]["mean_abs"] < 1e-5


def test_sweep_uses_pool_prefix():
    """Candidate i is scored on exactly the first n_i pool samples."""
    d, g = synth.tile_pool(500, 6, 3, 1, seed=2)
    counts = synth.sample_counts(3, lo=100, hi=400)
    res = sweep.sweep(4, 3, 1, np.array([1.5, 1.6, 1.7]), None, counts, d, g)
    for i, c in enumerate((1.5, 1.6, 1.7)):
        n = int(counts[i])
        mats = fp.mats_f32(tc.family_points(6, c), 4, 3)
        e = fp.l1_errors(fp.tile_1d_f32(mats, d[:n], g[:n]), fp.direct_tile_f64(d[:n], g[:n]))
        assert res[i]["abs_sum"] == e["abs_sum"] and res[i]["count"] == n * 4


def test_sample_counts_range_and_determinism():
    a = synth.sample_counts(4096)
    assert a.min() >= 500 and a.max() <= 2000 and len(set(a.tolist())) > 1000
    assert np.array_equal(a, synth.sample_counts(4096))
    # SplitMix64 reference value: first output for state 0 (Vigna's test vector)
    assert synth.splitmix64(0) == 0xE220A8397B1DCDAF


def test_argmin_ties_to_smaller_grid_value():
    assert sweep.argmin([3.0, 1.0, 1.0, math.inf], [0.5, 0.7, 0.6, 0.1]) == (2, 0.6)


# ----------------------------------------------------------------------------
# Surrogate reference
# ----------------------------------------------------------------------------
def test_gelu_values():
    z = np.array([0.0, 1.0, -1.0, 2.5])
    g = mlp.gelu(z)
    assert g[0] == 0.0
    assert g[1] == pytest.approx(0.8413447460685429, rel=1e-15)       # Phi(1)
    assert g[1] - g[2] == pytest.approx(1.0, rel=1e-15)                # gelu(x) - gelu(-x) = x
    h = 1e-6
    assert mlp.gelu_grad(z) == pytest.approx((mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), rel=1e-8, abs=1e-9)


def _small_params(seed):
    p = synth.mlp_init((4, 7, 6, 5, 1), seed=seed)
    rng = np.random.default_rng(seed)
    return [(W.astype(np.float64), rng.standard_normal(b.shape) * 0.1) for W, b in p]


def test_gradients_match_central_differences():
    params = _small_params(3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((9, 4))
    t = rng.standard_normal(9)
    loss, grads = mlp.loss_and_grads(params, X, t)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr, garr in ((W, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gflat = garr.reshape(-1)
            for idx in range(0, flat.size, max(1, flat.size // 7)):
                old = flat[idx]
                flat[idx] = old + h
                lp, _ = mlp.loss_and_grads(params, X, t)
                flat[idx] = old - h
                lm, _ = mlp.loss_and_grads(params, X, t)
                flat[idx] = old
                assert gflat[idx] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-9)


def test_adam_first_step_closed_form():
    """At t = 1 the bias-corrected moments are g and g^2, so every parameter
    moves by -lr g / (|g| + eps)."""
    params = _small_params(5)
    rng = np.random.default_rng(6)
    grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in params]
    new = mlp.adam_step(params, grads, mlp.zero_state(params), 1, lr=0.01)
    for (W, b), (gW, gb), (nW, nb) in zip(params, grads, new):
        assert np.allclose(nW - W, -0.01 * gW / (np.abs(gW) + 1e-8), rtol=1e-12, atol=1e-15)
        assert np.allclose(nb - b, -0.01 * gb / (np.abs(gb) + 1e-8), rtol=1e-12, atol=1e-15)


def test_training_reduces_loss():
    params = [(W.astype(np.float64), b.astype(np.float64)) for W, b in synth.mlp_init((4, 16, 16, 16, 1), seed=1)]
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (256, 4))
    t = np.sin(2 * X[:, 0]) + X[:, 2] ** 2
    state = mlp.zero_state(params)
    l0, _ = mlp.loss_and_grads(params, X, t)
    for step in range(1, 201):
        _, gr = mlp.loss_and_grads(params, X, t)
        params = mlp.adam_step(params, gr, state, step, lr=1e-2)
    l1, _ = mlp.loss_and_grads(params, X, t)
    assert l1 < 0.1 * l0


def test_parameter_count():
    p = synth.mlp_init(mlp.WIDTHS)
    assert mlp.flatten(p).size == 33793
