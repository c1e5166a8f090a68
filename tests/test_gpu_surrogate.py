"""GPU checks of the surrogate network kernels against the float64 oracle,
and of what the trained surrogate gains over the plain sweep."""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _wg():
    from paper_2201_10369_amd import wg
    return wg


def _data(n, seed):
    rng = np.random.default_rng(seed)
    pairs = synth.surrogate_pairs(n, seed=seed)
    sizes = np.array(synth.SURROGATE_SIZES)[rng.integers(0, 12, n)]
    target = rng.standard_normal(n).astype(np.float32) - 6.0
    return pairs[:, 0], pairs[:, 1], sizes[:, 0].astype(np.int32), sizes[:, 1].astype(np.int32), target


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _params(seed=3):
    p = synth.mlp_init(omlp.WIDTHS, seed=seed)
    rng = np.random.default_rng(seed)
    return [(W, (rng.standard_normal(b.shape) * 0.05).astype(np.float32)) for W, b in p]


def test_gradient_matches_oracle():
    wg = _wg()
    params = _params()
    c1, c2, m, r, t = _data(300, 1)
    ctx = wg.Mlp(512)
    g, loss = ctx.gradient(_dev(wg.mlp_pack(params)), _dev(c1), _dev(c2), _dev(m), _dev(r), _dev(t))
    g = wg.mlp_unpack(g.cpu().numpy())
    X = omlp.features(c1, c2, m, r)
    l64, g64 = omlp.loss_and_grads([(W.astype(np.float64), b.astype(np.float64)) for W, b in params], X, t)
    assert loss.item() == pytest.approx(l64, rel=1e-5)
    for (gW, gb), (oW, ob) in zip(g, g64):
        for a, b in ((gW, oW), (gb, ob)):
            assert np.linalg.norm(a - b) <= 2e-4 * np.linalg.norm(b) + 1e-9


@pytest.mark.parametrize("n", [1, 17, 1000, 4096])
def test_gradient_matches_oracle_at_training_batches(n):
    """The batch of the training runs (4096 samples: 256 forward blocks, the
    weight gradients over 8 slices), a ragged one (1000 = 62 blocks of 16
    and one of 8) and the degenerate ones (one sample: one block, one slice;
    17: a second block holding one sample), twice: the two results are
    bitwise equal."""
    wg = _wg()
    params = _params(6)
    c1, c2, m, r, t = _data(n, 7)
    ctx = wg.Mlp(4096)
    args = (_dev(wg.mlp_pack(params)), _dev(c1), _dev(c2), _dev(m), _dev(r), _dev(t))
    g, loss = ctx.gradient(*args)
    g2, loss2 = ctx.gradient(*args)
    assert torch.equal(g, g2) and torch.equal(loss, loss2)
    X = omlp.features(c1, c2, m, r)
    l64, g64 = omlp.loss_and_grads([(W.astype(np.float64), b.astype(np.float64)) for W, b in params], X, t)
    assert loss.item() == pytest.approx(l64, rel=1e-5)
    for (gW, gb), (oW, ob) in zip(wg.mlp_unpack(g.cpu().numpy()), g64):
        for a, b in ((gW, oW), (gb, ob)):
            assert np.linalg.norm(a - b) <= 2e-4 * np.linalg.norm(b) + 1e-9


def test_training_from_device_permutations_and_bad_entries():
    """Training with the minibatch orders already on the GPU gives the same
    bits as from the host; an order entry outside [0, n) gives NaN losses for
    its minibatch, not an out-of-range read."""
    from paper_2201_10369_amd import surrogate as sg
    wg = _wg()
    n = 512
    c1, c2, m, r, t = _data(n, 8)
    data = {"c1": c1, "c2": c2, "m": m, "r": r, "target": t.astype(np.float64)}
    perm = synth.minibatch_order(n, 2, seed=4)
    init = _params(7)
    a, la = sg.train(data, init, perm, batch=128)
    b, lb = sg.train(data, init, _dev(perm), batch=128)
    assert torch.equal(la, lb) and torch.equal(a.params, b.params)
    bad = perm.copy()
    bad[1, 5] = n + 7
    ctx = wg.Mlp(128)
    P = _dev(wg.mlp_pack(init))
    adam = torch.zeros(2 * P.numel(), dtype=torch.float32, device="cuda")
    losses = ctx.train(P, adam, 1, 1e-3, _dev(c1), _dev(c2), _dev(m), _dev(r),
                       _dev(((t - t.mean()) / t.std()).astype(np.float32)), _dev(bad), 128).cpu().numpy()
    assert np.all(np.isfinite(losses[:4])) and np.isnan(losses[4])


def test_predict_matches_oracle():
    wg = _wg()
    params = _params(4)
    c1, c2, m, r, _ = _data(1000, 2)
    out = wg.mlp_predict(_dev(wg.mlp_pack(params)), _dev(c1), _dev(c2), _dev(m), _dev(r)).cpu().numpy()
    ref, _ = omlp.forward(params, omlp.features(c1, c2, m, r))
    assert np.allclose(out, ref, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("batch", [128, 100])
def test_adam_training_matches_oracle(batch):
    """Adam steps on the same minibatches (batch 128: five steps; batch 100:
    six steps of 7 forward blocks, the last one partial, over 7 slices): the
    loss of every step agrees with the float64 oracle, and the parameters
    stay close."""
    wg = _wg()
    params = _params(5)
    n, epochs = 640, 1
    c1, c2, m, r, t = _data(n, 3)
    perm = synth.minibatch_order(n, epochs, seed=9)
    P = _dev(wg.mlp_pack(params))
    adam = torch.zeros(2 * P.numel(), dtype=torch.float32, device="cuda")
    ctx = wg.Mlp(batch)
    losses = ctx.train(P, adam, 1, 1e-3, _dev(c1), _dev(c2), _dev(m), _dev(r), _dev(t), _dev(perm), batch)
    p64 = [(W.astype(np.float64), b.astype(np.float64)) for W, b in params]
    state = omlp.zero_state(p64)
    X = omlp.features(c1, c2, m, r)
    ref_losses = []
    for step in range(n // batch):
        idx = perm[0, step * batch:(step + 1) * batch]
        loss, grads = omlp.loss_and_grads(p64, X[idx], t[idx])
        ref_losses.append(loss)
        p64 = omlp.adam_step(p64, grads, state, step + 1, lr=1e-3)
    assert np.allclose(losses.cpu().numpy(), ref_losses, rtol=1e-4)
    # every parameter group separately (W1, b1, ..., W4, b4): its distance to
    # the oracle is a small part of how far the group moved, and nearly every
    # entry is within 1% of its own move (Adam's normalised step can turn the
    # sign of a few updates whose gradient is at float32 rounding level)
    got = wg.mlp_unpack(P.cpu().numpy())
    for li, ((gW, gb), (oW, ob), (iW, ib)) in enumerate(zip(got, p64, params)):
        for name, g_, o_, i_ in (("W", gW, oW, iW), ("b", gb, ob, ib)):
            moved = np.abs(o_ - i_.astype(np.float64))
            d = np.abs(g_.astype(np.float64) - o_)
            ratio = np.linalg.norm(d) / np.linalg.norm(moved)
            frac = np.mean(d <= 1e-2 * moved + 1e-7)
            print(f"layer {li + 1} {name}: |got-ref|/|moved| = {ratio:.2e}, within 1% of the move: {frac:.4f}")
            assert np.linalg.norm(moved) > 0
            assert ratio <= 2e-2, (li, name, ratio)
            assert frac >= (0.98 if g_.size > 1 else 1.0), (li, name, frac)


def test_topk_matches_numpy():
    wg = _wg()
    rng = np.random.default_rng(4)
    v = rng.standard_normal(70000).astype(np.float32)
    v[123] = v[456] = -10.0                       # a tie: smaller index first
    v[7] = np.nan
    idx = wg.topk_min(_dev(v), 40).cpu().numpy()
    order = np.argsort(np.where(np.isnan(v), np.inf, v), kind="stable")[:40]
    assert np.array_equal(idx, order)
    assert list(idx[:2]) == [123, 456]


def test_topk_infinities_nan_and_short_input():
    wg = _wg()
    v = np.array([3.0, np.inf, -np.inf, np.nan, 3.0, np.inf, -1.0, np.nan, -np.inf, 0.5], np.float32)
    idx = wg.topk_min(_dev(v), 12).cpu().numpy()
    ok = np.flatnonzero(~np.isnan(v))
    order = ok[np.argsort(v[ok], kind="stable")]
    assert list(idx) == list(order) + [-1] * (12 - len(order))
    assert list(idx[:2]) == [2, 8] and list(idx[5:8]) == [4, 1, 5]


@pytest.mark.parametrize("m,r", [(4, 3), (2, 3), (6, 5)])
def test_surrogate_gain_over_plain_and_random_search(m, r):
    """Hold out one tile size: the surrogate is trained on sweep errors of the
    other 11 tile sizes (F(2..8,3), F(2..6,5); 2D), plus 64 exact samples of
    the held-out size, all of which count as evaluations.  Its 32 best
    proposals on a 4096-point grid over c in [0.05, 20] and the four best of
    those 64 samples are scored exactly, then three 32-point local
    refinements from the best proposal and three from the best sample (for
    the two-parameter family of F(6x6,5x5) proposals come from a 128 x 128
    (c, d) grid, three refinements each in c and in d run from the best
    point, and the plain search is a 64 x 64 grid).  With 292
    evaluations, more than 10x fewer than the 4096 of the plain search, the
    best error is within 1% of the plain search's best, and no worse than
    random search with the same budget."""
    from paper_2201_10369_amd import surrogate as sg
    sizes = synth.SURROGATE_SIZES
    sweeps = {s: sg.sweep_for(*s, *synth.tile_pool(sg.POOL, s[0] + s[1] - 1, s[1], 2)) for s in sizes}
    others = [s for s in sizes if s != (m, r)]
    pairs, counts = synth.surrogate_inputs(sizes, 83334, seed=5)
    data = sg.make_dataset(sweeps, {s: pairs[s] for s in others}, {s: counts[s] for s in others})
    pairs, counts = synth.surrogate_inputs(sizes, 64, seed=11)
    shots = sg.make_dataset(sweeps, {(m, r): pairs[(m, r)]}, {(m, r): counts[(m, r)]})
    both = sg.concat(data, shots)
    n = len(both["c1"])
    model, losses = sg.train(both, synth.mlp_init(omlp.WIDTHS, seed=7), synth.minibatch_order(n, 20, seed=8))
    losses = losses.cpu().numpy()
    assert losses[-20:].mean() < 0.2 * losses[:20].mean()
    S = sweeps[(m, r)]
    pc1, pc2, qc1, qc2, two = sg.search_grids(m + r - 1)
    plain = sg.score(S, pc1, pc2, np.full(4096, sg.POOL))
    best_plain = float(np.min(plain))
    assert np.isfinite(best_plain)
    err, c1, c2, used = sg.guided_search(model, S, m, r, qc1, qc2, k=32, refine=32, refine_c2=two,
                                         extra=sg.best_samples(shots, 4))
    assert used == 32 + 4 + 3 * 32 * 2
    used += 64
    assert used * 10 <= 4096
    rng = np.random.default_rng(12)
    pick = rng.choice(4096, used, replace=False)
    rand = sg.score(S, pc1[pick], pc2[pick], np.full(used, sg.POOL))
    print(f"F({m},{r}): plain best {best_plain:.4e} at c={pc1[np.argmin(plain)]:.4f},{pc2[np.argmin(plain)]:.4f}; "
          f"surrogate {err:.4e} at c={c1:.4f},{c2:.4f} with {used} evaluations; random search "
          f"{np.min(rand):.4e}; final loss {losses[-20:].mean():.4f}")
    assert err <= 1.01 * best_plain
    assert err <= np.min(rand)
