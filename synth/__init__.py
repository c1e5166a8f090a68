"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws random numbers and lays them out; it holds none of the
Winograd arithmetic.  Everything the method would otherwise draw at random
(tile pools, per-candidate sample counts, candidate grids, surrogate training
pairs, initial network weights, minibatch orders) is produced here and passed
to both sides as an input.

Distributions follow the paper's evaluation protocol (Section 6: uniform random
inputs, many samples per evaluation) and the layer workloads used for the
throughput measurement (uniform[-1,1] for the small F(2x2,3x3) layer; N(0,1)
activations with N(0, 1/sqrt(9C)) filters for the large layers).
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1


# ----------------------------------------------------------------------------
# Layer workloads
# ----------------------------------------------------------------------------
#: name -> shape and distribution of each synthetic layer workload.
LAYERS = {
    # F(2x2,3x3), points {0,1,-1,inf}: small layer, uniform[-1,1] data
    "f2x2_n1_c16_k16_32x32": dict(N=1, C=16, K=16, H=32, W=32, r=3, m=2,
                                  padding="same", dist="uniform"),
    # F(4x4,3x3), points {0,inf,+-c,+-1/c}
    "f4x4_n32_c256_k256_56x56": dict(N=32, C=256, K=256, H=56, W=56, r=3, m=4,
                                     padding="same", dist="normal"),
    # F(6x6,3x3), points {0,inf,+-1,+-c,+-1/c}
    "f6x6_n64_c256_k256_28x28": dict(N=64, C=256, K=256, H=28, W=28, r=3, m=6,
                                     padding="same", dist="normal"),
    # F(4x4,5x5), the same 8-point family, 5x5 filters
    "f4x4r5_n64_c256_k256_28x28": dict(N=64, C=256, K=256, H=28, W=28, r=5, m=4,
                                       padding="same", dist="normal"),
}


def layer_inputs(N, C, K, H, W, r, dist="normal", seed_x=0, seed_w=1):
    """Activations x (N,C,H,W) and filters w (K,C,r,r), float32, C-contiguous.

    dist="uniform": both i.i.d. uniform[-1,1].
    dist="normal":  x ~ N(0,1); w ~ N(0, sigma) with sigma = 1/sqrt(r*r*C).
    Drawn in float64 with numpy's default generator, then rounded to float32.
    """
    gx = np.random.default_rng(seed_x)
    gw = np.random.default_rng(seed_w)
    if dist == "uniform":
        x = gx.uniform(-1.0, 1.0, size=(N, C, H, W))
        w = gw.uniform(-1.0, 1.0, size=(K, C, r, r))
    elif dist == "normal":
        x = gx.standard_normal(size=(N, C, H, W))
        w = gw.standard_normal(size=(K, C, r, r)) / np.sqrt(r * r * C)
    else:
        raise ValueError(dist)
    return (np.ascontiguousarray(x, dtype=np.float32),
            np.ascontiguousarray(w, dtype=np.float32))


def exact_small_ints(shape, seed, lo=-4, hi=4):
    """Small integer-valued float32 data (exactly representable), for tests
    whose expected values are computed in rational arithmetic."""
    g = np.random.default_rng(seed)
    return g.integers(lo, hi + 1, size=shape).astype(np.float32)


# ----------------------------------------------------------------------------
# Tile pools for the error sweep (one tile + one filter per sample)
# ----------------------------------------------------------------------------
def tile_pool(n, alpha, r, dims, seed=2):
    """Pool of n samples: input tiles d and filters g, i.i.d. uniform[-1,1].

    dims=1: d (n, alpha), g (n, r).   dims=2: d (n, alpha, alpha), g (n, r, r).
    The generator is keyed on (seed, alpha, r, dims) so every tile size has its
    own reproducible pool; float64 draws are rounded to float32.
    """
    g_ = np.random.default_rng([seed, alpha, r, dims])
    if dims == 1:
        d = g_.uniform(-1.0, 1.0, size=(n, alpha))
        g = g_.uniform(-1.0, 1.0, size=(n, r))
    elif dims == 2:
        d = g_.uniform(-1.0, 1.0, size=(n, alpha, alpha))
        g = g_.uniform(-1.0, 1.0, size=(n, r, r))
    else:
        raise ValueError(dims)
    return (np.ascontiguousarray(d, dtype=np.float32),
            np.ascontiguousarray(g, dtype=np.float32))


def splitmix64(x):
    """SplitMix64 output function applied to one 64-bit counter value
    (Steele, Lea and Flood, OOPSLA 2014; constants as published there)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_array(x):
    """splitmix64 over a uint64 array (numpy's uint64 arithmetic wraps modulo
    2^64, which is what the published definition asks for)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def sample_counts(n_cand, seed=2, lo=500, hi=2000):
    """Uneven per-candidate sample counts in [lo, hi]: candidate i scores the
    pool prefix [0, n_i) with n_i = lo + splitmix64(seed ^ i) mod (hi-lo+1)."""
    span = hi - lo + 1
    i = np.arange(n_cand, dtype=np.uint64) ^ np.uint64(seed & MASK64)
    return (lo + splitmix64_array(i) % np.uint64(span)).astype(np.int32)


def candidate_grid(n=4096, lo=0.05, hi=20.0):
    """n candidate values of c, log-spaced over [lo, hi] (float64)."""
    return np.exp(np.linspace(np.log(lo), np.log(hi), n))


def linear_grid(lo, hi, step):
    """Evenly spaced grid lo, lo+step, ... <= hi (float64), e.g. the
    [1.1, 2.5] step 1e-3 curve of the paper's Section 6.1."""
    k = int(np.floor((hi - lo) / step + 1e-9)) + 1
    return lo + step * np.arange(k, dtype=np.float64)


# ----------------------------------------------------------------------------
# Surrogate training inputs
# ----------------------------------------------------------------------------
#: tile sizes (m, r) the surrogate is trained on: F(2..8, 3) and F(2..6, 5)
SURROGATE_SIZES = [(m, 3) for m in range(2, 9)] + [(m, 5) for m in range(2, 7)]


def surrogate_pairs(n, seed=5, lo=0.05, hi=20.0):
    """n (c1, c2) pairs, each coordinate log-uniform over [lo, hi]."""
    g = np.random.default_rng(seed)
    u = g.uniform(np.log(lo), np.log(hi), size=(n, 2))
    return np.exp(u)


def surrogate_inputs(sizes, n_per_size, seed=5):
    """Per tile size (m, r) of `sizes` (k-th entry): n_per_size (c1, c2)
    pairs and pool-prefix counts, both keyed on seed * 1000 + k.  Returns
    two dicts keyed by (m, r)."""
    pairs, counts = {}, {}
    for k, s in enumerate(sizes):
        pairs[tuple(s)] = surrogate_pairs(n_per_size, seed=seed * 1000 + k)
        counts[tuple(s)] = sample_counts(n_per_size, seed=seed * 1000 + k)
    return pairs, counts


def mlp_init(widths, seed=7):
    """Initial weights for a fully connected net with the given layer widths.

    Returns a list of (W (out, in), b (out,)) float32 pairs.  W is uniform in
    +-sqrt(6/(in+out)) (Glorot and Bengio, 2010); biases start at zero.
    """
    g = np.random.default_rng(seed)
    params = []
    for fan_in, fan_out in zip(widths[:-1], widths[1:]):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        W = g.uniform(-lim, lim, size=(fan_out, fan_in)).astype(np.float32)
        b = np.zeros(fan_out, dtype=np.float32)
        params.append((W, b))
    return params


def minibatch_order(n, epochs, seed=11):
    """Per-epoch random permutations of range(n), int32, shape (epochs, n)."""
    g = np.random.default_rng(seed)
    return np.stack([g.permutation(n) for _ in range(epochs)]).astype(np.int32)
