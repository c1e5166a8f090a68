"""Pins for the oracle's 16-bit Hadamard stage (float16 / bfloat16 operands,
float32 channel sums), against what the mathematics fixes rather than against
the oracle's own formulas:

* exactness (Section 4.1: the algorithm is exact in exact arithmetic): with
  dyadic points, small-integer data and channel magnitudes spread over many
  binades, every scaled operand is representable in 16 bits, so the 16-bit
  layer must equal the exact direct convolution element by element, whatever
  the per-channel scales are;
* a rigorous forward-error bound: on N(0,1) data at F(4x4,3x3) and
  F(6x6,3x3) every output lies within the propagated bound built from the
  16-bit unit roundoff on the scaled operands, the float32 channel sum
  (Higham's gamma_C) and the float32 transforms;
* the defining properties of the operands: each scaled operand is a value of
  the 16-bit format (checked bitwise / by its significand, not by casting) and
  lies within half an ulp of the float32 transform it rounds;
* the balancing property of the power-of-two scale (the exponent of the
  scaled input bound and of the scaled filter bound differ by less than 4).
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import synth
from oracle import fp
from oracle import toomcook as tc

U32 = 2.0 ** -24
UNIT16 = {"f16": 2.0 ** -11, "bf16": 2.0 ** -8}
# absolute rounding error of the smallest values: half the float16 subnormal
# spacing (2^-24); bfloat16 shares float32's exponent range
TINY16 = {"f16": 2.0 ** -25, "bf16": 2.0 ** -134}

DYADIC = [[Fr(0), Fr(1), Fr(-1)], [Fr(0), Fr(2), Fr(-2)], [Fr(-1, 2), Fr(0), Fr(1, 2)]]


def _gamma(n, u=U32):
    return n * u / (1 - n * u)


def _spread_channels(x, spread):
    """Multiply channel c by 2^(c mod spread - spread//2): channel maxima then
    span several binades, so the per-channel exponents differ."""
    C = x.shape[1]
    f = np.array([2.0 ** (c % spread - spread // 2) for c in range(C)], dtype=np.float32)
    return (x * f[None, :, None, None]).astype(np.float32)


# ----------------------------------------------------------------------------
# exactness on dyadic points
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("pts", DYADIC)
@pytest.mark.parametrize("padding,H,W", [("same", 11, 9), ("valid", 10, 13)])
@pytest.mark.parametrize("with_absmax", [False, True])
def test_16bit_layer_exact_on_dyadic_points(dtype, pts, padding, H, W, with_absmax):
    """F(2x2,3x3) with points whose normalisers are powers of two and
    integer data in [-2, 2] (input channels scaled by 2^-3 .. 2^3, filter
    channels by 2^-1 .. 2^1): U = G g G^T and
    V = B^T d B are short dyadic numbers, exact in float16 and bfloat16 once
    scaled by any power of two in range, the products are exact in float32
    and so are the channel sums, so the 16-bit layer must equal the exact
    direct convolution.  A scale applied to one operand and not undone by
    the other, a transposed operand or a wrong tile index breaks equality."""
    mats = fp.mats_f32(pts, 2, 3)
    x = _spread_channels(synth.exact_small_ints((2, 7, H, W), 3, -2, 2), 7)
    w = _spread_channels(synth.exact_small_ints((5, 7, 3, 3), 4, -2, 2), 3)
    ax = np.abs(x).max(axis=(0, 2, 3)) if with_absmax else None
    s = fp.scale_exponents(mats, w, ax)
    assert (s != s[..., :1]).any()                    # the scales differ between channels
    y = fp.winograd_layer(x, w, mats, 2, padding, dtype, x_absmax=ax)
    exact = tc.direct_layer([[[[Fr(float(v)) for v in row] for row in ch] for ch in im] for im in x],
                            [[[[Fr(float(v)) for v in row] for row in ch] for ch in k] for k in w], padding)
    assert np.array_equal(y.astype(np.float64), np.array(exact, dtype=np.float64))


# ----------------------------------------------------------------------------
# forward-error bound on random data
# ----------------------------------------------------------------------------
def _abs2(P, X):
    """|P| |X| |P|^T over the last two axes, float64."""
    P = np.abs(np.asarray(P, dtype=np.float64))
    return np.einsum("ik,...kl,jl->...ij", P, np.abs(X), P)


def _exact2(P, X):
    P = np.asarray(P, dtype=np.float64)
    return np.einsum("ik,...kl,jl->...ij", P, X, P)


def forward_error_bound(pts, m, x, w, padding, dtype, x_absmax):
    """Elementwise bound on |y16 - y| (y the exact convolution) for output
    tiles (K, P, m, m), propagated step by step:

      |U32 - U| <= eU Ug,  Ug = |G||g||G|^T, eU = 2 gamma_r + gamma_r^2 + eM
      |V32 - V| <= eV Vb,  Vb = |B^T||d||B|, eV = 2 gamma_a + gamma_a^2 + eM
        (gamma_n with u = 2^-24; eM covers the rounding of the exact matrices
        to float32, 2u + u^2 with u slightly above 2^-24 for the double
        rounding)
      |Uh - U| <= dU = u16 (|U| + eU Ug) + eU Ug + tiny16 2^-s    (likewise V, 2^+s)
      |Mh - M| <= dM = sum_c (dU |V| + |U| dV + dU dV)
                       + gamma_C sum_c (|U| + dU)(|V| + dV)
        (16-bit products are exact in float32; the sum over C channels)
      |Yh - y| <= |A^T| dM |A| + eY |A^T| (|M| + dM) |A|,
        eY = 2 gamma_a + gamma_a^2 + eM.
    U, V and M are the exact values (float64 einsums of the exact matrices,
    1e-15 relative; covered by a 1e-12 slack)."""
    AT, G, BT = (np.array([[float(v) for v in row] for row in M_], dtype=np.float64)
                 for M_ in tc.transforms(pts, m, 3))
    a = BT.shape[0]
    u16, tiny = UNIT16[dtype], TINY16[dtype]
    eMat = 2 * (U32 + 2.0 ** -52) + (U32 + 2.0 ** -52) ** 2
    eU = 2 * _gamma(3) + _gamma(3) ** 2 + eMat
    eV = 2 * _gamma(a) + _gamma(a) ** 2 + eMat
    eY = eV
    d = fp.input_tiles(x, m, 3, padding).astype(np.float64)         # (P, C, a, a)
    g = np.asarray(w, dtype=np.float64)                              # (K, C, 3, 3)
    U, V = _exact2(G, g), _exact2(BT, d)
    Ug, Vb = _abs2(G, g), _abs2(BT, d)
    s = np.moveaxis(fp.scale_exponents(fp.mats_f32(pts, m, 3), w, x_absmax), 2, 0)   # (C, a, a)
    dU = u16 * (np.abs(U) + eU * Ug) + eU * Ug + tiny * 2.0 ** (-s)[None]
    dV = u16 * (np.abs(V) + eV * Vb) + eV * Vb + tiny * 2.0 ** s[None]
    K, C, P = g.shape[0], g.shape[1], d.shape[0]

    def csum(A_, B_):                                                # sum_c A[k,c] B[p,c] -> (K, P, a, a)
        return np.einsum("kcij,pcij->kpij", A_, B_)

    M = csum(U, V)
    dM = csum(dU, np.abs(V)) + csum(np.abs(U), dV) + csum(dU, dV) + \
        _gamma(C) * csum(np.abs(U) + dU, np.abs(V) + dV)
    bound = _abs2(AT, dM) + eY * _abs2(AT, np.abs(M) + dM)
    y = _exact2(AT, M)
    return bound * (1 + 1e-12) + 1e-12 * np.abs(y), y


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("alpha,c,C", [(6, 1.622, 4), (6, 2.0, 32), (8, 2.0, 4), (8, 2.0, 32), (8, 1.37, 16)])
def test_16bit_layer_within_forward_error_bound(dtype, alpha, c, C):
    """N(0,1) activations with channel magnitudes over several binades and
    N(0, 1/sqrt(9C)) filters, per-channel input maxima given: every output of
    the oracle's 16-bit layer is within the propagated bound of the exact
    convolution, and the bound is not vacuous (the largest error uses a
    visible part of it)."""
    m = alpha - 2
    pts = tc.family_points(alpha, Fr(c), Fr(1))
    x, w = synth.layer_inputs(1, C, 3, 2 * m + 3, 2 * m + 1, 3, "normal")
    x = _spread_channels(x, 5)
    ax = np.abs(x).max(axis=(0, 2, 3))
    Y = fp.winograd_layer_tiles(x, w, fp.mats_f32(pts, m, 3), m, "same", dtype, x_absmax=ax)
    bound, yx = forward_error_bound(pts, m, x, w, "same", dtype, ax)
    err = np.abs(Y.astype(np.float64) - yx)
    ratio = err / bound
    assert np.all(ratio <= 1.0), ratio.max()
    assert ratio.max() > 1e-3
    # the float32 layer's error is far below the 16-bit one (the 16-bit
    # rounding is really applied)
    Y32 = fp.winograd_layer_tiles(x, w, fp.mats_f32(pts, m, 3), m, "same", "f32")
    assert np.abs(Y32 - yx).mean() * 20 < err.mean()


# ----------------------------------------------------------------------------
# the operands themselves
# ----------------------------------------------------------------------------
def _is_16bit_value(v, dtype):
    """True where v (float32) is a value of the 16-bit format: bfloat16 keeps
    the upper 16 bits of a float32; a float16 value has at most 11
    significant bits at its binade (normal) or is a multiple of 2^-24
    (subnormal), and magnitude at most 65504."""
    v = np.asarray(v, dtype=np.float32)
    if dtype == "bf16":
        return (v.view(np.uint32) & 0xFFFF) == 0
    a = np.abs(v.astype(np.float64))
    _, e = np.frexp(a)                                # a = f 2^e, 0.5 <= f < 1
    step = np.where(a >= 2.0 ** -14, np.ldexp(1.0, e - 11), 2.0 ** -24)
    return (np.mod(a, step) == 0) & (a <= 65504.0)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("alpha,c", [(4, 1.0), (6, 1.622), (8, 2.0), (8, 0.4)])
def test_16bit_operands_are_nearest_values_of_the_scaled_transforms(dtype, alpha, c):
    """Each operand the 16-bit Hadamard stage consumes (the transform times
    its power of two) is a value of the 16-bit format within half an ulp (u16 relative,
    or the subnormal half-spacing) of the scaled float32 transform: round to
    nearest, applied after the scaling."""
    m = alpha - 2
    pts = [Fr(0), Fr(1), Fr(-1)] if alpha == 4 else tc.family_points(alpha, Fr(c), Fr(1))
    x, w = synth.layer_inputs(1, 12, 5, 2 * m + 1, 2 * m + 2, 3, "normal")
    x = _spread_channels(x, 6)
    ax = np.abs(x).max(axis=(0, 2, 3))
    mats = fp.mats_f32(pts, m, 3)
    U32, V32 = fp.transformed_operands(x, w, mats, m, "same", "f32")
    # the operands come scaled: U' = U 2^s, V' = V 2^-s, each rounded
    Us, Vs = fp.transformed_operands(x, w, mats, m, "same", dtype, x_absmax=ax)
    s = np.moveaxis(fp.scale_exponents(mats, w, ax), 2, 0)[None]       # (1, C, a, a)
    assert _is_16bit_value(Us, dtype).all() and _is_16bit_value(Vs, dtype).all()
    for got, ref in ((Us, np.ldexp(U32.astype(np.float64), s)), (Vs, np.ldexp(V32.astype(np.float64), -s))):
        lim = np.maximum(UNIT16[dtype] * np.abs(ref), TINY16[dtype])
        assert np.all(np.abs(got.astype(np.float64) - ref) <= lim)


@pytest.mark.parametrize("alpha,c", [(4, 1.0), (6, 1.622), (8, 2.0), (8, 0.05), (8, 20.0), (10, 1.3)])
def test_scale_balances_the_operand_bounds(alpha, c):
    """Section-6 scaling reading: the power of two moves the bound of the
    transformed input, |B^T row e1|_1 |B^T row e2|_1 max|x_c|, and that of
    the transformed filter, |G row e1|_1 |G row e2|_1 max_k|w_{k,c}|, to the
    same binade up to the rounding of exponents: their base-2 logarithms
    differ by less than 4 after scaling (a wrong sign, a missing channel
    part or a transposed element index breaks this)."""
    m = alpha - 2
    pts = [Fr(0), Fr(1), Fr(-1)] if alpha == 4 else tc.family_points(alpha, Fr(c), Fr(2.7))
    mats = fp.mats_f32(pts, m, 3)
    AT, G, BT = (np.abs(M_.astype(np.float64)) for M_ in mats)
    x, w = synth.layer_inputs(1, 9, 4, 8, 8, 3, "normal")
    x = _spread_channels(x, 9)
    ax = np.abs(x).max(axis=(0, 2, 3)).astype(np.float64)
    aw = np.abs(w).max(axis=(0, 2, 3)).astype(np.float64)
    nb, ng = BT.sum(axis=1), G.sum(axis=1)
    s = fp.scale_exponents(mats, w, ax.astype(np.float32))               # (a, a, C)
    vb = np.log2(nb[:, None, None] * nb[None, :, None] * ax[None, None, :]) - s
    ub = np.log2(ng[:, None, None] * ng[None, :, None] * aw[None, None, :]) + s
    assert np.all(np.abs(vb - ub) < 4.0)
    assert (s != s[..., :1]).any()                                      # depends on the channel
