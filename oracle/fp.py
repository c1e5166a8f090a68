"""Floating-point Winograd evaluation, direct convolution and error metrics
(oracle).  Test infrastructure only (see the package docstring).

What is computed
----------------
* Transform matrices in float32: each exact entry (rational construction of
  Sections 4.1/4.2) rounded to the nearest float64 and then to the nearest
  float32 (round-to-nearest-even both times).
* Winograd tiles in float32 (the precision the paper scores): 1D
  Y = A^T[(Gg) (.) (B^T d)] (eq. conv_1d) and the nested 2D form
  Y = A^T[(G g G^T) (.) (B^T d B)] A (eq. conv_2d), evaluated as nested
  matrix products, never as a Kronecker product (Section 7 found that worse).
  Every inner product is accumulated in ascending index order, each term
  added with a fused multiply-add (acc <- RN32(m * x + acc), one rounding per
  term, starting from acc = 0).  A 2D product P X P^T is evaluated as (P X)
  first, then (P X) P^T.  (The paper does not state the operation order; this
  is the order every float32 Winograd result here follows.)
* The convolution layer (eq. conv with the channel sum): the image is cut
  into tiles of m x m outputs; the Hadamard products of the transformed
  filters and inputs are summed over the input channels c in ascending
  order, then the output transform is applied (Section 4.1 notes that the
  transforms are amortised and that the channel sum is a matrix product).
* Reduced-precision Hadamard stage: transformed tiles are scaled by powers of
  two per (tile element, channel) and rounded to float16 or bfloat16; the
  products are accumulated in float32.  Power-of-two scaling of one operand
  by 2^-s and of the other by 2^+s leaves every product unchanged.
* Direct convolution in float64 (the reference every error is measured
  against, Section 6) and in float32 with sequential accumulation (the
  "n = 0" rows of the paper's state-of-the-art tables).
* The L1 error of Section 6: absolute differences summed in float64; reported
  both normalised by the number of outputs (mean absolute error) and by the
  L1 norm of the reference (relative L1).
"""
from __future__ import annotations

import math

import numpy as np

from . import toomcook as tc

F32 = np.float32
F64 = np.float64


# ----------------------------------------------------------------------------
# Matrices
# ----------------------------------------------------------------------------
def to_f32(mat):
    """Exact matrix -> float32 array via float64 (both round-to-nearest-even)."""
    return np.array([[np.float32(float(v)) for v in row] for row in mat], dtype=F32)


def mats_f32(points, m, r, modified=True):
    """(A^T, G, B^T) in float32 for ordered points (exact construction first)."""
    AT, G, BT = tc.transforms(points, m, r, modified)
    return to_f32(AT), to_f32(G), to_f32(BT)


# ----------------------------------------------------------------------------
# Fused multiply-add and fixed-order float32 matrix application
# ----------------------------------------------------------------------------
def fma32(a, b, c):
    """Correctly rounded float32 a*b + c (a single rounding, ties to even).

    p = a*b is exact in float64.  s = p + c rounds once in float64, and the
    TwoSum error term e (Knuth) makes p + c = s + e exact.  Rounding s to
    float32 gives the correctly rounded result unless s lies exactly halfway
    between two float32 values and e != 0; then the exact value lies on the
    side of the midpoint that e points to."""
    scalar = np.ndim(a) == 0 and np.ndim(b) == 0 and np.ndim(c) == 0
    a64 = np.atleast_1d(np.asarray(a, dtype=F32)).astype(F64)
    b64 = np.atleast_1d(np.asarray(b, dtype=F32)).astype(F64)
    c64 = np.atleast_1d(np.asarray(c, dtype=F32)).astype(F64)
    p = a64 * b64
    s = p + c64
    bv = s - p
    e = (p - (s - bv)) + (c64 - bv)
    r = s.astype(F32)
    d = s - r.astype(F64)
    toward = np.where(d > 0, np.float32(np.inf), np.float32(-np.inf)).astype(F32)
    nb = np.nextafter(r, toward)
    with np.errstate(invalid="ignore", over="ignore"):
        mid = (d != 0) & (s == (r.astype(F64) + nb.astype(F64)) / 2)
    fix = mid & (e != 0) & (np.sign(e) == np.sign(d))
    r = np.where(fix, nb, r)
    return r[0] if scalar else r


def apply_left(Mat, X, axis):
    """Z[..i..] = sum_l Mat[i,l] X[..l..] along `axis` in float32: ascending l,
    acc <- fma(Mat[i,l], X[l], acc) from acc = 0."""
    Mat = np.asarray(Mat, dtype=F32)
    X = np.moveaxis(np.asarray(X, dtype=F32), axis, 0)
    out = np.empty((Mat.shape[0],) + X.shape[1:], dtype=F32)
    for i in range(Mat.shape[0]):
        acc = np.zeros(X.shape[1:], dtype=F32)
        for l in range(Mat.shape[1]):
            acc = fma32(Mat[i, l], X[l], acc)
        out[i] = acc
    return np.moveaxis(out, 0, axis)


def xform2d(Mat, X):
    """Mat X Mat^T over the last two axes: rows first, then columns."""
    return apply_left(Mat, apply_left(Mat, X, -2), -1)


# ----------------------------------------------------------------------------
# Single tiles (the paper's per-kernel experiments)
# ----------------------------------------------------------------------------
def tile_1d_f32(mats, d, g):
    """float32 1D Winograd on a batch: d (n, alpha), g (n, r) -> (n, m)."""
    AT, G, BT = mats
    u = apply_left(G, g, -1)
    v = apply_left(BT, d, -1)
    return apply_left(AT, u * v, -1)


def tile_2d_f32(mats, d, g):
    """float32 2D Winograd on a batch: d (n, a, a), g (n, r, r) -> (n, m, m)."""
    AT, G, BT = mats
    U = xform2d(G, g)
    V = xform2d(BT, d)
    return xform2d(AT, U * V)


# ----------------------------------------------------------------------------
# Mixed precision (Section 6): float64 transforms, float32 Hadamard product
# ----------------------------------------------------------------------------
def apply_left_f64(Mat, X, axis):
    """Z[..i..] = sum_l Mat[i,l] X[..l..] along `axis` in float64: ascending
    l, acc <- acc + Mat[i,l] * X[l] from acc = 0 (product and sum each
    rounded; no fused multiply-add)."""
    Mat = np.asarray(Mat, dtype=F64)
    X = np.moveaxis(np.asarray(X, dtype=F64), axis, 0)
    out = np.empty((Mat.shape[0],) + X.shape[1:], dtype=F64)
    for i in range(Mat.shape[0]):
        acc = np.zeros(X.shape[1:], dtype=F64)
        for l in range(Mat.shape[1]):
            acc = acc + Mat[i, l] * X[l]
        out[i] = acc
    return np.moveaxis(out, 0, axis)


def xform2d_f64(Mat, X):
    return apply_left_f64(Mat, apply_left_f64(Mat, X, -2), -1)


def tile_1d_mixed(mats64, d, g):
    """Mixed-precision 1D tiles: U = G g and V = B^T d in float64 with the
    float64 matrices, each rounded to float32; their product in float32;
    Y = A^T (U V) in float64, rounded to float32."""
    AT, G, BT = mats64
    U = apply_left_f64(G, g, -1).astype(F32)
    V = apply_left_f64(BT, d, -1).astype(F32)
    return apply_left_f64(AT, (U * V).astype(F64), -1).astype(F32)


def tile_2d_mixed(mats64, d, g):
    """Mixed-precision 2D tiles (as tile_1d_mixed, two-sided products taken
    rows first)."""
    AT, G, BT = mats64
    U = xform2d_f64(G, g).astype(F32)
    V = xform2d_f64(BT, d).astype(F32)
    return xform2d_f64(AT, (U * V).astype(F64)).astype(F32)


def mats_f64(points, m, r, modified=True):
    """(A^T, G, B^T) in float64 for ordered points (exact, then rounded)."""
    AT, G, BT = tc.transforms(points, m, r, modified)
    return tuple(np.array([[float(v) for v in row] for row in M_], dtype=F64) for M_ in (AT, G, BT))


def direct_tile_f64(d, g):
    """Correlation of each tile with its filter in float64 (1D or 2D batch)."""
    d = np.asarray(d, dtype=F64)
    g = np.asarray(g, dtype=F64)
    r = g.shape[-1]
    if d.ndim == 2:
        m = d.shape[1] - r + 1
        y = np.zeros((d.shape[0], m), dtype=F64)
        for k in range(r):
            y += d[:, k:k + m] * g[:, k:k + 1]
        return y
    m = d.shape[1] - r + 1
    y = np.zeros((d.shape[0], m, m), dtype=F64)
    for u in range(r):
        for v in range(r):
            y += d[:, u:u + m, v:v + m] * g[:, u:u + 1, v:v + 1]
    return y


def direct_tile_f32(d, g):
    """Correlation in float32, accumulating the r (1D) or r*r (2D) products
    sequentially in (u, v) order, separately rounded: the direct-convolution
    rows of the paper's Tables 7 and 8."""
    d = np.asarray(d, dtype=F32)
    g = np.asarray(g, dtype=F32)
    r = g.shape[-1]
    m = d.shape[1] - r + 1
    if d.ndim == 2:
        acc = d[:, 0:m] * g[:, 0:1]
        for k in range(1, r):
            acc = acc + d[:, k:k + m] * g[:, k:k + 1]
        return acc
    acc = None
    for u in range(r):
        for v in range(r):
            t = d[:, u:u + m, v:v + m] * g[:, u:u + 1, v:v + 1]
            acc = t if acc is None else acc + t
    return acc


# ----------------------------------------------------------------------------
# Errors
# ----------------------------------------------------------------------------
def l1_errors(y, yref):
    """L1 error of y against the float64 reference (Section 6): returns
    abs_sum = sum|y - yref|, ref_sum = sum|yref| (both float64), rel_l1 and
    mean_abs (abs_sum per output element)."""
    y = np.asarray(y, dtype=F64)
    yref = np.asarray(yref, dtype=F64)
    se = float(np.abs(y - yref).sum())
    sr = float(np.abs(yref).sum())
    n = y.size
    return dict(abs_sum=se, ref_sum=sr, rel_l1=se / sr if sr else math.inf,
                mean_abs=se / n if n else math.nan, count=n)


# ----------------------------------------------------------------------------
# Reduced precision rounding
# ----------------------------------------------------------------------------
def round_f16(x32):
    """float32 -> nearest float16 (ties to even), returned as float32."""
    return np.asarray(x32, dtype=F32).astype(np.float16).astype(F32)


def round_bf16(x32):
    """float32 -> nearest bfloat16 (ties to even), returned as float32: keep
    the upper 16 bits after adding 0x7FFF plus the lowest kept bit."""
    x32 = np.ascontiguousarray(x32, dtype=F32)
    b = x32.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    out = b.astype(np.uint32).view(F32)
    return np.where(np.isnan(x32), x32, out)


def _exp2_of(v):
    """Binary exponent E with v = f * 2^E, 0.5 <= |f| < 1; E(0) = 0."""
    return math.frexp(v)[1] if v != 0.0 else 0


def scale_exponents(mats, w, x_absmax=None):
    """Per (tile element e=(e1,e2), input channel c) power-of-two exponents
    s[e1, e2, c] for the reduced-precision Hadamard stage.

    The transformed input V[e,c] is bounded by |B^T row e1|_1 |B^T row e2|_1
    max|x_c| and the transformed filter U[e,k,c] by |G row e1|_1 |G row e2|_1
    max_k|w[k,c]|.  With E() the binary exponent of such a bound,
      s = floor((E_V - E_U) / 2)
    gives V*2^-s and U*2^+s bounds of equal exponent.  The row norms are summed
    in float64 in ascending order of the float32 matrix entries.  x_absmax
    (per channel) defaults to 1.
    """
    AT, G, BT = mats
    alpha = BT.shape[0]
    C = w.shape[1]

    def rownorm_exps(M):
        out = []
        for i in range(M.shape[0]):
            acc = 0.0
            for l in range(M.shape[1]):
                acc += abs(float(M[i, l]))
            out.append(_exp2_of(acc))
        return out

    eb = rownorm_exps(BT)
    eg = rownorm_exps(G)
    aw = np.abs(np.asarray(w, dtype=F32)).max(axis=(0, 2, 3))
    ax = np.ones(C) if x_absmax is None else np.asarray(x_absmax, dtype=F32)
    s = np.empty((alpha, alpha, C), dtype=np.int64)
    for c in range(C):
        ex = _exp2_of(float(ax[c]))
        ew = _exp2_of(float(aw[c]))
        for e1 in range(alpha):
            for e2 in range(alpha):
                ev = eb[e1] + eb[e2] + ex
                eu = eg[e1] + eg[e2] + ew
                s[e1, e2, c] = (ev - eu) // 2
    return s


# ----------------------------------------------------------------------------
# Convolution layer
# ----------------------------------------------------------------------------
def layer_geometry(H, W, r, m, padding):
    p = tc.pad_amount(r, padding)
    Ho, Wo = H + 2 * p - r + 1, W + 2 * p - r + 1
    Th, Tw = -(-Ho // m), -(-Wo // m)
    return p, Ho, Wo, Th, Tw


def input_tiles(x, m, r, padding, tiles=None):
    """alpha x alpha input windows, shape (P, C, alpha, alpha), for tile index
    p = (n*Th + th)*Tw + tw (all tiles, or the listed ones).  Window of tile
    (th, tw) starts at row th*m - p, column tw*m - p; zeros outside."""
    N, C, H, W = x.shape
    alpha = m + r - 1
    p, Ho, Wo, Th, Tw = layer_geometry(H, W, r, m, padding)
    Hp, Wp = Th * m + r - 1, Tw * m + r - 1
    xp = np.zeros((N, C, max(Hp, p + H), max(Wp, p + W)), dtype=F32)
    xp[:, :, p:p + H, p:p + W] = x
    if tiles is None:
        tiles = np.arange(N * Th * Tw)
    tiles = np.asarray(tiles)
    n = tiles // (Th * Tw)
    th = (tiles // Tw) % Th
    tw = tiles % Tw
    out = np.empty((len(tiles), C, alpha, alpha), dtype=F32)
    for a in range(alpha):
        for b in range(alpha):
            out[:, :, a, b] = xp[n, :, th * m + a, tw * m + b]
    return out


def transformed_operands(x, w, mats, m, padding, dtype="f32", x_absmax=None, tiles=None):
    """U (K, C, a, a) and V (P, C, a, a) as the Hadamard stage consumes them:
    float32, or scaled by 2^(+-s) and rounded to float16/bfloat16; with
    dtype "mixed" (mats in float64) the float64 transforms of Section 6
    rounded to float32."""
    AT, G, BT = mats
    r = G.shape[1]
    d = input_tiles(x, m, r, padding, tiles)
    if dtype == "mixed":
        return (xform2d_f64(G, np.asarray(w, dtype=F32)).astype(F32),
                xform2d_f64(BT, d).astype(F32))
    V = xform2d(BT, d)
    U = xform2d(G, np.asarray(w, dtype=F32))
    if dtype == "f32":
        return U, V
    s = scale_exponents(mats, w, x_absmax)           # (a, a, C)
    sc = np.moveaxis(s, 2, 0)                       # (C, a, a)
    Vs = np.ldexp(V, -sc[None]).astype(F32)
    Us = np.ldexp(U, sc[None]).astype(F32)
    rnd = round_f16 if dtype == "f16" else round_bf16
    return rnd(Us), rnd(Vs)


def hadamard_channel_sum(U, V):
    """M[k, p, e] = sum_c U[k, c, e] V[p, c, e]: float32 products, ascending c."""
    acc = U[:, None, 0] * V[None, :, 0]
    for c in range(1, U.shape[1]):
        acc = acc + U[:, None, c] * V[None, :, c]
    return acc


def winograd_layer_tiles(x, w, mats, m, padding, dtype="f32", x_absmax=None, tiles=None):
    """Output tiles (K, P, m, m) of the float Winograd layer (all tiles or
    the listed tile indices)."""
    AT, G, BT = mats
    U, V = transformed_operands(x, w, mats, m, padding, dtype, x_absmax, tiles)
    Mh = hadamard_channel_sum(U, V)
    if dtype == "mixed":
        return xform2d_f64(AT, Mh).astype(F32)
    return xform2d(AT, Mh)


def assemble_tiles(Y, N, Th, Tw, Ho, Wo):
    """Output tiles (K, P, m, m) -> image layout (N, K, Ho, Wo); the parts of
    edge tiles past the output are discarded."""
    K, P, m, _ = Y.shape
    Y = Y.reshape(K, N, Th, Tw, m, m).transpose(1, 0, 2, 4, 3, 5)
    Y = Y.reshape(N, K, Th * m, Tw * m)
    return np.ascontiguousarray(Y[:, :, :Ho, :Wo])


def winograd_layer(x, w, mats, m, padding, dtype="f32", x_absmax=None):
    """Full float Winograd layer: x (N,C,H,W), w (K,C,r,r) -> y (N,K,Ho,Wo)."""
    N, C, H, W = x.shape
    K, r = w.shape[0], w.shape[2]
    p, Ho, Wo, Th, Tw = layer_geometry(H, W, r, m, padding)
    Y = winograd_layer_tiles(x, w, mats, m, padding, dtype, x_absmax)
    return assemble_tiles(Y, N, Th, Tw, Ho, Wo)


def direct_layer_f64(x, w, padding):
    """float64 direct convolution layer (eq. conv as a zero-padded
    cross-correlation); a float64 tensor contraction per filter tap."""
    x = np.asarray(x, dtype=F64)
    w = np.asarray(w, dtype=F64)
    N, C, H, W = x.shape
    K, r = w.shape[0], w.shape[2]
    p = tc.pad_amount(r, padding)
    Ho, Wo = H + 2 * p - r + 1, W + 2 * p - r + 1
    xp = np.zeros((N, C, H + 2 * p, W + 2 * p), dtype=F64)
    xp[:, :, p:p + H, p:p + W] = x
    y = np.zeros((N, K, Ho, Wo), dtype=F64)
    for u in range(r):
        for v in range(r):
            y += np.einsum("nchw,kc->nkhw", xp[:, :, u:u + Ho, v:v + Wo], w[:, :, u, v],
                           optimize=True)
    return y


def direct_points_f64(x, w, padding, coords):
    """float64 direct convolution at the listed output coordinates
    (rows of (n, k, i, j)), computed one output at a time."""
    x = np.asarray(x, dtype=F64)
    w = np.asarray(w, dtype=F64)
    N, C, H, W = x.shape
    r = w.shape[2]
    p = tc.pad_amount(r, padding)
    out = np.empty(len(coords), dtype=F64)
    for t, (n, k, i, j) in enumerate(coords):
        acc = 0.0
        for u in range(r):
            ii = i + u - p
            if not 0 <= ii < H:
                continue
            for v in range(r):
                jj = j + v - p
                if not 0 <= jj < W:
                    continue
                acc += float(np.dot(x[n, :, ii, jj], w[k, :, u, v]))
        out[t] = acc
    return out
