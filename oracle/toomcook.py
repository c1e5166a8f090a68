"""Exact Toom-Cook / Winograd construction from a point set (oracle).

Test infrastructure only (see the package docstring).

The paper writes 1D Winograd convolution as Y = A^T [ (G g) (.) (B^T d) ]
(eq. conv_1d, obtained from the Toom-Cook form eq. toom_cook by the matrix
exchange of eq. mat_exch) and the 2D algorithm by nesting it with itself,
Y = A^T [ (G g G^T) (.) (B^T d B) ] A (eq. conv_2d).

Section 4.1 gives the matrices for points a_0..a_{n-1}:
  * A^T is the (transposed) Vandermonde matrix of the points, A^T[j][i] = a_i^j;
  * G is the Vandermonde matrix of the points over the kernel length, with the
    Lagrange normalisation N_i = prod_{j != i} (a_i - a_j) folded into its rows
    (the paper prefers folding it into G rather than into the product);
  * B^T holds the coefficients of the Lagrange numerators
    M_i(x) = M(x) / (x - a_i), M(x) = prod_j (x - a_j).
Section 4.2 gives the modified algorithm used for every experiment: only
alpha-1 finite points are used, and a last row/column for the point at
infinity is appended: A^T gets a last column e_{m-1}, G a last row e_{r-1},
and B^T a last row holding the coefficients of the full product polynomial
M'(x) of the finite points (its last column is e_{alpha-1}).

Reading adopted where the printed general form is garbled: G[i][k] is
a_i^k / N_i (division, not multiplication by N_i, and no column of ones); this
is what the printed examples eq. f2_3a, f2_3b, f4_3a and f4_3d contain.

All functions are generic over the scalar type: they only use +, -, * and /,
so they run on fractions.Fraction (exact rationals) as well as on sympy
symbols (used by the tests to compare with the printed symbolic matrices).
"""
from __future__ import annotations

from fractions import Fraction


# ----------------------------------------------------------------------------
# Polynomials (ascending coefficient lists)
# ----------------------------------------------------------------------------
def poly_from_roots(roots):
    """Coefficients (ascending powers) of prod_{a in roots} (x - a)."""
    coeffs = [1]
    for a in roots:
        nxt = [0] * (len(coeffs) + 1)
        for i, co in enumerate(coeffs):
            nxt[i + 1] = nxt[i + 1] + co       # x * co x^i
            nxt[i] = nxt[i] - a * co           # -a * co x^i
        coeffs = nxt
    return coeffs


def node_normaliser(points, i):
    """N_i = prod_{j != i} (a_i - a_j) (Section 4.1, Lagrange normalisation)."""
    prod = 1
    for j, a in enumerate(points):
        if j != i:
            prod = prod * (points[i] - a)
    return prod


# ----------------------------------------------------------------------------
# Transform matrices
# ----------------------------------------------------------------------------
class SingularPoints(ValueError):
    """Two points coincide, so some N_i is zero and no interpolation exists."""


def transforms(points, m, r, modified=True):
    """Exact A^T (m x alpha), G (alpha x r), B^T (alpha x alpha).

    points: ordered finite points.  With modified=True (the paper's form,
    Section 4.2) there must be alpha-1 = m+r-2 of them and the point at
    infinity is appended last; with modified=False (plain Toom-Cook,
    Section 4.1) there must be alpha = m+r-1 finite points.
    Points are used in the given order; the order only permutes rows/columns.
    Returns lists of lists of the scalar type of the points.
    """
    alpha = m + r - 1
    pts = list(points)
    nf = len(pts)
    if m < 1 or r < 1:
        raise ValueError("m and r must be >= 1")
    if modified and nf != alpha - 1:
        raise ValueError(f"modified form needs {alpha - 1} finite points, got {nf}")
    if not modified and nf != alpha:
        raise ValueError(f"plain form needs {alpha} finite points, got {nf}")

    norms = [node_normaliser(pts, i) for i in range(nf)]
    for nv in norms:
        if nv == 0:
            raise SingularPoints("two interpolation points coincide")

    zero, one = 0, 1
    AT = [[zero] * alpha for _ in range(m)]
    G = [[zero] * r for _ in range(alpha)]
    BT = [[zero] * alpha for _ in range(alpha)]

    for i, a in enumerate(pts):
        # A^T column i: powers a^0 .. a^{m-1}  (0^0 = 1)
        pw = one
        for j in range(m):
            AT[j][i] = pw
            pw = pw * a
        # G row i: a^k / N_i
        pw = one
        for k in range(r):
            G[i][k] = pw / norms[i]
            pw = pw * a
        # B^T row i: coefficients of M_i(x) = prod_{j != i} (x - a_j)
        Mi = poly_from_roots([b for j, b in enumerate(pts) if j != i])
        for l, co in enumerate(Mi):
            BT[i][l] = co

    if modified:
        last = alpha - 1
        AT[m - 1][last] = one            # A^T last column e_{m-1}
        G[last][r - 1] = one             # G last row e_{r-1}
        Mfull = poly_from_roots(pts)     # M'(x), monic of degree alpha-1
        for l, co in enumerate(Mfull):
            BT[last][l] = co             # includes BT[last][last] = 1
    return AT, G, BT


def exactness_defect(AT, G, BT):
    """Max over (j,k,l) of |sum_i AT[j][i] G[i][k] BT[i][l] - [l == j+k]|.

    The Winograd tile computes Y_j = sum_k g_k d_{j+k} for every input iff this
    trilinear identity holds exactly; it is zero for every valid construction.
    """
    m, alpha = len(AT), len(AT[0])
    r = len(G[0])
    worst = 0
    for j in range(m):
        for k in range(r):
            for l in range(alpha):
                s = 0
                for i in range(alpha):
                    s = s + AT[j][i] * G[i][k] * BT[i][l]
                target = 1 if l == j + k else 0
                dv = abs(s - target)
                if dv > worst:
                    worst = dv
    return worst


# ----------------------------------------------------------------------------
# Point families of Section 5 (orders follow the printed matrices)
# ----------------------------------------------------------------------------
def family_points(alpha, c1, c2=None):
    """Finite points (the point at infinity is implicit and last) of the
    one/two-parameter families used for a tile of alpha = m+r-1 points.

    Section 5 proposes {0, inf} plus {-c, c} (eq. ps0) for alpha=4,
    {-1/c, -c, c, 1/c} (eq. ps1) for alpha=6, and the two-parameter set
    {+-c, +-1/c, +-d, +-1/d} (eq. ps2) for alpha=10; smaller and in-between
    sizes take subsets (eq. ps3 and the d-subsets for alpha>6).  One canonical
    subset is used per size here (c2 plays the role of d):
      4: -c, 0, c                    5: 0, -c, c, 1/c
      6: -1/c, -c, 0, c, 1/c         7: alpha-6 set, d
      8: alpha-6 set, -d, d          9: alpha-6 set, -1/d, -d, d
     10: alpha-6 set, -1/d, -d, d, 1/d
    Arguments may be Fractions (exact) or floats (converted exactly).
    """
    c = c1 if isinstance(c1, Fraction) else Fraction(c1)
    if alpha in (4, 5, 6):
        if alpha == 4:
            return [-c, Fraction(0), c]
        if alpha == 5:
            return [Fraction(0), -c, c, 1 / c]
        return [-1 / c, -c, Fraction(0), c, 1 / c]
    if c2 is None:
        raise ValueError("families with alpha > 6 need a second parameter")
    d = c2 if isinstance(c2, Fraction) else Fraction(c2)
    base = [-1 / c, -c, Fraction(0), c, 1 / c]
    extra = {7: [d], 8: [-d, d], 9: [-1 / d, -d, d], 10: [-1 / d, -d, d, 1 / d]}
    if alpha not in extra:
        raise ValueError(f"no family for alpha={alpha}")
    return base + extra[alpha]


def family_points_f64(alpha, c1, c2=None):
    """The family's points as a float64 program holds them: each point of
    family_points rounded to the nearest float64 (ties to even), kept as the
    exact rational it denotes.  -c and c are exact; 1/c and 1/d are the float64
    values nearest to them, which is what a float64 computation of 1/c gives."""
    return [Fraction(float(p)) for p in family_points(alpha, c1, c2)]


def chebyshev_nodes(n):
    """Chebyshev nodes x_k = cos((2k-1) pi / (2n)), k=1..n (Section 2), as
    floats; the comparison family of the paper's network experiments."""
    import math
    return [math.cos((2 * k - 1) * math.pi / (2 * n)) for k in range(1, n + 1)]


# ----------------------------------------------------------------------------
# Exact evaluation (rational arithmetic)
# ----------------------------------------------------------------------------
def matvec(Mat, v):
    return [sum((Mat[i][l] * v[l] for l in range(len(v))), 0) for i in range(len(Mat))]


def matmul(A, B):
    n, k, mcol = len(A), len(B), len(B[0])
    return [[sum((A[i][l] * B[l][j] for l in range(k)), 0) for j in range(mcol)]
            for i in range(n)]


def transpose(A):
    return [list(row) for row in zip(*A)]


def tile_1d(AT, G, BT, d, g):
    """Y = A^T [ (G g) (.) (B^T d) ]  (eq. conv_1d), exact."""
    u = matvec(G, g)
    v = matvec(BT, d)
    return matvec(AT, [a * b for a, b in zip(u, v)])


def tile_2d(AT, G, BT, d, g):
    """Y = A^T [ (G g G^T) (.) (B^T d B) ] A  (eq. conv_2d), exact."""
    U = matmul(matmul(G, g), transpose(G))
    V = matmul(matmul(BT, d), transpose(BT))
    Mh = [[U[i][j] * V[i][j] for j in range(len(U[0]))] for i in range(len(U))]
    return matmul(matmul(AT, Mh), transpose(AT))


def direct_1d(d, g):
    """Correlation y_j = sum_k d_{j+k} g_k, j < len(d)-len(g)+1 (the CNN form
    of eq. conv in one dimension)."""
    r = len(g)
    return [sum((d[j + k] * g[k] for k in range(r)), 0) for j in range(len(d) - r + 1)]


def direct_2d(d, g):
    r = len(g)
    n = len(d) - r + 1
    return [[sum((d[i + u][j + v] * g[u][v] for u in range(r) for v in range(r)), 0)
             for j in range(n)] for i in range(n)]


def pad_amount(r, padding):
    if padding == "same":
        if r % 2 == 0:
            raise ValueError("'same' padding needs an odd kernel size")
        return (r - 1) // 2
    if padding == "valid":
        return 0
    raise ValueError(padding)


def direct_layer(x, w, padding):
    """Exact direct convolution layer (eq. conv, read as a cross-correlation
    with zero padding): y[n][k][i][j] = sum_{c,u,v} x[n][c][i+u-p][j+v-p] w[k][c][u][v].
    x, w are nested lists of exact scalars."""
    N, C, H, W = len(x), len(x[0]), len(x[0][0]), len(x[0][0][0])
    K, r = len(w), len(w[0][0])
    p = pad_amount(r, padding)
    Ho, Wo = H + 2 * p - r + 1, W + 2 * p - r + 1

    def at(n, c, i, j):
        return x[n][c][i][j] if (0 <= i < H and 0 <= j < W) else 0

    return [[[[sum((at(n, c, i + u - p, j + v - p) * w[k][c][u][v]
                    for c in range(C) for u in range(r) for v in range(r)), 0)
               for j in range(Wo)] for i in range(Ho)] for k in range(K)] for n in range(N)]


def winograd_layer(x, w, AT, G, BT, padding):
    """Exact tiled Winograd layer: the same tiling as the float oracle (tiles of
    m x m outputs, stride m, input windows of alpha x alpha starting at
    (t_h m - p, t_w m - p), zeros outside the image, outputs past the edge
    discarded), with every tile computed by the exact eq. conv_2d and the
    Hadamard products summed over channels before the output transform."""
    N, C, H, W = len(x), len(x[0]), len(x[0][0]), len(x[0][0][0])
    K, r = len(w), len(w[0][0])
    m, alpha = len(AT), len(AT[0])
    p = pad_amount(r, padding)
    Ho, Wo = H + 2 * p - r + 1, W + 2 * p - r + 1
    Th, Tw = -(-Ho // m), -(-Wo // m)
    GT, B = transpose(G), transpose(BT)
    A = transpose(AT)

    def at(n, c, i, j):
        return x[n][c][i][j] if (0 <= i < H and 0 <= j < W) else 0

    U = [[matmul(matmul(G, w[k][c]), GT) for c in range(C)] for k in range(K)]
    y = [[[[None] * Wo for _ in range(Ho)] for _ in range(K)] for _ in range(N)]
    for n in range(N):
        for th in range(Th):
            for tw in range(Tw):
                V = []
                for c in range(C):
                    d = [[at(n, c, th * m - p + a, tw * m - p + b) for b in range(alpha)]
                         for a in range(alpha)]
                    V.append(matmul(matmul(BT, d), B))
                for k in range(K):
                    Mh = [[sum((U[k][c][i][j] * V[c][i][j] for c in range(C)), 0)
                           for j in range(alpha)] for i in range(alpha)]
                    Y = matmul(matmul(AT, Mh), A)
                    for i in range(m):
                        for j in range(m):
                            oi, oj = th * m + i, tw * m + j
                            if oi < Ho and oj < Wo:
                                y[n][k][oi][oj] = Y[i][j]
    return y
