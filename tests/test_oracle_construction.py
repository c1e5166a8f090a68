"""Pins for the exact construction in the oracle (Sections 4.1, 4.2, 5)."""
import random
from fractions import Fraction as Fr

import pytest
import sympy as sp

from conftest import GOLDEN, read_sections, read_table
from oracle import toomcook as tc


def _sym(expr, syms):
    return sp.sympify(expr, locals=syms)


@pytest.mark.parametrize("name", ["f2_3a", "f2_3b", "f4_3a", "f4_3bcd"])
def test_printed_symbolic_matrices(name):
    """The construction reproduces the matrices the paper prints (symbolic)."""
    sec = read_sections(f"{GOLDEN}/printed_matrices.txt")[name]
    syms = {s: sp.Symbol(s) for s in sec["symbols"].split()}
    pts = [_sym(p, syms) for p in sec["points"].split(",")]
    m, r = int(sec["m"]), int(sec["r"])
    AT, G, BT = tc.transforms(pts, m, r)
    for key, mine in (("BT", BT), ("G", G)):
        printed = [[_sym(v, syms) for v in row.split(",")] for row in sec[key]]
        assert len(printed) == len(mine) and len(printed[0]) == len(mine[0]), key
        for i, row in enumerate(printed):
            for j, v in enumerate(row):
                assert sp.simplify(sp.sympify(mine[i][j]) - v) == 0, (name, key, i, j)
    # A^T is the Vandermonde of the points plus the infinity column e_{m-1}
    for j in range(m):
        for i, a in enumerate(pts):
            assert sp.simplify(sp.sympify(AT[j][i]) - a ** j) == 0
        assert AT[j][m + r - 2] == (1 if j == m - 1 else 0)


def test_classic_f23_up_to_diagonal_scaling():
    """Points {0, 1, -1, inf}: the textbook F(2,3) matrices (Lavin and Gray)
    equal the paper-form construction up to the diagonal rescaling
    B^T -> D1 B^T, G -> D2 G, A^T -> A^T (D1 D2)^-1, which leaves the
    algorithm exact."""
    AT, G, BT = tc.transforms([Fr(0), Fr(1), Fr(-1)], 2, 3)
    classic_BT = [[1, 0, -1, 0], [0, 1, 1, 0], [0, -1, 1, 0], [0, 1, 0, -1]]
    classic_G = [[1, 0, 0], [Fr(1, 2), Fr(1, 2), Fr(1, 2)], [Fr(1, 2), Fr(-1, 2), Fr(1, 2)], [0, 0, 1]]
    classic_AT = [[1, 1, 1, 0], [0, 1, -1, -1]]
    D1 = [-1, 1, 1, -1]
    D2 = [-1, 1, 1, 1]
    for i in range(4):
        assert [D1[i] * v for v in BT[i]] == classic_BT[i]
        assert [D2[i] * v for v in G[i]] == classic_G[i]
    for j in range(2):
        assert [AT[j][i] / (D1[i] * D2[i]) for i in range(4)] == classic_AT[j]
    # and the classic set is itself exact
    assert tc.exactness_defect(classic_AT, classic_G, classic_BT) == 0


def _random_points(rng, n):
    pts = set()
    while len(pts) < n:
        pts.add(Fr(rng.randint(-9, 9), rng.randint(1, 7)))
    out = list(pts)
    rng.shuffle(out)
    return out


@pytest.mark.parametrize("m,r", [(2, 3), (3, 3), (4, 3), (6, 3), (8, 3), (2, 5), (4, 5), (6, 5), (1, 3), (3, 2)])
def test_exactness_identity(m, r):
    """sum_i A^T[j,i] G[i,k] B^T[i,l] = [l = j+k] for random rational points,
    for both the modified (infinity) and the plain construction."""
    rng = random.Random(1000 * m + r)
    alpha = m + r - 1
    for _ in range(3):
        assert tc.exactness_defect(*tc.transforms(_random_points(rng, alpha - 1), m, r)) == 0
        assert tc.exactness_defect(*tc.transforms(_random_points(rng, alpha), m, r, modified=False)) == 0


def test_identity_fails_for_a_planted_mistake():
    """The identity is sharp: dropping the infinity row of B^T breaks it."""
    AT, G, BT = tc.transforms([Fr(0), Fr(1), Fr(-1), Fr(2), Fr(-2)], 4, 3)
    BT[-1] = [0] * len(BT[-1])
    assert tc.exactness_defect(AT, G, BT) != 0


def _rand_rat(rng):
    return Fr(rng.randint(-20, 20), rng.randint(1, 5))


@pytest.mark.parametrize("m,r", [(2, 3), (4, 3), (6, 3), (2, 5), (3, 5)])
def test_exact_tiles_equal_direct(m, r):
    """Exact 1D and 2D Winograd tiles (eq. conv_1d, conv_2d) equal the direct
    correlation, for non-symmetric data (catches transposed operands)."""
    rng = random.Random(7 * m + r)
    alpha = m + r - 1
    AT, G, BT = tc.transforms(_random_points(rng, alpha - 1), m, r)
    d = [_rand_rat(rng) for _ in range(alpha)]
    g = [_rand_rat(rng) for _ in range(r)]
    assert tc.tile_1d(AT, G, BT, d, g) == tc.direct_1d(d, g)
    d2 = [[_rand_rat(rng) for _ in range(alpha)] for _ in range(alpha)]
    g2 = [[_rand_rat(rng) for _ in range(r)] for _ in range(r)]
    assert tc.tile_2d(AT, G, BT, d2, g2) == tc.direct_2d(d2, g2)


@pytest.mark.parametrize("m,padding,H,W", [(2, "same", 7, 5), (4, "same", 9, 6), (4, "valid", 9, 10), (3, "valid", 5, 5)])
def test_exact_layer_equals_direct_layer(m, padding, H, W):
    """Tiling, zero padding and the discarded ragged edge are exact."""
    rng = random.Random(H * 100 + W + m)
    r = 3
    N, C, K = 2, 2, 3
    x = [[[[Fr(rng.randint(-3, 3)) for _ in range(W)] for _ in range(H)] for _ in range(C)] for _ in range(N)]
    w = [[[[Fr(rng.randint(-3, 3)) for _ in range(r)] for _ in range(r)] for _ in range(C)] for _ in range(K)]
    AT, G, BT = tc.transforms(_random_points(rng, m + r - 2), m, r)
    assert tc.winograd_layer(x, w, AT, G, BT, padding) == tc.direct_layer(x, w, padding)


def test_singular_points_rejected():
    with pytest.raises(tc.SingularPoints):
        tc.transforms([Fr(0), Fr(1), Fr(1)], 2, 3)
    with pytest.raises(tc.SingularPoints):
        tc.transforms(tc.family_points(6, Fr(1)), 4, 3)     # c = 1 makes c = 1/c
    with pytest.raises(ValueError):
        tc.transforms([Fr(0), Fr(1)], 2, 3)                  # wrong point count


def test_family_special_cases():
    """{+-c, +-1/c} at c=2 is {+-2, +-1/2}; the alpha=8 family at c=2, d=1 is the
    Barabasz et al. set P8 = {0, -1, 1, 1/2, -1/2, 2, -2} (Table tab:sota_1d)."""
    assert set(tc.family_points(6, 2.0)) == {Fr(0), Fr(2), Fr(-2), Fr(1, 2), Fr(-1, 2)}
    assert set(tc.family_points(8, 2.0, 1.0)) == {Fr(0), Fr(-1), Fr(1), Fr(1, 2), Fr(-1, 2), Fr(2), Fr(-2)}
    assert tc.family_points(4, 3.0) == [Fr(-3), Fr(0), Fr(3)]
    for alpha in range(4, 11):
        pts = tc.family_points(alpha, 1.7, 2.9)
        assert len(pts) == alpha - 1 and len(set(pts)) == alpha - 1


def test_table1_multiplies_per_output():
    """Table tab:block-size: 2D Winograd needs alpha^2 multiplies for m^2 outputs."""
    for row in read_table(f"{GOLDEN}/table1_multiplies.txt"):
        alpha = int(row[0])
        for mcol, vcol in ((1, 2), (3, 4)):
            if row[mcol] == "-":
                continue
            m = int(row[mcol])
            assert round(alpha * alpha / (m * m), 2) == pytest.approx(float(row[vcol]), abs=1e-9)


def test_chebyshev_nodes():
    nodes = tc.chebyshev_nodes(4)
    assert len(nodes) == 4
    import math
    assert nodes[0] == pytest.approx(math.cos(math.pi / 8))
    assert sum(nodes) == pytest.approx(0.0, abs=1e-12)
