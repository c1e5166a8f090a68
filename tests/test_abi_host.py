"""CPU-only checks of the C ABI: the library loads and exports every declared
symbol; the host-side construction, families, validation and plan layout
agree with the oracle and the documented contract.  No GPU work is launched."""
import ctypes
import math
import os
import re
from fractions import Fraction as Fr

import numpy as np
import pytest

from conftest import ROOT
from oracle import fp
from oracle import toomcook as tc
from paper_2201_10369_amd import wg

HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include")) if f.endswith(".h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[\w\s\*]+?\b(wg_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = wg.lib()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding knows every one of them
    unbound = [n for n in names if n not in wg._SIGS]
    assert not unbound, unbound


def test_version_and_supported():
    assert wg.lib().wg_version() >= 10000
    assert wg.supported(6, 3) and wg.supported(2, 5) and not wg.supported(9, 3) and not wg.supported(4, 4)


def _ulps32(a, b):
    """Distance in float32 units in the last place (+0 and -0 are equal)."""
    def ordinal(v):
        i = np.ascontiguousarray(v, np.float32).view(np.int32).astype(np.int64)
        return np.where(i < 0, -(i & 0x7FFFFFFF), i)
    return np.abs(ordinal(a) - ordinal(b))


@pytest.mark.parametrize("alpha,c1,c2", [(4, 1.054, None), (5, 1.5, None), (6, 1.622, None), (6, 2.0, None),
                                         (7, 2.22, 1.0), (8, 2.0, 1.0), (8, 0.45, 1.0), (9, 1.305, 2.485),
                                         (10, 1.272, 2.099), (10, 19.7, 0.06)])
def test_host_construction_matches_oracle(alpha, c1, c2):
    m = alpha - 2
    pts = wg.family_points(alpha, c1, c2 if c2 is not None else 1.0)
    exact_pts = [Fr(float(p)) for p in pts]                 # the same doubles, exactly
    AT, G, BT = wg.transforms(m, 3, pts)
    ATx, Gx, BTx = tc.transforms(exact_pts, m, 3)
    for mine, ex in ((AT, ATx), (G, Gx), (BT, BTx)):
        # every entry is the exact value rounded once to the nearest float64
        assert np.array_equal(mine, np.array([[float(v) for v in row] for row in ex]))
    AT32, G32, BT32 = wg.transforms(m, 3, pts, f32=True)
    for mine, ref in zip((AT32, G32, BT32), fp.mats_f32(exact_pts, m, 3)):
        assert np.array_equal(mine, ref) and _ulps32(mine, ref).max() == 0


@pytest.mark.parametrize("seed", range(6))
def test_host_construction_random_points(seed):
    """Random points over many binades, both forms, r = 3 and 5."""
    rng = np.random.default_rng(seed)
    for m, r in ((2, 3), (6, 3), (3, 5), (6, 5)):
        for modified in (True, False):
            n = m + r - 2 if modified else m + r - 1
            pts = rng.choice([-1, 1], n) * np.exp(rng.uniform(-6, 6, n))
            AT, G, BT = wg.transforms(m, r, pts, modified)
            ex = tc.transforms([Fr(float(p)) for p in pts], m, r, modified)
            for mine, e in zip((AT, G, BT), ex):
                assert np.array_equal(mine, np.array([[float(v) for v in row] for row in e]))


def test_symmetric_family_gives_exact_zeros():
    """{-1/c, -c, 0, c, 1/c}: the row of B^T for the point 0 is
    [1, 0, -(c^4+1)/c^2, 0, 1, 0] (eq. f4_3a); the odd coefficients cancel
    exactly for any float64 c.  (The constant term is c^2 fl(1/c)^2, which
    rounds to 1 in float32.)"""
    for c in (1.622, 2.71828, 0.3):
        BT = wg.transforms(4, 3, wg.family_points(6, c))[2]
        assert BT[2, 1] == 0.0 and BT[2, 3] == 0.0 and BT[2, 5] == 0.0 and BT[2, 4] == 1.0
        BT32 = wg.transforms(4, 3, wg.family_points(6, c), f32=True)[2]
        assert BT32[2, 0] == 1.0


def test_family_points_match_oracle():
    for alpha in range(4, 11):
        got = wg.family_points(alpha, 1.7, 2.9)
        ref = [float(p) for p in tc.family_points(alpha, 1.7, 2.9)]
        assert np.array_equal(got, np.array(ref))


def test_validation_errors():
    with pytest.raises(wg.WGError) as e:
        wg.transforms(2, 3, [0.0, 1.0, 1.0])
    assert e.value.status == -2                               # WG_ESINGULAR
    with pytest.raises(wg.WGError) as e:
        wg.transforms(2, 3, [0.0, 1.0])
    assert e.value.status == -1                               # WG_EINVAL: wrong point count
    with pytest.raises(wg.WGError) as e:
        wg.transforms(2, 3, [0.0, 1.0, float("nan")])
    assert e.value.status == -1
    with pytest.raises(wg.WGError) as e:
        wg.family_points(11, 2.0)
    assert e.value.status == -1
    pts = wg.family_points(6, 2.0)
    with pytest.raises(wg.WGError) as e:
        wg.Plan(4, 3, pts, 1, 4, 4, 8, 8, dtype="f32", padding="same").__class__(4, 4, pts, 1, 4, 4, 8, 8)
    assert e.value.status == -3                               # WG_EUNSUPPORTED: r = 4
    with pytest.raises(wg.WGError) as e:
        wg.Plan(4, 3, wg.family_points(6, 1.0), 1, 4, 4, 8, 8)
    assert e.value.status == -2                               # c = 1: -c = -1/c
    with pytest.raises(wg.WGError) as e:
        wg.Plan(4, 3, pts, 0, 4, 4, 8, 8)
    assert e.value.status == -1
    with pytest.raises(wg.WGError) as e:
        wg.Plan(4, 3, pts, 1, 4, 4, 2, 2, padding="valid")      # empty output
    assert e.value.status == -1
    assert "empty" in wg.lib().wg_last_error().decode()


def test_plan_layout_contract():
    pts = wg.family_points(8, 2.0, 1.0)
    plan = wg.Plan(6, 3, pts, 64, 256, 256, 28, 28, "same", "f16")
    L = plan.layout
    assert (L["alpha"], L["Hout"], L["Wout"], L["Th"], L["Tw"], L["P"]) == (8, 28, 28, 5, 5, 1600)
    assert L["P_pad"] % 64 == 0 and L["P_pad"] >= 1600 and L["K_pad"] >= 256 and L["C_pad"] >= 256
    assert L["elem_bytes"] == 2 and L["C_pad"] * 2 % 128 == 0
    E = 64
    assert L["scale_offset"] >= E * L["K_pad"] * L["C_pad"] * 2
    assert L["filter_bytes"] >= L["scale_offset"] + E * L["C_pad"] * 4
    assert L["m_offset"] >= E * L["P_pad"] * L["C_pad"] * 2
    assert L["workspace_bytes"] >= L["m_offset"] + E * L["K_pad"] * L["P_pad"] * 4
    # the plan's float32 matrices are the host construction's
    AT, G, BT = plan.matrices()
    AT2, G2, BT2 = wg.transforms(6, 3, pts, f32=True)
    assert np.array_equal(AT, AT2) and np.array_equal(G, G2) and np.array_equal(BT, BT2)
    # ragged valid-padding geometry
    p2 = wg.Plan(4, 3, wg.family_points(6, 1.6), 2, 3, 5, 11, 9, "valid", "f32")
    assert (p2.layout["Hout"], p2.layout["Wout"], p2.layout["Th"], p2.layout["Tw"]) == (9, 7, 3, 2)
    assert p2.layout["C_pad"] % 32 == 0 and p2.layout["pad"] == 0


def test_score_workspace_is_positive():
    assert wg.lib().wg_score_workspace_bytes(1) >= 16
    assert wg.lib().wg_score_workspace_bytes(10 ** 9) <= 1024 * 16


def test_gemm_tiles_knob_validation():
    plan = wg.Plan(6, 3, [0, 1, -1, 2, -2, 0.5, -0.5], 2, 8, 8, 12, 12)
    assert plan.gemm_tiles == 1
    plan.gemm_tiles = 4
    assert plan.gemm_tiles == 4
    for bad in (0, 17, -3):
        with pytest.raises(wg.WGError):
            plan.gemm_tiles = bad
    assert plan.gemm_tiles == 4


def test_gemm_autotune_argument_checks():
    """Argument errors are reported before any device work."""
    L = wg.lib()
    plan = wg.Plan(6, 3, [0, 1, -1, 2, -2, 0.5, -0.5], 2, 8, 8, 12, 12)
    chosen = ctypes.c_int(0)
    fake = ctypes.c_void_p(256)
    assert L.wg_plan_autotune_gemm(None, fake, fake, 1 << 30, 4, ctypes.byref(chosen), None) == -1
    assert L.wg_plan_autotune_gemm(plan.handle, None, fake, 1 << 30, 4, ctypes.byref(chosen), None) == -1
    assert L.wg_plan_autotune_gemm(plan.handle, fake, fake, 1 << 30, 0, ctypes.byref(chosen), None) == -1
    assert L.wg_plan_autotune_gemm(plan.handle, fake, fake, 16, 4, ctypes.byref(chosen), None) == -4
    assert chosen.value == 0 and plan.gemm_tiles == 1


def test_sweep_points_argument_checks():
    L = wg.lib()
    assert L.wg_sweep_run_points(None, None, None, 1, None, None) == -1     # null sweep
    assert L.wg_sweep_autotune(None, None, None, None, 1, None, None) == -1


def test_point_sets_of_the_tables():
    """Comparison sets of Tables tab:sota_1d / tab:sota_2d (P4 ... P10), the
    Chebyshev nodes of Section 2 and the subsets of eq. subset_points."""
    from paper_2201_10369_amd import pointsets as ps
    for dims in (1, 2):
        for alpha in range(4, 11):
            s = ps.comparison_set(alpha, dims)
            assert len(s) == alpha - 1 and len(set(s)) == alpha - 1 and s[:3] == [0.0, -1.0, 1.0]
    assert ps.comparison_set(9, 1) == [0.0, -1.0, 1.0, 0.5, -0.5, 2.0, -2.0, -0.25]
    assert ps.comparison_set(10, 2)[-2:] == [-0.25, 4.0]
    assert ps.comparison_set(6, 1)[-1] == -3.0 and ps.comparison_set(6, 2)[-1] == -2.0
    with pytest.raises(ValueError):
        ps.comparison_set(11, 1)
    for alpha in range(4, 11):
        nodes = ps.chebyshev(alpha)
        ref = tc.chebyshev_nodes(alpha - 1)
        assert len(nodes) == alpha - 1
        for a, b in zip(nodes, ref):
            assert abs(a - b) < 1e-15                       # the oracle's nodes (middle one 6e-17 there)
        if (alpha - 1) % 2 == 1:
            assert nodes[(alpha - 2) // 2] == 0.0
        assert all(abs(a + b) < 1e-15 for a, b in zip(nodes, nodes[::-1]))   # symmetric
    # eq. subset_points for F(4,3) with base {1, -1}: the six pairs of proposed points
    subs = ps.base_subsets(6, [1.0, -1.0])
    assert len(subs) == 6 and ("-1/c", "-c") in subs and ("c", "1/c") in subs
    assert ps.base_subsets(6, []) == [("-1/c", "-c", "c", "1/c")]
    lists = ps.subset_lists([-3.0], ("-1/c", "c", "1/c"), [2.0, 4.0])
    assert lists.tolist() == [[0.0, -3.0, -0.5, 2.0, 0.5], [0.0, -3.0, -0.25, 4.0, 0.25]]
    with pytest.raises(ValueError):
        ps.base_subsets(4, [1.0, -1.0, 3.0])
    fam = ps.family_lists(10, [2.0, 1.5], [3.0, 1.25])
    assert fam.shape == (2, 9) and np.array_equal(fam[0], wg.family_points(10, 2.0, 3.0))


def test_launch_size_limits_are_rejected_before_any_launch():
    """The 32-bit byte-offset limits of the layer kernels (one image of x,
    one row of alpha planes of M, 128 rows of a plane) give WG_EUNSUPPORTED
    from the host checks, before anything is launched.  The buffers are
    placeholders that are never dereferenced; the test is skipped where a GPU
    is present, so a missing check can never launch on them."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("host-only check with placeholder device pointers")
    L = wg.lib()
    fake = ctypes.c_void_p(1 << 40)
    pts = wg.family_points(8, 2.0, 1.0)
    # one image of x: C_pad * H * W * 4 = 2 GiB
    p = wg.Plan(6, 3, pts, 1, 8192, 64, 256, 256, "same", "f16")
    assert L.wg_input_transform(p.handle, fake, fake, fake, p.workspace_bytes, None) == -3
    assert "2 GB" in L.wg_last_error().decode()
    assert L.wg_transform_filters_and_input(p.handle, fake, None, fake, fake, fake, p.workspace_bytes, None) == -3
    # one row of alpha planes of M: alpha * K_pad * P_pad * 4 >= 2 GiB
    p = wg.Plan(6, 3, pts, 16384, 16, 256, 28, 28, "same", "f32")
    assert L.wg_output_transform(p.handle, fake, p.workspace_bytes, fake, None) == -3
    assert "planes of M" in L.wg_last_error().decode()


def test_surrogate_train_rejects_bad_permutations_before_any_gpu_work():
    """surrogate.train checks the minibatch orders on the host: a tensor must
    be contiguous int32 on the GPU, and an array must have shape (epochs, n);
    both are rejected before anything is uploaded or launched."""
    torch = pytest.importorskip("torch")
    from paper_2201_10369_amd import surrogate as sg
    n = 8
    data = {"c1": np.ones(n), "c2": np.ones(n), "m": np.full(n, 4, np.int32), "r": np.full(n, 3, np.int32),
            "target": np.zeros(n, np.float32)}
    with pytest.raises(ValueError, match="int32 on the GPU"):
        sg.train(data, None, torch.zeros((2, n), dtype=torch.int64))
    with pytest.raises(ValueError, match="int32 on the GPU"):
        sg.train(data, None, torch.zeros((2, n), dtype=torch.int32))          # on the host
    with pytest.raises(ValueError, match="shape"):
        sg.train(data, None, np.zeros((2, n + 1), np.int32))
    with pytest.raises(ValueError, match="shape"):
        sg.train(data, None, np.zeros(n, np.int32))
