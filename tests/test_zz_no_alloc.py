"""The allocation-free scoring entry point (static device scratch) against
wg_score_error with a caller workspace, called through the C ABI twice in a
row, the second time with a smaller input."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_noalloc_score_matches_workspace_score_twice():
    from paper_2201_10369_amd import wg
    rng = np.random.default_rng(21)
    for n in (3_000_017, 70_001):
        yref = rng.standard_normal(n)
        y = (yref + rng.standard_normal(n) * 1e-5).astype(np.float32)
        yd, rd = torch.from_numpy(y).cuda(), torch.from_numpy(yref).cuda()
        ref = wg.score_error(yd, rd)
        out = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
        wg.score_error_noalloc(yd, rd, out)
        torch.cuda.synchronize()
        # the same kernels and partial-sum grid: equal bit for bit
        assert torch.equal(out, ref), (n, out.cpu().numpy(), ref.cpu().numpy())
        s = np.abs(y.astype(np.float64) - yref).sum()
        assert out[0].item() == pytest.approx(s, rel=1e-12)
        assert out[1].item() == pytest.approx(np.abs(yref).sum(), rel=1e-12)


def test_noalloc_score_rejects_bad_arguments():
    from paper_2201_10369_amd import wg
    y = torch.zeros(4, dtype=torch.float32, device="cuda")
    r = torch.zeros(4, dtype=torch.float64, device="cuda")
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    lib = wg.lib()
    assert lib.wg_score_error_noalloc(None, wg._tptr(r), 4, wg._tptr(out), None) == -1
    assert lib.wg_score_error_noalloc(wg._tptr(y), wg._tptr(r), 0, wg._tptr(out), None) == -1
