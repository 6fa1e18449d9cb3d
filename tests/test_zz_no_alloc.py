"""voldor_residual_bins_noalloc (the binning pass with the library's static
device scratch, for callers that cannot allocate) against voldor_residual_bins
with a caller-allocated workspace: the same kernels, so the same bins bit for
bit, on two calls in a row (the second smaller, over the first call's partials
left in the shared array), and sizes beyond the array rejected before any
launch."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vo():
    import paper_2104_06789_amd as m
    m.lib()
    return m


def _pair(torch, n, seed):
    g = torch.Generator().manual_seed(seed)
    X = (torch.randn((n, 2), generator=g) * 12.0).float()
    G = (X + torch.randn((n, 2), generator=g) * 0.4).float()
    X[::97, 0] = float("nan")   # items with a missing component are skipped
    return X.cuda(), G.cuda()


def test_noalloc_matches_workspace_entry_point(vo):
    import torch
    for n, nbins, seed in [(1_500_000, 40, 0), (100_003, 17, 1)]:
        X, G = _pair(torch, n, seed)
        ref = vo.residual_bins(X, G, nbins=nbins, v_max=40.0)
        out = torch.full((nbins, 4), -1.0, dtype=torch.float64, device="cuda")
        vo.residual_bins_noalloc(X, G, out, nbins=nbins, v_max=40.0)
        torch.cuda.synchronize()
        print(n, nbins, float(out[:, 0].sum()), float(ref[:, 0].sum()))
        assert float(out[:, 0].sum()) > 0.9 * n
        assert torch.equal(out, ref)


def test_noalloc_rejects_sizes_beyond_its_scratch(vo):
    import torch
    n, nbins = 600_000, 256          # 293 workgroups x 256 bins x 4 > 262144 doubles
    assert vo.lib().voldor_residual_workspace(n, nbins) > 262144
    X, G = _pair(torch, n, 2)
    out = torch.zeros((nbins, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(vo.VoldorError) as e:
        vo.residual_bins_noalloc(X, G, out, nbins=nbins)
    assert e.value.code == vo.EINVAL
    torch.cuda.synchronize()
    assert torch.count_nonzero(out) == 0
